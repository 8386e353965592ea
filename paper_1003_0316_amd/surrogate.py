"""Learned correction for the unoccupied bands above a cutoff: loading the
trained perceptron and marshalling the library's learned polarization call.
Every arithmetic step runs in libgw (gw_polarization_learned):
  1. P_ret  = the explicit sum over unoccupied bands [0, cut)
  2. X      = features of P_ret, band energies, frequencies;  Y = perceptron(X)
             (column 0: y = log(d_I / |P_ret,II|))
  3. judge  = the left-out bands [cut, n_unocc) projected explicitly for a
              sample of occupied bands spread over the occupied range; the
              predicted and the sampled left-out trace are compared
  4. P      = P_ret + D P_ret D if the judge passes, otherwise the explicit
              sum over the left-out bands is added (fallback; P is then the
              full-band result).
predict() and apply() expose steps 2 and 4 alone (training, ablations).
"""
from __future__ import annotations

import os
from typing import Optional, Sequence

import numpy as np
import torch

from . import binding as gw

N_IN, WIDTH, N_OUT = 32, 256, 32
DEFAULT_MODEL = os.path.join(os.path.dirname(os.path.abspath(__file__)), "surrogate_model.npz")


class Surrogate:
    def __init__(self, mlp: gw.Mlp, judge_tol: float = 0.25, meta: Optional[dict] = None):
        self.mlp = mlp
        self.judge_tol = judge_tol
        self.meta = meta or {}
        self._buf = {}

    # ------------------------------------------------------------- persistence
    @classmethod
    def load(cls, path: str, device, judge_tol: float = 0.25) -> "Surrogate":
        with np.load(path, allow_pickle=False) as z:
            master = z["master"]
            dims = [int(x) for x in z["dims"]]
            meta = {k: z[k].tolist() for k in z.files if k not in ("master", "dims")}
        mlp = gw.Mlp(*dims, device=device, master=master, train=False)
        return cls(mlp, judge_tol, meta)

    @classmethod
    def load_default(cls, device, judge_tol: float = 0.25) -> "Surrogate":
        if not os.path.exists(DEFAULT_MODEL):
            raise FileNotFoundError(f"no trained surrogate at {DEFAULT_MODEL}")
        return cls.load(DEFAULT_MODEL, device, judge_tol)

    @staticmethod
    def save(mlp: gw.Mlp, path: str, **meta) -> None:
        np.savez(path, master=mlp.master.cpu().numpy(), dims=np.array([mlp.n_in, mlp.width, mlp.n_out]),
                 **{k: np.asarray(v) for k, v in meta.items()})

    # -------------------------------------------------------------- inference
    def _tensor(self, name, shape, dtype, device):
        t = self._buf.get(name)
        if t is None or tuple(t.shape) != tuple(shape) or t.device != device:
            t = torch.empty(shape, dtype=dtype, device=device)
            self._buf[name] = t
        return t

    def predict(self, P_ret: torch.Tensor, eps_dev: torch.Tensor, omega, n_occ: int, cut: int, kq=None):
        """Y [n_omega*N][n_out] (column 0 is y) and the marshalled descriptor."""
        args = gw.SurrogateArgs(P_ret, eps_dev, omega, n_occ, cut, kq, n_in=self.mlp.n_in)
        rows = P_ret.shape[0] * P_ret.shape[1]
        X = self._tensor("X", (rows, self.mlp.n_in), torch.float32, P_ret.device)
        Y = self._tensor("Y", (rows, self.mlp.n_out), torch.float32, P_ret.device)
        act = self._tensor("act", (rows, 4 * self.mlp.width), torch.float32, P_ret.device)
        gw.gw_surrogate_features(args, X)
        self.mlp.forward(X, Y, act)
        return Y, args

    def apply(self, P: torch.Tensor, eps_dev: torch.Tensor, omega, n_occ: int, cut: int, kq=None):
        """P <- P + D P D in place (P holds the explicit sum to the cutoff)."""
        Y, _ = self.predict(P, eps_dev, omega, n_occ, cut, kq)
        gw.gw_surrogate_apply(P, Y, self.mlp.n_out)
        return Y

    def learned_call(self, U, psi, eps_host, eps_dev, omega, n_occ: int, cut: int, kq=None, *,
                     precision="split_bf16", P=None, n_sample_occ: int = 2, judge: bool = True,
                     flags: int = 0) -> gw.LearnedCall:
        """The marshalled library call for P over all bands with the bands
        above `cut` replaced by the correction (judged, with fallback)."""
        pol = gw.PolarizationCall(U, psi, eps_host, omega, n_occ, precision=precision, eps_dev=eps_dev, P=P, kq=kq,
                                  flags=flags)
        return gw.LearnedCall(pol, self.mlp, cut, judge=judge, n_sample_occ=n_sample_occ, judge_tol=self.judge_tol)
