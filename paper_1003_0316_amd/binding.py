"""Thin Python binding of libgw (ctypes).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.  PyTorch provides
device memory and the stream.

Functions carry the C names: gw_project, gw_polarization, gw_screen, ...
If the shared library is missing this module raises on import -- there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgw.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libgw.so not found at {LIB_PATH}; build it with "
                      f"`python -m paper_1003_0316_amd.build` (no CPU fallback exists)")
_lib = ctypes.CDLL(LIB_PATH)

GW_FP64, GW_FP32, GW_SPLIT_BF16, GW_SPLIT_FP16, GW_FP16 = 0, 1, 2, 3, 4
PRECISIONS = {"fp64": GW_FP64, "fp32": GW_FP32, "split_bf16": GW_SPLIT_BF16, "split_fp16": GW_SPLIT_FP16,
              "fp16": GW_FP16}
STATUS = {0: "GW_OK", -1: "GW_ERR_INVALID_ARG", -2: "GW_ERR_UNSUPPORTED", -3: "GW_ERR_WORKSPACE",
          -4: "GW_ERR_HIP", -5: "GW_ERR_NONFINITE", -6: "GW_ERR_NOT_HPD"}
GW_CHECK_FINITE, GW_CHECK_HPD = 1, 2


class GwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class GwPolDesc(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int), ("n_k", ctypes.c_int), ("N", ctypes.c_int), ("R", ctypes.c_int),
        ("n_occ", ctypes.c_int), ("n_unocc", ctypes.c_int),
        ("occ_begin", ctypes.c_int), ("occ_end", ctypes.c_int),
        ("unocc_begin", ctypes.c_int), ("unocc_end", ctypes.c_int),
        ("n_omega", ctypes.c_int),
        ("omega_host", ctypes.POINTER(ctypes.c_double)),
        ("kq_host", ctypes.POINTER(ctypes.c_int)),
        ("k_list_host", ctypes.POINTER(ctypes.c_int)),
        ("n_k_list", ctypes.c_int),
        ("U", ctypes.c_void_p), ("psi", ctypes.c_void_p),
        ("eps", ctypes.c_void_p), ("eps_host", ctypes.POINTER(ctypes.c_double)),
        ("P", ctypes.c_void_p),
        ("accumulate", ctypes.c_int), ("chunk_pairs", ctypes.c_int),
        ("real_inputs", ctypes.c_int),
        ("n_nodes", ctypes.c_int), ("nodes_host", ctypes.POINTER(ctypes.c_double)),
        ("flags", ctypes.c_int),
    ]


class GwSigmaDesc(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int), ("n_k", ctypes.c_int), ("N", ctypes.c_int), ("R", ctypes.c_int),
        ("n_bands", ctypes.c_int),
        ("n_mesh", ctypes.c_int), ("mesh_host", ctypes.POINTER(ctypes.c_double)),
        ("n_out", ctypes.c_int), ("omega_out_host", ctypes.POINTER(ctypes.c_double)),
        ("n_states", ctypes.c_int),
        ("state_set_host", ctypes.POINTER(ctypes.c_int)), ("state_band_host", ctypes.POINTER(ctypes.c_int)),
        ("mu", ctypes.c_double),
        ("U", ctypes.c_void_p), ("psi", ctypes.c_void_p),
        ("eps", ctypes.c_void_p), ("eps_host", ctypes.POINTER(ctypes.c_double)),
        ("W_host", ctypes.POINTER(ctypes.c_void_p)), ("v", ctypes.c_void_p),
        ("sigma", ctypes.c_void_p),
    ]


_sz = ctypes.c_size_t
_vp = ctypes.c_void_p
_ci = ctypes.c_int
_lib.gw_last_error.restype = ctypes.c_char_p
_lib.gw_version.restype = _ci
_lib.gw_project_workspace_size.argtypes = [_ci, _ci, _ci, _ci, _ci, ctypes.POINTER(_sz)]
_lib.gw_project.argtypes = [_vp, _ci, _ci, _ci, _ci, _ci, _vp, _vp, _vp, _vp, _vp, _sz]
_lib.gw_polarization_workspace_size.argtypes = [ctypes.POINTER(GwPolDesc), ctypes.POINTER(_sz)]
_lib.gw_polarization.argtypes = [_vp, ctypes.POINTER(GwPolDesc), _vp, _sz]
_lib.gw_screen_workspace_size.argtypes = [_ci, _ci, ctypes.POINTER(_sz)]
_lib.gw_screen.argtypes = [_vp, _ci, _ci, _vp, _vp, _vp, _vp, _vp, _sz]
_lib.gw_screen_ex.argtypes = [_vp, _ci, _ci, _vp, _vp, _vp, _vp, _ci, _vp, _sz]
_lib.gw_screen_noalloc.argtypes = [_vp, _ci, _ci, _vp, _vp, _vp, _vp]
_lib.gw_screen_noalloc_max_bytes.restype = _sz
_lib.gw_screen_noalloc_max_bytes.argtypes = []

class GwMlp(ctypes.Structure):
    _fields_ = [("n_in", ctypes.c_int), ("width", ctypes.c_int), ("n_out", ctypes.c_int),
                ("master", ctypes.c_void_p), ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p),
                ("wt", ctypes.c_void_p), ("wk", ctypes.c_void_p)]


class GwSurrDesc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("n_omega", ctypes.c_int), ("omega_host", ctypes.POINTER(ctypes.c_double)),
                ("n_k", ctypes.c_int), ("n_occ", ctypes.c_int), ("n_unocc", ctypes.c_int), ("cut", ctypes.c_int),
                ("kq_host", ctypes.POINTER(ctypes.c_int)), ("eps", ctypes.c_void_p), ("P_ret", ctypes.c_void_p),
                ("n_in", ctypes.c_int)]


class GwLearnedDesc(ctypes.Structure):
    _fields_ = [("mlp", ctypes.POINTER(GwMlp)), ("cut", ctypes.c_int), ("judge", ctypes.c_int),
                ("n_sample_occ", ctypes.c_int), ("judge_tol", ctypes.c_double),
                ("judge_err_host", ctypes.POINTER(ctypes.c_double)), ("used_fallback_host", ctypes.POINTER(ctypes.c_int))]


_pm = ctypes.POINTER(GwMlp)
_ps = ctypes.POINTER(GwSurrDesc)
_f = ctypes.c_float
_lib.gw_mlp_sizes.argtypes = [_ci, _ci, _ci, ctypes.POINTER(_sz), ctypes.POINTER(_sz)]
_lib.gw_mlp_sync_bf16.argtypes = [_vp, _pm]
_lib.gw_mlp_forward.argtypes = [_vp, _pm, _vp, _ci, _vp, _vp]
_lib.gw_mlp_loss.argtypes = [_vp, _ci, _ci, _ci, _vp, _vp, _vp, _vp, _vp]
_lib.gw_mlp_workspace_size.argtypes = [_ci, _ci, ctypes.POINTER(_sz)]
_lib.gw_mlp_backward.argtypes = [_vp, _pm, _vp, _vp, _vp, _ci, _vp, _vp, _vp, _sz]
_lib.gw_mlp_adam_step.argtypes = [_vp, _pm, _vp, _f, _f, _f, _f, _ci]
_lib.gw_surrogate_workspace_size.argtypes = [_ps, ctypes.POINTER(_sz)]
_lib.gw_surrogate_features.argtypes = [_vp, _ps, _vp, _vp, _sz]
_lib.gw_surrogate_targets.argtypes = [_vp, _ci, _ci, _vp, _vp, _vp, _vp]
_lib.gw_surrogate_apply.argtypes = [_vp, _ci, _ci, _vp, _ci, _vp]
_lib.gw_surrogate_judge.argtypes = [_vp, _ps, _vp, _ci, _vp, _ci, ctypes.POINTER(_ci), ctypes.POINTER(_ci), _vp, _vp,
                                    _sz]

_pl = ctypes.POINTER(GwLearnedDesc)
_lib.gw_polarization_learned_workspace_size.argtypes = [ctypes.POINTER(GwPolDesc), _pl, ctypes.POINTER(_sz)]
_lib.gw_polarization_learned.argtypes = [_vp, ctypes.POINTER(GwPolDesc), _pl, _vp, _sz]

_lib.gw_set_tuning.argtypes = [ctypes.c_char_p, _ci]
_lib.gw_get_tuning.argtypes = [ctypes.c_char_p, ctypes.POINTER(_ci)]
_lib.gw_profile_enable.argtypes = [_ci]
_lib.gw_profile_reset.argtypes = []
_lib.gw_profile_query.argtypes = [ctypes.c_char_p, ctypes.POINTER(_ci), ctypes.POINTER(ctypes.c_double)]

_lib.gw_sigma_c_workspace_size.argtypes = [ctypes.POINTER(GwSigmaDesc), ctypes.POINTER(_sz)]
_lib.gw_sigma_c.argtypes = [_vp, ctypes.POINTER(GwSigmaDesc), _vp, _sz]

_lib.gw_basis_select_count.argtypes = [_ci, ctypes.POINTER(ctypes.c_double), ctypes.c_double, ctypes.POINTER(_ci)]
_lib.gw_basis_select.argtypes = [_vp, _ci, _ci, _ci, _vp, _vp, ctypes.c_double, _ci, _vp, _vp, _vp]

EXPORTED = ("gw_last_error", "gw_version", "gw_project_workspace_size", "gw_project",
            "gw_polarization_workspace_size", "gw_polarization", "gw_screen_workspace_size", "gw_screen",
            "gw_screen_noalloc_max_bytes", "gw_screen_noalloc", "gw_screen_ex",
            "gw_polarization_learned_workspace_size", "gw_polarization_learned",
            "gw_profile_enable", "gw_profile_reset", "gw_profile_query",
            "gw_mlp_sizes", "gw_mlp_sync_bf16", "gw_mlp_forward", "gw_mlp_loss", "gw_mlp_workspace_size",
            "gw_mlp_backward", "gw_mlp_adam_step", "gw_surrogate_workspace_size", "gw_surrogate_features",
            "gw_surrogate_targets", "gw_surrogate_apply", "gw_surrogate_judge", "gw_set_tuning", "gw_get_tuning",
            "gw_sigma_c_workspace_size", "gw_sigma_c", "gw_basis_select_count", "gw_basis_select")


def lib():
    return _lib


def _check(status: int) -> None:
    if status != 0:
        raise GwError(status, _lib.gw_last_error().decode())


def gw_last_error() -> str:
    return _lib.gw_last_error().decode()


def gw_version() -> int:
    return _lib.gw_version()


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _cdtype(prec: int):
    return torch.complex128 if prec == GW_FP64 else torch.complex64


def _dev_tensor(t: torch.Tensor, name: str, dtype=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


_ws_cache: dict = {}


def workspace(nbytes: int, device, tag: str = "default") -> torch.Tensor:
    """A cached device byte buffer of at least nbytes (per device, stream tag)."""
    key = (str(device), tag)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        _ws_cache.pop(key, None)
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def gw_project_workspace_size(precision, N, R, n_occ, n_unocc) -> int:
    out = _sz(0)
    _check(_lib.gw_project_workspace_size(_prec(precision), N, R, n_occ, n_unocc, ctypes.byref(out)))
    return out.value


def gw_project(U: torch.Tensor, psi_occ: torch.Tensor, psi_unocc: torch.Tensor, precision="fp64",
               M: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """M[I, n*n_unocc + n'] = sum_r U[I,r] conj(psi_occ[n,r]) psi_unocc[n',r]."""
    prec = _prec(precision)
    dt = _cdtype(prec)
    _dev_tensor(U, "U", dt)
    _dev_tensor(psi_occ, "psi_occ", dt)
    _dev_tensor(psi_unocc, "psi_unocc", dt)
    N, R = U.shape
    n_occ, n_unocc = psi_occ.shape[0], psi_unocc.shape[0]
    if psi_occ.shape[1] != R or psi_unocc.shape[1] != R:
        raise ValueError("grid sizes differ")
    if M is None:
        M = torch.empty((N, n_occ * n_unocc), dtype=dt, device=U.device)
    _dev_tensor(M, "M", dt)
    if tuple(M.shape) != (N, n_occ * n_unocc):
        raise ValueError("M has the wrong shape")
    nbytes = gw_project_workspace_size(prec, N, R, n_occ, n_unocc)
    ws = workspace(nbytes, U.device, "project") if nbytes else None
    _check(_lib.gw_project(_stream(stream), prec, N, R, n_occ, n_unocc, U.data_ptr(), psi_occ.data_ptr(),
                           psi_unocc.data_ptr(), M.data_ptr(), ws.data_ptr() if ws is not None else None,
                           ws.numel() if ws is not None else 0))
    return M


class PolarizationCall:
    """Marshalled arguments of one gw_polarization call (keeps host arrays alive)."""

    def __init__(self, U, psi, eps_host, omega, n_occ, *, precision="fp64", eps_dev=None, P=None,
                 k_list=None, kq=None, occ_range=None, unocc_range=None, accumulate=False, chunk_pairs=0,
                 real=False, nodes=None, flags=0):
        prec = _prec(precision)
        dt = torch.float32 if real else _cdtype(prec)
        _dev_tensor(U, "U", dt)
        _dev_tensor(psi, "psi", dt)
        N, R = U.shape
        n_k, nb = psi.shape[0], psi.shape[1]
        if psi.shape[2] != R:
            raise ValueError("psi grid size differs from U")
        n_unocc = nb - n_occ
        self.eps_host = np.ascontiguousarray(eps_host, dtype=np.float64)
        if self.eps_host.shape != (n_k, nb):
            raise ValueError(f"eps must be [{n_k}][{nb}]")
        self.eps_dev = eps_dev if eps_dev is not None else torch.from_numpy(self.eps_host).to(U.device)
        _dev_tensor(self.eps_dev, "eps_dev", torch.float64)
        self.omega = np.ascontiguousarray(omega, dtype=np.float64)
        n_om = self.omega.shape[0]
        if P is None:
            P = torch.empty((n_om, N, N), dtype=torch.complex128, device=U.device)
        _dev_tensor(P, "P", torch.complex128)
        if tuple(P.shape) != (n_om, N, N):
            raise ValueError("P has the wrong shape")
        self.P = P
        self.kq = None if kq is None else np.ascontiguousarray(kq, dtype=np.int32)
        self.k_list = None if k_list is None else np.ascontiguousarray(k_list, dtype=np.int32)
        o0, o1 = (0, n_occ) if occ_range is None else occ_range
        u0, u1 = (0, n_unocc) if unocc_range is None else unocc_range
        self.tensors = (U, psi)
        d = GwPolDesc()
        d.precision, d.n_k, d.N, d.R = prec, n_k, N, R
        d.n_occ, d.n_unocc = n_occ, n_unocc
        d.occ_begin, d.occ_end, d.unocc_begin, d.unocc_end = o0, o1, u0, u1
        d.n_omega = n_om
        d.omega_host = self.omega.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.kq_host = self.kq.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if self.kq is not None else None
        if self.k_list is not None:
            d.k_list_host = self.k_list.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
            d.n_k_list = int(self.k_list.shape[0])
        else:
            d.k_list_host = None
            d.n_k_list = 0
        d.U, d.psi = U.data_ptr(), psi.data_ptr()
        d.eps = self.eps_dev.data_ptr()
        d.eps_host = self.eps_host.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.P = P.data_ptr()
        d.accumulate = 1 if accumulate else 0
        d.chunk_pairs = int(chunk_pairs)
        d.real_inputs = 1 if real else 0
        self.nodes = None if nodes is None else np.ascontiguousarray(nodes, dtype=np.float64)
        if self.nodes is not None:
            d.n_nodes = int(self.nodes.shape[0])
            d.nodes_host = self.nodes.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        else:
            d.n_nodes = 0
            d.nodes_host = None
        d.flags = int(flags)
        self.desc = d

    def workspace_size(self) -> int:
        out = _sz(0)
        _check(_lib.gw_polarization_workspace_size(ctypes.byref(self.desc), ctypes.byref(out)))
        return out.value

    def run(self, ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        nbytes = self.workspace_size()
        if ws is None:
            ws = workspace(nbytes, self.P.device, "polarization")
        _check(_lib.gw_polarization(_stream(stream), ctypes.byref(self.desc), ws.data_ptr(), ws.numel()))
        return self.P


def gw_polarization(U, psi, eps_host, omega, n_occ, **kw) -> torch.Tensor:
    """P[j] = sum_k sum_{n occ} sum_{n' unocc} w M M^H (see gw.h); with
    nodes=[...] the spectral route on those transition-energy nodes.  Returns P
    (complex128 [n_omega][N][N]); the work is enqueued on the current stream."""
    ws = kw.pop("ws", None)
    stream = kw.pop("stream", None)
    return PolarizationCall(U, psi, eps_host, omega, n_occ, **kw).run(ws, stream)


def gw_polarization_workspace_size(U, psi, eps_host, omega, n_occ, **kw) -> int:
    return PolarizationCall(U, psi, eps_host, omega, n_occ, **kw).workspace_size()


class LearnedCall:
    """Marshalled arguments of one gw_polarization_learned call: the explicit
    sum to the cutoff, the learned correction for the bands above it, the
    judge and the fallback, in the library (see gw.h)."""

    def __init__(self, pol: PolarizationCall, mlp, cut: int, *, judge: bool = True, n_sample_occ: int = 2,
                 judge_tol: float = 0.25):
        self.pol = pol
        self.mlp = mlp
        n_om = pol.desc.n_omega
        self.err = np.zeros(n_om, dtype=np.float64)
        self.fb = ctypes.c_int(0)
        l = GwLearnedDesc()
        l.mlp = ctypes.pointer(mlp.desc)
        l.cut = int(cut)
        l.judge = 1 if judge else 0
        l.n_sample_occ = int(n_sample_occ)
        l.judge_tol = float(judge_tol)
        l.judge_err_host = self.err.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        l.used_fallback_host = ctypes.pointer(self.fb)
        self.desc = l

    def workspace_size(self) -> int:
        out = _sz(0)
        _check(_lib.gw_polarization_learned_workspace_size(ctypes.byref(self.pol.desc), ctypes.byref(self.desc),
                                                           ctypes.byref(out)))
        return out.value

    def run(self, ws: Optional[torch.Tensor] = None, stream=None):
        """Returns (P, report); report has judge_err (per frequency, judged
        calls) and used_fallback."""
        nbytes = self.workspace_size()
        if ws is None:
            ws = workspace(nbytes, self.pol.P.device, "learned")
        _check(_lib.gw_polarization_learned(_stream(stream), ctypes.byref(self.pol.desc), ctypes.byref(self.desc),
                                            ws.data_ptr(), ws.numel()))
        rep = {"used_fallback": bool(self.fb.value)}
        if self.desc.judge:
            rep["judge_err"] = self.err.tolist()
            rep["judge_err_max"] = float(self.err.max())
        return self.pol.P, rep


def gw_screen_workspace_size(N: int, n_omega: int) -> int:
    out = _sz(0)
    _check(_lib.gw_screen_workspace_size(N, n_omega, ctypes.byref(out)))
    return out.value


def gw_screen(P: torch.Tensor, v: torch.Tensor, W: Optional[torch.Tensor] = None, info=None, stream=None,
              flags: int = 0):
    """W[j] = (1 - diag(v) P[j])^-1 diag(v) in FP64.  Returns (W, info) with
    info an int32 device tensor (0 = ok, c+1 = pivot failure at column c).
    flags: GW_CHECK_FINITE / GW_CHECK_HPD (gw_screen_ex)."""
    _dev_tensor(P, "P", torch.complex128)
    _dev_tensor(v, "v", torch.float64)
    n_om, N = P.shape[0], P.shape[1]
    if W is None:
        W = torch.empty_like(P)
    _dev_tensor(W, "W", torch.complex128)
    if info is None:
        info = torch.empty(n_om, dtype=torch.int32, device=P.device)
    nbytes = gw_screen_workspace_size(N, n_om)
    ws = workspace(nbytes, P.device, "screen")
    _check(_lib.gw_screen_ex(_stream(stream), N, n_om, P.data_ptr(), v.data_ptr(), W.data_ptr(), info.data_ptr(),
                             int(flags), ws.data_ptr(), ws.numel()))
    return W, info


def gw_screen_noalloc_max_bytes() -> int:
    return int(_lib.gw_screen_noalloc_max_bytes())


def gw_screen_noalloc(P: torch.Tensor, v: torch.Tensor, W: torch.Tensor, info: torch.Tensor, stream=None):
    """gw_screen on the library's fixed scratch array (no workspace, no
    allocation in the call): W and info must be given."""
    _dev_tensor(P, "P", torch.complex128)
    _dev_tensor(v, "v", torch.float64)
    _dev_tensor(W, "W", torch.complex128)
    _dev_tensor(info, "info", torch.int32)
    n_om, N = P.shape[0], P.shape[1]
    _check(_lib.gw_screen_noalloc(_stream(stream), N, n_om, P.data_ptr(), v.data_ptr(), W.data_ptr(),
                                  info.data_ptr()))
    return W, info


def gw_profile_enable(on: bool = True) -> None:
    _check(_lib.gw_profile_enable(1 if on else 0))


def gw_profile_reset() -> None:
    _check(_lib.gw_profile_reset())


def gw_profile_query(kernel: str):
    """(launches, total_ms) of the recorded launches of `kernel` (synchronises)."""
    n = ctypes.c_int(0)
    ms = ctypes.c_double(0.0)
    _check(_lib.gw_profile_query(kernel.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


# ------------------------------------------------------------------ perceptron

def gw_mlp_sizes(n_in: int, width: int, n_out: int):
    a, b = _sz(0), _sz(0)
    _check(_lib.gw_mlp_sizes(n_in, width, n_out, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


class Mlp:
    """Device-resident parameters of the 3-layer perceptron (see gw.h)."""

    def __init__(self, n_in: int, width: int, n_out: int, device, master: Optional[np.ndarray] = None,
                 train: bool = True):
        self.n_in, self.width, self.n_out = n_in, width, n_out
        n_p, n_b = gw_mlp_sizes(n_in, width, n_out)
        self.device = torch.device(device)
        self.master = torch.zeros(n_p, dtype=torch.float32, device=self.device)
        if master is not None:
            if master.size != n_p:
                raise ValueError(f"master has {master.size} values, expected {n_p}")
            self.master.copy_(torch.from_numpy(np.ascontiguousarray(master, dtype=np.float32)))
        self.adam_m = torch.zeros_like(self.master) if train else None
        self.adam_v = torch.zeros_like(self.master) if train else None
        self.wt = torch.zeros(n_b, dtype=torch.int16, device=self.device)
        self.wk = torch.zeros(n_b, dtype=torch.int16, device=self.device)
        self.step = 0
        self.desc = GwMlp(n_in, width, n_out, self.master.data_ptr(),
                          self.adam_m.data_ptr() if train else None, self.adam_v.data_ptr() if train else None,
                          self.wt.data_ptr(), self.wk.data_ptr())
        self.sync()

    @staticmethod
    def flat_from_dict(p: dict, n_in: int, width: int, n_out: int) -> np.ndarray:
        """Master layout from {W1,b1,W2,b2,W3,b3} (zero-padded to the layer sizes)."""
        def pad(a, shape):
            out = np.zeros(shape)
            a = np.asarray(a)
            out[tuple(slice(0, s) for s in a.shape)] = a
            return out
        parts = [pad(p["W1"], (n_in, width)), pad(p["b1"], (width,)), pad(p["W2"], (width, width)),
                 pad(p["b2"], (width,)), pad(p["W3"], (width, n_out)), pad(p["b3"], (n_out,))]
        return np.concatenate([x.reshape(-1) for x in parts]).astype(np.float32)

    def to_dict(self) -> dict:
        m = self.master.cpu().numpy().astype(np.float64)
        a, w, o = self.n_in, self.width, self.n_out
        offs = np.cumsum([0, a * w, w, w * w, w, w * o, o])
        return {"W1": m[offs[0]:offs[1]].reshape(a, w), "b1": m[offs[1]:offs[2]],
                "W2": m[offs[2]:offs[3]].reshape(w, w), "b2": m[offs[3]:offs[4]],
                "W3": m[offs[4]:offs[5]].reshape(w, o), "b3": m[offs[5]:offs[6]]}

    def sync(self, stream=None):
        _check(_lib.gw_mlp_sync_bf16(_stream(stream), ctypes.byref(self.desc)))

    def forward(self, X: torch.Tensor, Y: Optional[torch.Tensor] = None, act: Optional[torch.Tensor] = None,
                stream=None):
        _dev_tensor(X, "X", torch.float32)
        rows = X.shape[0]
        if Y is None:
            Y = torch.empty((rows, self.n_out), dtype=torch.float32, device=X.device)
        if act is None:
            act = torch.empty((rows, 4 * self.width), dtype=torch.float32, device=X.device)
        _check(_lib.gw_mlp_forward(_stream(stream), ctypes.byref(self.desc), X.data_ptr(), rows, Y.data_ptr(),
                                   act.data_ptr()))
        return Y, act

    def loss(self, Y, T, mask=None, n_used: int = 1, stream=None):
        rows = Y.shape[0]
        dY = torch.empty_like(Y)
        L = torch.empty(1, dtype=torch.float32, device=Y.device)
        _check(_lib.gw_mlp_loss(_stream(stream), rows, self.n_out, n_used, Y.data_ptr(), T.data_ptr(),
                                mask.data_ptr() if mask is not None else None, dY.data_ptr(), L.data_ptr()))
        return L, dY

    def backward(self, X, act, dY, grad=None, want_dx=False, stream=None):
        rows = X.shape[0]
        if grad is None:
            grad = torch.empty_like(self.master)
        dX = torch.empty_like(X) if want_dx else None
        n = _sz(0)
        _check(_lib.gw_mlp_workspace_size(rows, self.width, ctypes.byref(n)))
        ws = workspace(n.value, X.device, "mlp")
        _check(_lib.gw_mlp_backward(_stream(stream), ctypes.byref(self.desc), X.data_ptr(), act.data_ptr(),
                                    dY.data_ptr(), rows, grad.data_ptr(), dX.data_ptr() if dX is not None else None,
                                    ws.data_ptr(), ws.numel()))
        return grad, dX

    def adam(self, grad, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        self.step += 1
        _check(_lib.gw_mlp_adam_step(_stream(stream), ctypes.byref(self.desc), grad.data_ptr(), lr, b1, b2, eps,
                                     self.step))


# ------------------------------------------------------------ surrogate kernels

class SurrogateArgs:
    """Marshalled gw_surr_desc (keeps the host arrays alive)."""

    def __init__(self, P_ret: torch.Tensor, eps_dev: torch.Tensor, omega, n_occ: int, cut: int, kq=None,
                 n_in: int = 32):
        _dev_tensor(P_ret, "P_ret", torch.complex128)
        _dev_tensor(eps_dev, "eps", torch.float64)
        self.omega = np.ascontiguousarray(omega, dtype=np.float64)
        n_k, nb = eps_dev.shape
        self.kq = None if kq is None else np.ascontiguousarray(kq, dtype=np.int32)
        d = GwSurrDesc()
        d.N, d.n_omega = P_ret.shape[1], self.omega.shape[0]
        d.omega_host = self.omega.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.n_k, d.n_occ, d.n_unocc, d.cut = n_k, n_occ, nb - n_occ, cut
        d.kq_host = self.kq.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if self.kq is not None else None
        d.eps, d.P_ret, d.n_in = eps_dev.data_ptr(), P_ret.data_ptr(), n_in
        self.desc = d
        self.tensors = (P_ret, eps_dev)

    def workspace(self, device):
        n = _sz(0)
        _check(_lib.gw_surrogate_workspace_size(ctypes.byref(self.desc), ctypes.byref(n)))
        return workspace(n.value, device, "surrogate")


def gw_surrogate_features(args: SurrogateArgs, X: Optional[torch.Tensor] = None, stream=None):
    d = args.desc
    if X is None:
        X = torch.empty((d.N * d.n_omega, d.n_in), dtype=torch.float32, device=args.tensors[0].device)
    ws = args.workspace(X.device)
    _check(_lib.gw_surrogate_features(_stream(stream), ctypes.byref(d), X.data_ptr(), ws.data_ptr(), ws.numel()))
    return X


def gw_surrogate_targets(P_ret, P_full, stream=None):
    n_om, N = P_ret.shape[0], P_ret.shape[1]
    T = torch.empty(n_om * N, dtype=torch.float32, device=P_ret.device)
    mask = torch.empty_like(T)
    _check(_lib.gw_surrogate_targets(_stream(stream), N, n_om, P_ret.data_ptr(), P_full.data_ptr(), T.data_ptr(),
                                     mask.data_ptr()))
    return T, mask


def gw_surrogate_apply(P: torch.Tensor, Y: torch.Tensor, ldy: int, stream=None):
    _dev_tensor(P, "P", torch.complex128)
    _check(_lib.gw_surrogate_apply(_stream(stream), P.shape[1], P.shape[0], Y.data_ptr(), ldy, P.data_ptr()))
    return P


def gw_surrogate_judge(args: SurrogateArgs, Y, ldy, P_sample, sample_rows, stream=None):
    ks = np.ascontiguousarray([r[0] for r in sample_rows], dtype=np.int32)
    os_ = np.ascontiguousarray([r[1] for r in sample_rows], dtype=np.int32)
    err = torch.empty(args.desc.n_omega, dtype=torch.float64, device=P_sample.device)
    ws = args.workspace(P_sample.device)
    _check(_lib.gw_surrogate_judge(_stream(stream), ctypes.byref(args.desc), Y.data_ptr(), ldy, P_sample.data_ptr(),
                                   len(sample_rows), ks.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                   os_.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), err.data_ptr(), ws.data_ptr(),
                                   ws.numel()))
    return err


def gw_get_tuning(key: str) -> int:
    v = ctypes.c_int(0)
    _check(_lib.gw_get_tuning(key.encode(), ctypes.byref(v)))
    return v.value


def gw_set_tuning(key: str, value: int) -> None:
    _check(_lib.gw_set_tuning(key.encode(), int(value)))


class SigmaCall:
    """Marshalled arguments of one gw_sigma_c call (keeps host arrays alive)."""

    def __init__(self, U, psi, eps_host, W_by_transfer, v, mesh, omega_out, states, mu, *, precision="fp64",
                 eps_dev=None, sigma=None):
        prec = _prec(precision)
        dt = _cdtype(prec)
        _dev_tensor(U, "U", dt)
        _dev_tensor(psi, "psi", dt)
        N, R = U.shape
        n_k, nb = psi.shape[0], psi.shape[1]
        self.eps_host = np.ascontiguousarray(eps_host, dtype=np.float64)
        if self.eps_host.shape != (n_k, nb):
            raise ValueError(f"eps must be [{n_k}][{nb}]")
        self.eps_dev = eps_dev if eps_dev is not None else torch.from_numpy(self.eps_host).to(U.device)
        _dev_tensor(self.eps_dev, "eps_dev", torch.float64)
        if len(W_by_transfer) != n_k:
            raise ValueError("one W per momentum transfer (n_k of them) is required")
        self.mesh = np.ascontiguousarray(mesh, dtype=np.float64)
        for W in W_by_transfer:
            _dev_tensor(W, "W", torch.complex128)
            if tuple(W.shape) != (self.mesh.shape[0], N, N):
                raise ValueError("W has the wrong shape")
        _dev_tensor(v, "v", torch.float64)
        self.omega_out = np.ascontiguousarray(omega_out, dtype=np.float64)
        st = np.asarray(states, dtype=np.int32).reshape(-1, 2)
        self.state_set = np.ascontiguousarray(st[:, 0])
        self.state_band = np.ascontiguousarray(st[:, 1])
        if sigma is None:
            sigma = torch.empty((st.shape[0], self.omega_out.shape[0]), dtype=torch.complex128, device=U.device)
        _dev_tensor(sigma, "sigma", torch.complex128)
        self.sigma = sigma
        self.W_ptrs = (ctypes.c_void_p * n_k)(*[W.data_ptr() for W in W_by_transfer])
        self.tensors = (U, psi, v, tuple(W_by_transfer))
        d = GwSigmaDesc()
        d.precision, d.n_k, d.N, d.R, d.n_bands = prec, n_k, N, R, nb
        d.n_mesh = int(self.mesh.shape[0])
        d.mesh_host = self.mesh.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.n_out = int(self.omega_out.shape[0])
        d.omega_out_host = self.omega_out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.n_states = int(st.shape[0])
        d.state_set_host = self.state_set.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        d.state_band_host = self.state_band.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        d.mu = float(mu)
        d.U, d.psi = U.data_ptr(), psi.data_ptr()
        d.eps = self.eps_dev.data_ptr()
        d.eps_host = self.eps_host.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.W_host = ctypes.cast(self.W_ptrs, ctypes.POINTER(ctypes.c_void_p))
        d.v = v.data_ptr()
        d.sigma = sigma.data_ptr()
        self.desc = d

    def workspace_size(self) -> int:
        out = _sz(0)
        _check(_lib.gw_sigma_c_workspace_size(ctypes.byref(self.desc), ctypes.byref(out)))
        return out.value

    def run(self, ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        nbytes = self.workspace_size()
        if ws is None:
            ws = workspace(nbytes, self.sigma.device, "sigma")
        _check(_lib.gw_sigma_c(_stream(stream), ctypes.byref(self.desc), ws.data_ptr(), ws.numel()))
        return self.sigma


def gw_sigma_c(U, psi, eps_host, W_by_transfer, v, mesh, omega_out, states, mu, **kw) -> torch.Tensor:
    """Diagonal correlation self-energy sigma[state][o] on the imaginary axis
    (Eq. SEc_AC, see gw.h): complex128 [n_states][n_out], enqueued on the
    current stream.  W_by_transfer[t] is W(t) [n_mesh][N][N] (not W - v)."""
    ws = kw.pop("ws", None)
    stream = kw.pop("stream", None)
    return SigmaCall(U, psi, eps_host, W_by_transfer, v, mesh, omega_out, states, mu, **kw).run(ws, stream)


def gw_basis_select(U: torch.Tensor, v: torch.Tensor, v_min: float, stream=None):
    """Keep the basis functions with v >= v_min (Sec. "Optimization of the
    MPB"): returns (U_out [n_keep][R], v_out [n_keep], src_of_dst [n_keep])."""
    if U.dim() != 2 or not U.is_cuda or not U.is_contiguous():
        raise ValueError("U must be a contiguous device matrix")
    _dev_tensor(v, "v", torch.float64)
    N, R = U.shape
    v_host = np.ascontiguousarray(v.cpu().numpy(), dtype=np.float64)
    n = _ci(0)
    _check(_lib.gw_basis_select_count(N, v_host.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(v_min),
                                      ctypes.byref(n)))
    U_out = torch.empty((n.value, R), dtype=U.dtype, device=U.device)
    v_out = torch.empty((n.value,), dtype=torch.float64, device=U.device)
    src = torch.empty((max(1, n.value),), dtype=torch.int32, device=U.device)
    _check(_lib.gw_basis_select(_stream(stream), N, R, U.element_size(), U.data_ptr(), v.data_ptr(), float(v_min),
                                n.value, U_out.data_ptr(), v_out.data_ptr(), src.data_ptr()))
    return U_out, v_out, src[:n.value]

