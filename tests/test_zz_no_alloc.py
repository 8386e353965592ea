"""The allocation-free screening entry point against gw_screen (same kernels,
workspace from the caller): two calls in a row on the library's fixed array,
the second smaller, each bit-identical to gw_screen and within the FP64 bar of
the oracle."""
import numpy as np
import pytest
import torch

import gwsynth
from oracle import polarization as orc

pytestmark = pytest.mark.gpu


def _case(N, n_om, seed):
    shp = gwsynth.make_shape(n_k=2, n_b=N + 20, R=2 * N, N=N, n_occ=3, n_unocc=N // 2, omega="c1")
    inp = gwsynth.generate(shp, seed=seed, omega=gwsynth.omega_mesh("c1")[:n_om])
    P = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=inp.kq)
    return P, inp.v


def test_screen_noalloc_matches_screen_twice(lib):
    dev = torch.device("cuda:0")
    for N, n_om, seed in ((300, 6, 41), (77, 3, 42)):
        print(f"no-alloc screening case N={N} n_omega={n_om} seed={seed}", flush=True)
        P, v = _case(N, n_om, seed)
        Pd = torch.from_numpy(P).to(dev)
        vd = torch.from_numpy(v).to(dev)
        W_ref, info_ref = lib.gw_screen(Pd, vd)
        W = torch.full_like(Pd, float("nan"))
        info = torch.full((n_om,), -7, dtype=torch.int32, device=dev)
        lib.gw_screen_noalloc(Pd, vd, W, info)
        torch.cuda.synchronize()
        assert torch.equal(info.cpu(), info_ref.cpu()) and int(info.abs().sum()) == 0
        assert torch.equal(W.cpu(), W_ref.cpu())
        Wo = orc.screened_interaction(P, v)
        assert orc.rel_fro(W.cpu().numpy(), Wo).max() < 1e-10
