"""FP64 HIP path vs the CPU FP64 oracle (relative Frobenius error <= 1e-10 per
frequency), through the C ABI.  Shapes span several tiles with ragged tails."""
import numpy as np
import pytest

import gwsynth
from oracle import polarization as orc

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _to_dev(inp, dtype):
    import torch
    U = torch.from_numpy(np.ascontiguousarray(inp.U)).to("cuda", dtype)
    psi = torch.from_numpy(np.ascontiguousarray(inp.psi)).to("cuda", dtype)
    return U, psi


def test_project_fp64_ragged(lib):
    import torch
    shp = gwsynth.make_shape(n_k=1, n_b=40, R=100, N=130, n_occ=3, n_unocc=37)
    inp = gwsynth.generate(shp, seed=21)
    U, psi = _to_dev(inp, torch.complex128)
    M = lib.gw_project(U, psi[0, :3].contiguous(), psi[0, 3:].contiguous(), "fp64")
    torch.cuda.synchronize()
    ref = orc.projections(inp.U, inp.psi[0, :3], inp.psi[0, 3:])
    err = np.linalg.norm(M.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err < 1e-13


@pytest.mark.parametrize("shape", [
    dict(n_k=2, n_b=40, R=100, N=130, n_occ=3, n_unocc=37),
    dict(n_k=3, n_b=20, R=17, N=1, n_occ=1, n_unocc=1),
    dict(n_k=1, n_b=64, R=300, N=65, n_occ=5, n_unocc=70),
])
def test_polarization_fp64_ragged(lib, shape):
    import torch
    inp = gwsynth.generate(gwsynth.make_shape(**shape), seed=8, omega=gwsynth.omega_mesh("c1"))
    U, psi = _to_dev(inp, torch.complex128)
    P = lib.gw_polarization(U, psi, inp.eps, inp.omega, shape["n_occ"], precision="fp64", kq=inp.kq)
    torch.cuda.synchronize()
    ref = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, shape["n_occ"], kq=inp.kq)
    Pg = P.cpu().numpy()
    err = orc.rel_fro(Pg, ref)
    assert err.max() < TOL, err
    # stored exactly Hermitian with a real diagonal
    for j in range(Pg.shape[0]):
        assert np.array_equal(Pg[j], Pg[j].conj().T)


def test_polarization_fp64_config1(lib):
    import torch
    inp = gwsynth.generate("c1")
    U, psi = _to_dev(inp, torch.complex128)
    P = lib.gw_polarization(U, psi, inp.eps, inp.omega, 4, precision="fp64", kq=inp.kq)
    torch.cuda.synchronize()
    ref = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 4, kq=inp.kq)
    err = orc.rel_fro(P.cpu().numpy(), ref)
    print("config1 fp64 rel err per omega", err)
    assert err.max() < TOL


def test_polarization_fp64_small_chunks_and_subsets(lib):
    """Chunking over pairs, k subsets, band sub-ranges and accumulation."""
    import torch
    inp = gwsynth.generate("c1")
    U, psi = _to_dev(inp, torch.complex128)
    ref = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 4, kq=inp.kq, k_list=[0, 5, 7],
                           occ_range=(1, 4), unocc_range=(3, 50))
    P = lib.gw_polarization(U, psi, inp.eps, inp.omega, 4, precision="fp64", kq=inp.kq, k_list=[0, 5],
                            occ_range=(1, 4), unocc_range=(3, 50), chunk_pairs=40)
    lib.gw_polarization(U, psi, inp.eps, inp.omega, 4, precision="fp64", kq=inp.kq, k_list=[7],
                        occ_range=(1, 4), unocc_range=(3, 50), P=P, accumulate=True, chunk_pairs=7)
    torch.cuda.synchronize()
    assert orc.rel_fro(P.cpu().numpy(), ref).max() < TOL


def test_polarization_deterministic(lib):
    import torch
    inp = gwsynth.generate("c1")
    U, psi = _to_dev(inp, torch.complex128)
    P1 = lib.gw_polarization(U, psi, inp.eps, inp.omega, 4, precision="fp64", kq=inp.kq).clone()
    P2 = lib.gw_polarization(U, psi, inp.eps, inp.omega, 4, precision="fp64", kq=inp.kq).clone()
    torch.cuda.synchronize()
    assert torch.equal(P1, P2)


@pytest.mark.parametrize("N", [120, 1, 33, 130, 200, 257])
def test_screen_fp64(lib, N):
    import torch
    shp = gwsynth.make_shape(n_k=2, n_b=60, R=256, N=N, n_occ=3, n_unocc=20)
    inp = gwsynth.generate(shp, seed=4, omega=gwsynth.omega_mesh("c1"))
    P = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=inp.kq)
    Wref = orc.screened_interaction(P, inp.v)
    Pd = torch.from_numpy(P).to("cuda")
    vd = torch.from_numpy(inp.v).to("cuda")
    W, info = lib.gw_screen(Pd, vd)
    torch.cuda.synchronize()
    assert int(info.abs().sum()) == 0
    err = orc.rel_fro(W.cpu().numpy(), Wref)
    assert err.max() < TOL, err


def test_screen_config1_from_gpu_p(lib):
    """P and W of config 1 end to end on the GPU vs the oracle."""
    import torch
    inp = gwsynth.generate("c1")
    U, psi = _to_dev(inp, torch.complex128)
    P = lib.gw_polarization(U, psi, inp.eps, inp.omega, 4, precision="fp64", kq=inp.kq)
    W, info = lib.gw_screen(P, torch.from_numpy(inp.v).to("cuda"))
    torch.cuda.synchronize()
    Pref = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 4, kq=inp.kq)
    Wref = orc.screened_interaction(Pref, inp.v)
    assert int(info.abs().sum()) == 0
    assert orc.rel_fro(W.cpu().numpy(), Wref).max() < TOL


def test_screen_reports_indefinite(lib):
    """A polarization with a positive eigenvalue large enough to make
    1 - sqrt(v) P sqrt(v) indefinite is reported through info (host-forced
    condition; every kernel still runs to completion)."""
    import torch
    N = 40
    v = np.ones(N)
    P = np.zeros((2, N, N), dtype=complex)
    P[0] = -0.1 * np.eye(N)
    P[1] = -0.1 * np.eye(N)
    P[1, 35, 35] = 3.0      # eps_35,35 = 1 - 3 < 0
    W, info = lib.gw_screen(torch.from_numpy(P).to("cuda"), torch.from_numpy(v).to("cuda"))
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    assert info[0] == 0
    assert info[1] == 36
    np.testing.assert_allclose(W[0].cpu().numpy(), np.eye(N) / 1.1, rtol=1e-14, atol=1e-15)
