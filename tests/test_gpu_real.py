"""Real inputs (the inversion-symmetric case, Eq. condition_inv): the real
form of the split-BF16 path vs the CPU FP64 oracle on the same real,
float32-rounded inputs.  P must be real (imaginary parts exactly zero),
symmetric, and within 1e-4 relative Frobenius error per frequency."""
import numpy as np
import pytest

import gwsynth
from oracle import polarization as orc

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _real(inp):
    return (np.ascontiguousarray(inp.U.real, dtype=np.float32), np.ascontiguousarray(inp.psi.real, dtype=np.float32))


@pytest.mark.parametrize("shape", [
    dict(n_k=2, n_b=60, R=1000, N=300, n_occ=3, n_unocc=150),
    dict(n_k=3, n_b=64, R=513, N=129, n_occ=2, n_unocc=63),
    dict(n_k=1, n_b=20, R=33, N=7, n_occ=1, n_unocc=5),
])
def test_real_path_ragged(lib, shape):
    import torch
    inp = gwsynth.generate(gwsynth.make_shape(**shape), seed=13, omega=gwsynth.omega_mesh("m16"))
    U, psi = _real(inp)
    P = lib.gw_polarization(torch.from_numpy(U).to("cuda"), torch.from_numpy(psi).to("cuda"), inp.eps, inp.omega,
                            shape["n_occ"], precision="split_bf16", kq=inp.kq, real=True)
    torch.cuda.synchronize()
    Pg = P.cpu().numpy()
    ref = orc.polarization(U.astype(np.complex128), psi.astype(np.complex128), inp.eps, inp.omega, shape["n_occ"],
                           kq=inp.kq)
    err = orc.rel_fro(Pg, ref)
    print(f"real path {shape}: max rel err {err.max():.2e}")
    assert err.max() < TOL
    assert np.all(Pg.imag == 0.0)
    assert np.array_equal(Pg, np.transpose(Pg, (0, 2, 1)))


def test_real_path_chunked_matches_unchunked(lib):
    import torch
    inp = gwsynth.generate(gwsynth.make_shape(n_k=2, n_b=40, R=256, N=150, n_occ=4, n_unocc=40), seed=3,
                           omega=gwsynth.omega_mesh("c1"))
    U, psi = _real(inp)
    Ud, pd = torch.from_numpy(U).to("cuda"), torch.from_numpy(psi).to("cuda")
    P1 = lib.gw_polarization(Ud, pd, inp.eps, inp.omega, 4, precision="split_bf16", kq=inp.kq, real=True).clone()
    P2 = lib.gw_polarization(Ud, pd, inp.eps, inp.omega, 4, precision="split_bf16", kq=inp.kq, real=True,
                             chunk_pairs=37).clone()
    torch.cuda.synchronize()
    assert orc.rel_fro(P1.cpu().numpy(), P2.cpu().numpy()).max() < 1e-5


def test_real_path_largest_size_sampled(lib):
    """Real inputs of the largest workload's shape (N=6000, R=65536, 16
    frequencies), k = 0, occupied bands 0..5 x unoccupied 0..1499 at the
    default chunk size; the oracle evaluates the sampled block P[S, S]."""
    import torch
    shp = gwsynth.SHAPES["c5"]
    nb = shp.n_occ + shp.n_unocc_cut
    inp = gwsynth.generate_torch(shp, torch.device("cuda"), k_subset=[0, 1], band_limit=nb)
    U = inp.U.real.contiguous()
    psi = inp.psi.real.contiguous()
    eps = np.ascontiguousarray(inp.eps[:, :nb])
    occ = (0, 6)
    P = lib.gw_polarization(U, psi, eps, inp.omega, shp.n_occ, precision="split_bf16", k_list=[0], occ_range=occ,
                            real=True)
    torch.cuda.synchronize()
    rng = np.random.default_rng(2)
    S = np.sort(np.concatenate([[0, shp.N - 1], rng.choice(np.arange(1, shp.N - 1), 14, replace=False)]))
    idx = torch.as_tensor(S, device="cuda")
    Pg = P.index_select(1, idx).index_select(2, idx).cpu().numpy()
    psi_h = np.zeros((2, nb, shp.R), dtype=np.float32)
    psi_h[0, :occ[1]] = psi[0, :occ[1]].cpu().numpy()
    psi_h[1, shp.n_occ:] = psi[1, shp.n_occ:].cpu().numpy()
    ref = orc.polarization(U[S].cpu().numpy().astype(np.complex128), psi_h.astype(np.complex128), eps[:2],
                           inp.omega, shp.n_occ, kq=[1, 0], k_list=[0], occ_range=occ, unocc_range=(0, shp.n_unocc_cut))
    err = orc.rel_fro(Pg, ref)
    print(f"real path c5 shape: sampled max rel err {err.max():.2e}")
    assert err.max() < TOL
    assert np.all(Pg.imag == 0.0)


@pytest.mark.parametrize("shape", [
    dict(n_k=2, n_b=60, R=1000, N=300, n_occ=3, n_unocc=150),   # 32 real K stages: the ring's 4-step tail
    dict(n_k=3, n_b=64, R=513, N=129, n_occ=2, n_unocc=63),     # 17 stages: the 2-step tail
    dict(n_k=1, n_b=20, R=33, N=7, n_occ=1, n_unocc=5),         # 2 stages: fewer steps than the copy lead
])
def test_real_cores_bitwise(lib, shape):
    """The two real GEMM cores (the 8-wave register-staged core, real_core 1;
    the six-slot core, real_core 2, the default, at leads 3 to 5) issue the
    same MFMAs on every accumulator in the same order (hi hi, hi lo, lo hi per
    16 k, k ascending), so P agrees bit for bit."""
    import torch
    inp = gwsynth.generate(gwsynth.make_shape(**shape), seed=17, omega=gwsynth.omega_mesh("m16"))
    U, psi = _real(inp)
    Ud, pd = torch.from_numpy(U).to("cuda"), torch.from_numpy(psi).to("cuda")
    out = {}
    try:
        for core, lead in ((1, 4), (2, 3), (2, 4), (2, 5)):
            lib.gw_set_tuning("real_core", core)
            lib.gw_set_tuning("gemm3m_lead", lead)
            P = lib.gw_polarization(Ud, pd, inp.eps, inp.omega, shape["n_occ"], precision="split_bf16", kq=inp.kq,
                                    real=True)
            torch.cuda.synchronize()
            out[core, lead] = P.cpu().numpy()
    finally:
        lib.gw_set_tuning("real_core", 2)
        lib.gw_set_tuning("gemm3m_lead", 4)
    for key in ((2, 3), (2, 4), (2, 5)):
        assert np.array_equal(out[1, 4], out[key]), key
