"""Reduced-precision paths at the full sizes of the supercell-shaped and the
largest workload, in the launch configuration bench.py times (default chunk
sizes), against the CPU FP64 oracle on sampled outputs.

P_IJ depends on rows I and J of U only, so the oracle evaluates the sampled
block P[S, S] exactly from U[S] (16 rows spread over the basis) with the same
complex64-rounded wave functions; the GPU computes the full matrices.  At the
largest size W is checked through its defining equation on the sampled rows:
(1 - v P) W = v, i.e. W[S, :] - v_S (P[S, :] W) = diag(v)[S, :]."""
import numpy as np
import pytest

import gwsynth
from oracle import polarization as orc

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _sample_rows(N, n=16, seed=0):
    rng = np.random.default_rng(seed)
    S = np.sort(rng.choice(np.arange(1, N - 1), size=n - 2, replace=False))
    return np.concatenate([[0], S, [N - 1]])      # first and last row of the basis included


def _block(P, S):
    import torch
    idx = torch.as_tensor(S, device=P.device)
    return P.index_select(1, idx).index_select(2, idx).cpu().numpy()


def _oracle_block(U, psi, eps, omega, n_occ, sets, kq_local, k_local, occ, unocc, S):
    """Oracle P[S, S] with wave functions of the listed k-sets only (set i of
    the oracle arrays is set sets[i] of the full input)."""
    R = U.shape[1]
    nb = psi.shape[1]
    U_S = U[S].cpu().numpy().astype(np.complex128)
    psi_h = np.zeros((len(sets), nb, R), dtype=np.complex64)
    for i, k in enumerate(sets):
        psi_h[i] = psi[k].cpu().numpy()
    eps_h = np.ascontiguousarray(eps[sets])
    return orc.polarization(U_S, psi_h, eps_h, omega, n_occ, kq=kq_local, k_list=k_local, occ_range=occ,
                            unocc_range=unocc)


@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_supercell_size_sampled(lib, prec):
    """N_k=8, N=3000, R=32768, 128 + 2000 bands, 16 frequencies; k in {0, 4}
    (unoccupied states from sets 1 and 5), occupied bands 0..7, all 2000
    unoccupied bands: two chunks per k at the default chunk size."""
    import torch
    shp = gwsynth.SHAPES["c3"]
    sets = [0, 1, 4, 5]
    inp = gwsynth.generate_torch(shp, torch.device("cuda"), k_subset=sets)
    occ = (0, 8)
    P = lib.gw_polarization(inp.U, inp.psi, inp.eps, inp.omega, shp.n_occ, precision=prec, k_list=[0, 4],
                            occ_range=occ)
    torch.cuda.synchronize()
    S = _sample_rows(shp.N)
    Pg = _block(P, S)
    del P
    ref = _oracle_block(inp.U, inp.psi, inp.eps, inp.omega, shp.n_occ, sets, [1, 1, 3, 3], [0, 2], occ,
                        (0, shp.n_unocc), S)
    err = orc.rel_fro(Pg, ref)
    print(f"c3 {prec}: sampled P max rel err {err.max():.2e} (per frequency {np.array2string(err, precision=1)})")
    assert err.max() < TOL


def test_largest_size_sampled_with_screening(lib):
    """N_k=4, N=6000, R=65536, 16 frequencies, the explicit bands of the
    surrogate path (unoccupied 0..1499); k = 0, occupied bands 0..5: one
    full 6912-pair chunk and a partial one, split BF16; then W in FP64."""
    import torch
    shp = gwsynth.SHAPES["c5"]
    cut = shp.n_unocc_cut
    nb = shp.n_occ + cut
    inp = gwsynth.generate_torch(shp, torch.device("cuda"), k_subset=[0, 1], band_limit=nb)
    eps = np.ascontiguousarray(inp.eps[:, :nb])
    occ = (0, 6)
    P = lib.gw_polarization(inp.U, inp.psi, eps, inp.omega, shp.n_occ, precision="split_bf16", k_list=[0],
                            occ_range=occ)
    torch.cuda.synchronize()
    S = _sample_rows(shp.N, seed=1)
    Pg = _block(P, S)
    ref = _oracle_block(inp.U, inp.psi, eps, inp.omega, shp.n_occ, [0, 1], [1, 0], [0], occ, (0, cut), S)
    err = orc.rel_fro(Pg, ref)
    print(f"c5 split_bf16: sampled P max rel err {err.max():.2e}")
    assert err.max() < TOL

    v = torch.from_numpy(gwsynth.coulomb_diag(shp.N)).to("cuda")
    W, info = lib.gw_screen(P, v)
    torch.cuda.synchronize()
    assert int(info.abs().sum()) == 0
    idx = torch.as_tensor(S, device="cuda")
    vS = v.index_select(0, idx).to(torch.complex128)
    worst = 0.0
    for j in range(P.shape[0]):
        PS = P[j].index_select(0, idx)
        WS = W[j].index_select(0, idx)
        lhs = WS - vS[:, None] * (PS @ W[j])
        rhs = torch.zeros_like(lhs)
        rhs[torch.arange(len(S), device="cuda"), idx] = vS
        worst = max(worst, float(torch.linalg.norm(lhs - rhs) / torch.linalg.norm(rhs)))
    print(f"c5 screening: max relative residual of (1 - vP) W = v on the sampled rows {worst:.2e}")
    assert worst < 1e-10


def test_largest_size_top_bands_sampled(lib):
    """N_k=4, N=6000, R=65536, 16 frequencies, the explicit bands of the
    surrogate path: k = 2 with the six highest occupied bands (250..255, the
    smallest gaps and largest weights), unoccupied bands 0..1499 of set 3,
    split BF16, sampled block against the oracle."""
    import torch
    shp = gwsynth.SHAPES["c5"]
    cut = shp.n_unocc_cut
    nb = shp.n_occ + cut
    inp = gwsynth.generate_torch(shp, torch.device("cuda"), k_subset=[2, 3], band_limit=nb)
    eps = np.ascontiguousarray(inp.eps[:, :nb])
    occ = (shp.n_occ - 6, shp.n_occ)
    P = lib.gw_polarization(inp.U, inp.psi, eps, inp.omega, shp.n_occ, precision="split_bf16", k_list=[2],
                            occ_range=occ)
    torch.cuda.synchronize()
    S = _sample_rows(shp.N, seed=2)
    Pg = _block(P, S)
    del P
    ref = _oracle_block(inp.U, inp.psi, eps, inp.omega, shp.n_occ, [2, 3], [1, 0], [0], occ, (0, cut), S)
    err = orc.rel_fro(Pg, ref)
    print(f"c5 split_bf16, k=2, top occupied bands: sampled P max rel err {err.max():.2e}")
    assert err.max() < TOL
