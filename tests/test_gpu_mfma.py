"""Reduced-precision HIP paths (FP32 MFMA, split BF16, split FP16) vs the CPU
FP64 oracle on the same complex64-rounded inputs; tolerance 1e-4 relative
Frobenius error per frequency (the reduced-precision bar), measured values are
printed.  Shapes span several 128-wide tiles and ragged tails."""
import numpy as np
import pytest

import gwsynth
from oracle import polarization as orc

pytestmark = pytest.mark.gpu
TOL = 1e-4
PRECS = ["fp32", "split_bf16", "split_fp16"]


def _dev(inp):
    import torch
    U = torch.from_numpy(np.ascontiguousarray(inp.U)).to("cuda", torch.complex64)
    psi = torch.from_numpy(np.ascontiguousarray(inp.psi)).to("cuda", torch.complex64)
    return U, psi


def _rounded(inp):
    """The c64 values the GPU receives, widened to c128 for the oracle."""
    return inp.U.astype(np.complex64).astype(np.complex128), inp.psi.astype(np.complex64).astype(np.complex128)


def _supported(lib, prec):
    try:
        lib.gw_project_workspace_size(prec, 4, 4, 1, 1)
        return True
    except lib.GwError:
        return False


@pytest.mark.parametrize("prec", PRECS)
def test_project_ragged(lib, prec):
    import torch
    shp = gwsynth.make_shape(n_k=1, n_b=50, R=1000, N=300, n_occ=3, n_unocc=50)
    inp = gwsynth.generate(shp, seed=31)
    U, psi = _dev(inp)
    M = lib.gw_project(U, psi[0, :3].contiguous(), psi[0, 3:].contiguous(), prec)
    torch.cuda.synchronize()
    Ur, pr = _rounded(inp)
    ref = orc.projections(Ur, pr[0, :3], pr[0, 3:])
    err = np.linalg.norm(M.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"{prec} projection rel err {err:.2e}")
    assert err < 1e-5


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("shape", [
    dict(n_k=2, n_b=60, R=1000, N=300, n_occ=3, n_unocc=150),
    dict(n_k=1, n_b=20, R=33, N=7, n_occ=1, n_unocc=5),
    dict(n_k=3, n_b=64, R=512, N=129, n_occ=2, n_unocc=63),
])
def test_polarization_ragged(lib, prec, shape):
    import torch
    inp = gwsynth.generate(gwsynth.make_shape(**shape), seed=9, omega=gwsynth.omega_mesh("m16"))
    U, psi = _dev(inp)
    P = lib.gw_polarization(U, psi, inp.eps, inp.omega, shape["n_occ"], precision=prec, kq=inp.kq)
    torch.cuda.synchronize()
    Ur, pr = _rounded(inp)
    ref = orc.polarization(Ur, pr, inp.eps, inp.omega, shape["n_occ"], kq=inp.kq)
    Pg = P.cpu().numpy()
    err = orc.rel_fro(Pg, ref)
    print(f"{prec} {shape} max rel err {err.max():.2e}")
    assert err.max() < TOL, err
    for j in range(Pg.shape[0]):
        assert np.array_equal(Pg[j], Pg[j].conj().T)


@pytest.mark.parametrize("prec", PRECS)
def test_polarization_chunked_matches_unchunked(lib, prec):
    """Chunk size only changes where FP32 partial sums are flushed to FP64."""
    import torch
    inp = gwsynth.generate(gwsynth.make_shape(n_k=2, n_b=40, R=256, N=150, n_occ=4, n_unocc=40), seed=3,
                           omega=gwsynth.omega_mesh("c1"))
    U, psi = _dev(inp)
    P1 = lib.gw_polarization(U, psi, inp.eps, inp.omega, 4, precision=prec, kq=inp.kq).clone()
    P2 = lib.gw_polarization(U, psi, inp.eps, inp.omega, 4, precision=prec, kq=inp.kq, chunk_pairs=37).clone()
    torch.cuda.synchronize()
    d = orc.rel_fro(P1.cpu().numpy(), P2.cpu().numpy())
    assert d.max() < 1e-5


def test_config2_fp32_sampled_k(lib):
    """Config 2 (N_k=64, N=500, R=4096, 16 occ + 500 unocc, 13 frequencies) on
    two sampled k-points: FP32 GPU vs FP64 oracle, then W in FP64."""
    import torch
    inp = gwsynth.generate("c2")
    U, psi = _dev(inp)
    ks = [0, 37]
    P = lib.gw_polarization(U, psi, inp.eps, inp.omega, 16, precision="fp32", kq=inp.kq, k_list=ks)
    W, info = lib.gw_screen(P, torch.from_numpy(inp.v).to("cuda"))
    torch.cuda.synchronize()
    Ur, pr = _rounded(inp)
    ref = orc.polarization(Ur, pr, inp.eps, inp.omega, 16, kq=inp.kq, k_list=ks)
    err = orc.rel_fro(P.cpu().numpy(), ref)
    Wref = orc.screened_interaction(ref, inp.v)
    werr = orc.rel_fro(W.cpu().numpy(), Wref)
    print(f"config2 fp32 k={ks}: P err max {err.max():.2e}, W err max {werr.max():.2e}")
    assert int(info.abs().sum()) == 0
    assert err.max() < TOL and werr.max() < TOL


@pytest.mark.parametrize("prec", PRECS)
def test_deterministic(lib, prec):
    import torch
    inp = gwsynth.generate("c1")
    U, psi = _dev(inp)
    P1 = lib.gw_polarization(U, psi, inp.eps, inp.omega, 4, precision=prec, kq=inp.kq).clone()
    P2 = lib.gw_polarization(U, psi, inp.eps, inp.omega, 4, precision=prec, kq=inp.kq).clone()
    torch.cuda.synchronize()
    assert torch.equal(P1, P2)


@pytest.mark.parametrize("prec", PRECS)
def test_poisoned_workspace(lib, prec):
    """The result does not depend on stale workspace contents."""
    import torch
    inp = gwsynth.generate("c1")
    U, psi = _dev(inp)
    call = lib.PolarizationCall(U, psi, inp.eps, inp.omega, 4, precision=prec, kq=inp.kq)
    n = call.workspace_size()
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    ws.fill_(0)
    P1 = call.run(ws).clone()
    ws.fill_(0xFF)   # NaN patterns everywhere
    P2 = call.run(ws).clone()
    torch.cuda.synchronize()
    assert torch.equal(P1, P2)


@pytest.mark.parametrize("pipeline,pv,staging", [(1, 1, 1), (1, 2, 1), (2, 2, 1), (2, 2, 2), (2, 2, 3), (2, 2, 4)])
def test_split_bf16_kernel_variants(lib, pipeline, pv, staging):
    """Every kernel variant of the split-BF16 path meets the same bar (N spans
    two 256-row tiles with a ragged tail; R and the pair count are ragged):
    operands staged inside the GEMM kernels with either projection tiling, and
    pre-tiled operands on the shared GEMM core (4 waves staged through
    registers or copied straight into LDS, or 8 waves in lockstep or in
    ping-pong)."""
    import torch
    shape = dict(n_k=2, n_b=60, R=1000, N=300, n_occ=3, n_unocc=150)
    inp = gwsynth.generate(gwsynth.make_shape(**shape), seed=9, omega=gwsynth.omega_mesh("m16"))
    U, psi = _dev(inp)
    try:
        lib.gw_set_tuning("complex_product", 4)
        lib.gw_set_tuning("bf16_pipeline", pipeline)
        lib.gw_set_tuning("projection_variant", pv)
        lib.gw_set_tuning("gemm_staging", staging)
        P = lib.gw_polarization(U, psi, inp.eps, inp.omega, 3, precision="split_bf16", kq=inp.kq)
        M = lib.gw_project(U, psi[0, :3].contiguous(), psi[0, 3:].contiguous(), "split_bf16")
        torch.cuda.synchronize()
    finally:
        lib.gw_set_tuning("complex_product", 3)
        lib.gw_set_tuning("bf16_pipeline", 2)
        lib.gw_set_tuning("projection_variant", 2)
        lib.gw_set_tuning("gemm_staging", 3)
    Ur, pr = _rounded(inp)
    ref = orc.polarization(Ur, pr, inp.eps, inp.omega, 3, kq=inp.kq)
    err = orc.rel_fro(P.cpu().numpy(), ref)
    Mref = orc.projections(Ur, pr[0, :3], pr[0, 3:])
    merr = np.linalg.norm(M.cpu().numpy() - Mref) / np.linalg.norm(Mref)
    print(f"pipeline {pipeline} projection variant {pv} staging {staging}: P max rel err {err.max():.2e}, M rel err {merr:.2e}")
    assert err.max() < TOL
    assert merr < 1e-5


@pytest.mark.parametrize("real", [False, True])
@pytest.mark.parametrize("N,R", [(1, 1), (1, 40), (5, 1)])
def test_extreme_shapes_max_frequencies(lib, real, N, R):
    """Degenerate sizes (one basis function, one grid point) with the maximum
    of 64 frequencies on the default split-BF16 pipeline (complex and real)."""
    import torch
    shape = dict(n_k=2, n_b=8, R=R, N=N, n_occ=2, n_unocc=5)
    om = np.concatenate([[0.0], np.geomspace(0.01, 50.0, 63)])
    inp = gwsynth.generate(gwsynth.make_shape(**shape), seed=17, omega=om)
    if real:
        U = np.ascontiguousarray(inp.U.real, dtype=np.float32)
        psi = np.ascontiguousarray(inp.psi.real, dtype=np.float32)
        Ud, pd = torch.from_numpy(U).to("cuda"), torch.from_numpy(psi).to("cuda")
        U64, p64 = U.astype(np.complex128), psi.astype(np.complex128)
    else:
        Ud, pd = _dev(inp)
        U64, p64 = _rounded(inp)
    P = lib.gw_polarization(Ud, pd, inp.eps, om, 2, precision="split_bf16", kq=inp.kq, real=real)
    torch.cuda.synchronize()
    ref = orc.polarization(U64, p64, inp.eps, om, 2, kq=inp.kq)
    err = orc.rel_fro(P.cpu().numpy(), ref)
    assert err.max() < TOL, err.max()


def test_single_fp16_ablation_misses_the_bar(lib):
    """GW_FP16 (hi words only, the split path's scaling): the ablation that
    motivates the split.  Its error sits well above the split FP16 error and
    around the 1e-4 bar; P stays Hermitian."""
    import torch
    shape = dict(n_k=2, n_b=60, R=1000, N=300, n_occ=3, n_unocc=150)
    inp = gwsynth.generate(gwsynth.make_shape(**shape), seed=9, omega=gwsynth.omega_mesh("m16"))
    U, psi = _dev(inp)
    Ur, pr = _rounded(inp)
    ref = orc.polarization(Ur, pr, inp.eps, inp.omega, 3, kq=inp.kq)
    P1 = lib.gw_polarization(U, psi, inp.eps, inp.omega, 3, precision="fp16", kq=inp.kq).cpu().numpy()
    P2 = lib.gw_polarization(U, psi, inp.eps, inp.omega, 3, precision="split_fp16", kq=inp.kq).cpu().numpy()
    M1 = lib.gw_project(U, psi[0, :3].contiguous(), psi[0, 3:].contiguous(), "fp16").cpu().numpy()
    torch.cuda.synchronize()
    e1, e2 = orc.rel_fro(P1, ref), orc.rel_fro(P2, ref)
    mref = orc.projections(Ur, pr[0, :3], pr[0, 3:])
    em = np.linalg.norm(M1 - mref) / np.linalg.norm(mref)
    print(f"single FP16: P max rel err {e1.max():.2e} (split FP16 {e2.max():.2e}), projection {em:.2e}")
    assert 2e-5 < e1.max() < 5e-3 and e2.max() < 0.1 * e1.max()
    assert 5e-5 < em < 2e-3
    for j in range(P1.shape[0]):
        assert np.array_equal(P1[j], P1[j].conj().T)


@pytest.mark.parametrize("shape", [
    dict(n_k=2, n_b=60, R=1000, N=300, n_occ=3, n_unocc=150),
    dict(n_k=1, n_b=20, R=33, N=7, n_occ=1, n_unocc=5),
    dict(n_k=3, n_b=64, R=512, N=129, n_occ=2, n_unocc=63),
])
def test_three_product_core(lib, shape):
    """The three-multiplication (Gauss) form of the GEMM core (complex_product
    3, the default): polarization (projection and accumulation) and row-major projections
    on ragged multi-tile shapes, within the reduced-precision bar; P
    Hermitian; the judge's row projections in the learned path use it too."""
    import torch
    inp = gwsynth.generate(gwsynth.make_shape(**shape), seed=9, omega=gwsynth.omega_mesh("m16"))
    U, psi = _dev(inp)
    n_occ = shape["n_occ"]
    try:
        lib.gw_set_tuning("complex_product", 3)
        P = lib.gw_polarization(U, psi, inp.eps, inp.omega, n_occ, precision="split_bf16", kq=inp.kq)
        M = lib.gw_project(U, psi[0, :n_occ].contiguous(), psi[0, n_occ:].contiguous(), "split_bf16")
        Pc = lib.gw_polarization(U, psi, inp.eps, inp.omega, n_occ, precision="split_bf16", kq=inp.kq,
                                 chunk_pairs=256)
        torch.cuda.synchronize()
    finally:
        lib.gw_set_tuning("complex_product", 3)
    Ur, pr = _rounded(inp)
    ref = orc.polarization(Ur, pr, inp.eps, inp.omega, n_occ, kq=inp.kq)
    Pg = P.cpu().numpy()
    err = orc.rel_fro(Pg, ref)
    errc = orc.rel_fro(Pc.cpu().numpy(), ref)
    Mref = orc.projections(Ur, pr[0, :n_occ], pr[0, n_occ:])
    merr = np.linalg.norm(M.cpu().numpy() - Mref) / np.linalg.norm(Mref)
    print(f"three-product core {shape}: P max rel err {err.max():.2e} (chunked {errc.max():.2e}), M {merr:.2e}")
    assert err.max() < TOL and errc.max() < TOL
    assert merr < 2e-5
    for j in range(Pg.shape[0]):
        assert np.array_equal(Pg[j], Pg[j].conj().T)


@pytest.mark.parametrize("shape", [
    dict(n_k=2, n_b=60, R=1000, N=300, n_occ=3, n_unocc=150),    # 63 K stages: the six-slot ring's tail
    dict(n_k=1, n_b=20, R=33, N=7, n_occ=1, n_unocc=5),          # 3 stages: fewer than the ring's depth
    dict(n_k=3, n_b=64, R=512, N=129, n_occ=2, n_unocc=63),      # 32 stages
])
@pytest.mark.parametrize("prec", ["split_bf16", "split_fp16"])
def test_three_product_core_pipelines_bitwise(lib, shape, prec):
    """The two staging schemes of the three-multiplication core (two 72 KB
    stage buffers; six 24 KB plane slots copied 3, 4 (the default) or 5
    plane steps ahead) issue
    the same MFMAs in the same order on every accumulator, so P and M agree
    bit for bit; the slot ring also meets the reduced-precision bar against
    the oracle.  Split FP16 runs on the three-product core (fp16_core 2)."""
    import torch
    inp = gwsynth.generate(gwsynth.make_shape(**shape), seed=21, omega=gwsynth.omega_mesh("m16"))
    U, psi = _dev(inp)
    n_occ = shape["n_occ"]
    out = {}
    try:
        lib.gw_set_tuning("fp16_core", 2)
        for pipe, lead in ((2, 4), (6, 3), (6, 4), (6, 5)):
            lib.gw_set_tuning("gemm3m_pipeline", pipe)
            lib.gw_set_tuning("gemm3m_lead", lead)
            P = lib.gw_polarization(U, psi, inp.eps, inp.omega, n_occ, precision=prec, kq=inp.kq)
            M = lib.gw_project(U, psi[0, :n_occ].contiguous(), psi[0, n_occ:].contiguous(), prec)
            torch.cuda.synchronize()
            out[pipe, lead] = (P.cpu().numpy(), M.cpu().numpy())
    finally:
        lib.gw_set_tuning("gemm3m_pipeline", 6)
        lib.gw_set_tuning("gemm3m_lead", 4)
        lib.gw_set_tuning("fp16_core", 1)
    for key in ((6, 3), (6, 4), (6, 5)):
        assert np.array_equal(out[2, 4][0], out[key][0]) and np.array_equal(out[2, 4][1], out[key][1]), key
    Ur, pr = _rounded(inp)
    ref = orc.polarization(Ur, pr, inp.eps, inp.omega, n_occ, kq=inp.kq)
    err = orc.rel_fro(out[6, 4][0], ref)
    print(f"three-product core, six-slot ring, {prec} {shape}: P max rel err {err.max():.2e}")
    assert err.max() < TOL


@pytest.mark.parametrize("core", [1, 2])
def test_split_fp16_cores(lib, core):
    """Split FP16 on both kernel families: the operands staged inside the GEMM
    kernels with main and correction accumulators (fp16_core 1, the default:
    FP32-level accuracy), and the three-multiplication core on power-of-two
    scaled plane words with one accumulator set (fp16_core 2: twice as fast,
    accuracy of the split-BF16 class); ragged multi-tile shape, projection and
    polarization."""
    import torch
    shape = dict(n_k=2, n_b=60, R=1000, N=300, n_occ=3, n_unocc=150)
    inp = gwsynth.generate(gwsynth.make_shape(**shape), seed=13, omega=gwsynth.omega_mesh("m16"))
    U, psi = _dev(inp)
    try:
        lib.gw_set_tuning("fp16_core", core)
        P = lib.gw_polarization(U, psi, inp.eps, inp.omega, 3, precision="split_fp16", kq=inp.kq)
        M = lib.gw_project(U, psi[0, :3].contiguous(), psi[0, 3:].contiguous(), "split_fp16")
        torch.cuda.synchronize()
    finally:
        lib.gw_set_tuning("fp16_core", 1)
    Ur, pr = _rounded(inp)
    ref = orc.polarization(Ur, pr, inp.eps, inp.omega, 3, kq=inp.kq)
    err = orc.rel_fro(P.cpu().numpy(), ref)
    Mref = orc.projections(Ur, pr[0, :3], pr[0, 3:])
    merr = np.linalg.norm(M.cpu().numpy() - Mref) / np.linalg.norm(Mref)
    print(f"split FP16, core {core}: P max rel err {err.max():.2e}, M rel err {merr:.2e}")
    assert err.max() < (1e-6 if core == 1 else 1e-5) and merr < 2e-6
