"""Perceptron kernels and surrogate kernels vs the CPU FP64 oracle.

The GPU multiplies with BF16 copies of the FP32 master weights; the oracle
gets the same BF16 values, rounded on the host from the IEEE definition.
Activations enter the MFMA as hi + lo BF16 pairs, so forward outputs agree to
about 1e-5 relative; gradients (FP32 accumulation over the rows) to 1e-4."""
import os

import numpy as np
import pytest

import gwsynth
from oracle import mlp as omlp
from oracle import polarization as orc
from oracle import surrogate as osg
from oracle.precision import round_bf16

pytestmark = pytest.mark.gpu

DIMS = (32, 256, 32)


def _params(seed=3):
    p = gwsynth.mlp_init(*DIMS, seed=seed)
    rng = np.random.default_rng(seed)
    p["b1"] = rng.normal(0, 0.1, DIMS[1])
    p["b2"] = rng.normal(0, 0.1, DIMS[1])
    p["b3"] = rng.normal(0, 0.1, DIMS[2])
    p["W3"] = p["W3"] * 10
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def _oracle_params(p):
    """Weights as the GPU multiplies them: BF16 values; biases FP32."""
    q = dict(p)
    for k in ("W1", "W2", "W3"):
        q[k] = round_bf16(p[k]).astype(np.float64)
    return q


def _mlp(lib, p):
    import torch
    return lib.Mlp(*DIMS, torch.device("cuda"), master=lib.Mlp.flat_from_dict(p, *DIMS))


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_mlp_forward_matches_oracle(lib):
    import torch
    p = _params()
    m = _mlp(lib, p)
    rng = np.random.default_rng(1)
    X = rng.normal(0, 1, (1000, 32)).astype(np.float32)
    Y, act = m.forward(torch.from_numpy(X).cuda())
    torch.cuda.synchronize()
    Yr, cache = omlp.forward(_oracle_params(p), X.astype(np.float64), keep=True)
    assert _rel(Y.cpu().numpy(), Yr) < 1e-5
    a = act.cpu().numpy().reshape(4, 1000, 256)   # z1, h1, z2, h2 blocks
    assert _rel(a[1], cache[2]) < 1e-5
    assert _rel(a[3], cache[4]) < 1e-5


def test_mlp_loss_backward_match_oracle(lib):
    import torch
    p = _params(5)
    m = _mlp(lib, p)
    rng = np.random.default_rng(2)
    rows = 777
    X = rng.normal(0, 1, (rows, 32)).astype(np.float32)
    T = rng.normal(0, 1, (rows, 1)).astype(np.float32)
    M = (rng.uniform(size=(rows, 1)) > 0.1).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    Y, act = m.forward(Xd)
    L, dY = m.loss(Y, torch.from_numpy(T).cuda(), torch.from_numpy(M).cuda(), n_used=1)
    grad, dX = m.backward(Xd, act, dY, want_dx=True)
    torch.cuda.synchronize()
    q = _oracle_params(p)
    Yr, cache = omlp.forward(q, X.astype(np.float64), keep=True)
    Tfull = np.zeros_like(Yr)
    Tfull[:, :1] = T
    Mfull = np.zeros_like(Yr)
    Mfull[:, :1] = M
    Lr, dYr = omlp.loss(Yr, Tfull, Mfull)
    gr, dXr = omlp.backward(q, cache, dYr)
    assert abs(float(L.cpu()) - Lr) < 1e-5 * abs(Lr)
    assert _rel(dY.cpu().numpy(), dYr) < 1e-5
    gd = lib.Mlp.flat_from_dict(gr, *DIMS)
    gg = grad.cpu().numpy()
    offs = np.cumsum([0, 32 * 256, 256, 256 * 256, 256, 256 * 32, 32])
    for a, b, name in zip(offs[:-1], offs[1:], ["W1", "b1", "W2", "b2", "W3", "b3"]):
        assert _rel(gg[a:b], gd[a:b]) < 1e-4, name
    assert _rel(dX.cpu().numpy(), dXr) < 1e-4


def test_adam_step_matches_oracle_and_refreshes_bf16(lib):
    import torch
    p = _params(7)
    m = _mlp(lib, p)
    rng = np.random.default_rng(3)
    g = rng.normal(0, 1e-2, m.master.numel()).astype(np.float32)
    gd = torch.from_numpy(g).cuda()
    m.adam(gd, lr=1e-3)
    m.adam(gd * 0.5, lr=1e-3)
    torch.cuda.synchronize()
    flat = lib.Mlp.flat_from_dict(p, *DIMS).astype(np.float64)
    P = {"x": flat.copy()}
    mm = {"x": np.zeros_like(flat)}
    vv = {"x": np.zeros_like(flat)}
    omlp.adam_step(P, {"x": g.astype(np.float64)}, mm, vv, 1, lr=1e-3)
    omlp.adam_step(P, {"x": 0.5 * g.astype(np.float64)}, mm, vv, 2, lr=1e-3)
    got = m.master.cpu().numpy()
    assert np.abs(got - P["x"]).max() < 1e-6
    # wk holds BF16(master) in master layout for W1
    wk = m.wk.cpu().numpy().view(np.uint16)[:32 * 256]
    w1 = np.frombuffer((wk.astype(np.uint32) << 16).tobytes(), dtype=np.float32)
    np.testing.assert_array_equal(w1, round_bf16(got[:32 * 256]))


def test_mlp_training_reduces_loss(lib):
    import torch
    init = gwsynth.mlp_init(*DIMS, seed=9)
    m = lib.Mlp(*DIMS, torch.device("cuda"), master=lib.Mlp.flat_from_dict(init, *DIMS))
    rng = np.random.default_rng(4)
    X = rng.uniform(-1, 1, (4096, 32)).astype(np.float32)
    T = (np.sin(2 * X[:, :1]) + X[:, 1:2] * X[:, 2:3]).astype(np.float32)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    first = None
    for step in range(300):
        Y, act = m.forward(Xd)
        L, dY = m.loss(Y, Td, None, n_used=1)
        grad, _ = m.backward(Xd, act, dY)
        m.adam(grad, lr=2e-3)
        if first is None:
            first = float(L.cpu())
    last = float(L.cpu())
    assert last < 0.05 * first, (first, last)


@pytest.fixture(scope="module")
def surr_case():
    shp = gwsynth.make_shape(n_k=3, n_b=80, R=512, N=150, n_occ=3, n_unocc=60)
    inp = gwsynth.generate(shp, seed=23, omega=gwsynth.omega_mesh("m16"))
    Pr = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=inp.kq, unocc_range=(0, 20))
    Pf = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=inp.kq)
    return inp, Pr, Pf


def test_surrogate_features_targets_match_oracle(lib, surr_case):
    import torch
    inp, Pr, Pf = surr_case
    Prd = torch.from_numpy(Pr).cuda()
    eps = torch.from_numpy(inp.eps).cuda()
    args = lib.SurrogateArgs(Prd, eps, inp.omega, 3, 20, inp.kq)
    X = lib.gw_surrogate_features(args)
    T, M = lib.gw_surrogate_targets(Prd, torch.from_numpy(Pf).cuda())
    torch.cuda.synchronize()
    Xr = osg.features(Pr, inp.eps, inp.omega, 3, 20, inp.kq)
    np.testing.assert_allclose(X.cpu().numpy(), Xr, rtol=1e-5, atol=1e-6)
    Tr, Mr = osg.targets(Pr, Pf)
    np.testing.assert_array_equal(M.cpu().numpy(), Mr)
    np.testing.assert_allclose(T.cpu().numpy(), Tr, rtol=1e-6, atol=1e-6)


def test_surrogate_apply_and_judge_match_oracle(lib, surr_case):
    import torch
    inp, Pr, Pf = surr_case
    N, n_om = Pr.shape[1], Pr.shape[0]
    rng = np.random.default_rng(5)
    y = rng.normal(-0.5, 0.7, (n_om * N, 32)).astype(np.float32)
    Pd = torch.from_numpy(Pr).cuda()
    Yd = torch.from_numpy(y).cuda()
    lib.gw_surrogate_apply(Pd, Yd, 32)
    ref = osg.apply(Pr, y[:, 0].astype(np.float64))
    assert orc.rel_fro(Pd.cpu().numpy(), ref).max() < 1e-13
    # judge with a sample of occupied rows
    rows = [(k, n) for k in range(3) for n in range(1)]
    Ps = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=inp.kq, occ_range=(0, 1),
                          unocc_range=(20, 60))
    args = lib.SurrogateArgs(torch.from_numpy(Pr).cuda(), torch.from_numpy(inp.eps).cuda(), inp.omega, 3, 20,
                             inp.kq)
    err = lib.gw_surrogate_judge(args, Yd, 32, torch.from_numpy(Ps).cuda(), rows)
    torch.cuda.synchronize()
    eref = osg.judge(Pr, y[:, 0].astype(np.float64), Ps, inp.eps, 3, 20, inp.omega, rows, inp.kq)
    np.testing.assert_allclose(err.cpu().numpy(), eref, rtol=1e-6)


def test_surrogate_path_parity_with_trained_model(lib, surr_case):
    """GPU (features -> perceptron -> correction) vs oracle (same features
    definition, FP64 perceptron with the same BF16-valued weights, same
    correction) on identical P_ret: within 1e-4."""
    import torch
    from paper_1003_0316_amd.surrogate import DEFAULT_MODEL, Surrogate
    if not os.path.exists(DEFAULT_MODEL):
        pytest.skip("no trained model committed yet")
    inp, Pr, Pf = surr_case
    sur = Surrogate.load_default(torch.device("cuda"))
    Pd = torch.from_numpy(Pr).cuda()
    sur.apply(Pd, torch.from_numpy(inp.eps).cuda(), inp.omega, 3, 20, inp.kq)
    torch.cuda.synchronize()
    p = sur.mlp.to_dict()
    X = osg.features(Pr, inp.eps, inp.omega, 3, 20, inp.kq)
    y = omlp.forward(_oracle_params(p), X)[:, 0]
    ref = osg.apply(Pr, y)
    err = orc.rel_fro(Pd.cpu().numpy(), ref)
    assert err.max() < 1e-4, err


def test_surrogate_gain_over_truncation(lib):
    """On held-out seeds (not used in training) the corrected P is closer to
    the full-band P than the truncated sum, at every frequency.  The model
    error itself has no closed form to pin; this measures it against the
    explicit full-band sum."""
    import torch
    from paper_1003_0316_amd.surrogate import DEFAULT_MODEL, Surrogate
    from paper_1003_0316_amd import train_surrogate as ts
    if not os.path.exists(DEFAULT_MODEL):
        pytest.skip("no trained model committed yet")
    sur = Surrogate.load_default(torch.device("cuda"))
    seeds = [gwsynth.BASE_SEED + ts.SEED0 + 210, gwsynth.BASE_SEED + ts.SEED0 + 219]
    ev = ts.evaluate(sur, seeds, torch.device("cuda"), cuts=(300,))
    r = ev["300"]
    print("held-out: truncation", r["trunc_per_omega_mean"], "corrected", r["model_per_omega_mean"])
    assert np.all(np.array(r["model_per_omega_mean"]) < np.array(r["trunc_per_omega_mean"]))
    assert r["model_mean"] < 0.5 * r["trunc_mean"]


def test_surrogate_judge_forces_fallback(lib):
    """judge_tol = 0 always fails the judge: the path must return the explicit
    full-band sum (host-forced condition)."""
    import torch
    from paper_1003_0316_amd.surrogate import DEFAULT_MODEL, Surrogate
    if not os.path.exists(DEFAULT_MODEL):
        pytest.skip("no trained model committed yet")
    shp = gwsynth.make_shape(n_k=2, n_b=80, R=512, N=150, n_occ=3, n_unocc=60)
    inp = gwsynth.generate(shp, seed=29, omega=gwsynth.omega_mesh("m16"))
    dev = torch.device("cuda")
    U = torch.from_numpy(inp.U).to(dev, torch.complex64)
    psi = torch.from_numpy(inp.psi).to(dev, torch.complex64)
    eps = torch.from_numpy(inp.eps).to(dev)
    sur = Surrogate.load_default(dev, judge_tol=0.0)
    P, rep = sur.learned_call(U, psi, inp.eps, eps, inp.omega, 3, 20, inp.kq, precision="split_bf16").run()
    torch.cuda.synchronize()
    assert rep["used_fallback"]
    Ur = inp.U.astype(np.complex64).astype(np.complex128)
    pr = inp.psi.astype(np.complex64).astype(np.complex128)
    ref = orc.polarization(Ur, pr, inp.eps, inp.omega, 3, kq=inp.kq)
    assert orc.rel_fro(P.cpu().numpy(), ref).max() < 1e-4
