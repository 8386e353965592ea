"""The learned path in one library call (gw_polarization_learned) against the
oracle by composition: the explicit sum to the cutoff, the features, the
FP64 perceptron with the same BF16-valued weights and the congruence, all in
the oracle, on the same inputs; the judge against the oracle's judge on the
same sample rows; the forced fallback against the all-band sum; and the
optional checks (GW_ERR_NONFINITE, GW_ERR_NOT_HPD) forced from the host."""
import numpy as np
import pytest

import gwsynth
from oracle import mlp as omlp
from oracle import polarization as orc
from oracle import surrogate as osg
from oracle.precision import round_bf16

pytestmark = pytest.mark.gpu

DIMS = (32, 256, 32)
N_OCC, CUT = 4, 21


def sample_rows(n_k, n_s, n_occ):
    """The library's judge sample: n_s occupied bands per k-set, evenly from
    the lowest to the highest (the middle band when n_s = 1)."""
    def band(i):
        return n_occ // 2 if n_s == 1 else (i * (n_occ - 1) + (n_s - 1) // 2) // (n_s - 1)
    return [(k, band(i)) for k in range(n_k) for i in range(n_s)]


def _params(seed=5):
    p = gwsynth.mlp_init(*DIMS, seed=seed)
    rng = np.random.default_rng(seed)
    p["b1"] = rng.normal(0, 0.1, DIMS[1])
    p["b2"] = rng.normal(0, 0.1, DIMS[1])
    p["b3"] = rng.normal(-1.0, 0.2, DIMS[2])
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def _oracle_params(p):
    q = dict(p)
    for k in ("W1", "W2", "W3"):
        q[k] = round_bf16(p[k]).astype(np.float64)
    return q


@pytest.fixture(scope="module")
def case():
    shp = gwsynth.make_shape(n_k=3, n_b=90, R=600, N=140, n_occ=N_OCC, n_unocc=70)
    inp = gwsynth.generate(shp, seed=31, omega=gwsynth.omega_mesh("m16"))
    return inp


def _inputs(inp, precision):
    import torch
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    U = torch.from_numpy(inp.U).cuda().to(dt)
    psi = torch.from_numpy(inp.psi).cuda().to(dt)
    if precision == "fp64":
        Uo, po = inp.U, inp.psi
    else:
        Uo = inp.U.astype(np.complex64).astype(np.complex128)
        po = inp.psi.astype(np.complex64).astype(np.complex128)
    return U, psi, Uo, po


def _learned(lib, inp, U, psi, precision, p, judge=True, tol=1e30, n_s=2, P=None, flags=0):
    import torch
    mlp = lib.Mlp(*DIMS, torch.device("cuda"), master=lib.Mlp.flat_from_dict(p, *DIMS), train=False)
    eps = torch.from_numpy(inp.eps).cuda()
    pol = lib.PolarizationCall(U, psi, inp.eps, inp.omega, N_OCC, precision=precision, eps_dev=eps, kq=inp.kq, P=P,
                               flags=flags)
    call = lib.LearnedCall(pol, mlp, CUT, judge=judge, n_sample_occ=n_s, judge_tol=tol)
    return call, mlp


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-4), ("split_bf16", 1e-4)])
def test_learned_call_matches_oracle_composition(lib, case, precision, bar):
    """P = P_ret + D P_ret D with y from the perceptron: the GPU call against
    the oracle's explicit sum, features, FP64 perceptron (BF16-valued weights)
    and congruence.  The perceptron's BF16 products bound the agreement (the
    FP64 sum alone agrees to 1e-10)."""
    import torch
    inp = case
    p = _params()
    U, psi, Uo, po = _inputs(inp, precision)
    print(f"learned call {precision}: N=140 R=600 n_k=3 cut={CUT}", flush=True)
    call, _ = _learned(lib, inp, U, psi, precision, p)
    P, rep = call.run()
    torch.cuda.synchronize()
    assert not rep["used_fallback"]
    Pr = orc.polarization(Uo, po, inp.eps, inp.omega, N_OCC, kq=inp.kq, unocc_range=(0, CUT))
    X = osg.features(Pr, inp.eps, inp.omega, N_OCC, CUT, inp.kq)
    y = omlp.forward(_oracle_params(p), X)[:, 0]
    ref = osg.apply(Pr, y)
    err = orc.rel_fro(P.cpu().numpy(), ref)
    print(f"  max rel err {err.max():.2e}")
    assert err.max() < bar, err
    # the judge: same sample rows, the oracle's left-out sample explicitly summed
    rows = sample_rows(3, 2, N_OCC)
    Ps = np.zeros_like(Pr)
    for (k, n) in rows:
        Ps += orc.polarization(Uo, po, inp.eps, inp.omega, N_OCC, kq=inp.kq, k_list=[k], occ_range=(n, n + 1),
                               unocc_range=(CUT, 70))
    eref = osg.judge(Pr, y, Ps, inp.eps, N_OCC, CUT, inp.omega, rows, inp.kq)
    np.testing.assert_allclose(rep["judge_err"], eref, rtol=1e-3, atol=1e-6)


def test_learned_call_unjudged_equals_judged_pass(lib, case):
    """judge = 0 applies the same correction without the sample (asynchronous
    call): bit-identical P."""
    import torch
    inp = case
    p = _params()
    U, psi, _, _ = _inputs(inp, "split_bf16")
    a, _ = _learned(lib, inp, U, psi, "split_bf16", p)
    Pa = a.run()[0].clone()
    b, _ = _learned(lib, inp, U, psi, "split_bf16", p, judge=False)
    Pb, rep = b.run()
    torch.cuda.synchronize()
    assert not rep["used_fallback"] and "judge_err" not in rep
    assert torch.equal(Pa, Pb)


@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("split_bf16", 1e-4)])
def test_learned_call_fallback_is_the_all_band_sum(lib, case, precision, bar):
    """judge_tol = 0 fails the judge (host-forced): P is the explicit sum over
    all bands."""
    import torch
    inp = case
    U, psi, Uo, po = _inputs(inp, precision)
    call, _ = _learned(lib, inp, U, psi, precision, _params(), tol=0.0, n_s=1)
    P, rep = call.run()
    torch.cuda.synchronize()
    assert rep["used_fallback"] and rep["judge_err_max"] > 0.0
    ref = orc.polarization(Uo, po, inp.eps, inp.omega, N_OCC, kq=inp.kq)
    assert orc.rel_fro(P.cpu().numpy(), ref).max() < bar


def test_nonfinite_input_is_reported_before_any_work(lib, case):
    import torch
    inp = case
    U, psi, _, _ = _inputs(inp, "split_bf16")
    U = U.clone()
    U[7, 11] = complex(float("nan"), 0.0)
    P = torch.full((inp.omega.size, 140, 140), 3.0 + 0j, dtype=torch.complex128, device="cuda")
    pol = lib.PolarizationCall(U, psi, inp.eps, inp.omega, N_OCC, precision="split_bf16", kq=inp.kq, P=P,
                               flags=lib.GW_CHECK_FINITE)
    with pytest.raises(lib.GwError) as e:
        pol.run()
    assert e.value.status == -5
    torch.cuda.synchronize()
    assert bool((P == 3.0).all())          # nothing was computed
    call, _ = _learned(lib, inp, U, psi, "split_bf16", _params(), flags=lib.GW_CHECK_FINITE)
    with pytest.raises(lib.GwError) as e:
        call.run()
    assert e.value.status == -5
    # clean inputs with the check on: same result as without it
    U2, psi2, _, _ = _inputs(inp, "split_bf16")
    a = lib.PolarizationCall(U2, psi2, inp.eps, inp.omega, N_OCC, precision="split_bf16", kq=inp.kq,
                             flags=lib.GW_CHECK_FINITE).run().clone()
    b = lib.PolarizationCall(U2, psi2, inp.eps, inp.omega, N_OCC, precision="split_bf16", kq=inp.kq).run()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_screen_checks(lib, case):
    """GW_CHECK_HPD: a positive P makes eps indefinite -> GW_ERR_NOT_HPD with
    the failing column in info; GW_CHECK_FINITE on a NaN in P; a valid P
    passes both checks with the result of the unchecked call."""
    import torch
    inp = case
    Pr = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega[:3], N_OCC, kq=inp.kq)
    P = torch.from_numpy(Pr).cuda()
    v = torch.from_numpy(inp.v).cuda()
    W0, _ = lib.gw_screen(P, v)
    W1, info = lib.gw_screen(P, v, flags=lib.GW_CHECK_FINITE | lib.GW_CHECK_HPD)
    torch.cuda.synchronize()
    assert int(info.abs().sum()) == 0 and torch.equal(W0, W1)
    with pytest.raises(lib.GwError) as e:
        lib.gw_screen(-P, v, flags=lib.GW_CHECK_HPD)
    assert e.value.status == -6
    W2, info2 = lib.gw_screen(-P, v)
    torch.cuda.synchronize()
    assert int(info2.cpu().max()) > 0
    Pn = P.clone()
    Pn[1, 5, 3] = complex(float("inf"), 0.0)
    with pytest.raises(lib.GwError) as e:
        lib.gw_screen(Pn, v, flags=lib.GW_CHECK_FINITE)
    assert e.value.status == -5
