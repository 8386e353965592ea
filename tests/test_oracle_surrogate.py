"""Pins of the surrogate oracle: brute-force loops for the weight sums and
band edges, and closed-form properties of the correction."""
import numpy as np

import gwsynth
from oracle import polarization as orc
from oracle import surrogate as osg


def _small():
    shp = gwsynth.make_shape(n_k=2, n_b=30, R=64, N=10, n_occ=2, n_unocc=12)
    return gwsynth.generate(shp, seed=17, omega=(0.0, 0.3, 4.0))


def test_weight_sums_bruteforce():
    inp = _small()
    lo, hi = osg.weight_sums(inp.eps, 2, 5, inp.omega, inp.kq)
    for j, w in enumerate(inp.omega):
        a = b = 0.0
        for k in range(2):
            for n in range(2):
                for u in range(12):
                    d = inp.eps[k, n] - inp.eps[(k + 1) % 2, 2 + u]
                    x = abs(4 * d / (d * d + w * w))
                    if u < 5:
                        a += x
                    else:
                        b += x
        assert abs(lo[j] - a) < 1e-12 * a and abs(hi[j] - b) < 1e-12 * b


def test_band_edges_bruteforce():
    inp = _small()
    e = osg.band_edges(inp.eps, 2, 5)
    ref = [np.mean([inp.eps[k][i] for k in range(2)]) for i in (0, 1, 2, 6, 13)]
    np.testing.assert_allclose(e, ref, rtol=1e-15)


def test_apply_adds_predicted_diagonal_and_stays_nsd():
    inp = _small()
    P = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 2, kq=inp.kq, unocc_range=(0, 5))
    rng = np.random.default_rng(0)
    y = rng.normal(-1, 1, P.shape[0] * P.shape[1])
    Q = osg.apply(P, y)
    d = np.real(np.einsum("jii->ji", Q - P)).reshape(-1)
    pr = np.abs(np.real(np.einsum("jii->ji", P))).reshape(-1)
    np.testing.assert_allclose(-d, pr * np.exp(y), rtol=1e-13)
    for j in range(Q.shape[0]):
        assert np.abs(Q[j] - Q[j].conj().T).max() < 1e-14 * np.abs(Q[j]).max()
        assert np.linalg.eigvalsh(Q[j]).max() < 1e-12 * np.abs(Q[j]).max()


def test_exact_target_recovers_full_diagonal():
    """With y equal to the target the corrected diagonal is the full-band one."""
    inp = _small()
    Pr = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 2, kq=inp.kq, unocc_range=(0, 5))
    Pf = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 2, kq=inp.kq)
    t, m = osg.targets(Pr, Pf)
    assert m.all()
    Q = osg.apply(Pr, t)
    np.testing.assert_allclose(np.einsum("jii->ji", Q).real, np.einsum("jii->ji", Pf).real, rtol=1e-12)


def test_features_shape_and_definitions():
    inp = _small()
    Pr = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 2, kq=inp.kq, unocc_range=(0, 5))
    X = osg.features(Pr, inp.eps, inp.omega, 2, 5, inp.kq)
    N = 10
    assert X.shape == (3 * N, 32) and np.all(X[:, 12:] == 0)
    lo, hi = osg.weight_sums(inp.eps, 2, 5, inp.omega, inp.kq)
    np.testing.assert_allclose(X[N:2 * N, 1], np.log(hi[1] / lo[1]))
    np.testing.assert_allclose(X[:N, 2], 0.0, atol=1e-15)
    np.testing.assert_allclose(X[:N, 4], np.arange(N) / N)
    np.testing.assert_allclose(X[:, 9], 5 / 12)


def test_judge_zero_when_sample_is_everything():
    """Sample = all rows: f = 1 and TR_s is the exact left-out trace, so the
    judge error is zero exactly when y is the exact target."""
    inp = _small()
    Pr = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 2, kq=inp.kq, unocc_range=(0, 5))
    Pf = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 2, kq=inp.kq)
    t, _ = osg.targets(Pr, Pf)
    rows = [(k, n) for k in range(2) for n in range(2)]
    err = osg.judge(Pr, t, Pf - Pr, inp.eps, 2, 5, inp.omega, rows, inp.kq)
    assert err.max() < 1e-12
    err2 = osg.judge(Pr, t + 0.5, Pf - Pr, inp.eps, 2, 5, inp.omega, rows, inp.kq)
    assert err2.min() > 0.3


# ----------------------------------------------------- hand-worked fixtures
import json
import math
import os
from fractions import Fraction

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "surrogate_hand.json")


def _hand():
    with open(GOLDEN) as fh:
        return json.load(fh)


def _val(expr, names=None):
    """Evaluate a fixture expression: exact fractions, log, abs, sqrt."""
    env = {"log": math.log, "abs": abs, "sqrt": math.sqrt}
    env.update(names or {})
    e = expr
    if not any(c.isalpha() for c in expr):
        return float(sum(Fraction(t.strip()) for t in expr.split("+")))
    return float(eval(e, {"__builtins__": {}}, env))


def _bands(h):
    b = h["bands"]
    eps = np.array(b["eps"])
    S = {"Sl0": _val(b["S_lo"][0]), "Sl1": _val(b["S_lo"][1]), "Sh0": _val(b["S_hi"][0]),
         "Sh1": _val(b["S_hi"][1])}
    return b, eps, S


def _diag_P(diag):
    d = np.asarray(diag, dtype=np.float64)
    P = np.zeros((d.shape[0], d.shape[1], d.shape[1]), dtype=np.complex128)
    for j in range(d.shape[0]):
        P[j] = np.diag(d[j])
        P[j][0, 1], P[j][1, 0] = 0.25 - 0.5j, 0.25 + 0.5j     # off-diagonals must not matter
    return P


def test_hand_weight_sums_and_edges():
    h = _hand()
    b, eps, S = _bands(h)
    lo, hi = osg.weight_sums(eps, b["n_occ"], b["cut"], b["omega"], b["kq"])
    np.testing.assert_allclose(lo, [S["Sl0"], S["Sl1"]], rtol=1e-14)
    np.testing.assert_allclose(hi, [S["Sh0"], S["Sh1"]], rtol=1e-14)
    np.testing.assert_allclose(osg.band_edges(eps, b["n_occ"], b["cut"]), [_val(e) for e in b["edges"]], rtol=1e-15)


def test_hand_feature_rows():
    h = _hand()
    b, eps, S = _bands(h)
    P = _diag_P(h["features"]["P_ret_diag"])
    X = osg.features(P, eps, b["omega"], b["n_occ"], b["cut"], b["kq"])
    want = np.array([[_val(e, S) for e in row] for row in h["features"]["rows"]])
    np.testing.assert_allclose(X[:, :12], want, rtol=1e-13, atol=1e-14)


def test_hand_judge_with_a_partial_sample():
    """One sampled row of four: the share f is 144/335 at w = 0, so an inverted
    share or a share over the wrong rows gives a different error."""
    h = _hand()
    b, eps, S = _bands(h)
    P = _diag_P(h["features"]["P_ret_diag"])
    Ps = _diag_P(h["judge"]["P_sample_diag"])
    rows = [tuple(r) for r in h["judge"]["sample_rows"]]
    err = osg.judge(P, np.array(h["judge"]["y"]), Ps, eps, b["n_occ"], b["cut"], b["omega"], rows, b["kq"])
    want = [_val(e, S) for e in h["judge"]["err"]]
    np.testing.assert_allclose(err, want, rtol=1e-13)
    assert abs(want[0] - 97 / 432) < 1e-15


def test_hand_rel_fro_per_frequency():
    from oracle import polarization as orc
    r = _hand()["rel_fro"]
    x = np.array(r["x_re"]) + 1j * np.array(r["x_im"])
    ref = np.array(r["ref_re"]) + 1j * np.array(r["ref_im"])
    np.testing.assert_allclose(orc.rel_fro(x, ref), [_val(e) for e in r["err"]], rtol=1e-15)
    np.testing.assert_allclose(orc.rel_fro(x[1], ref[1]), [math.sqrt(5) / 3], rtol=1e-15)


# ------------------------------------------------ brute force from the definitions

def _bracket_abs(d, w):
    return abs(4.0 * d / (d * d + w * w))


def _brute_sums(eps, n_occ, cut, omega, kq, rows):
    n_unocc = eps.shape[1] - n_occ
    lo = [0.0] * len(omega)
    hi = [0.0] * len(omega)
    for j, w in enumerate(omega):
        for (k, n) in rows:
            for u in range(n_unocc):
                x = _bracket_abs(eps[k][n] - eps[kq[k]][n_occ + u], w)
                if u < cut:
                    lo[j] += x
                else:
                    hi[j] += x
    return lo, hi


def test_features_every_column_bruteforce():
    """All twelve columns on a 3-set case with a nontrivial k+q map, each
    computed with plain loops from the definitions."""
    shp = gwsynth.make_shape(n_k=3, n_b=30, R=64, N=7, n_occ=3, n_unocc=9)
    inp = gwsynth.generate(shp, seed=23, omega=(0.0, 0.4, 3.0))
    kq = [2, 0, 1]
    cut = 4
    Pr = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=kq, unocc_range=(0, cut))
    X = osg.features(Pr, inp.eps, inp.omega, 3, cut, kq)
    n_k, N, eps, om = 3, 7, inp.eps, list(inp.omega)
    all_rows = [(k, n) for k in range(n_k) for n in range(3)]
    lo, hi = _brute_sums(eps, 3, cut, om, kq, all_rows)
    e0 = sum(eps[k][0] for k in range(n_k)) / n_k
    e1 = sum(eps[k][2] for k in range(n_k)) / n_k
    e2 = sum(eps[k][3] for k in range(n_k)) / n_k
    e3 = sum(eps[k][3 + cut - 1] for k in range(n_k)) / n_k
    e4 = sum(eps[k][3 + 9 - 1] for k in range(n_k)) / n_k
    for j, w in enumerate(om):
        p = [abs(Pr[j][I][I].real) for I in range(N)]
        p0 = [abs(Pr[0][I][I].real) for I in range(N)]
        pm = sum(p) / N
        for I in range(N):
            want = [w / (1 + w), math.log(hi[j]) - math.log(lo[j]), math.log(p[I]) - math.log(p0[I]),
                    math.log(p[I]) - math.log(pm), I / N, e3 - e2, e4 - e3, e1 - e0, e2 - e1, cut / 9,
                    (math.log(hi[j]) - math.log(lo[j])) - (math.log(hi[0]) - math.log(lo[0])),
                    math.log(lo[j]) - math.log(lo[0])]
            np.testing.assert_allclose(X[j * N + I, :12], want, rtol=1e-12, atol=1e-13)
            assert np.all(X[j * N + I, 12:] == 0)


def test_judge_partial_sample_bruteforce():
    """Sample of two rows out of nine, spread over the occupied range; share,
    traces and error by plain loops."""
    shp = gwsynth.make_shape(n_k=3, n_b=30, R=64, N=6, n_occ=3, n_unocc=8)
    inp = gwsynth.generate(shp, seed=29, omega=(0.0, 1.0))
    kq = [1, 2, 0]
    cut = 3
    Pr = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=kq, unocc_range=(0, cut))
    rows = [(0, 2), (2, 0)]
    Ps = np.zeros_like(Pr)
    for (k, n) in rows:
        Ps += orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=kq, k_list=[k], occ_range=(n, n + 1),
                               unocc_range=(cut, 8))
    rng = np.random.default_rng(3)
    y = rng.normal(-0.5, 0.7, 2 * 6)
    err = osg.judge(Pr, y, Ps, inp.eps, 3, cut, inp.omega, rows, kq)
    all_rows = [(k, n) for k in range(3) for n in range(3)]
    _, hi_all = _brute_sums(inp.eps, 3, cut, list(inp.omega), kq, all_rows)
    _, hi_s = _brute_sums(inp.eps, 3, cut, list(inp.omega), kq, rows)
    for j in range(2):
        tp = sum(abs(Pr[j][I][I].real) * math.exp(y[j * 6 + I]) for I in range(6))
        ts = sum(abs(Ps[j][I][I].real) for I in range(6))
        f = hi_s[j] / hi_all[j]
        assert 0.05 < f < 0.6
        assert abs(err[j] - abs(ts / f - tp) / tp) < 1e-12 * max(1.0, err[j])
