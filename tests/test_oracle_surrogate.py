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
