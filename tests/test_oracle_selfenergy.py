"""Pins of the self-energy oracle (Eq. SEc_AC) against things other than itself:
a library spline, adaptive quadrature, residue calculus for a plasmon-pole
W^c, and brute-force loops for the matrix elements."""
import numpy as np
import pytest
from scipy import integrate, interpolate

from oracle import polarization as orc
from oracle import selfenergy as ose

MESH = np.concatenate([[0.0], np.geomspace(0.01, 20.0, 15)])   # 16 points, as the workloads use


def test_spline_matches_library_clamped_spline():
    rng = np.random.default_rng(1)
    q = rng.normal(size=MESH.size)
    L = ose.lam(MESH)
    end = -2.0 * q[-1] / MESH[-1] / (1.0 - L[-1]) ** 2
    ref = interpolate.CubicSpline(L, q, bc_type=((1, 0.0), (1, end)))
    w = np.concatenate([MESH, np.geomspace(1e-3, 19.0, 50)])
    got = ose.spline_eval(MESH, q, w)
    assert np.allclose(got, ref(ose.lam(w)), rtol=1e-12, atol=1e-12)
    # the tail continues the spline with its value and slope
    e = 1e-6 * MESH[-1]
    left = ose.spline_eval(MESH, q, [MESH[-1] - e, MESH[-1]])
    right = ose.spline_eval(MESH, q, [MESH[-1], MESH[-1] + e])
    assert abs((left[1] - left[0]) - (right[1] - right[0])) < 1e-8 * abs(q[-1])


def _quad_integral(q, w, e):
    """int_{-inf}^{inf} q(w') / (i w + i w' - e) dw' by adaptive quadrature of
    the interpolant (even in w'), split at the mesh points and the tail."""
    def f(x, part):
        val = ose.spline_eval(MESH, q, [x])[0]
        k = 1.0 / (1j * (w + x) - e) + 1.0 / (1j * (w - x) - e)
        return (val * k).real if part == 0 else (val * k).imag
    tot = 0.0 + 0.0j
    pts = list(MESH)
    for a, b in zip(pts[:-1], pts[1:]):
        extra = [x for x in (w, abs(e)) if a < x < b]
        for part in (0, 1):
            v, _ = integrate.quad(f, a, b, args=(part,), points=extra or None, epsabs=1e-13, epsrel=1e-12, limit=400)
            tot += v if part == 0 else 1j * v
    for part in (0, 1):
        v, _ = integrate.quad(f, MESH[-1], np.inf, args=(part,), epsabs=1e-13, epsrel=1e-12, limit=400)
        tot += v if part == 0 else 1j * v
    return tot


@pytest.mark.parametrize("w,e", [(0.0, 0.02), (0.0, -0.3), (0.51, 1.7), (3.9234, -0.02), (20.0, 0.5), (35.0, -2.2)])
def test_weights_match_adaptive_quadrature(w, e):
    rng = np.random.default_rng(7)
    q = -np.abs(rng.normal(size=MESH.size)) / (1.0 + MESH ** 2)
    W = ose.freq_weights(MESH, [w], [e])[0, 0]
    got = W @ q
    ref = _quad_integral(q, w, e)
    assert abs(got - ref) <= 1e-9 * abs(ref)


def test_plasmon_pole_limit():
    """W^c(i w') = -2 a Omega / (Omega^2 + w'^2) has (residues)
    int dw' W^c / (i w + i w' - e) = 2 pi a / (sgn(e) Omega + e - i w);
    the spline-plus-tail integral converges to it as the mesh is refined."""
    a, Om = 0.7, 0.9
    for w, e in [(0.0, 0.05), (0.3, -0.4), (2.0, 1.1)]:
        exact = 2 * np.pi * a / (np.sign(e) * Om + e - 1j * w)
        errs = []
        for n in (16, 64, 256):
            mesh = np.concatenate([[0.0], np.geomspace(0.005, 400.0, n - 1)])
            q = -2 * a * Om / (Om ** 2 + mesh ** 2)
            got = ose.freq_weights(mesh, [w], [e])[0, 0] @ q
            errs.append(abs(got - exact) / abs(exact))
        assert errs[2] < 1e-5 and errs[2] < errs[1] < errs[0], errs


def test_quad_forms_brute_force():
    rng = np.random.default_rng(3)
    N, R, nb, nw = 4, 6, 3, 2
    U = rng.normal(size=(N, R)) + 1j * rng.normal(size=(N, R))
    ps = rng.normal(size=R) + 1j * rng.normal(size=R)
    pa = rng.normal(size=(nb, R)) + 1j * rng.normal(size=(nb, R))
    X = rng.normal(size=(nw, N, N)) + 1j * rng.normal(size=(nw, N, N))
    Wc = X + np.conj(np.transpose(X, (0, 2, 1)))
    got = ose.quad_forms(U, ps, pa, Wc)
    for j in range(nw):
        for b in range(nb):
            m = [sum(U[I, r] * np.conj(ps[r]) * pa[b, r] for r in range(R)) for I in range(N)]
            val = sum(np.conj(m[i]) * Wc[j, i, k] * m[k] for i in range(N) for k in range(N))
            assert abs(val.imag) < 1e-12 * abs(val)
            assert abs(got[j, b] - val.real) < 1e-12 * abs(val)


def test_sigma_c_plasmon_pole_matrix():
    """W^c_j = f(w_j) B with f the plasmon pole and B Hermitian: every band
    contributes -(m^H B m) a / (sgn(e) Omega + e - i w) in the dense-mesh limit."""
    rng = np.random.default_rng(11)
    N, R, nb, n_k = 3, 5, 4, 2
    U = rng.normal(size=(N, R)) + 1j * rng.normal(size=(N, R))
    psi = (rng.normal(size=(n_k, nb, R)) + 1j * rng.normal(size=(n_k, nb, R))) / np.sqrt(R)
    eps = np.sort(rng.uniform(-1.0, 1.0, size=(n_k, nb)), axis=1)
    mu = 0.013
    X = rng.normal(size=(N, N)) + 1j * rng.normal(size=(N, N))
    B = X @ X.conj().T
    a, Om = 1.0, 0.8
    mesh = np.concatenate([[0.0], np.geomspace(0.005, 400.0, 255)])
    f = -2 * a * Om / (Om ** 2 + mesh ** 2)
    Wc = [f[:, None, None] * B[None]] * n_k
    w_out = [0.0, 0.37, 2.5]
    got = ose.sigma_c(U, psi, eps, Wc, mesh, w_out, [(0, 1)], mu)[0]
    ref = np.zeros(len(w_out), dtype=np.complex128)
    for t in range(n_k):
        s2 = (0 + t) % n_k
        M = orc.projections(U, psi[0, 1][None], psi[s2])
        for b in range(nb):
            e = eps[s2, b] - mu
            qb = np.real(M[:, b].conj() @ B @ M[:, b])
            ref += -qb * a / (np.sign(e) * Om + e - 1j * np.asarray(w_out))
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-5


def test_weights_reject_bad_mesh_and_fermi_level():
    with pytest.raises(ValueError):
        ose.spline_basis([0.1, 1.0, 2.0])
    with pytest.raises(ValueError):
        ose.freq_weights(MESH, [0.0], [0.0])
