"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test would fail for a plausible slip in the oracle: a dropped conjugate,
a transposed operand, a wrong sign or factor in the frequency bracket, a wrong
k+q map, a wrong row/column scaling in the screening.
"""
import json
import math
import os

import numpy as np
import pytest

import gwsynth
from oracle import polarization as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def tiny(n_k=2, n_b=6, R=8, N=5, n_occ=2, n_unocc=3, seed=11, omega=(0.0, 0.3, 2.0)):
    shp = gwsynth.make_shape(n_k=n_k, n_b=n_b, R=R, N=N, n_occ=n_occ, n_unocc=n_unocc)
    return gwsynth.generate(shp, seed=seed, omega=omega)


# ----------------------------------------------------------------- projections

def test_projection_bruteforce_loops():
    inp = tiny(n_k=1, n_b=6, R=16, N=6, n_occ=2, n_unocc=3)
    U, psi = inp.U, inp.psi[0]
    po, pu = psi[:2], psi[2:]
    M = orc.projections(U, po, pu)
    for I in range(6):
        for n in range(2):
            for m in range(3):
                acc = 0j
                for r in range(16):
                    acc += U[I, r] * po[n, r].conjugate() * pu[m, r]
                assert abs(M[I, n * 3 + m] - acc) < 1e-14 * max(1.0, abs(acc))


def test_projection_identity_basis():
    # U = identity on the grid: the projection reads off the pointwise product.
    inp = tiny(n_k=1, R=7, N=7)
    psi = inp.psi[0]
    M = orc.projections(np.eye(7), psi[:2], psi[2:])
    for n in range(2):
        for m in range(3):
            np.testing.assert_allclose(M[:, n * 3 + m], np.conj(psi[n]) * psi[2 + m], rtol=0, atol=1e-15)


def test_projection_linear_in_basis():
    inp = tiny(n_k=1, R=12, N=4)
    rng = np.random.default_rng(0)
    V = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    psi = inp.psi[0]
    M1 = orc.projections(V @ inp.U, psi[:2], psi[2:])
    M2 = V @ orc.projections(inp.U, psi[:2], psi[2:])
    np.testing.assert_allclose(M1, M2, rtol=1e-12, atol=1e-14)


# --------------------------------------------------------------------- weights

def test_weight_closed_forms():
    eo = np.array([-0.5, -0.01])
    eu = np.array([0.02, 1.3, 2.0])
    om = np.array([0.0, 0.1, 1.0, 1e3])
    w = orc.transition_weights(eo, eu, om).reshape(4, 2, 3)
    d = eo[:, None] - eu[None, :]
    # static limit 4/Delta (two spins x 2/Delta), strictly negative, bounded by 4/|Delta|
    np.testing.assert_allclose(w[0], 4.0 / d, rtol=1e-15)
    assert np.all(w < 0)
    assert np.all(np.abs(w) <= 4.0 / np.abs(d)[None] * (1 + 1e-15))
    # large-frequency tail 4*Delta/omega^2 with relative deviation (Delta/omega)^2
    tail = 4.0 * d / om[3] ** 2
    assert np.all(np.abs(w[3] / tail - 1.0) <= (np.abs(d) / om[3]) ** 2 * 1.0001)
    # decreasing magnitude with omega
    assert np.all(np.abs(w[1:]) < np.abs(w[:-1]))


def test_weight_from_spectral_function():
    """The paper's other route (text after Eq. polar_MB): the imaginary part of
    the bracket on the real axis is a pair of delta peaks, and a Hilbert
    transform gives P at complex frequencies.  With Lorentzian peaks of width
    gamma the transform evaluated at i*nu equals the bracket at i*(nu+gamma);
    here it is done by brute numerical quadrature."""
    from scipy.integrate import quad

    e_o, e_u = -0.3, 0.45
    d = e_o - e_u
    gam = 0.05
    a = abs(d)

    def spec(x):
        # spectral weight of 1/(z-|D|) - 1/(z+|D|): +delta at |D|, -delta at -|D|
        return (gam / math.pi) * (1.0 / ((x - a) ** 2 + gam ** 2) - 1.0 / ((x + a) ** 2 + gam ** 2))

    for nu in (0.02, 0.2, 1.7):
        def re_int(x):
            return (spec(x) / (1j * nu - x)).real

        val = 0.0
        h = 10 * gam
        for lo, hi in ((-np.inf, -a - h), (-a - h, -a + h), (-a + h, a - h), (a - h, a + h), (a + h, np.inf)):
            if hi > lo:
                val += quad(re_int, lo, hi, limit=400, epsabs=1e-13, epsrel=1e-12)[0]
        spin = 2.0
        w_or = orc.transition_weights([e_o], [e_u], [nu + gam])[0, 0]
        assert abs(spin * val - w_or) < 1e-8 * abs(w_or)


# ---------------------------------------------------------------- polarization

def test_polarization_bruteforce_realspace():
    """Eq. polar_r first (real-space polarisation from the wave functions),
    then a change of basis P_IJ = sum_{r,r'} U_Ir P(r,r') conj(U_Jr') -- a
    different order of operations from the oracle, with pure-Python loops."""
    inp = tiny(n_k=2, n_b=6, R=6, N=4, n_occ=2, n_unocc=3, omega=(0.0, 0.7))
    n_occ, nb = 2, 5
    P_or = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, n_occ, kq=inp.kq)
    R, N = 6, 4
    for j, om in enumerate(inp.omega):
        Pr = np.zeros((R, R), dtype=complex)
        for k in range(2):
            kk = (k + 1) % 2
            for n in range(n_occ):
                for m in range(n_occ, nb):
                    dlt = inp.eps[k, n] - inp.eps[kk, m]
                    wgt = 4.0 * dlt / (dlt * dlt + om * om)
                    for r in range(R):
                        for s in range(R):
                            Pr[r, s] += (wgt * inp.psi[k, n, r].conjugate() * inp.psi[kk, m, r]
                                         * inp.psi[k, n, s] * inp.psi[kk, m, s].conjugate())
        for I in range(N):
            for J in range(N):
                acc = 0j
                for r in range(R):
                    for s in range(R):
                        acc += inp.U[I, r] * Pr[r, s] * inp.U[J, s].conjugate()
                assert abs(P_or[j, I, J] - acc) < 1e-13 * max(1.0, abs(P_or[j]).max())


@pytest.fixture(scope="module")
def small():
    shp = gwsynth.make_shape(n_k=3, n_b=40, R=64, N=24, n_occ=3, n_unocc=9)
    inp = gwsynth.generate(shp, seed=5, omega=gwsynth.omega_mesh("m13"))
    P = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=inp.kq)
    return inp, P


def test_polarization_hermitian(small):
    _, P = small
    for j in range(P.shape[0]):
        assert np.abs(P[j] - P[j].conj().T).max() <= 1e-14 * np.abs(P[j]).max()


def test_polarization_negative_semidefinite(small):
    _, P = small
    for j in range(P.shape[0]):
        lam = np.linalg.eigvalsh(P[j])
        assert lam.max() <= 1e-12 * np.abs(lam).max()


def test_polarization_single_transition():
    inp = tiny(n_k=1, n_b=6, R=10, N=5, n_occ=1, n_unocc=1, omega=(0.0, 0.4))
    P = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 1)
    m = inp.U @ (np.conj(inp.psi[0, 0]) * inp.psi[0, 1])
    d = inp.eps[0, 0] - inp.eps[0, 1]
    for j, om in enumerate(inp.omega):
        lam = np.linalg.eigvalsh(P[j])
        wgt = 4 * d / (d * d + om * om)
        assert abs(lam[0] - wgt * np.vdot(m, m).real) < 1e-12 * abs(lam[0])
        assert np.all(np.abs(lam[1:]) < 1e-12 * abs(lam[0]))  # rank one


def test_polarization_tail():
    """Large-frequency behaviour: omega^2 P(i omega) -> 4 M diag(Delta) M^H,
    relative deviation bounded by (Delta_max/omega)^2 (the omega^-2 asymptotics
    used for the frequency tail in the paper)."""
    inp = tiny(n_k=2, n_b=10, R=16, N=6, n_occ=2, n_unocc=4, omega=(1e3,))
    P = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 2, kq=inp.kq)[0]
    ref = np.zeros_like(P)
    dmax = 0.0
    for k in range(2):
        kk = (k + 1) % 2
        M = orc.projections(inp.U, inp.psi[k, :2], inp.psi[kk, 2:])
        d = (inp.eps[k, :2, None] - inp.eps[kk, None, 2:]).reshape(-1)
        dmax = max(dmax, np.abs(d).max())
        ref += (M * (4 * d)[None, :]) @ M.conj().T
    rel = np.linalg.norm(1e6 * P - ref) / np.linalg.norm(ref)
    assert rel <= (dmax / 1e3) ** 2 * 1.01


def test_polarization_loewner_monotone(small):
    _, P = small
    for j in range(P.shape[0] - 1):
        lam = np.linalg.eigvalsh(P[j + 1] - P[j])
        assert lam.min() >= -1e-12 * np.abs(P[j]).max()


def test_polarization_additive(small):
    inp, P = small
    Pa = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=inp.kq, k_list=[0, 2])
    Pb = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=inp.kq, k_list=[1])
    np.testing.assert_allclose(Pa + Pb, P, rtol=0, atol=1e-13 * np.abs(P).max())
    P1 = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=inp.kq, unocc_range=(0, 4))
    P2 = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=inp.kq, unocc_range=(4, 9))
    P3 = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=inp.kq, occ_range=(0, 1))
    P4 = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, 3, kq=inp.kq, occ_range=(1, 3))
    np.testing.assert_allclose(P1 + P2, P, rtol=0, atol=1e-13 * np.abs(P).max())
    np.testing.assert_allclose(P3 + P4, P, rtol=0, atol=1e-13 * np.abs(P).max())


def test_polarization_phase_and_basis_covariance(small):
    inp, P = small
    rng = np.random.default_rng(3)
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, inp.psi.shape[:2]))
    P_ph = orc.polarization(inp.U, inp.psi * ph[:, :, None], inp.eps, inp.omega, 3, kq=inp.kq)
    np.testing.assert_allclose(P_ph, P, rtol=0, atol=1e-13 * np.abs(P).max())
    Q, _ = np.linalg.qr(rng.standard_normal((24, 24)) + 1j * rng.standard_normal((24, 24)))
    P_q = orc.polarization(Q @ inp.U, inp.psi, inp.eps, inp.omega, 3, kq=inp.kq)
    for j in range(P.shape[0]):
        np.testing.assert_allclose(P_q[j], Q @ P[j] @ Q.conj().T, rtol=0, atol=1e-12 * np.abs(P[j]).max())


def test_polarization_trace(small):
    inp, P = small
    tr = np.zeros(P.shape[0])
    for k in range(3):
        kk = (k + 1) % 3
        M = orc.projections(inp.U, inp.psi[k, :3], inp.psi[kk, 3:])
        d = (inp.eps[k, :3, None] - inp.eps[kk, None, 3:]).reshape(-1)
        nrm = np.sum(np.abs(M) ** 2, axis=0)
        for j, om in enumerate(inp.omega):
            tr[j] += np.sum(4 * d / (d * d + om * om) * nrm)
    np.testing.assert_allclose(np.trace(P, axis1=1, axis2=2).real, tr, rtol=1e-12)


def test_polarization_rejects_metal():
    inp = tiny()
    eps = inp.eps.copy()
    eps[1, 0] = 0.5   # an "occupied" level above the unoccupied ones at k+q of k=1
    with pytest.raises(ValueError):
        orc.check_insulator(eps, 2, inp.kq)
    orc.check_insulator(inp.eps, 2, inp.kq)


# ------------------------------------------------------------------- screening

def test_screen_scalar_closed_form():
    P = np.array([[[-0.37 + 0j]]])
    v = np.array([2.5])
    W = orc.screened_interaction(P, v)
    assert abs(W[0, 0, 0] - 2.5 / (1 - 2.5 * -0.37)) < 1e-15


def test_screen_zero_polarization():
    v = gwsynth.coulomb_diag(9)
    W = orc.screened_interaction(np.zeros((2, 9, 9), complex), v)
    np.testing.assert_allclose(W[0], np.diag(v), atol=0)


def test_screen_dyson_and_symmetrized(small):
    inp, P = small
    v = inp.v
    W = orc.screened_interaction(P, v)
    Ws = orc.screened_interaction_symmetrized(P, v)
    for j in range(P.shape[0]):
        # Eq. W_Dyson: W = v + v P W
        res = W[j] - np.diag(v) - (v[:, None] * P[j]) @ W[j]
        assert np.abs(res).max() <= 1e-11 * np.abs(W[j]).max()
        np.testing.assert_allclose(Ws[j], W[j], rtol=0, atol=1e-11 * np.abs(W[j]).max())
        # Hermitian positive definite, below v in the Loewner order, W^c = W - v NSD
        assert np.abs(W[j] - W[j].conj().T).max() <= 1e-11 * np.abs(W[j]).max()
        lw = np.linalg.eigvalsh(0.5 * (W[j] + W[j].conj().T))
        assert lw.min() > 0
        lc = np.linalg.eigvalsh(0.5 * (W[j] + W[j].conj().T) - np.diag(v))
        assert lc.max() <= 1e-10 * np.abs(W[j]).max()


def test_screen_neumann_series_small_p(small):
    inp, P = small
    v = inp.v
    Ps = P[-1] * (0.01 / (np.abs(P[-1]).max() * v.max()))
    W = orc.screened_interaction(Ps, v)
    V = np.diag(v)
    ser = V.copy().astype(complex)
    term = V.astype(complex)
    for _ in range(12):
        term = (v[:, None] * Ps) @ term
        ser += term
    np.testing.assert_allclose(W, ser, rtol=0, atol=1e-14 * np.abs(W).max())


def test_screen_large_frequency_limit(small):
    inp, _ = small
    P = orc.polarization(inp.U, inp.psi, inp.eps, [2e3], 3, kq=inp.kq)[0]
    W = orc.screened_interaction(P, inp.v)
    lead = inp.v[:, None] * P * inp.v[None, :]
    err = np.linalg.norm(W - np.diag(inp.v) - lead) / np.linalg.norm(lead)
    assert err < 1e-3


# -------------------------------------------------------------- worked example

def test_hand_worked_examples():
    """Fixtures computed by hand (derivations in the fixture file)."""
    with open(os.path.join(GOLDEN, "hand_examples.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        U = np.array(c["U_re"]) + 1j * np.array(c["U_im"])
        psi = np.array(c["psi_re"]) + 1j * np.array(c["psi_im"])
        eps = np.array(c["eps"])
        P = orc.polarization(U, psi, eps, c["omega"], c["n_occ"])
        Pexp = np.array(c["P_re"]) + 1j * np.array(c["P_im"])
        np.testing.assert_allclose(P, Pexp, rtol=1e-14, atol=1e-15)
        W = orc.screened_interaction(P, np.array(c["v"]))
        Wexp = np.array(c["W_re"]) + 1j * np.array(c["W_im"])
        np.testing.assert_allclose(W, Wexp, rtol=1e-13, atol=1e-15)


def test_real_inputs_give_real_symmetric_P():
    """With a real basis and real wave functions (the inversion-symmetric case
    of Eq. condition_inv) the matrix elements are real and P is real
    symmetric (text after Eq. polar_MB)."""
    rng = np.random.default_rng(21)
    n_k, N, R, n_occ, n_unocc = 2, 5, 12, 2, 3
    U = rng.normal(size=(N, R)).astype(np.complex128)
    psi = rng.normal(size=(n_k, n_occ + n_unocc, R)).astype(np.complex128)
    eps = np.tile(np.array([-0.4, -0.1, 0.2, 0.5, 1.1]), (n_k, 1))
    P = orc.polarization(U, psi, eps, [0.0, 0.7], n_occ)
    assert np.all(P.imag == 0.0)
    assert np.allclose(P, np.transpose(P, (0, 2, 1)), rtol=0, atol=1e-13 * np.abs(P).max())
