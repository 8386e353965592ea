"""CPU FP64 oracle for the correlation self-energy on the imaginary axis.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Plain NumPy, written after
Sec. "Correlation self-energy" of the paper: Eq. SEc_AC (the analytically
continued form), the interpolation of W^c between the imaginary mesh points by
cubic splines in lambda with omega(lambda) = lambda / (1 - lambda), the
stepwise analytic integration and the omega^-2 tail fitted to the last mesh
point.

    Sigma_c^n(i w) = -(1/2pi) sum_t sum_n' sum_{mu,nu} <n'|n E_mu> <E_nu n|n'>
                     * int_{-inf}^{inf} dw' W^c_{mu nu}(t, i w') / (i w + i w' - e_n')

Readings (the paper leaves these open; the HIP path takes the same ones):
* Matrix elements.  With the projection convention of oracle.polarization
  (U_Ir stands for conj(E_I(r)) times the grid weight), <n'|n E_mu> =
  conj(M_mu) and <E_nu n|n'> = M_nu with M_I = sum_r U_Ir conj(psi_n) psi_n',
  so the matrix part is q(i w') = m^H W^c(i w') m, real for Hermitian W^c.
* Momentum transfers.  Transfer t pairs the state's set s with set
  (s + t) mod N_k; W^c(t) is the screened interaction whose polarization pairs
  every set k with (k + t) mod N_k.  Energies e_n' are measured from a
  chemical potential mu inside the gap.  No Gamma-point (k -> 0) terms.
* Evenness.  P(i w) depends on w^2, so W^c(i w') is even in w' and the integral
  is folded onto w' >= 0:  K(w') = 1/(i(w + w') - e') + 1/(i(w - w') - e').
* Spline.  Clamped cubic spline in lambda through (lambda_j, q_j) with zero
  slope at lambda = 0 (evenness; the mesh must start at w = 0) and, at the last
  point, the slope of the tail q_L (w_L / w')^2 (continuous derivative).
* Tail.  q(w') = q_L (w_L / w')^2 for w' > w_L.
"""
from __future__ import annotations

import numpy as np

from . import polarization as pol


def lam(omega):
    """lambda(w) = w / (1 + w): [0, inf) -> [0, 1)."""
    omega = np.asarray(omega, dtype=np.float64)
    return omega / (1.0 + omega)


def spline_basis(omega_mesh) -> np.ndarray:
    """Coefficients C [n_int][4][n_mesh] of the clamped spline as a linear map
    of the data: on interval i, q(lambda) = sum_p sum_j C[i,p,j] q_j (lambda -
    lambda_i)^p.  Built by solving, for every unit data vector, the full
    linear system of interpolation, C1/C2 continuity and the two end slopes."""
    om = np.asarray(omega_mesh, dtype=np.float64)
    if om.ndim != 1 or om.size < 2 or om[0] != 0.0 or np.any(np.diff(om) <= 0):
        raise ValueError("the mesh must start at 0 and increase strictly")
    L = lam(om)
    n = om.size
    ni = n - 1
    h = np.diff(L)
    A = np.zeros((4 * ni, 4 * ni))
    rows = []
    r = 0
    # unknowns: a_i0, a_i1, a_i2, a_i3 for interval i at index 4i..4i+3
    for i in range(ni):            # value at the left and right end
        A[r, 4 * i] = 1.0
        rows.append(("val", i)); r += 1
        for p in range(4):
            A[r, 4 * i + p] = h[i] ** p
        rows.append(("val", i + 1)); r += 1
    for i in range(ni - 1):        # first and second derivative continuity at knot i+1
        for p in range(1, 4):
            A[r, 4 * i + p] = p * h[i] ** (p - 1)
        A[r, 4 * (i + 1) + 1] = -1.0
        rows.append(("zero", None)); r += 1
        for p in range(2, 4):
            A[r, 4 * i + p] = p * (p - 1) * h[i] ** (p - 2)
        A[r, 4 * (i + 1) + 2] = -2.0
        rows.append(("zero", None)); r += 1
    A[r, 1] = 1.0                  # slope 0 at lambda = 0
    rows.append(("zero", None)); r += 1
    for p in range(1, 4):          # slope at the end equals the tail's slope
        A[r, 4 * (ni - 1) + p] = p * h[ni - 1] ** (p - 1)
    rows.append(("end", None)); r += 1
    assert r == 4 * ni
    # tail q_L (w_L/w)^2: dq/dw = -2 q_L / w_L at w_L; dw/dlambda = 1/(1 - lambda)^2
    end_slope = -2.0 / om[-1] / (1.0 - L[-1]) ** 2
    C = np.zeros((ni, 4, n))
    for j in range(n):
        b = np.zeros(4 * ni)
        for k, (kind, idx) in enumerate(rows):
            if kind == "val":
                b[k] = 1.0 if idx == j else 0.0
            elif kind == "end":
                b[k] = end_slope if j == n - 1 else 0.0
        x = np.linalg.solve(A, b)
        C[:, :, j] = x.reshape(ni, 4)
    return C


def spline_eval(omega_mesh, q, omega):
    """Value of the interpolant (spline inside the mesh, tail beyond it)."""
    om = np.asarray(omega_mesh, dtype=np.float64)
    C = spline_basis(om)
    L = lam(om)
    q = np.asarray(q)
    w = np.atleast_1d(np.asarray(omega, dtype=np.float64))
    out = np.empty(w.shape, dtype=np.result_type(q, np.float64))
    for idx, x in enumerate(w):
        if x >= om[-1]:
            out[idx] = q[-1] * (om[-1] / x) ** 2
            continue
        lx = x / (1.0 + x)
        i = min(int(np.searchsorted(L, lx, side="right")) - 1, L.size - 2)
        t = lx - L[i]
        out[idx] = sum((C[i, p] @ q) * t ** p for p in range(4))
    return out


def _F(p, d, h):
    """int_0^h x^p / (x + d) dx for complex d (no zero of x + d on [0, h]).

    |d| > 2h: the convergent series sum_m (-1)^m h^(p+m+1) / ((p+m+1) d^(m+1));
    otherwise the recurrence F_p = h^p/p - d F_{p-1} from F_0 = log(1 + h/d)."""
    if abs(d) > 2.0 * h:
        s = 0.0 + 0.0j
        term_ratio = -h / d
        t = h ** (p + 1) / d
        for m in range(80):
            s += t / (p + m + 1)
            t *= term_ratio
            if abs(t) < 1e-30 * abs(s):
                break
        return s
    F = np.log(1.0 + h / d)
    for k in range(1, p + 1):
        F = h ** k / k - d * F
    return F


def freq_weights(omega_mesh, omega_out, eps_rel) -> np.ndarray:
    """w [n_eps][n_out][n_mesh] with

        int_{-inf}^{inf} dw' q(i w') / (i w + i w' - e')  =  sum_j w_j(w, e') q_j

    for the spline-plus-tail interpolant q of the data q_j on the mesh.

    On spline interval i, with a = i w - e' the folded kernel times
    dw'/dlambda is  -i/(lambda + c1) + i/(lambda + c2),  c1 = a/(i - a),
    c2 = a/(-i - a)  (partial fractions of 1/((1-lambda)(a + (+-i - a) lambda));
    the 1/(1 - lambda) parts cancel between the two terms), integrated against
    (lambda - lambda_i)^p.  The tail gives
    w_L^2 (2/a) [1/w_L - (1/a)((pi/2) sgn(-e') - atan(w_L / a))]."""
    om = np.asarray(omega_mesh, dtype=np.float64)
    C = spline_basis(om)
    L = lam(om)
    h = np.diff(L)
    wl = om[-1]
    out = np.zeros((len(eps_rel), len(omega_out), om.size), dtype=np.complex128)
    for ie, e in enumerate(np.asarray(eps_rel, dtype=np.float64)):
        if e == 0.0:
            raise ValueError("energies must not sit at the chemical potential")
        for io, w in enumerate(np.asarray(omega_out, dtype=np.float64)):
            a = 1j * w - e
            c1 = a / (1j - a)
            c2 = a / (-1j - a)
            acc = np.zeros(om.size, dtype=np.complex128)
            for i in range(h.size):
                for p in range(4):
                    J = -1j * _F(p, L[i] + c1, h[i]) + 1j * _F(p, L[i] + c2, h[i])
                    acc += C[i, p] * J
            tail = wl ** 2 * (2.0 / a) * (1.0 / wl - (1.0 / a) * (0.5 * np.pi * np.sign(-e) - np.arctan(wl / a)))
            acc[-1] += tail
            out[ie, io] = acc
    return out


def correlation_w(U, psi, eps, omega_mesh, n_occ, v, t) -> np.ndarray:
    """W^c = W - v for momentum transfer t: P from every set k paired with
    (k + t) mod N_k (Eq. polar_MB), then W = (1 - vP)^-1 v (Eq. W_Dyson)."""
    n_k = psi.shape[0]
    kq = (np.arange(n_k) + t) % n_k
    P = pol.polarization(U, psi, eps, omega_mesh, n_occ, kq=kq)
    W = pol.screened_interaction(P, v)
    return W - np.diag(np.asarray(v, dtype=np.float64))[None]


def quad_forms(U, psi_state, psi_all, Wc) -> np.ndarray:
    """q[j][n'] = m_n'^H W^c_j m_n' with m_n' the projection of
    conj(psi_state) psi_n' (Eq. proj_MB); the real part (W^c is Hermitian)."""
    M = pol.projections(U, psi_state[None, :], psi_all)          # [N][n_b]
    q = np.empty((Wc.shape[0], M.shape[1]))
    for j in range(Wc.shape[0]):
        Y = Wc[j] @ M
        q[j] = np.real(np.sum(np.conj(M) * Y, axis=0))
    return q


def sigma_c(U, psi, eps, Wc_by_transfer, omega_mesh, omega_out, states, mu) -> np.ndarray:
    """Eq. SEc_AC for the diagonal elements of the listed states (set s, band n):
    Sigma [n_states][n_out] complex128.  Wc_by_transfer[t] is W^c(t) on the
    mesh, [n_mesh][N][N]."""
    n_k = psi.shape[0]
    out = np.zeros((len(states), len(omega_out)), dtype=np.complex128)
    for si, (s, n) in enumerate(states):
        for t, Wc in enumerate(Wc_by_transfer):
            s2 = (s + t) % n_k
            q = quad_forms(U, psi[s, n], psi[s2], Wc)                   # [n_mesh][n_b]
            w = freq_weights(omega_mesh, omega_out, eps[s2] - mu)       # [n_b][n_out][n_mesh]
            out[si] += -np.einsum("boj,jb->o", w, q) / (2.0 * np.pi)
    return out
