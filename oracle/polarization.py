"""CPU FP64 oracle for the RPA polarization and the screened interaction.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module; the product path never does.
It shares no code with the HIP library.

Everything is plain NumPy in float64/complex128, written step by step after
the paper (Friedrich, Bluegel, Schindlmayr, "Efficient implementation of the GW
approximation within the all-electron FLAPW method"):

* projections          Sec. "Formulation in the MPB", Eq. proj_MB
* polarization matrix  Eq. polar_MB, with the frequency bracket taken on the
                       imaginary axis (the text after Eq. polar_MB: the bracket
                       is real there and P becomes Hermitian) and the spin sum
                       over two degenerate spin channels
* screening            Eq. W_Dyson in matrix form, W = (1 - vP)^-1 v, solved by
                       LU (numpy.linalg.solve); the symmetrised form of
                       Eqs. dielec_MB / screen_MB is provided separately

Readings of points the paper leaves open (index conventions of the synthetic
workload):
* U_Ir stands for conj(M~_I(r)) times the grid quadrature weight, so
  M_I^{nn'} = sum_r U_Ir conj(psi_n(r)) psi_n'(r)  (no conjugation on U).
* The Brillouin-zone sum is a plain sum over the k-points given (no 1/N_k);
  the wave functions at k+q are the set kq[k].
* Only insulators: every occupied energy lies below every unoccupied one, so
  eta -> 0 is taken before evaluating on the imaginary axis.
"""
from __future__ import annotations

import numpy as np


def projections(U: np.ndarray, psi_occ: np.ndarray, psi_unocc: np.ndarray) -> np.ndarray:
    """Eq. proj_MB on a grid: M[I, n*n_unocc + n'] = sum_r U[I,r] conj(psi_occ[n,r]) psi_unocc[n',r].

    U [N][R], psi_occ [n_occ][R], psi_unocc [n_unocc][R]  ->  M [N][n_occ*n_unocc].
    For each occupied band the integrand conj(psi_n) * psi_n' is formed and
    integrated against every row of U (one matrix product per occupied band).
    """
    U = np.asarray(U, dtype=np.complex128)
    po = np.asarray(psi_occ, dtype=np.complex128)
    pu = np.asarray(psi_unocc, dtype=np.complex128)
    N = U.shape[0]
    n_occ, n_unocc = po.shape[0], pu.shape[0]
    M = np.empty((N, n_occ * n_unocc), dtype=np.complex128)
    for n in range(n_occ):
        G = U * np.conj(po[n])[None, :]           # U_Ir conj(psi_n(r))
        M[:, n * n_unocc:(n + 1) * n_unocc] = G @ pu.T
    return M


def bracket_imag_axis(e_occ, e_unocc, omega) -> np.ndarray:
    """The frequency bracket of Eq. polar_MB,
        1/(w + e_n - e_n' + i eta) - 1/(w - e_n + e_n' - i eta),
    evaluated at w -> i*omega with eta -> 0 (complex arithmetic, real part kept;
    the imaginary part vanishes on the imaginary axis).

    Shapes broadcast: e_occ [..], e_unocc [..], omega [..].
    """
    z = 1j * np.asarray(omega, dtype=np.float64)
    d = np.asarray(e_occ, dtype=np.float64) - np.asarray(e_unocc, dtype=np.float64)
    b = 1.0 / (z + d) - 1.0 / (z - d)
    return b.real


def transition_weights(eps_occ: np.ndarray, eps_unocc: np.ndarray, omega: np.ndarray,
                       n_spin: int = 2) -> np.ndarray:
    """w[iw, n*n_unocc + n'] = sum over spins of the bracket (two degenerate spins).

    eps_occ [n_occ], eps_unocc [n_unocc], omega [n_omega] -> [n_omega][n_occ*n_unocc].
    """
    eo = np.asarray(eps_occ, dtype=np.float64)
    eu = np.asarray(eps_unocc, dtype=np.float64)
    om = np.asarray(omega, dtype=np.float64)
    b = bracket_imag_axis(eo[None, :, None], eu[None, None, :], om[:, None, None])
    return n_spin * b.reshape(om.shape[0], -1)


def check_insulator(eps: np.ndarray, n_occ: int, kq: np.ndarray) -> None:
    for k in range(eps.shape[0]):
        if not np.max(eps[k, :n_occ]) < np.min(eps[kq[k], n_occ:]):
            raise ValueError(f"k={k}: occupied and unoccupied energies overlap (not an insulator)")


def polarization(U, psi, eps, omega, n_occ: int, *, kq=None, k_list=None,
                 occ_range=None, unocc_range=None) -> np.ndarray:
    """Eq. polar_MB on the imaginary axis:

        P_IJ(q, i w) = sum_k sum_{n occ} sum_{n' unocc} w_{k n n'}(w) M_I^{knn'} conj(M_J^{knn'})

    with M from Eq. proj_MB using psi at k (occupied) and psi at kq[k]
    (unoccupied), and w the spin-summed bracket.  Returns P [n_omega][N][N]
    complex128 (full matrix).

    occ_range = (n0, n1) restricts the occupied bands, unocc_range = (m0, m1)
    the unoccupied ones (indices relative to the first unoccupied band).
    """
    U = np.asarray(U, dtype=np.complex128)
    n_k = psi.shape[0]
    nb = psi.shape[1]
    n_unocc = nb - n_occ
    kq = ((np.arange(n_k) + 1) % n_k) if kq is None else np.asarray(kq)
    ks = range(n_k) if k_list is None else list(k_list)
    o0, o1 = (0, n_occ) if occ_range is None else occ_range
    u0, u1 = (0, n_unocc) if unocc_range is None else unocc_range
    om = np.asarray(omega, dtype=np.float64)
    N = U.shape[0]
    P = np.zeros((om.shape[0], N, N), dtype=np.complex128)
    for k in ks:
        kk = int(kq[k])
        po = np.asarray(psi[k, o0:o1], dtype=np.complex128)
        pu = np.asarray(psi[kk, n_occ + u0:n_occ + u1], dtype=np.complex128)
        if po.shape[0] == 0 or pu.shape[0] == 0:
            continue
        M = projections(U, po, pu)
        w = transition_weights(eps[k, o0:o1], eps[kk, n_occ + u0:n_occ + u1], om)
        MH = M.conj().T
        for j in range(om.shape[0]):
            P[j] += (M * w[j][None, :]) @ MH
    return P


def hat_weights(x, nodes) -> np.ndarray:
    """h[b, t]: the share of a transition at energy x_t given to node b when
    its spectral weight is split linearly between the two nodes around it
    (x_t inside [nodes[0], nodes[-1]], nodes strictly increasing)."""
    x = np.asarray(x, dtype=np.float64)
    nd = np.asarray(nodes, dtype=np.float64)
    if nd.ndim != 1 or nd.size < 2 or np.any(np.diff(nd) <= 0):
        raise ValueError("nodes must increase strictly (at least two)")
    if x.size and (x.min() < nd[0] or x.max() > nd[-1]):
        raise ValueError("a transition energy lies outside the nodes")
    h = np.zeros((nd.size, x.size))
    for t, xt in enumerate(x):
        b = min(int(np.searchsorted(nd, xt, side="right")) - 1, nd.size - 2)
        f = (xt - nd[b]) / (nd[b + 1] - nd[b])
        h[b, t] += 1.0 - f
        h[b + 1, t] += f
    return h


def spectral_weights(U, psi, eps, n_occ: int, nodes, *, kq=None, k_list=None, occ_range=None,
                     unocc_range=None) -> np.ndarray:
    """S[b] = sum over the transitions of h_b(x_t) M_t M_t^H with x_t = e_n' - e_n
    > 0: the spectral function of P (the imaginary part of Eq. polar_MB on the
    real axis, a sum of delta functions at the transition energies) with every
    delta moved onto the two nodes around it.  [n_nodes][N][N] complex128."""
    U = np.asarray(U, dtype=np.complex128)
    n_k = psi.shape[0]
    n_unocc = psi.shape[1] - n_occ
    kq = ((np.arange(n_k) + 1) % n_k) if kq is None else np.asarray(kq)
    ks = range(n_k) if k_list is None else list(k_list)
    o0, o1 = (0, n_occ) if occ_range is None else occ_range
    u0, u1 = (0, n_unocc) if unocc_range is None else unocc_range
    nd = np.asarray(nodes, dtype=np.float64)
    N = U.shape[0]
    S = np.zeros((nd.size, N, N), dtype=np.complex128)
    for k in ks:
        kk = int(kq[k])
        po = np.asarray(psi[k, o0:o1], dtype=np.complex128)
        pu = np.asarray(psi[kk, n_occ + u0:n_occ + u1], dtype=np.complex128)
        M = projections(U, po, pu)
        x = (np.asarray(eps[kk, n_occ + u0:n_occ + u1])[None, :] - np.asarray(eps[k, o0:o1])[:, None]).reshape(-1)
        h = hat_weights(x, nd)
        MH = M.conj().T
        for b in range(nd.size):
            S[b] += (M * h[b][None, :]) @ MH
    return S


def polarization_spectral(U, psi, eps, omega, n_occ: int, nodes, **kw) -> np.ndarray:
    """P(i w) from the node spectral weights by the Hilbert transform of each
    node's delta function (the route of the text after Eq. polar_MB):
    P(i w) = sum_b -4 x_b / (x_b^2 + w^2) S[b], the same spin-summed bracket as
    the direct sum evaluated at the node energy.  Exact when every transition
    sits on a node; otherwise the bracket is interpolated linearly in x
    between the nodes."""
    S = spectral_weights(U, psi, eps, n_occ, nodes, **kw)
    nd = np.asarray(nodes, dtype=np.float64)
    om = np.asarray(omega, dtype=np.float64)
    c = -4.0 * nd[None, :] / (nd[None, :] ** 2 + om[:, None] ** 2)      # [n_omega][n_nodes]
    return np.einsum("jb,bxy->jxy", c, S)


def screened_interaction(P: np.ndarray, v: np.ndarray) -> np.ndarray:
    """W = (1 - v P)^-1 v for diagonal v (Eq. W_Dyson in matrix form), per
    frequency, by LU solve of (I - diag(v) P) W = diag(v)."""
    P = np.asarray(P, dtype=np.complex128)
    v = np.asarray(v, dtype=np.float64)
    N = v.shape[0]
    single = P.ndim == 2
    Ps = P[None] if single else P
    W = np.empty_like(Ps)
    I = np.eye(N)
    V = np.diag(v).astype(np.complex128)
    for j in range(Ps.shape[0]):
        W[j] = np.linalg.solve(I - v[:, None] * Ps[j], V)
    return W[0] if single else W


def screened_interaction_symmetrized(P: np.ndarray, v: np.ndarray) -> np.ndarray:
    """Eqs. dielec_MB / screen_MB in the Coulomb eigenbasis (v diagonal):
    eps_{mu nu} = delta - sqrt(v_mu) P_{mu nu} sqrt(v_nu),  W = sqrt(v) eps^-1 sqrt(v)."""
    P = np.asarray(P, dtype=np.complex128)
    s = np.sqrt(np.asarray(v, dtype=np.float64))
    single = P.ndim == 2
    Ps = P[None] if single else P
    W = np.empty_like(Ps)
    N = s.shape[0]
    for j in range(Ps.shape[0]):
        eps = np.eye(N) - s[:, None] * Ps[j] * s[None, :]
        W[j] = s[:, None] * np.linalg.inv(eps) * s[None, :]
    return W[0] if single else W


def rel_fro(x: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Relative Frobenius error per leading index (per frequency)."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    if x.ndim == 2:
        return np.array([np.linalg.norm(x - ref) / np.linalg.norm(ref)])
    d = (x - ref).reshape(x.shape[0], -1)
    r = ref.reshape(ref.shape[0], -1)
    return np.linalg.norm(d, axis=1) / np.linalg.norm(r, axis=1)
