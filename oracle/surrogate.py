"""CPU FP64 oracle of the learned high-band correction (features, targets,
application, judge).  TEST INFRASTRUCTURE ONLY; shares no code with the HIP
library.

Definitions (a reading of the band-truncation correction; the paper's own
correction for the same truncation is the extrapolar approximation in the
section on convergence with the number of bands):

* weight sums  S_lo(w) = sum_{k,n occ, n' < cut} |w_knn'(w)|,
               S_hi(w) = sum_{k,n occ, n' >= cut} |w_knn'(w)|
  with |w| the magnitude of the spin-summed imaginary-axis bracket of Eq.
  polar_MB (unoccupied bands at kq[k]).
* band edges (means over k-sets): lowest occupied e0, highest occupied e1,
  lowest unoccupied e2, highest retained unoccupied e3, highest unoccupied e4.
* features of row r = j*N + I (frequency j, basis function I):
    f0 = w/(1+w)                 f1 = log S_hi(w) - log S_lo(w)
    f2 = log p - log p_ref       f3 = log p - log mean_I p
    f4 = I/N                     f5 = e3 - e2,  f6 = e4 - e3,  f7 = e1 - e0,  f8 = e2 - e1
    f9 = cut/n_unocc             f10 = f1 - f1(w_ref)
    f11 = log S_lo(w) - log S_lo(w_ref)
  with p = |Re P_ret,II(w)| and w_ref the first frequency.
* target t = log((Re P_ret,II - Re P_full,II) / |Re P_ret,II|) (masked where
  undefined).
* correction P = P_ret + D P_ret D, D = diag(exp(y/2)), y clamped to [-30, 30].
* judge err(w) = |TR_s/f - TR_p| / TR_p with TR_p = sum_I |P_ret,II| e^{y_I},
  TR_s the trace of an explicit sample of left-out transitions and f the
  sample's share of S_hi.
"""
from __future__ import annotations

import numpy as np

from .polarization import transition_weights

NF = 12


def weight_sums(eps, n_occ, cut, omega, kq=None, rows=None):
    """(S_lo, S_hi) per frequency; rows = list of (k, n) or None for all."""
    eps = np.asarray(eps, dtype=np.float64)
    n_k = eps.shape[0]
    kq = ((np.arange(n_k) + 1) % n_k) if kq is None else np.asarray(kq)
    if rows is None:
        rows = [(k, n) for k in range(n_k) for n in range(n_occ)]
    om = np.asarray(omega, dtype=np.float64)
    lo = np.zeros(om.shape[0])
    hi = np.zeros(om.shape[0])
    for k, n in rows:
        w = np.abs(transition_weights([eps[k, n]], eps[kq[k], n_occ:], om))
        lo += w[:, :cut].sum(axis=1)
        hi += w[:, cut:].sum(axis=1)
    return lo, hi


def band_edges(eps, n_occ, cut):
    eps = np.asarray(eps, dtype=np.float64)
    return np.array([eps[:, 0].mean(), eps[:, n_occ - 1].mean(), eps[:, n_occ].mean(),
                     eps[:, n_occ + cut - 1].mean(), eps[:, -1].mean()])


def features(P_ret, eps, omega, n_occ, cut, kq=None, n_in=32):
    P_ret = np.asarray(P_ret)
    n_om, N = P_ret.shape[0], P_ret.shape[1]
    n_unocc = eps.shape[1] - n_occ
    om = np.asarray(omega, dtype=np.float64)
    lo, hi = weight_sums(eps, n_occ, cut, om, kq)
    e = band_edges(eps, n_occ, cut)
    p = np.abs(np.real(np.einsum("jii->ji", P_ret)))
    lg = lambda x: np.log(np.maximum(x, 1e-300))
    X = np.zeros((n_om * N, n_in))
    for j in range(n_om):
        r = slice(j * N, (j + 1) * N)
        X[r, 0] = om[j] / (1 + om[j])
        X[r, 1] = lg(hi[j]) - lg(lo[j])
        X[r, 2] = lg(p[j]) - lg(p[0])
        X[r, 3] = lg(p[j]) - lg(p[j].mean())
        X[r, 4] = np.arange(N) / N
        X[r, 5] = e[3] - e[2]
        X[r, 6] = e[4] - e[3]
        X[r, 7] = e[1] - e[0]
        X[r, 8] = e[2] - e[1]
        X[r, 9] = cut / n_unocc
        X[r, 10] = X[r, 1] - (lg(hi[0]) - lg(lo[0]))
        X[r, 11] = lg(lo[j]) - lg(lo[0])
    return X


def targets(P_ret, P_full):
    pr = np.real(np.einsum("jii->ji", np.asarray(P_ret))).reshape(-1)
    pf = np.real(np.einsum("jii->ji", np.asarray(P_full))).reshape(-1)
    d = pr - pf
    ok = (np.abs(pr) > 0) & (d > 0) & np.isfinite(d)
    t = np.where(ok, np.log(np.where(ok, d, 1.0) / np.where(ok, np.abs(pr), 1.0)), 0.0)
    return t, ok.astype(np.float64)


def apply(P_ret, y):
    """P_ret + D P_ret D with D = diag(exp(y/2)); y [n_omega*N] frequency-major."""
    P_ret = np.asarray(P_ret, dtype=np.complex128)
    n_om, N = P_ret.shape[0], P_ret.shape[1]
    yy = np.clip(np.asarray(y, dtype=np.float64).reshape(n_om, N), -30, 30)
    d = np.exp(0.5 * yy)
    return P_ret + d[:, :, None] * P_ret * d[:, None, :]


def judge(P_ret, y, P_sample, eps, n_occ, cut, omega, sample_rows, kq=None):
    n_om, N = P_ret.shape[0], P_ret.shape[1]
    yy = np.clip(np.asarray(y, dtype=np.float64).reshape(n_om, N), -30, 30)
    pr = np.abs(np.real(np.einsum("jii->ji", P_ret)))
    ps = np.abs(np.real(np.einsum("jii->ji", P_sample)))
    tp = (pr * np.exp(yy)).sum(axis=1)
    ts = ps.sum(axis=1)
    _, hi = weight_sums(eps, n_occ, cut, omega, kq)
    _, shi = weight_sums(eps, n_occ, cut, omega, kq, rows=sample_rows)
    f = shi / hi
    return np.abs(ts / f - tp) / tp
