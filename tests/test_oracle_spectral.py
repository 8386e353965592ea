"""Pins of the spectral route of the oracle (spectral weights on energy nodes,
then the Hilbert transform of each node to the imaginary axis) against the
direct sum of Eq. polar_MB, brute force and the properties of linear
interpolation."""
import numpy as np
import pytest

import gwsynth
from oracle import polarization as orc


def _small(seed=2):
    shape = gwsynth.make_shape(n_k=2, n_b=12, R=16, N=5, n_occ=2, n_unocc=4)
    return gwsynth.generate(shape, seed=seed, omega=np.array([0.0, 0.3, 2.0, 15.0]))


def _energies(inp, n_occ):
    kq = inp.kq
    xs = [inp.eps[kq[k], n_occ:][None, :] - inp.eps[k, :n_occ][:, None] for k in range(inp.eps.shape[0])]
    return np.concatenate([x.reshape(-1) for x in xs])


def test_hat_weights_partition_and_linear_reproduction():
    nodes = np.array([0.02, 0.05, 0.3, 0.31, 2.5])
    x = np.concatenate([nodes, np.random.default_rng(0).uniform(0.02, 2.5, 200)])
    h = orc.hat_weights(x, nodes)
    assert np.all(h >= 0)
    assert np.allclose(h.sum(axis=0), 1.0, atol=1e-15)
    assert np.allclose(nodes @ h, x, rtol=1e-14)              # linear functions are reproduced
    assert np.all((h > 0).sum(axis=0) <= 2)
    for b, xb in enumerate(nodes):                             # a transition on a node goes to that node only
        assert h[b, b] == 1.0
    with pytest.raises(ValueError):
        orc.hat_weights([0.01], nodes)
    with pytest.raises(ValueError):
        orc.hat_weights([0.1], [0.3, 0.2])


def test_nodes_on_every_transition_reproduce_the_direct_sum():
    inp = _small()
    n_occ = 2
    nodes = np.unique(_energies(inp, n_occ))
    P = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, n_occ, kq=inp.kq)
    Ps = orc.polarization_spectral(inp.U, inp.psi, inp.eps, inp.omega, n_occ, nodes, kq=inp.kq)
    assert orc.rel_fro(Ps, P).max() < 1e-13


def test_spectral_weights_sum_to_the_unweighted_transition_sum():
    inp = _small(5)
    n_occ = 2
    x = _energies(inp, n_occ)
    nodes = np.geomspace(x.min(), x.max(), 7)
    S = orc.spectral_weights(inp.U, inp.psi, inp.eps, n_occ, nodes, kq=inp.kq)
    N, R = inp.U.shape
    ref = np.zeros((N, N), dtype=complex)
    for k in range(inp.eps.shape[0]):
        kk = inp.kq[k]
        for n in range(n_occ):
            for u in range(inp.psi.shape[1] - n_occ):
                m = np.array([sum(inp.U[I, r] * np.conj(inp.psi[k, n, r]) * inp.psi[kk, n_occ + u, r]
                                  for r in range(R)) for I in range(N)])
                ref += np.outer(m, m.conj())
    assert np.abs(S.sum(axis=0) - ref).max() < 1e-12 * np.abs(ref).max()
    for b in range(len(nodes)):                                 # every node matrix is Hermitian PSD
        assert np.abs(S[b] - S[b].conj().T).max() < 1e-14 * max(1.0, np.abs(S[b]).max())
        assert np.linalg.eigvalsh(S[b]).min() > -1e-12 * max(1.0, np.abs(S[b]).max())


def test_error_falls_as_the_square_of_the_node_spacing():
    shape = gwsynth.make_shape(n_k=2, n_b=80, R=64, N=12, n_occ=4, n_unocc=40)
    inp = gwsynth.generate(shape, seed=3, omega=np.array([0.0, 0.5, 5.0]))
    n_occ = 4
    x = _energies(inp, n_occ)
    P = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, n_occ, kq=inp.kq)
    errs = []
    for B in (16, 32, 64):
        nodes = np.geomspace(x.min(), x.max(), B)
        Ps = orc.polarization_spectral(inp.U, inp.psi, inp.eps, inp.omega, n_occ, nodes, kq=inp.kq)
        errs.append(orc.rel_fro(Ps, P).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, errs
