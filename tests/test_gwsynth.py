"""The seeded input generator: determinism and the recipe's stated properties."""
import numpy as np

import gwsynth


def test_deterministic_and_seed_dependent():
    a = gwsynth.generate("c1")
    b = gwsynth.generate("c1")
    c = gwsynth.generate("c1", seed=77)
    assert np.array_equal(a.psi, b.psi) and np.array_equal(a.U, b.U) and np.array_equal(a.eps, b.eps)
    assert not np.array_equal(a.psi, c.psi)


def test_shapes_and_ranges():
    s = gwsynth.SHAPES["c1"]
    inp = gwsynth.generate(s)
    assert inp.U.shape == (s.N, s.R) and inp.psi.shape == (s.n_k, s.n_bands, s.R)
    assert inp.eps.shape == (s.n_k, s.n_bands)
    eo, eu = inp.eps[:, :s.n_occ], inp.eps[:, s.n_occ:]
    assert eo.min() >= -0.5 and eo.max() <= 0 and eu.min() >= 0.02 and eu.max() <= 2.0
    assert np.all(np.diff(eo, axis=1) >= 0) and np.all(np.diff(eu, axis=1) >= 0)
    np.testing.assert_array_equal(inp.kq, (np.arange(s.n_k) + 1) % s.n_k)
    np.testing.assert_allclose(inp.omega, [0, 0.05, 0.2, 0.5, 1.5, 5])
    assert abs(inp.v[0] - 4 * np.pi / 0.05) < 1e-12


def test_band_gram_matches_recipe():
    # psi = z^T A / sqrt(N_b) with orthonormal z: psi psi^H = z^T (A A^H / N_b) conj(z);
    # its trace over bands equals sum_b z-weighted row norms of A, about R per band.
    s = gwsynth.make_shape(n_k=1, n_b=50, R=4096, N=8, n_occ=3, n_unocc=20)
    inp = gwsynth.generate(s, seed=3)
    nrm = np.sum(np.abs(inp.psi[0]) ** 2, axis=1)
    assert np.all(np.abs(nrm / (4096 / 50) - 1) < 0.15)


def test_blockwise_orthonormal_when_more_bands_than_coefficients():
    rng = np.random.default_rng(0)
    z = gwsynth._orthonormal_columns(gwsynth._cn(rng, (10, 23)))
    for c0, c1 in ((0, 10), (10, 20), (20, 23)):
        q = z[:, c0:c1]
        np.testing.assert_allclose(q.conj().T @ q, np.eye(c1 - c0), atol=1e-13)


def test_omega_meshes():
    m13 = gwsynth.omega_mesh("m13")
    m16 = gwsynth.omega_mesh("m16")
    assert m13.size == 13 and m16.size == 16 and m13[0] == 0 and m16[0] == 0
    np.testing.assert_allclose([m16[1], m16[-1]], [0.01, 20.0])


def test_device_orthonormalisation_matches_householder_up_to_phases():
    """The torch backend's shifted Cholesky QR spans the same columns as a
    LAPACK Householder QR: each column agrees up to a unit-modulus factor."""
    import torch
    rng = np.random.default_rng(5)
    for m, n in ((300, 300), (700, 530), (90, 7)):
        Z = gwsynth._cn(rng, (m, n))
        Q = gwsynth.cholesky_qr(torch.from_numpy(Z)).numpy()
        np.testing.assert_allclose(Q.conj().T @ Q, np.eye(n), atol=1e-13)
        q, _ = np.linalg.qr(Z)
        ph = np.sum(q.conj() * Q, axis=0)
        np.testing.assert_allclose(np.abs(ph), 1.0, atol=1e-12)
        np.testing.assert_allclose(Q, q * ph[None, :], atol=1e-12)


def test_device_orthonormalisation_of_an_ill_conditioned_block():
    """Condition number 1e7: the shifted first pass keeps the factorisation
    defined and the later passes restore orthonormality."""
    import torch
    rng = np.random.default_rng(6)
    m, n = 400, 200
    a, _ = np.linalg.qr(gwsynth._cn(rng, (m, n)))
    b, _ = np.linalg.qr(gwsynth._cn(rng, (n, n)))
    Z = (a * np.geomspace(1.0, 1e-7, n)[None, :]) @ b
    Q = gwsynth.cholesky_qr(torch.from_numpy(Z)).numpy()
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(n), atol=1e-12)
    # same column space as Z
    proj = Q @ (Q.conj().T @ Z)
    assert np.linalg.norm(proj - Z) < 1e-10 * np.linalg.norm(Z)


def test_torch_backend_on_the_host_is_deterministic():
    import torch
    s = gwsynth.make_shape(n_k=2, n_b=40, R=64, N=6, n_occ=2, n_unocc=50)   # 52 bands > 40: two QR blocks
    a = gwsynth.generate_torch(s, torch.device("cpu"), seed=4)
    b = gwsynth.generate_torch(s, torch.device("cpu"), seed=4)
    assert torch.equal(a.psi, b.psi) and torch.equal(a.U, b.U) and np.array_equal(a.eps, b.eps)
    assert a.psi.shape == (2, 52, 64) and a.psi.dtype == torch.complex64
