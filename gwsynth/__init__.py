"""Seeded synthetic inputs for the RPA polarization path.

This module only draws and shapes inputs: wave functions, band energies, the
basis-projection matrix U, the Coulomb eigenvalues v, the frequency mesh and
initial network weights.  It holds none of the polarization/screening
arithmetic, so the CPU oracle and the GPU path can both consume its output
without sharing any of the method's code.

Workload recipe (the paper's real crystals are replaced by random data with
the paper's shapes; Sec. "Formulation in the MPB", Eq. proj_MB / polar_MB):

* per k-point: A ~ CN(0,1)^{N_b x R};  z = Q of a reduced QR of
  CN(0,1)^{N_b x n_bands} (done blockwise when n_bands > N_b);
  psi_k = z^T A / sqrt(N_b)  (bands x grid, grid contiguous);
  occupied energies ~ U[-0.5, 0] Ha sorted, unoccupied ~ U[0.02, 2.0] Ha sorted.
  The wave functions at k+q are the set at (k+1) mod N_k.
* U = CN(0,1)^{N x R} * exp(-2 I / N) / sqrt(R)   (rows decay with basis index)
* v_I = 4 pi / (0.05 + (I/N)^2)   (a diagonal stand-in for the Coulomb
  eigenvalues of Eq. dielec_MB)

CN(0,1) means real and imaginary parts i.i.d. N(0, 1/2).

Two backends draw the same recipe:
* ``numpy`` -- everything on the host, bit-reproducible per seed.  Seeds:
  ``SeedSequence([20100316, cfg_id]).spawn(N_k + 1)``; child k draws, in this
  order, Re A, Im A, Re z, Im z, eps_occ, eps_unocc; child N_k draws Re U, Im U.
* ``torch`` -- for the large workloads: the Gaussian arrays (A, z, U) are drawn
  on the device with torch's counter-based generator seeded from the same
  SeedSequence children; the energies still come from numpy on the host.  z is
  orthonormalised in complex128 on the device by shifted Cholesky QR (three
  passes of Gram matrix, Cholesky factor and triangular solve, every step a
  matrix product except the factorisation and inversion of small diagonal
  blocks, done by host LAPACK), so no device solver library is involved; z^T A
  runs in complex64 on the device.  Values differ from the numpy backend; each
  run's oracle consumes the very tensors the GPU path consumes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

BASE_SEED = 20100316


def omega_mesh(kind: str) -> np.ndarray:
    """Imaginary-frequency meshes (Hartree), dense near zero.

    'c1'  : {0, 0.05, 0.2, 0.5, 1.5, 5}
    'm13' : {0} + 12 log-spaced points in [0.01, 20]
    'm16' : {0} + 15 log-spaced points in [0.01, 20]
    """
    if kind == "c1":
        return np.array([0.0, 0.05, 0.2, 0.5, 1.5, 5.0])
    if kind == "m13":
        return np.concatenate([[0.0], np.geomspace(0.01, 20.0, 12)])
    if kind == "m16":
        return np.concatenate([[0.0], np.geomspace(0.01, 20.0, 15)])
    raise ValueError(kind)


@dataclasses.dataclass(frozen=True)
class Shape:
    name: str
    cfg_id: int
    n_k: int
    n_b: int
    R: int
    N: int
    n_occ: int
    n_unocc: int
    omega: str = "m16"
    n_unocc_cut: Optional[int] = None  # explicit unoccupied bands on the surrogate path

    @property
    def n_bands(self) -> int:
        return self.n_occ + self.n_unocc


# Workload presets.  Sizes follow the paper's workload shapes (MPB of a few
# hundred to a few thousand functions, 4x4x4 k-meshes, ~200+ unoccupied bands,
# ~10-16 imaginary frequencies, a 128-atom supercell at few k-points).
SHAPES = {
    "c1": Shape("c1", 1, n_k=8, n_b=100, R=512, N=120, n_occ=4, n_unocc=60, omega="c1"),
    "c2": Shape("c2", 2, n_k=64, n_b=600, R=4096, N=500, n_occ=16, n_unocc=500, omega="m13"),
    "c3": Shape("c3", 3, n_k=8, n_b=3000, R=32768, N=3000, n_occ=128, n_unocc=2000),
    "c4": Shape("c4", 4, n_k=8, n_b=3000, R=32768, N=3000, n_occ=128, n_unocc=2000,
                n_unocc_cut=300),
    # full-band training runs for the high-band surrogate
    "c4train": Shape("c4train", 40, n_k=4, n_b=1600, R=8192, N=1000, n_occ=64,
                     n_unocc=1500),
    "c5": Shape("c5", 5, n_k=4, n_b=6000, R=65536, N=6000, n_occ=256, n_unocc=6000,
                n_unocc_cut=1500),
}


@dataclasses.dataclass
class Inputs:
    """One workload instance.  Arrays are numpy (host) or torch (device)."""
    shape: Shape
    U: object          # [N][R] complex
    psi: object        # [n_k][n_bands][R] complex; bands [0,n_occ) occupied
    eps: np.ndarray    # [n_k][n_bands] float64 (always host)
    v: np.ndarray      # [N] float64
    omega: np.ndarray  # [n_omega] float64
    kq: np.ndarray     # [n_k] int32, index of the k+q set
    seed: int


def _cn(rng: np.random.Generator, shape) -> np.ndarray:
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) * math.sqrt(0.5)


def _orthonormal_columns(zraw: np.ndarray) -> np.ndarray:
    """Reduced QR; when there are more columns than rows the columns are
    orthonormalised in independent blocks of at most n_rows columns."""
    n_b, n_cols = zraw.shape
    out = np.empty_like(zraw)
    for c0 in range(0, n_cols, n_b):
        c1 = min(n_cols, c0 + n_b)
        q, _ = np.linalg.qr(zraw[:, c0:c1], mode="reduced")
        out[:, c0:c1] = q
    return out



def _cholesky_lower(G, block: int = 512):
    """Lower Cholesky factor L (G = L L^H) of a Hermitian positive definite
    torch matrix, blocked right-looking: each diagonal block is factored and
    inverted by host LAPACK; the panel and the trailing update are matrix
    products on G's device.  Returns (L, list of the inverted diagonal blocks)."""
    import torch

    n = G.shape[0]
    A = G.clone()
    L = torch.zeros_like(G)
    inv_blocks = []
    for j0 in range(0, n, block):
        j1 = min(n, j0 + block)
        d = A[j0:j1, j0:j1].cpu().numpy()
        d = 0.5 * (d + d.conj().T)
        Ljj = np.linalg.cholesky(d)
        Linv = np.linalg.inv(Ljj)
        Linv = np.tril(Linv)
        Ljj_t = torch.from_numpy(Ljj).to(G.device)
        Linv_t = torch.from_numpy(Linv).to(G.device)
        inv_blocks.append(Linv_t)
        L[j0:j1, j0:j1] = Ljj_t
        if j1 < n:
            X = A[j1:, j0:j1] @ Linv_t.conj().transpose(0, 1)      # panel L21 = A21 L11^-H
            L[j1:, j0:j1] = X
            A[j1:, j1:] -= X @ X.conj().transpose(0, 1)
    return L, inv_blocks


def _right_solve_upper(Z, L, inv_blocks, block: int = 512):
    """Q with Q L^H = Z (L lower, so L^H is upper), by block columns:
    Q_j = (Z_j - sum_{i<j} Q_i (L^H)_ij) (L_jj^H)^-1, all matrix products."""
    import torch

    n = L.shape[0]
    Q = torch.empty_like(Z)
    for b, j0 in enumerate(range(0, n, block)):
        j1 = min(n, j0 + block)
        rhs = Z[:, j0:j1]
        if j0 > 0:
            rhs = rhs - Q[:, :j0] @ L[j0:j1, :j0].conj().transpose(0, 1)
        Q[:, j0:j1] = rhs @ inv_blocks[b].conj().transpose(0, 1)
    return Q


def cholesky_qr(Z, passes: int = 3):
    """Orthonormal columns spanning those of the complex128 matrix Z (rows >=
    columns): shifted Cholesky QR.  Each pass forms the Gram matrix G = Z^H Z,
    its Cholesky factor G = L L^H and Z <- Z L^-H; the first pass factors
    G + s I with s = 11 (m n + n (n + 1)) u ||Z||_2^2 (u the unit roundoff, the
    2-norm bounded by the Frobenius norm) so that the factorisation exists
    for any full-rank Z, the later passes restore orthonormality to rounding
    level (Fukaya, Kannan, Nakatsukasa, Yamamoto, Yanagisawa, SIAM J. Sci.
    Comput. 42 (2020), shifted CholeskyQR3).  The columns equal those of a
    Householder QR up to a unit-modulus factor per column."""
    import torch

    m, n = Z.shape
    if n > m:
        raise ValueError("cholesky_qr needs at least as many rows as columns")
    u = float(np.finfo(np.float64).eps) / 2.0
    Q = Z
    for p in range(passes):
        G = Q.conj().transpose(0, 1) @ Q
        G = 0.5 * (G + G.conj().transpose(0, 1))
        if p == 0:
            nrm2 = float((Q.real.square() + Q.imag.square()).sum().item())
            s = 11.0 * (m * n + n * (n + 1)) * u * nrm2
            G = G + s * torch.eye(n, dtype=G.dtype, device=G.device)
        L, inv_blocks = _cholesky_lower(G)
        Q = _right_solve_upper(Q, L, inv_blocks)
    return Q


def coulomb_diag(N: int) -> np.ndarray:
    I = np.arange(N, dtype=np.float64)
    return 4.0 * math.pi / (0.05 + (I / N) ** 2)


def _u_decay(N: int, R: int) -> np.ndarray:
    I = np.arange(N, dtype=np.float64)
    return np.exp(-2.0 * I / N) / math.sqrt(R)


def make_shape(name: str = "custom", *, n_k: int, n_b: int, R: int, N: int, n_occ: int,
               n_unocc: int, omega: str = "m16", cfg_id: int = 99) -> Shape:
    return Shape(name, cfg_id, n_k=n_k, n_b=n_b, R=R, N=N, n_occ=n_occ, n_unocc=n_unocc,
                 omega=omega)


def generate(shape: Shape | str, seed: Optional[int] = None, *, omega: Optional[Sequence[float]] = None,
             base_seed: int = BASE_SEED) -> Inputs:
    """Host (numpy) generation, complex128.  ``seed`` overrides cfg_id."""
    if isinstance(shape, str):
        shape = SHAPES[shape]
    sid = shape.cfg_id if seed is None else seed
    ss = np.random.SeedSequence([base_seed, sid])
    children = ss.spawn(shape.n_k + 1)
    nb = shape.n_bands
    psi = np.empty((shape.n_k, nb, shape.R), dtype=np.complex128)
    eps = np.empty((shape.n_k, nb), dtype=np.float64)
    for k in range(shape.n_k):
        rng = np.random.default_rng(children[k])
        A = _cn(rng, (shape.n_b, shape.R))
        z = _orthonormal_columns(_cn(rng, (shape.n_b, nb)))
        eps[k, :shape.n_occ] = np.sort(rng.uniform(-0.5, 0.0, shape.n_occ))
        eps[k, shape.n_occ:] = np.sort(rng.uniform(0.02, 2.0, shape.n_unocc))
        psi[k] = (z.T @ A) / math.sqrt(shape.n_b)
    rng = np.random.default_rng(children[shape.n_k])
    U = _cn(rng, (shape.N, shape.R)) * _u_decay(shape.N, shape.R)[:, None]
    om = np.asarray(omega, dtype=np.float64) if omega is not None else omega_mesh(shape.omega)
    kq = ((np.arange(shape.n_k) + 1) % shape.n_k).astype(np.int32)
    return Inputs(shape, U, psi, eps, coulomb_diag(shape.N), om, kq, sid)


def generate_torch(shape: Shape | str, device, seed: Optional[int] = None, *,
                   omega: Optional[Sequence[float]] = None, base_seed: int = BASE_SEED,
                   k_subset: Optional[Sequence[int]] = None,
                   band_limit: Optional[int] = None, log=None) -> Inputs:
    """Device generation in complex64 (large workloads).

    Gaussian draws use torch's device generator seeded from the SeedSequence
    children; the energies come from numpy on the host.  The orthonormal
    basis z is computed blockwise by a complex128 QR on the device, and
    psi_k = z^T A / sqrt(N_b) by complex64 products.  ``band_limit`` keeps the
    first ``band_limit`` bands of each k-set (z is still drawn and
    orthonormalised at full width, so the kept bands equal those of a full
    draw); ``k_subset`` generates only those k-sets (others stay zero).
    """
    import torch

    if isinstance(shape, str):
        shape = SHAPES[shape]
    sid = shape.cfg_id if seed is None else seed
    ss = np.random.SeedSequence([base_seed, sid])
    children = ss.spawn(shape.n_k + 1)
    nb_full = shape.n_bands
    nb = nb_full if band_limit is None else min(nb_full, band_limit)
    psi = torch.zeros((shape.n_k, nb, shape.R), dtype=torch.complex64, device=device)
    eps = np.zeros((shape.n_k, nb_full), dtype=np.float64)
    ks = set(range(shape.n_k)) if k_subset is None else set(k_subset)
    scale = 1.0 / math.sqrt(shape.n_b)

    def cn(g, rows, cols, dtype=torch.float32):
        x = torch.complex(torch.randn((rows, cols), generator=g, device=device, dtype=dtype),
                          torch.randn((rows, cols), generator=g, device=device, dtype=dtype))
        return x.mul_(math.sqrt(0.5))

    for k in range(shape.n_k):
        rng = np.random.default_rng(children[k])
        dev_seed = int(rng.integers(0, 2**62))
        eps[k, :shape.n_occ] = np.sort(rng.uniform(-0.5, 0.0, shape.n_occ))
        eps[k, shape.n_occ:] = np.sort(rng.uniform(0.02, 2.0, shape.n_unocc))
        if k not in ks:
            continue
        g = torch.Generator(device=device)
        g.manual_seed(dev_seed)
        zraw = cn(g, shape.n_b, nb_full, torch.float64)
        z = torch.empty_like(zraw)
        for c0 in range(0, nb_full, shape.n_b):
            c1 = min(nb_full, c0 + shape.n_b)
            z[:, c0:c1] = cholesky_qr(zraw[:, c0:c1])
        zt = z[:, :nb].transpose(0, 1).contiguous().to(torch.complex64)
        del zraw, z
        acc = None
        rb = 1024
        for r0 in range(0, shape.n_b, rb):
            r1 = min(shape.n_b, r0 + rb)
            Ablk = cn(g, r1 - r0, shape.R)
            part = torch.matmul(zt[:, r0:r1].contiguous(), Ablk)
            acc = part if acc is None else acc.add_(part)
            del Ablk, part
        psi[k].copy_(acc.mul_(scale))
        del acc, zt
        if log:
            log(f"generated k-set {k}")
    rng = np.random.default_rng(children[shape.n_k])
    g = torch.Generator(device=device)
    g.manual_seed(int(rng.integers(0, 2**62)))
    U = cn(g, shape.N, shape.R)
    dec = torch.from_numpy(_u_decay(shape.N, shape.R)).to(device=device, dtype=torch.float32)
    U.mul_(dec[:, None])
    om = np.asarray(omega, dtype=np.float64) if omega is not None else omega_mesh(shape.omega)
    kq = ((np.arange(shape.n_k) + 1) % shape.n_k).astype(np.int32)
    return Inputs(shape, U, psi, eps, coulomb_diag(shape.N), om, kq, sid)


def mlp_init(n_in: int, width: int, n_out: int, seed: int = 7) -> dict:
    """Initial weights of a 3-layer perceptron (float64, He-style scaling).

    Layout: W1 [n_in][width], b1 [width], W2 [width][width], b2 [width],
    W3 [width][n_out], b3 [n_out]  (row-major, y = x W + b).
    """
    rng = np.random.default_rng(np.random.SeedSequence([BASE_SEED, 7000, seed]))
    W1 = rng.standard_normal((n_in, width)) * math.sqrt(2.0 / n_in)
    W2 = rng.standard_normal((width, width)) * math.sqrt(2.0 / width)
    W3 = rng.standard_normal((width, n_out)) * math.sqrt(1.0 / width) * 0.1
    return {"W1": W1, "b1": np.zeros(width), "W2": W2, "b2": np.zeros(width),
            "W3": W3, "b3": np.zeros(n_out)}
