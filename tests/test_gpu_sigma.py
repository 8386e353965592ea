"""Correlation self-energy (Eq. SEc_AC) through the C ABI vs the CPU FP64
oracle.  The oracle builds its own W^c for every momentum transfer from the
same inputs (the GPU's W is computed by the library's FP64 path); the FP64
self-energy path must agree to 1e-10, the split-BF16 one to 1e-4 (relative,
max over states of the vector of output frequencies)."""
import numpy as np
import pytest

import gwsynth
from oracle import polarization as orc
from oracle import selfenergy as ose

pytestmark = pytest.mark.gpu


def _gpu_W(lib, U64, psi64, eps, mesh, n_occ, v):
    """W(t) for every transfer t with the library's FP64 path."""
    import torch
    n_k = psi64.shape[0]
    Ws = []
    for t in range(n_k):
        kq = (np.arange(n_k) + t) % n_k
        P = lib.gw_polarization(U64, psi64, eps, mesh, n_occ, precision="fp64", kq=kq)
        W, info = lib.gw_screen(P, v)
        torch.cuda.synchronize()
        assert int(info.abs().sum()) == 0
        Ws.append(W)
    return Ws


def _oracle(U, psi, eps, mesh, n_occ, v, out, states, mu):
    n_k = psi.shape[0]
    Wc = [ose.correlation_w(U, psi, eps, mesh, n_occ, v, t) for t in range(n_k)]
    return ose.sigma_c(U, psi, eps, Wc, mesh, out, states, mu)


def _rel(a, b):
    return max(np.linalg.norm(a[i] - b[i]) / np.linalg.norm(b[i]) for i in range(b.shape[0]))


def _mu(eps, n_occ):
    return 0.5 * (eps[:, :n_occ].max() + eps[:, n_occ:].min())


def test_sigma_fp64_config1(lib):
    import torch
    inp = gwsynth.generate("c1")
    n_occ = 4
    mesh = inp.omega                     # starts at 0
    out = np.concatenate([mesh, [0.1, 3.0, 8.0]])      # on the mesh, between points and beyond the last
    states = [(0, 3), (0, 4), (5, 0), (7, 63)]
    mu = _mu(inp.eps, n_occ)
    U = torch.from_numpy(inp.U).to("cuda")
    psi = torch.from_numpy(inp.psi).to("cuda")
    v = torch.from_numpy(inp.v).to("cuda")
    Ws = _gpu_W(lib, U, psi, inp.eps, mesh, n_occ, v)
    sig = lib.gw_sigma_c(U, psi, inp.eps, Ws, v, mesh, out, states, mu, precision="fp64")
    torch.cuda.synchronize()
    ref = _oracle(inp.U, inp.psi, inp.eps, mesh, n_occ, inp.v, out, states, mu)
    err = _rel(sig.cpu().numpy(), ref)
    print(f"sigma_c fp64 c1: rel err {err:.2e}")
    assert err < 1e-10
    # on the imaginary axis Sigma_c(i w) = sum_p |A_p|^2 / (i w - E_p): real at w = 0,
    # negative imaginary part for w > 0
    s = sig.cpu().numpy()
    assert np.all(np.abs(s[:, 0].imag) <= 1e-12 * np.abs(s[:, 0]))
    assert np.all(s[:, out > 0].imag < 0)


@pytest.mark.parametrize("cp", [3, 4])
@pytest.mark.parametrize("shape", [
    dict(n_k=2, n_b=60, R=1000, N=300, n_occ=3, n_unocc=150),
    dict(n_k=3, n_b=64, R=513, N=129, n_occ=2, n_unocc=63),
])
def test_sigma_split_bf16(lib, shape, cp):
    """Split BF16 on both GEMM cores (complex_product 3: the three-product
    six-slot core, the default; 4: the four-product core) against the oracle."""
    import torch
    inp = gwsynth.generate(gwsynth.make_shape(**shape), seed=5, omega=gwsynth.omega_mesh("m16"))
    n_occ = shape["n_occ"]
    mesh = inp.omega
    out = np.array([0.0, 0.05, 0.5, 2.0, 30.0])
    nb = n_occ + shape["n_unocc"]
    states = [(0, n_occ - 1), (0, n_occ), (shape["n_k"] - 1, nb - 1)]
    mu = _mu(inp.eps, n_occ)
    U64 = inp.U.astype(np.complex64).astype(np.complex128)
    psi64 = inp.psi.astype(np.complex64).astype(np.complex128)
    v = torch.from_numpy(inp.v).to("cuda")
    Ws = _gpu_W(lib, torch.from_numpy(U64).to("cuda"), torch.from_numpy(psi64).to("cuda"), inp.eps, mesh, n_occ, v)
    U32 = torch.from_numpy(inp.U).to("cuda", torch.complex64)
    psi32 = torch.from_numpy(inp.psi).to("cuda", torch.complex64)
    try:
        lib.gw_set_tuning("complex_product", cp)
        sig = lib.gw_sigma_c(U32, psi32, inp.eps, Ws, v, mesh, out, states, mu, precision="split_bf16")
        torch.cuda.synchronize()
    finally:
        lib.gw_set_tuning("complex_product", 3)
    ref = _oracle(U64, psi64, inp.eps, mesh, n_occ, inp.v, out, states, mu)
    err = _rel(sig.cpu().numpy(), ref)
    print(f"sigma_c split_bf16 {shape}, complex_product {cp}: rel err {err:.2e}")
    assert err < 1e-4


def test_sigma_deterministic_and_workspace_reuse(lib):
    import torch
    inp = gwsynth.generate("c1")
    mesh = inp.omega
    U = torch.from_numpy(inp.U).to("cuda")
    psi = torch.from_numpy(inp.psi).to("cuda")
    v = torch.from_numpy(inp.v).to("cuda")
    Ws = _gpu_W(lib, U, psi, inp.eps, mesh, 4, v)
    call = lib.SigmaCall(U, psi, inp.eps, Ws, v, mesh, [0.0, 1.0], [(1, 2), (2, 9)], _mu(inp.eps, 4))
    ws = torch.empty(call.workspace_size(), dtype=torch.uint8, device="cuda")
    ws.fill_(0xFF)
    a = call.run(ws).clone()
    b = call.run(ws).clone()
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_sigma_split_bf16_batches(lib):
    """18 states: a full batch of 16 sharing each transfer's W^c operand and one
    partial batch of 2.  Every state equals, bit for bit, the same state
    computed alone (the columns of the batched products are independent), and
    all of them meet the oracle bar."""
    import torch
    shape = dict(n_k=3, n_b=64, R=513, N=129, n_occ=2, n_unocc=63)
    inp = gwsynth.generate(gwsynth.make_shape(**shape), seed=8, omega=gwsynth.omega_mesh("m16"))
    n_occ = shape["n_occ"]
    mesh = inp.omega
    out = np.array([0.0, 0.3, 4.0])
    states = [(k, b) for k in range(3) for b in (0, 1, 2, 5, 30, 64)]
    mu = _mu(inp.eps, n_occ)
    U64 = inp.U.astype(np.complex64).astype(np.complex128)
    psi64 = inp.psi.astype(np.complex64).astype(np.complex128)
    v = torch.from_numpy(inp.v).to("cuda")
    Ws = _gpu_W(lib, torch.from_numpy(U64).to("cuda"), torch.from_numpy(psi64).to("cuda"), inp.eps, mesh, n_occ, v)
    U32 = torch.from_numpy(inp.U).to("cuda", torch.complex64)
    psi32 = torch.from_numpy(inp.psi).to("cuda", torch.complex64)
    sig = lib.gw_sigma_c(U32, psi32, inp.eps, Ws, v, mesh, out, states, mu, precision="split_bf16").clone()
    for i in (0, 15, 16, 17):
        one = lib.gw_sigma_c(U32, psi32, inp.eps, Ws, v, mesh, out, [states[i]], mu, precision="split_bf16")
        torch.cuda.synchronize()
        assert torch.equal(sig[i], one[0]), i
    ref = _oracle(U64, psi64, inp.eps, mesh, n_occ, inp.v, out, states, mu)
    err = _rel(sig.cpu().numpy(), ref)
    print(f"sigma_c split_bf16, 18 states in batches of 16 + 2: rel err {err:.2e}")
    assert err < 1e-4
