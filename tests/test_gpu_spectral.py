"""The spectral route of the polarization (transitions split onto
transition-energy nodes, node matrices accumulated by the library's
polarization pass, P(i w) by the Hilbert transform of each node) through the C
ABI against the oracle's spectral route on the same inputs: FP64 1e-10,
reduced precisions 1e-4 (relative Frobenius, per frequency)."""
import numpy as np
import pytest

import gwsynth
from oracle import polarization as orc

pytestmark = pytest.mark.gpu


def _energies(eps, n_occ, kq):
    return np.concatenate([(eps[kq[k], n_occ:][None, :] - eps[k, :n_occ][:, None]).reshape(-1)
                           for k in range(eps.shape[0])])


def _nodes(eps, n_occ, kq, B):
    x = _energies(eps, n_occ, kq)
    return np.geomspace(x.min(), x.max(), B)


def test_spectral_fp64_config1(lib):
    import torch
    inp = gwsynth.generate("c1")
    n_occ = 4
    nodes = _nodes(inp.eps, n_occ, inp.kq, 40)
    U = torch.from_numpy(inp.U).to("cuda")
    psi = torch.from_numpy(inp.psi).to("cuda")
    P = lib.gw_polarization(U, psi, inp.eps, inp.omega, n_occ, precision="fp64", kq=inp.kq, nodes=nodes)
    torch.cuda.synchronize()
    ref = orc.polarization_spectral(inp.U, inp.psi, inp.eps, inp.omega, n_occ, nodes, kq=inp.kq)
    err = orc.rel_fro(P.cpu().numpy(), ref)
    direct = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, n_occ, kq=inp.kq)
    print(f"spectral fp64 c1 (40 nodes): {err.max():.2e} vs the oracle's route; "
          f"route error vs the direct sum {orc.rel_fro(ref, direct).max():.2e}")
    assert err.max() < 1e-10


def test_spectral_nodes_on_every_transition_equal_the_direct_sum(lib):
    import torch
    shape = gwsynth.make_shape(n_k=2, n_b=40, R=200, N=70, n_occ=2, n_unocc=20)
    inp = gwsynth.generate(shape, seed=6, omega=gwsynth.omega_mesh("c1"))
    n_occ = 2
    nodes = np.unique(_energies(inp.eps, n_occ, inp.kq))
    assert 2 <= nodes.size <= 256
    U = torch.from_numpy(inp.U).to("cuda")
    psi = torch.from_numpy(inp.psi).to("cuda")
    Ps = lib.gw_polarization(U, psi, inp.eps, inp.omega, n_occ, precision="fp64", kq=inp.kq, nodes=nodes).clone()
    Pd = lib.gw_polarization(U, psi, inp.eps, inp.omega, n_occ, precision="fp64", kq=inp.kq)
    torch.cuda.synchronize()
    assert orc.rel_fro(Ps.cpu().numpy(), Pd.cpu().numpy()).max() < 1e-12


@pytest.mark.parametrize("prec,B", [("split_bf16", 96), ("fp32", 33), ("split_fp16", 64)])
def test_spectral_reduced_precisions(lib, prec, B):
    """Ragged multi-tile shape; 96 nodes exercise more slots than frequencies."""
    import torch
    shape = dict(n_k=2, n_b=60, R=1000, N=300, n_occ=3, n_unocc=150)
    inp = gwsynth.generate(gwsynth.make_shape(**shape), seed=9, omega=gwsynth.omega_mesh("m16"))
    n_occ = 3
    nodes = _nodes(inp.eps, n_occ, inp.kq, B)
    U = torch.from_numpy(inp.U).to("cuda", torch.complex64)
    psi = torch.from_numpy(inp.psi).to("cuda", torch.complex64)
    P = lib.gw_polarization(U, psi, inp.eps, inp.omega, n_occ, precision=prec, kq=inp.kq, nodes=nodes)
    torch.cuda.synchronize()
    Ur = inp.U.astype(np.complex64).astype(np.complex128)
    pr = inp.psi.astype(np.complex64).astype(np.complex128)
    ref = orc.polarization_spectral(Ur, pr, inp.eps, inp.omega, n_occ, nodes, kq=inp.kq)
    err = orc.rel_fro(P.cpu().numpy(), ref)
    print(f"spectral {prec} ({B} nodes): {err.max():.2e}")
    assert err.max() < 1e-4


def test_spectral_accumulates_and_reuses_workspace(lib):
    """accumulate = 1 adds the spectral P to what P holds; a poisoned workspace
    does not change the result."""
    import torch
    inp = gwsynth.generate("c1")
    n_occ = 4
    nodes = _nodes(inp.eps, n_occ, inp.kq, 24)
    U = torch.from_numpy(inp.U).to("cuda")
    psi = torch.from_numpy(inp.psi).to("cuda")
    call = lib.PolarizationCall(U, psi, inp.eps, inp.omega, n_occ, precision="fp64", kq=inp.kq, nodes=nodes)
    ws = torch.empty(call.workspace_size(), dtype=torch.uint8, device="cuda")
    ws.fill_(0xFF)
    P1 = call.run(ws).clone()
    base = torch.randn(P1.shape, dtype=torch.float64, device="cuda").to(torch.complex128)
    acc = lib.PolarizationCall(U, psi, inp.eps, inp.omega, n_occ, precision="fp64", kq=inp.kq, nodes=nodes,
                               P=base.clone(), accumulate=True)
    P2 = acc.run(ws)
    torch.cuda.synchronize()
    assert torch.allclose(P2 - base, P1, rtol=1e-12, atol=1e-12 * float(P1.abs().max()))
