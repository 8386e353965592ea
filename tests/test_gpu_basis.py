"""Basis optimization by the Coulomb eigenvalue threshold (Sec. "Optimization
of the MPB") through the C ABI: the kept rows and entries must equal the
selection v >= v_min made on the host, bit for bit, in their original order."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,R", [("complex64", 1000), ("complex128", 33), ("float32", 513), ("float32", 7)])
def test_basis_select_matches_host_selection(lib, dtype, R):
    import torch
    rng = np.random.default_rng(4)
    N = 2500                                     # spans several 1024-row scan blocks
    v = rng.uniform(0.0, 10.0, N)
    U = rng.normal(size=(N, R))
    if dtype != "float32":
        U = U + 1j * rng.normal(size=(N, R))
    U = U.astype(dtype)
    Ud = torch.from_numpy(U).to("cuda")
    vd = torch.from_numpy(v).to("cuda")
    for v_min in (4.0, 0.0, 11.0, 9.99):
        Uo, vo, src = lib.gw_basis_select(Ud, vd, v_min)
        torch.cuda.synchronize()
        keep = np.nonzero(v >= v_min)[0]
        assert np.array_equal(src.cpu().numpy(), keep)
        assert np.array_equal(vo.cpu().numpy(), v[keep])
        assert np.array_equal(Uo.cpu().numpy(), U[keep])
