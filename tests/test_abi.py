"""The C ABI on the host: the library loads, exports every symbol gw.h
declares, answers workspace queries, and rejects invalid arguments with the
documented status before launching anything (no GPU needed).  Fake device
pointers are only used in calls whose validation must fail."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gw.h")
LIB = os.path.join(ROOT, "paper_1003_0316_amd", "libgw.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libgw.so not built")


def header_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gw_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def b():
    from paper_1003_0316_amd import binding
    return binding


def test_exports_every_declared_symbol(b):
    names = header_functions()
    assert "gw_polarization" in names and "gw_screen" in names and "gw_project" in names
    for n in names:
        assert hasattr(b.lib(), n), n
    assert set(b.EXPORTED) <= set(names)


def test_version(b):
    assert b.gw_version() >= 100


def _desc(b, n_k=2, N=8, R=16, n_occ=2, n_unocc=3, omega=(0.0, 1.0), eps=None, precision=0):
    keep = {}
    d = b.GwPolDesc()
    d.precision, d.n_k, d.N, d.R, d.n_occ, d.n_unocc = precision, n_k, N, R, n_occ, n_unocc
    d.occ_begin, d.occ_end, d.unocc_begin, d.unocc_end = 0, n_occ, 0, n_unocc
    keep["om"] = np.asarray(omega, dtype=np.float64)
    d.n_omega = len(omega)
    d.omega_host = keep["om"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    if eps is None:
        eps = np.concatenate([np.linspace(-0.5, -0.1, n_occ), np.linspace(0.1, 1.0, n_unocc)])
        eps = np.tile(eps, (n_k, 1))
    keep["eps"] = np.ascontiguousarray(eps, dtype=np.float64)
    d.eps_host = keep["eps"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    fake = 0x7F0000001000   # never dereferenced: every call below fails validation first
    d.U = d.psi = d.eps = d.P = fake
    d.kq_host = None
    d.k_list_host = None
    return d, keep


def test_workspace_queries(b):
    d, keep = _desc(b)
    n = ctypes.c_size_t(0)
    assert b.lib().gw_polarization_workspace_size(ctypes.byref(d), ctypes.byref(n)) == 0
    assert n.value >= 8 * 6 * 16
    assert b.gw_screen_workspace_size(100, 3) > 0
    assert b.gw_project_workspace_size("fp64", 4, 4, 1, 1) == 0


def _status(b, d):
    return b.lib().gw_polarization(None, ctypes.byref(d), ctypes.c_void_p(0x7F0000002000), 1 << 40)


@pytest.mark.parametrize("field,value", [
    ("N", 0), ("R", -1), ("n_omega", 0), ("occ_begin", 5), ("unocc_end", 9), ("precision", 7),
])
def test_rejects_bad_sizes(b, field, value):
    d, keep = _desc(b)
    setattr(d, field, value)
    assert _status(b, d) == -1
    assert b.gw_last_error() != ""


def test_rejects_negative_frequency(b):
    d, keep = _desc(b, omega=(0.0, -1.0))
    assert _status(b, d) == -1
    assert "frequenc" in b.gw_last_error()


def test_rejects_metal(b):
    eps = np.tile([-0.5, 0.3, 0.2, 0.4, 0.9], (2, 1))  # occupied 0.3 above unoccupied 0.2
    d, keep = _desc(b, eps=eps)
    assert _status(b, d) == -1
    assert "insulator" in b.gw_last_error()


def test_rejects_bad_k_maps(b):
    d, keep = _desc(b)
    kq = np.array([1, 5], dtype=np.int32)
    d.kq_host = kq.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    assert _status(b, d) == -1
    d, keep = _desc(b)
    kl = np.array([0, 2], dtype=np.int32)
    d.k_list_host = kl.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    d.n_k_list = 2
    assert _status(b, d) == -1


def test_rejects_too_many_frequencies(b):
    d, keep = _desc(b, omega=tuple(np.linspace(0, 1, 65)))
    assert _status(b, d) == -2


def test_rejects_small_workspace(b):
    d, keep = _desc(b)
    st = b.lib().gw_polarization(None, ctypes.byref(d), ctypes.c_void_p(0x7F0000002000), 16)
    assert st == -3
    st = b.lib().gw_polarization(None, ctypes.byref(d), None, 0)
    assert st == -3


def test_rejects_null_pointers(b):
    d, keep = _desc(b)
    d.P = None
    assert _status(b, d) == -1
    assert b.lib().gw_polarization(None, None, None, 0) == -1


def test_screen_validation(b):
    L = b.lib()
    fake = ctypes.c_void_p(0x7F0000003000)
    assert L.gw_screen(None, 0, 1, fake, fake, fake, fake, fake, 1 << 30) == -1
    assert L.gw_screen(None, 4, 1, None, fake, fake, fake, fake, 1 << 30) == -1
    assert L.gw_screen(None, 4, 1, fake, fake, fake, fake, fake, 1 << 30) == -1  # W aliases P
    other = ctypes.c_void_p(0x7F0000004000)
    assert L.gw_screen(None, 4, 1, fake, fake, other, fake, fake, 8) == -3


def test_project_validation(b):
    L = b.lib()
    fake = ctypes.c_void_p(0x7F0000003000)
    assert L.gw_project(None, 0, 0, 4, 1, 1, fake, fake, fake, fake, None, 0) == -1
    assert L.gw_project(None, 9, 4, 4, 1, 1, fake, fake, fake, fake, None, 0) == -1
    assert L.gw_project(None, 0, 4, 4, 1, 1, None, fake, fake, fake, None, 0) == -1


def test_tuning_switches_validate(b):
    """gw_set_tuning accepts the documented keys and values only (host-side)."""
    L = b.lib()
    for key, lo, hi, default in (("bf16_pipeline", 1, 2, 2), ("projection_variant", 1, 2, 2),
                                 ("gemm_staging", 1, 4, 3), ("complex_product", 3, 4, 3),
                                 ("fp16_core", 1, 2, 1), ("gemm3m_pipeline", 2, 6, 6),
                                 ("gemm3m_lead", 3, 5, 4), ("real_core", 1, 2, 2)):
        assert b.gw_get_tuning(key) == default
        for v in (lo, hi):
            assert L.gw_set_tuning(key.encode(), v) == 0
        for v in (lo - 1, hi + 1):
            assert L.gw_set_tuning(key.encode(), v) == -1
            assert key in L.gw_last_error().decode()
        assert L.gw_set_tuning(key.encode(), default) == 0
    assert L.gw_set_tuning(b"gemm3m_pipeline", 4) == -1   # two stage buffers or six plane slots only
    assert L.gw_set_tuning(b"no_such_key", 1) == -1
    assert L.gw_set_tuning(None, 1) == -1
    v = ctypes.c_int(0)
    assert L.gw_get_tuning(b"no_such_key", ctypes.byref(v)) == -1


def _sigma_desc(b, **over):
    keep = {}
    d = b.GwSigmaDesc()
    d.precision, d.n_k, d.N, d.R, d.n_bands = 0, 2, 8, 16, 5
    keep["mesh"] = np.asarray(over.pop("mesh", (0.0, 0.5, 2.0)), dtype=np.float64)
    d.n_mesh = keep["mesh"].size
    d.mesh_host = keep["mesh"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    keep["out"] = np.asarray(over.pop("out", (0.0, 1.0)), dtype=np.float64)
    d.n_out = keep["out"].size
    d.omega_out_host = keep["out"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    keep["ss"] = np.asarray(over.pop("sets", (0,)), dtype=np.int32)
    keep["sb"] = np.asarray(over.pop("bands", (1,)), dtype=np.int32)
    d.n_states = keep["ss"].size
    d.state_set_host = keep["ss"].ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    d.state_band_host = keep["sb"].ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    keep["eps"] = np.tile(np.array([-0.5, -0.2, 0.1, 0.4, 0.9]), (2, 1))
    d.eps_host = keep["eps"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.mu = over.pop("mu", 0.0)
    fake = 0x7F0000001000   # never dereferenced: every call below fails validation first
    d.U = d.psi = d.eps = d.v = d.sigma = fake
    keep["W"] = (ctypes.c_void_p * 2)(fake, fake)
    d.W_host = ctypes.cast(keep["W"], ctypes.POINTER(ctypes.c_void_p))
    for k, v in over.items():
        setattr(d, k, v)
    return d, keep


@pytest.mark.parametrize("kw,status", [
    (dict(mesh=(0.1, 0.5, 2.0)), -1),            # the mesh must start at 0
    (dict(mesh=(0.0, 0.5, 0.5)), -1),            # strictly increasing
    (dict(mesh=tuple(np.linspace(0, 1, 65))), -1),
    (dict(out=(-1.0,)), -1),
    (dict(mu=0.1), -1),                          # a band energy at the chemical potential
    (dict(bands=(5,)), -1),
    (dict(sets=(2,)), -1),
    (dict(precision=1), -2),                     # FP32 quadratic forms are not offered
])
def test_sigma_validation(b, kw, status):
    d, keep = _sigma_desc(b, **kw)
    out = ctypes.c_size_t(0)
    assert b.lib().gw_sigma_c_workspace_size(ctypes.byref(d), ctypes.byref(out)) == status
    assert b.lib().gw_sigma_c(None, ctypes.byref(d), None, 0) == status


def test_sigma_workspace_and_null_w(b):
    d, keep = _sigma_desc(b)
    out = ctypes.c_size_t(0)
    assert b.lib().gw_sigma_c_workspace_size(ctypes.byref(d), ctypes.byref(out)) == 0 and out.value > 0
    assert b.lib().gw_sigma_c(None, ctypes.byref(d), None, 0) == -3       # no workspace
    keep["W"][1] = None
    assert b.lib().gw_sigma_c_workspace_size(ctypes.byref(d), ctypes.byref(out)) == -1


def test_real_inputs_validation(b):
    d, keep = _desc(b, precision=0)
    d.real_inputs = 1
    out = ctypes.c_size_t(0)
    assert b.lib().gw_polarization_workspace_size(ctypes.byref(d), ctypes.byref(out)) == -2   # FP64: unsupported
    d.precision = 2
    d.real_inputs = 2
    assert b.lib().gw_polarization_workspace_size(ctypes.byref(d), ctypes.byref(out)) == -1
    d.real_inputs = 1
    assert b.lib().gw_polarization_workspace_size(ctypes.byref(d), ctypes.byref(out)) == 0 and out.value > 0


def test_basis_select_count(b):
    L = b.lib()
    v = np.array([5.0, 1.0, 3.0, 0.5, 3.0])
    n = ctypes.c_int(-1)
    ptr = v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.gw_basis_select_count(5, ptr, 3.0, ctypes.byref(n)) == 0 and n.value == 3
    assert L.gw_basis_select_count(5, ptr, 0.0, ctypes.byref(n)) == 0 and n.value == 5
    assert L.gw_basis_select_count(5, ptr, 9.0, ctypes.byref(n)) == 0 and n.value == 0
    assert L.gw_basis_select_count(0, ptr, 1.0, ctypes.byref(n)) == -1
    assert L.gw_basis_select_count(5, ptr, float("nan"), ctypes.byref(n)) == -1
    v[2] = np.inf
    assert L.gw_basis_select_count(5, ptr, 1.0, ctypes.byref(n)) == -1
    assert L.gw_basis_select(None, 4, 4, 12, 1, 1, 0.0, 1, 1, 1, 1) == -1      # element size


def _with_nodes(d, keep, nodes):
    keep["nodes"] = np.ascontiguousarray(nodes, dtype=np.float64)
    d.n_nodes = len(nodes)
    d.nodes_host = keep["nodes"].ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def test_spectral_route_validation(b):
    """Transition energies of the default descriptor span [0.2, 1.5]."""
    L = b.lib()
    out = ctypes.c_size_t(0)
    d, keep = _desc(b)
    assert L.gw_polarization_workspace_size(ctypes.byref(d), ctypes.byref(out)) == 0
    direct = out.value
    _with_nodes(d, keep, [0.2, 0.5, 1.5])
    assert L.gw_polarization_workspace_size(ctypes.byref(d), ctypes.byref(out)) == 0
    assert out.value >= direct + 3 * 8 * 8 * 16                   # the node matrices
    st = L.gw_polarization(None, ctypes.byref(d), ctypes.c_void_p(0x7F0000002000), 16)
    assert st == -3                                               # arguments valid, workspace too small
    for bad in ([0.25, 0.5, 1.5], [0.2, 0.5, 1.4], [0.2, 0.2, 1.5], [0.0, 0.5, 1.5], [0.2], [1.5, 0.5, 0.2]):
        d, keep = _desc(b)
        _with_nodes(d, keep, bad)
        assert _status(b, d) == -1, bad
        assert "node" in b.gw_last_error()
    d, keep = _desc(b)
    _with_nodes(d, keep, np.linspace(0.2, 1.5, 257))
    assert L.gw_polarization_workspace_size(ctypes.byref(d), ctypes.byref(out)) == -1
    assert _status(b, d) == -1
    d, keep = _desc(b, precision=3)                               # split FP16: at most 64 nodes
    _with_nodes(d, keep, np.linspace(0.2, 1.5, 65))
    assert _status(b, d) == -2


def test_screen_noalloc_validation(b):
    """The allocation-free screening rejects bad arguments and sizes whose
    panels exceed its fixed array, before touching the device."""
    L = b.lib()
    fake = ctypes.c_void_p(0x7F0000003000)
    other = ctypes.c_void_p(0x7F0000004000)
    assert b.gw_screen_noalloc_max_bytes() == 64 << 20
    assert L.gw_screen_noalloc(None, 0, 1, fake, fake, other, fake) == -1
    assert L.gw_screen_noalloc(None, 4, 1, None, fake, other, fake) == -1
    assert L.gw_screen_noalloc(None, 4, 1, fake, fake, fake, fake) == -1   # W aliases P
    # largest N at 16 frequencies that fits, and the next size up that does not
    fits = [N for N in range(64, 8193, 64) if b.gw_screen_workspace_size(N, 16) <= b.gw_screen_noalloc_max_bytes()]
    too_big = max(fits) + 64
    assert b.gw_screen_workspace_size(too_big, 16) > b.gw_screen_noalloc_max_bytes()
    assert L.gw_screen_noalloc(None, too_big, 16, fake, fake, other, fake) == -3
    assert "fixed array" in b.gw_last_error()


def _learned(b, d, keep, **kw):
    m = b.GwMlp(32, 256, 32, 0x7F0000005000, None, None, 0x7F0000006000, 0x7F0000007000)
    keep["mlp"] = m
    l = b.GwLearnedDesc()
    l.mlp = ctypes.pointer(m)
    l.cut, l.judge, l.n_sample_occ, l.judge_tol = 2, 1, 1, 0.25
    for k, v in kw.items():
        setattr(l, k, v)
    return l


def _lstatus(b, d, l):
    out = ctypes.c_size_t(0)
    return b.lib().gw_polarization_learned_workspace_size(ctypes.byref(d), ctypes.byref(l), ctypes.byref(out))


def test_learned_call_validation(b):
    """gw_polarization_learned rejects, before any launch: a missing
    perceptron, a cutoff outside [1, n_unocc), partial band ranges, k lists,
    accumulation and the spectral route, bad sample counts and tolerances."""
    d, keep = _desc(b, n_unocc=5)
    assert _lstatus(b, d, _learned(b, d, keep)) == 0
    L = b.lib()
    out = ctypes.c_size_t(0)
    assert L.gw_polarization_learned_workspace_size(ctypes.byref(d), None, ctypes.byref(out)) == -1
    for kw in ({"cut": 0}, {"cut": 5}, {"n_sample_occ": 0}, {"n_sample_occ": 3}, {"judge_tol": -1.0},
               {"judge_tol": float("nan")}, {"judge": 2}):
        assert _lstatus(b, d, _learned(b, d, keep, **kw)) == -1, kw
    l = _learned(b, d, keep)
    l.mlp.contents.n_in = 12
    assert _lstatus(b, d, l) == -1
    d2, keep2 = _desc(b, n_unocc=5)
    d2.unocc_end = 4
    assert _lstatus(b, d2, _learned(b, d2, keep2)) == -1
    d3, keep3 = _desc(b, n_unocc=5)
    d3.accumulate = 1
    assert _lstatus(b, d3, _learned(b, d3, keep3)) == -2
    d4, keep4 = _desc(b, n_unocc=5)
    keep4["kl"] = np.array([0], dtype=np.int32)
    d4.k_list_host = keep4["kl"].ctypes.data_as(ctypes.POINTER(ctypes.c_int))
    d4.n_k_list = 1
    assert _lstatus(b, d4, _learned(b, d4, keep4)) == -2
    # judge = 0 needs no sample
    assert _lstatus(b, d, _learned(b, d, keep, judge=0, n_sample_occ=0)) == 0
    # a valid call with too small a workspace
    l = _learned(b, d, keep)
    need = ctypes.c_size_t(0)
    assert L.gw_polarization_learned_workspace_size(ctypes.byref(d), ctypes.byref(l), ctypes.byref(need)) == 0
    assert L.gw_polarization_learned(None, ctypes.byref(d), ctypes.byref(l), ctypes.c_void_p(0x7F0000008000),
                                     need.value - 1) == -3


def test_check_flags_validation(b):
    d, keep = _desc(b)
    d.flags = 4
    out = ctypes.c_size_t(0)
    assert b.lib().gw_polarization(None, ctypes.byref(d), ctypes.c_void_p(0x7F0000008000), 1 << 40) == -1
    L = b.lib()
    fake = ctypes.c_void_p(0x7F0000003000)
    other = ctypes.c_void_p(0x7F0000004000)
    assert L.gw_screen_ex(None, 4, 1, fake, fake, other, fake, 8, fake, 1 << 30) == -1
    assert "unknown flags" in b.gw_last_error()
    assert b.STATUS[-5] == "GW_ERR_NONFINITE" and b.STATUS[-6] == "GW_ERR_NOT_HPD"
