"""Thin Python binding of libgw (ctypes).  Argument marshalling only: every
step of the computation runs in the library's HIP kernels.  PyTorch provides
device memory and the stream.

Functions carry the C names: gw_project, gw_polarization, gw_screen, ...
If the shared library is missing this module raises on import -- there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgw.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"libgw.so not found at {LIB_PATH}; build it with "
                      f"`python -m paper_1003_0316_amd.build` (no CPU fallback exists)")
_lib = ctypes.CDLL(LIB_PATH)

GW_FP64, GW_FP32, GW_SPLIT_BF16, GW_SPLIT_FP16 = 0, 1, 2, 3
PRECISIONS = {"fp64": GW_FP64, "fp32": GW_FP32, "split_bf16": GW_SPLIT_BF16, "split_fp16": GW_SPLIT_FP16}
STATUS = {0: "GW_OK", -1: "GW_ERR_INVALID_ARG", -2: "GW_ERR_UNSUPPORTED", -3: "GW_ERR_WORKSPACE",
          -4: "GW_ERR_HIP"}


class GwError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class GwPolDesc(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int), ("n_k", ctypes.c_int), ("N", ctypes.c_int), ("R", ctypes.c_int),
        ("n_occ", ctypes.c_int), ("n_unocc", ctypes.c_int),
        ("occ_begin", ctypes.c_int), ("occ_end", ctypes.c_int),
        ("unocc_begin", ctypes.c_int), ("unocc_end", ctypes.c_int),
        ("n_omega", ctypes.c_int),
        ("omega_host", ctypes.POINTER(ctypes.c_double)),
        ("kq_host", ctypes.POINTER(ctypes.c_int)),
        ("k_list_host", ctypes.POINTER(ctypes.c_int)),
        ("n_k_list", ctypes.c_int),
        ("U", ctypes.c_void_p), ("psi", ctypes.c_void_p),
        ("eps", ctypes.c_void_p), ("eps_host", ctypes.POINTER(ctypes.c_double)),
        ("P", ctypes.c_void_p),
        ("accumulate", ctypes.c_int), ("chunk_pairs", ctypes.c_int),
    ]


_sz = ctypes.c_size_t
_vp = ctypes.c_void_p
_ci = ctypes.c_int
_lib.gw_last_error.restype = ctypes.c_char_p
_lib.gw_version.restype = _ci
_lib.gw_project_workspace_size.argtypes = [_ci, _ci, _ci, _ci, _ci, ctypes.POINTER(_sz)]
_lib.gw_project.argtypes = [_vp, _ci, _ci, _ci, _ci, _ci, _vp, _vp, _vp, _vp, _vp, _sz]
_lib.gw_polarization_workspace_size.argtypes = [ctypes.POINTER(GwPolDesc), ctypes.POINTER(_sz)]
_lib.gw_polarization.argtypes = [_vp, ctypes.POINTER(GwPolDesc), _vp, _sz]
_lib.gw_screen_workspace_size.argtypes = [_ci, _ci, ctypes.POINTER(_sz)]
_lib.gw_screen.argtypes = [_vp, _ci, _ci, _vp, _vp, _vp, _vp, _vp, _sz]

_lib.gw_profile_enable.argtypes = [_ci]
_lib.gw_profile_reset.argtypes = []
_lib.gw_profile_query.argtypes = [ctypes.c_char_p, ctypes.POINTER(_ci), ctypes.POINTER(ctypes.c_double)]

EXPORTED = ("gw_last_error", "gw_version", "gw_project_workspace_size", "gw_project",
            "gw_polarization_workspace_size", "gw_polarization", "gw_screen_workspace_size", "gw_screen",
            "gw_profile_enable", "gw_profile_reset", "gw_profile_query")


def lib():
    return _lib


def _check(status: int) -> None:
    if status != 0:
        raise GwError(status, _lib.gw_last_error().decode())


def gw_last_error() -> str:
    return _lib.gw_last_error().decode()


def gw_version() -> int:
    return _lib.gw_version()


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _prec(p) -> int:
    return PRECISIONS[p] if isinstance(p, str) else int(p)


def _cdtype(prec: int):
    return torch.complex128 if prec == GW_FP64 else torch.complex64


def _dev_tensor(t: torch.Tensor, name: str, dtype=None) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


_ws_cache: dict = {}


def workspace(nbytes: int, device, tag: str = "default") -> torch.Tensor:
    """A cached device byte buffer of at least nbytes (per device, stream tag)."""
    key = (str(device), tag)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        _ws_cache.pop(key, None)
        buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def gw_project_workspace_size(precision, N, R, n_occ, n_unocc) -> int:
    out = _sz(0)
    _check(_lib.gw_project_workspace_size(_prec(precision), N, R, n_occ, n_unocc, ctypes.byref(out)))
    return out.value


def gw_project(U: torch.Tensor, psi_occ: torch.Tensor, psi_unocc: torch.Tensor, precision="fp64",
               M: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """M[I, n*n_unocc + n'] = sum_r U[I,r] conj(psi_occ[n,r]) psi_unocc[n',r]."""
    prec = _prec(precision)
    dt = _cdtype(prec)
    _dev_tensor(U, "U", dt)
    _dev_tensor(psi_occ, "psi_occ", dt)
    _dev_tensor(psi_unocc, "psi_unocc", dt)
    N, R = U.shape
    n_occ, n_unocc = psi_occ.shape[0], psi_unocc.shape[0]
    if psi_occ.shape[1] != R or psi_unocc.shape[1] != R:
        raise ValueError("grid sizes differ")
    if M is None:
        M = torch.empty((N, n_occ * n_unocc), dtype=dt, device=U.device)
    _dev_tensor(M, "M", dt)
    if tuple(M.shape) != (N, n_occ * n_unocc):
        raise ValueError("M has the wrong shape")
    nbytes = gw_project_workspace_size(prec, N, R, n_occ, n_unocc)
    ws = workspace(nbytes, U.device, "project") if nbytes else None
    _check(_lib.gw_project(_stream(stream), prec, N, R, n_occ, n_unocc, U.data_ptr(), psi_occ.data_ptr(),
                           psi_unocc.data_ptr(), M.data_ptr(), ws.data_ptr() if ws is not None else None,
                           ws.numel() if ws is not None else 0))
    return M


class PolarizationCall:
    """Marshalled arguments of one gw_polarization call (keeps host arrays alive)."""

    def __init__(self, U, psi, eps_host, omega, n_occ, *, precision="fp64", eps_dev=None, P=None,
                 k_list=None, kq=None, occ_range=None, unocc_range=None, accumulate=False, chunk_pairs=0):
        prec = _prec(precision)
        dt = _cdtype(prec)
        _dev_tensor(U, "U", dt)
        _dev_tensor(psi, "psi", dt)
        N, R = U.shape
        n_k, nb = psi.shape[0], psi.shape[1]
        if psi.shape[2] != R:
            raise ValueError("psi grid size differs from U")
        n_unocc = nb - n_occ
        self.eps_host = np.ascontiguousarray(eps_host, dtype=np.float64)
        if self.eps_host.shape != (n_k, nb):
            raise ValueError(f"eps must be [{n_k}][{nb}]")
        self.eps_dev = eps_dev if eps_dev is not None else torch.from_numpy(self.eps_host).to(U.device)
        _dev_tensor(self.eps_dev, "eps_dev", torch.float64)
        self.omega = np.ascontiguousarray(omega, dtype=np.float64)
        n_om = self.omega.shape[0]
        if P is None:
            P = torch.empty((n_om, N, N), dtype=torch.complex128, device=U.device)
        _dev_tensor(P, "P", torch.complex128)
        if tuple(P.shape) != (n_om, N, N):
            raise ValueError("P has the wrong shape")
        self.P = P
        self.kq = None if kq is None else np.ascontiguousarray(kq, dtype=np.int32)
        self.k_list = None if k_list is None else np.ascontiguousarray(k_list, dtype=np.int32)
        o0, o1 = (0, n_occ) if occ_range is None else occ_range
        u0, u1 = (0, n_unocc) if unocc_range is None else unocc_range
        self.tensors = (U, psi)
        d = GwPolDesc()
        d.precision, d.n_k, d.N, d.R = prec, n_k, N, R
        d.n_occ, d.n_unocc = n_occ, n_unocc
        d.occ_begin, d.occ_end, d.unocc_begin, d.unocc_end = o0, o1, u0, u1
        d.n_omega = n_om
        d.omega_host = self.omega.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.kq_host = self.kq.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if self.kq is not None else None
        if self.k_list is not None:
            d.k_list_host = self.k_list.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
            d.n_k_list = int(self.k_list.shape[0])
        else:
            d.k_list_host = None
            d.n_k_list = 0
        d.U, d.psi = U.data_ptr(), psi.data_ptr()
        d.eps = self.eps_dev.data_ptr()
        d.eps_host = self.eps_host.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.P = P.data_ptr()
        d.accumulate = 1 if accumulate else 0
        d.chunk_pairs = int(chunk_pairs)
        self.desc = d

    def workspace_size(self) -> int:
        out = _sz(0)
        _check(_lib.gw_polarization_workspace_size(ctypes.byref(self.desc), ctypes.byref(out)))
        return out.value

    def run(self, ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        nbytes = self.workspace_size()
        if ws is None:
            ws = workspace(nbytes, self.P.device, "polarization")
        _check(_lib.gw_polarization(_stream(stream), ctypes.byref(self.desc), ws.data_ptr(), ws.numel()))
        return self.P


def gw_polarization(U, psi, eps_host, omega, n_occ, **kw) -> torch.Tensor:
    """P[j] = sum_k sum_{n occ} sum_{n' unocc} w M M^H (see gw.h).  Returns P
    (complex128 [n_omega][N][N]); the work is enqueued on the current stream."""
    ws = kw.pop("ws", None)
    stream = kw.pop("stream", None)
    return PolarizationCall(U, psi, eps_host, omega, n_occ, **kw).run(ws, stream)


def gw_polarization_workspace_size(U, psi, eps_host, omega, n_occ, **kw) -> int:
    return PolarizationCall(U, psi, eps_host, omega, n_occ, **kw).workspace_size()


def gw_screen_workspace_size(N: int, n_omega: int) -> int:
    out = _sz(0)
    _check(_lib.gw_screen_workspace_size(N, n_omega, ctypes.byref(out)))
    return out.value


def gw_screen(P: torch.Tensor, v: torch.Tensor, W: Optional[torch.Tensor] = None, info=None, stream=None):
    """W[j] = (1 - diag(v) P[j])^-1 diag(v) in FP64.  Returns (W, info) with
    info an int32 device tensor (0 = ok, c+1 = pivot failure at column c)."""
    _dev_tensor(P, "P", torch.complex128)
    _dev_tensor(v, "v", torch.float64)
    n_om, N = P.shape[0], P.shape[1]
    if W is None:
        W = torch.empty_like(P)
    _dev_tensor(W, "W", torch.complex128)
    if info is None:
        info = torch.empty(n_om, dtype=torch.int32, device=P.device)
    nbytes = gw_screen_workspace_size(N, n_om)
    ws = workspace(nbytes, P.device, "screen")
    _check(_lib.gw_screen(_stream(stream), N, n_om, P.data_ptr(), v.data_ptr(), W.data_ptr(), info.data_ptr(),
                          ws.data_ptr(), ws.numel()))
    return W, info


def gw_profile_enable(on: bool = True) -> None:
    _check(_lib.gw_profile_enable(1 if on else 0))


def gw_profile_reset() -> None:
    _check(_lib.gw_profile_reset())


def gw_profile_query(kernel: str):
    """(launches, total_ms) of the recorded launches of `kernel` (synchronises)."""
    n = ctypes.c_int(0)
    ms = ctypes.c_double(0.0)
    _check(_lib.gw_profile_query(kernel.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value
