"""libgw from plain C (tests/c_abi/pol_screen_fp64.c): the program compiles and
links against include/gw.h and the library with the host C compiler (CPU);
on the GPU it computes P and W for the config-1 workload through the C ABI,
compared with the oracle at the FP64 bar."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import gwsynth
from oracle import polarization as orc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1003_0316_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def _compile(tmp_path):
    exe = tmp_path / "pol_screen_fp64"
    cmd = ["gcc", "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
           f"-I{os.path.join(ROOT, 'include')}", os.path.join(ROOT, "tests", "c_abi", "pol_screen_fp64.c"),
           f"-L{PKG}", "-lgw", f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{ROCM}/lib",
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


needs_toolchain = pytest.mark.skipif(
    shutil.which("gcc") is None or not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime_api.h"))
    or not os.path.exists(os.path.join(PKG, "libgw.so")), reason="needs gcc, the HIP headers and libgw.so")


@needs_toolchain
def test_c_program_compiles_and_links(tmp_path):
    exe = _compile(tmp_path)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 2 and "usage" in r.stderr


@needs_toolchain
@pytest.mark.gpu
def test_c_program_matches_oracle(tmp_path):
    exe = _compile(tmp_path)
    inp = gwsynth.generate("c1")
    n_k, nb, R = inp.psi.shape
    N, n_occ = inp.U.shape[0], 4
    assert np.array_equal(inp.kq, (np.arange(n_k) + 1) % n_k)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as f:
        np.array([n_k, N, R, n_occ, nb - n_occ, inp.omega.size], dtype="<i4").tofile(f)
        for a, dt in ((inp.omega, "<f8"), (inp.eps, "<f8"), (inp.v, "<f8"), (inp.U, "<c16"), (inp.psi, "<c16")):
            np.ascontiguousarray(a, dtype=dt).tofile(f)
    r = subprocess.run([str(exe), str(fin), str(fout)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    out = np.fromfile(fout, dtype="<c16")
    n_om = inp.omega.size
    P = out[:n_om * N * N].reshape(n_om, N, N)
    W = out[n_om * N * N:].reshape(n_om, N, N)
    Pref = orc.polarization(inp.U, inp.psi, inp.eps, inp.omega, n_occ, kq=inp.kq)
    Wref = orc.screened_interaction(Pref, inp.v)
    ep, ew = orc.rel_fro(P, Pref).max(), orc.rel_fro(W, Wref).max()
    print(f"C program: P {ep:.2e}, W {ew:.2e}")
    assert ep < 1e-10 and ew < 1e-10
