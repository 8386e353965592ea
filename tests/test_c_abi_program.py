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


def _compile_learned(tmp_path):
    exe = tmp_path / "learned_pol"
    cmd = ["gcc", "-std=c11", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
           f"-I{os.path.join(ROOT, 'include')}", os.path.join(ROOT, "tests", "c_abi", "learned_pol.c"),
           f"-L{PKG}", "-lgw", f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{ROCM}/lib",
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


@needs_toolchain
def test_c_learned_program_compiles_and_links(tmp_path):
    exe = _compile_learned(tmp_path)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 2 and "usage" in r.stderr


@needs_toolchain
@pytest.mark.gpu
@pytest.mark.parametrize("precision,tol", [("split_bf16", 1e30), ("split_bf16", 0.0), ("fp64", 1e30)])
def test_c_learned_program_matches_the_binding(tmp_path, precision, tol):
    """The learned path from C equals the binding's call on the same inputs bit
    for bit (P, judge errors, fallback decision), with and without the forced
    fallback."""
    import torch
    from paper_1003_0316_amd import binding as gw
    exe = _compile_learned(tmp_path)
    shp = gwsynth.make_shape(n_k=3, n_b=90, R=600, N=140, n_occ=4, n_unocc=70)
    inp = gwsynth.generate(shp, seed=37, omega=gwsynth.omega_mesh("m16"))
    dims = (32, 256, 32)
    p = gwsynth.mlp_init(*dims, seed=9)
    p["b3"] = p["b3"] - 1.0
    master = gw.Mlp.flat_from_dict(p, *dims).astype(np.float32)
    prec = gw.PRECISIONS[precision]
    cdt = "<c16" if precision == "fp64" else "<c8"
    cut, n_s = 21, 2
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as f:
        np.array([prec, 3, 140, 600, 4, 70, inp.omega.size, cut, n_s, *dims], dtype="<i4").tofile(f)
        np.array([tol], dtype="<f8").tofile(f)
        for a, dt in ((inp.omega, "<f8"), (inp.eps, "<f8"), (inp.U, cdt), (inp.psi, cdt), (master, "<f4")):
            np.ascontiguousarray(a, dtype=dt).tofile(f)
    print(f"C learned program: {precision}, judge_tol {tol}", flush=True)
    r = subprocess.run([str(exe), str(fin), str(fout)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    raw = open(fout, "rb").read()
    n_om = inp.omega.size
    nP = n_om * 140 * 140 * 16
    Pc = np.frombuffer(raw[:nP], dtype="<c16").reshape(n_om, 140, 140)
    errc = np.frombuffer(raw[nP:nP + 8 * n_om], dtype="<f8")
    fbc = int(np.frombuffer(raw[nP + 8 * n_om:], dtype="<i4")[0])
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    U = torch.from_numpy(inp.U).cuda().to(dt)
    psi = torch.from_numpy(inp.psi).cuda().to(dt)
    mlp = gw.Mlp(*dims, torch.device("cuda"), master=master, train=False)
    pol = gw.PolarizationCall(U, psi, inp.eps, inp.omega, 4, precision=precision, kq=inp.kq)
    P, rep = gw.LearnedCall(pol, mlp, cut, n_sample_occ=n_s, judge_tol=tol).run()
    torch.cuda.synchronize()
    assert fbc == int(rep["used_fallback"]) == (1 if tol == 0.0 else 0)
    assert np.array_equal(errc, np.asarray(rep["judge_err"]))
    assert np.array_equal(Pc, P.cpu().numpy())
