"""Package behaviour without the built library (fresh checkout): the build
module imports, and the binding fails loudly (no CPU fallback)."""
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _fresh_copy(tmp_path):
    dst = tmp_path / "paper_1003_0316_amd"
    shutil.copytree(os.path.join(ROOT, "paper_1003_0316_amd"), dst,
                    ignore=shutil.ignore_patterns("*.so", "_build", "__pycache__", "*.npz"))
    return str(tmp_path)


def _run(path, code):
    return subprocess.run([sys.executable, "-c", f"import sys; sys.path.insert(0, {path!r}); {code}"],
                          capture_output=True, text=True, timeout=120, cwd=path)


def test_build_module_imports_without_the_library(tmp_path):
    p = _fresh_copy(tmp_path)
    r = _run(p, "from paper_1003_0316_amd import build as b; assert b.ARCH == 'gfx950'; print(b.LIB)")
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().startswith(p)


def test_binding_fails_loudly_without_the_library(tmp_path):
    p = _fresh_copy(tmp_path)
    r = _run(p, "import paper_1003_0316_amd.binding")
    assert r.returncode != 0
    assert "libgw.so not found" in r.stderr
    r = _run(p, "from paper_1003_0316_amd import gw_polarization")
    assert r.returncode != 0 and "libgw.so not found" in r.stderr
