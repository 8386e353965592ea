"""The ctypes descriptors of the binding have the size and field offsets of
the C structs in include/gw.h (compiled by the host C compiler)."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1003_0316_amd import binding as b

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PAIRS = [("gw_pol_desc", b.GwPolDesc), ("gw_sigma_desc", b.GwSigmaDesc), ("gw_mlp", b.GwMlp),
         ("gw_surr_desc", b.GwSurrDesc), ("gw_learned_desc", b.GwLearnedDesc)]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs a host C compiler")
def test_descriptor_layouts_match_the_header(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gw.h"', "int main(void) {"]
    for cname, cls in PAIRS:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    r = subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, cls in PAIRS:
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
