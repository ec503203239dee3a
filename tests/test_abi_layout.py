"""The binding's ctypes mirrors of the C-ABI structs (qhp_params, qhp_wave,
qhp_info, qhp_gmres_info in include/qhp.h) against the header itself: a C
program compiled with gcc prints each struct's size and every field's
offset, which must equal the ctypes layout field for field (a field added to
one side only would shift every later one without any error)."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = {"qhp_params": "_Params", "qhp_wave": "_Wave", "qhp_info": "_Info", "qhp_gmres_info": "_GmresInfo"}


def _c_layout(tmp_path, mirrors):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "qhp.h"', "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in cls._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {}
    for ln in out.splitlines():
        a, b, v = ln.split()
        got[(a, b)] = int(v)
    return got


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_ctypes_mirrors_match_the_header(tmp_path):
    import paper_2312_06367_amd as qhp
    mirrors = {c: getattr(qhp, p) for c, p in STRUCTS.items()}
    got = _c_layout(tmp_path, mirrors)
    for cname, cls in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
