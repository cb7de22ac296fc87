"""The ctypes mirrors of the C-ABI structs (paper_1909_00149_amd/_lib.py,
net.py) against the headers themselves: a small C program built with the
host compiler prints sizeof and offsetof of every field, which must equal
ctypes' layout.  No GPU is involved."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_1909_00149_amd import _lib
from paper_1909_00149_amd.net import NetConfig

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = [("uot_params", _lib.Params), ("uot_state", _lib.State), ("uot_report", _lib.Report),
           ("uot_dr_report", _lib.DrReport), ("uotdf_params", _lib.DfParams), ("uotdf_report", _lib.DfReport),
           ("rpca_params", _lib.RpParams), ("rpca_report", _lib.RpReport), ("uotnet_config", NetConfig)]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    d = tmp_path_factory.mktemp("abi")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "uot.h"', '#include "uot_admm.h"',
             '#include "uotnet.h"', 'int main(void) {']
    for cname, cls in STRUCTS:
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True,
                   capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for line in out.splitlines():
        s, f, v = line.split()
        table[(s, f)] = int(v)
    return table


@pytest.mark.parametrize("cname,cls", STRUCTS, ids=[c for c, _ in STRUCTS])
def test_struct_layout_matches_header(c_layout, cname, cls):
    assert c_layout[(cname, "sizeof")] == ctypes.sizeof(cls), cname
    for f, _ in cls._fields_:
        assert c_layout[(cname, f)] == getattr(cls, f).offset, (cname, f)
