"""The binding's ctypes structures against the C header's own layout.

A small C program built with gcc from include/pic.h prints the size of every
struct the binding mirrors and the offset of each of its fields; the ctypes
classes must agree byte for byte (the library writes whole structs into the
binding's buffers).
"""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_2605_07083_amd import pic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = [("pic_config", pic.PicConfig), ("pic_tally", pic.PicTally), ("pic_diag", pic.PicDiag),
           ("pic_steady", pic.PicSteady), ("pic_derived", pic.PicDerived)]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not found")
    d = tmp_path_factory.mktemp("abi")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "pic.h"', "int main(void) {"]
    for cname, cls in STRUCTS:
        lines.append('    printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in cls._fields_:
            lines.append('    printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["    return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.check_call([gcc, "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)])
    out = {}
    for ln in subprocess.check_output([str(exe)], text=True).splitlines():
        sname, field, value = ln.split()
        out[(sname, field)] = int(value)
    return out


@pytest.mark.parametrize("cname,cls", STRUCTS)
def test_struct_matches_header(c_layout, cname, cls):
    assert C.sizeof(cls) == c_layout[(cname, "size")], cname
    for fname, _ in cls._fields_:
        assert getattr(cls, fname).offset == c_layout[(cname, fname)], (cname, fname)
