"""The ctypes structures of the binding match the C header's layout
(offsets and sizes from a C program compiled against include/paradiag.h)."""
import ctypes
import os
import shutil
import subprocess

import pytest

from paper_2304_12597_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _c_layout(tmp_path, struct, fields):
    src = tmp_path / "layout.c"
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "paradiag.h"',
             "int main(void) {", '  printf("%%zu\\n", sizeof(%s));' % struct]
    lines += ['  printf("%%zu\\n", offsetof(%s, %s));' % (struct, f) for f in fields]
    lines += ["  return 0;", "}"]
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o",
                    str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(v) for v in out[1:]]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
@pytest.mark.parametrize("cls,name", [(binding.pd_options, "pd_options"),
                                      (binding.pd_info, "pd_info")])
def test_struct_layout_matches_header(tmp_path, cls, name):
    fields = [f for f, _ in cls._fields_]
    size, offsets = _c_layout(tmp_path, name, fields)
    assert ctypes.sizeof(cls) == size
    assert [getattr(cls, f).offset for f in fields] == offsets
