"""The Python binding's ctypes structures match the C structures of
include/parac.h field by field: a C program built with the system compiler
prints each structure's size and every field's offset, and the ctypes
mirrors must give the same numbers (a field added on one side only, or in a
different place, shifts everything after it)."""
import os
import shutil
import subprocess

import pytest

from paper_2505_02977_amd import parac

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["parac_csr", "parac_factor_opts", "parac_factor_stats", "parac_pcg_opts",
           "parac_pcg_stats", "parac_block_shape", "parac_request", "parac_result",
           "parac_serve_opts", "parac_host_factor"]


def c_layout(tmp_path):
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "parac.h"', "int main(void) {"]
    for name in STRUCTS:
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (name, name))
        for field, _ in getattr(parac, name)._fields_:
            lines.append('  printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, field, name, field))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return dict(line.rsplit(" ", 1) for line in out.strip().splitlines())


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_ctypes_structures_match_the_header(tmp_path):
    got = c_layout(tmp_path)
    bad = []
    for name in STRUCTS:
        cls = getattr(parac, name)
        if int(got["%s size" % name]) != parac.C.sizeof(cls):
            bad.append((name, "size", got["%s size" % name], parac.C.sizeof(cls)))
        for field, _ in cls._fields_:
            off = getattr(cls, field).offset
            if int(got["%s.%s" % (name, field)]) != off:
                bad.append((name, field, got["%s.%s" % (name, field)], off))
    assert not bad, bad
