"""The ctypes structures of the binding have the size and field offsets of
the C structures in include/rpr.h, as a C compiler lays them out (no GPU
needed: the header is compiled by the host C compiler)."""
import ctypes as C
import os
import re
import shutil
import subprocess

import pytest

import paper_2411_06225_amd as rpr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = ["rpr_rhs", "rpr_propagator", "rpr_randnet", "rpr_options", "rpr_info"]


def c_fields(src, name):
    """Field names of `typedef struct { ... } name;` in declaration order."""
    body = re.search(r"typedef struct \{([^{}]*)\}\s*" + name + r"\s*;", src, flags=re.S).group(1)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        _, rest = decl.split(None, 1)  # type, then one or more declarators
        for d in rest.split(","):
            names.append(re.match(r"\s*([A-Za-z_]\w*)", d).group(1))
    return names


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs a host C compiler")
def test_binding_structs_match_the_header(tmp_path):
    src = open(os.path.join(ROOT, "include", "rpr.h")).read()
    src_nc = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    prog = ['#include <stdio.h>', '#include <stddef.h>', '#include "rpr.h"', "int main(void) {"]
    fields = {}
    for s in STRUCTS:
        fields[s] = c_fields(src_nc, s)
        prog.append(f'printf("{s} %zu", sizeof({s}));')
        for f in fields[s]:
            prog.append(f'printf(" %zu", offsetof({s}, {f}));')
        prog.append('printf("\\n");')
    prog.append("return 0; }")
    c_file, exe = tmp_path / "layout.c", tmp_path / "layout"
    c_file.write_text("\n".join(prog))
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(c_file), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    for line in out.strip().splitlines():
        name, size, *offs = line.split()
        cls = getattr(rpr, name)
        py_offs = [getattr(cls, f).offset for f, *_ in cls._fields_]
        assert C.sizeof(cls) == int(size), name
        assert py_offs == [int(o) for o in offs], (name, fields[name])
