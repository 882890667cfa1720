"""The ctypes structures of the binding have the layout of the C structures in
include/vms.h: a small C program built with the host compiler prints sizeof
and the offset of every field, and both sides must agree field by field."""
import ctypes as C
import os
import shutil
import subprocess

import pytest

from paper_1809_06350_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
STRUCTS = {
    "vms_material": L.Material,
    "vms_timeint": L.TimeInt,
    "vms_mesh": L.Mesh,
    "vms_state": L.State,
    "vms_matrix": L.Matrix,
    "vms_solver_opts": L.SolverOpts,
    "vms_solve_stats": L.SolveStats,
    "vms_newton_opts": L.NewtonOpts,
    "vms_step_stats": L.StepStats,
    "vms_amg_opts": L.AmgOpts,
}


def _c_layout(tmp_path):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "vms.h"', "int main(void) {"]
    for cname, cls in STRUCTS.items():
        lines.append(f'  printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'  printf("{cname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(line.split()[:2]): int(line.split()[2]) for line in out.splitlines()}


def test_ctypes_structures_match_the_header(tmp_path):
    c = _c_layout(tmp_path)
    for cname, cls in STRUCTS.items():
        assert C.sizeof(cls) == c[(cname, "sizeof")], cname
        for field, _ in cls._fields_:
            assert getattr(cls, field).offset == c[(cname, field)], f"{cname}.{field}"
