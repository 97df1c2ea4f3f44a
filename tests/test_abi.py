"""The C-ABI library loads on the CPU, exports every function declared in include/pb.h,
and rejects bad calls before touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2502_09323_amd import binding as B
from paper_2502_09323_amd import build as BB

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        BB.build()
    return B.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pb.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(pb_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("pb_build_coeffs", "pb_solve", "pb_energy", "pb_ctx_create", "pb_problem_free"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n
    for n in B.EXPORTED:
        assert n in declared_functions(), n


def test_struct_sizes_match_binding(tmp_path):
    """The ctypes structures have the size and field offsets of the C header (compiled here)."""
    import subprocess
    structs = {"pb_params": B.PbParams, "pb_solve_stats": B.PbSolveStats, "pb_energy_out": B.PbEnergyOut,
               "pb_refine_stats": B.PbRefineStats}
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "pb.h"', "int main(void) {"]
    for cname, py in structs.items():
        src.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            src.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    src.append("return 0; }")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(c), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines():
        cname, field, v = line.split()
        got[(cname, field)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "sizeof")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_null_arguments_are_rejected_without_a_gpu(lib):
    out = C.c_void_p()
    rc = lib.pb_ctx_create(0, None, B.ALLOC_FN(0), B.FREE_FN(0), None, 0, C.byref(out))
    assert rc == B.PB_EINVAL
    assert b"allocator" in lib.pb_last_error()
    rc = lib.pb_build_coeffs(None, None, 0, None, None, None, C.byref(out))
    assert rc == B.PB_EINVAL
    st = B.PbSolveStats()
    assert lib.pb_solve(None, C.byref(st)) == B.PB_EINVAL
    assert lib.pb_num_cut(None) == B.PB_EINVAL
    e = C.c_double(1.0)
    assert lib.pb_grid_energy(None, C.byref(e)) == B.PB_EINVAL
    assert lib.pb_grid_energy(None, None) == B.PB_EINVAL
    assert b"NULL" in lib.pb_last_error()
    assert lib.pb_cancel(None, 0) == B.PB_EINVAL
    assert lib.pb_server_set_timeout(None, 1.0) == B.PB_EINVAL
    assert lib.pb_server_memory(None, None, None, None) == B.PB_EINVAL
