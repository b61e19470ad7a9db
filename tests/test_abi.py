"""The C-ABI library loads and exports every function include/iedg.h
declares; the ctypes structures match the header's layout (compiled with
the host C compiler).  No compute call: these run without a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "iedg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"^[A-Za-z_][\w\s\*]*?\b(iedg_\w+)\s*\(", src, flags=re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_1605_01020_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1605_01020_amd.build import build_all
        build_all()
    return _lib


def test_header_declares_the_five_hot_path_calls():
    names = _declared()
    for fn in ("iedg_condense", "iedg_assemble", "iedg_factor_ilu0", "iedg_gmres_solve",
               "iedg_backsolve_local"):
        assert fn in names


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.strip()}
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    # the binding covers exactly the declared calls
    assert sorted(lib.SIGNATURES) == names


def test_library_loads_and_binds(lib):
    L = lib.load()
    for name in lib.SIGNATURES:
        assert getattr(L, name) is not None
    assert L.iedg_status_string(-2).decode()


def test_struct_layouts_match_header(lib, tmp_path):
    prog = tmp_path / "layout.c"
    prog.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "iedg.h"
int main(void) {
  printf("mesh_info %zu\n", sizeof(iedg_mesh_info));
  printf("gmres_opts %zu %zu %zu %zu %zu\n", sizeof(iedg_gmres_opts), offsetof(iedg_gmres_opts, rtol),
         offsetof(iedg_gmres_opts, inner_factor), offsetof(iedg_gmres_opts, precond), offsetof(iedg_gmres_opts, max_iters));
  printf("gmres_info %zu %zu\n", sizeof(iedg_gmres_info), offsetof(iedg_gmres_info, rel_resid));
  printf("segment %zu %zu %zu\n", sizeof(iedg_condense_segment), offsetof(iedg_condense_segment, A),
         offsetof(iedg_condense_segment, r));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-D__HIP_PLATFORM_AMD__", f"-I{ROOT}/include", "-I/opt/rocm/include",
                    str(prog), "-o", str(exe)], check=True)
    got = {}
    for ln in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        k, *v = ln.split()
        got[k] = [int(x) for x in v]
    assert got["mesh_info"] == [ctypes.sizeof(lib.MeshInfo)]
    O = lib.GmresOpts
    assert got["gmres_opts"] == [ctypes.sizeof(O), O.rtol.offset, O.inner_factor.offset, O.precond.offset,
                                 O.max_iters.offset]
    I = lib.GmresInfo
    assert got["gmres_info"] == [ctypes.sizeof(I), I.rel_resid.offset]
    S = lib.CondenseSegment
    assert got["segment"] == [ctypes.sizeof(S), S.A.offset, S.r.offset]
