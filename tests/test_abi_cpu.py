"""Host-side checks of the C ABI: the library loads, exports every symbol the
header declares, and the ctypes structures match the C layout (no GPU calls)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "rsr.h")
SO = os.path.join(ROOT, "paper_2306_15049_amd", "librsr.so")


def declared_functions():
    txt = open(HDR).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rsr_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(SO):
        from paper_2306_15049_amd import build
        build.build()
    return ctypes.CDLL(SO)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("rsr_set_operators", "rsr_update_weights", "rsr_set_recycle_space", "rsr_solve_shift_set",
                 "rsr_adjoint", "rsr_apply", "rsr_autotune", "rsr_weights_from_image"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_lists_every_export():
    from paper_2306_15049_amd import rsr
    assert sorted(rsr.EXPORTS) == declared_functions()


def test_version_string(lib):
    lib.rsr_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.rsr_version()


def test_null_context_is_rejected(lib):
    lib.rsr_apply.restype = ctypes.c_int
    assert lib.rsr_apply(None, 0, 0, ctypes.c_double(0.0), None, None, 1, ctypes.c_long(0), None) == -1
    lib.rsr_last_error.restype = ctypes.c_char_p
    assert lib.rsr_last_error(None) == b"null context"


def test_ctypes_struct_layout_matches_c():
    from paper_2306_15049_amd import rsr
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "rsr.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(rsr_instance), sizeof(rsr_solve_desc),
         offsetof(rsr_solve_desc, tol), offsetof(rsr_solve_desc, gamma_JL), offsetof(rsr_solve_desc, ld_x),
         offsetof(rsr_solve_desc, seed_lanczos), offsetof(rsr_solve_desc, seed_n_ritz),
         offsetof(rsr_solve_desc, seed_second), offsetof(rsr_solve_desc, solver),
         sizeof(rsr_shift_stats), offsetof(rsr_shift_stats, relres_init), offsetof(rsr_shift_stats, relres_true),
         sizeof(rsr_ct_instance), offsetof(rsr_ct_instance, spacing), offsetof(rsr_ct_instance, angles_host));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, c])
        vals = list(map(int, subprocess.check_output([exe]).split()))
    want = [ctypes.sizeof(rsr.Instance), ctypes.sizeof(rsr.SolveDesc), rsr.SolveDesc.tol.offset,
            rsr.SolveDesc.gamma_JL.offset, rsr.SolveDesc.ld_x.offset, rsr.SolveDesc.seed_lanczos.offset,
            rsr.SolveDesc.seed_n_ritz.offset, rsr.SolveDesc.seed_second.offset,
            rsr.SolveDesc.solver.offset, ctypes.sizeof(rsr.ShiftStats),
            rsr.ShiftStats.relres_init.offset, rsr.ShiftStats.relres_true.offset, ctypes.sizeof(rsr.CtInstance),
            rsr.CtInstance.spacing.offset, rsr.CtInstance.angles_host.offset]
    assert vals == want


def test_binding_argument_counts_match_the_header():
    # every prototype in the header has as many parameters as the binding passes
    from paper_2306_15049_amd import rsr
    txt = re.sub(r"/\*.*?\*/", "", open(HDR).read(), flags=re.S)
    protos = dict(re.findall(r"\b(rsr_[a-z_]+)\s*\(([^;{]*?)\)\s*;", txt))
    L = rsr.load()
    for name in rsr.EXPORTS:
        params = protos[name].strip()
        n = 0 if params in ("", "void") else params.count(",") + 1
        assert len(getattr(L, name).argtypes) == n, (name, n)
