"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/lgt.h declares, its structs have the ctypes layout, and
argument validation that happens before any device call."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lgt.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"LGT_API\s+[\w\s\*]+?\b(lgt_\w+)\s*\(", text)))


def test_header_declares_the_abi():
    names = declared_symbols()
    for n in ["lgt_create", "lgt_destroy", "lgt_last_error", "lgt_dslash", "lgt_cg_solve", "lgt_action",
              "lgt_fermion_force", "lgt_gauge_force", "lgt_md_step"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2602_20516_amd import _lib
    lib = _lib.load()
    for n in declared_symbols():
        assert hasattr(lib, n), n
        assert n in _lib.PROTOTYPES, n


def test_struct_layout_matches_c(tmp_path):
    from paper_2602_20516_amd import _lib
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "lgt.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n\", sizeof(lgt_geom),"
        " sizeof(lgt_solver_params), offsetof(lgt_solver_params, tol),"
        " offsetof(lgt_solver_params, reliable_delta), sizeof(lgt_solver_stats),"
        " offsetof(lgt_solver_stats, true_rel_residual), offsetof(lgt_solver_stats, ms),"
        " offsetof(lgt_solver_params, first_pass_factor), offsetof(lgt_solver_stats, corrections));return 0;}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    assert out == [ctypes.sizeof(_lib.Geom), ctypes.sizeof(_lib.SolverParams), _lib.SolverParams.tol.offset,
                   _lib.SolverParams.reliable_delta.offset, ctypes.sizeof(_lib.SolverStats),
                   _lib.SolverStats.true_rel_residual.offset, _lib.SolverStats.ms.offset,
                   _lib.SolverParams.first_pass_factor.offset, _lib.SolverStats.corrections.offset]


@pytest.mark.parametrize("dims,bc", [((4, 4, 3, 4), -1), ((0, 4, 4, 4), -1), ((4, 4, 4, 4), 0),
                                     ((4, 4, 4, 1), 1),
                                     # FP64 half-lattice spinor of 4 GiB or more (32-bit field offsets)
                                     ((64, 64, 64, 172), -1)])
def test_create_rejects_bad_geometry_before_touching_the_device(dims, bc):
    from paper_2602_20516_amd import _lib
    lib = _lib.load()
    g = _lib.Geom((ctypes.c_int32 * 4)(*dims), bc)
    ctx = ctypes.c_void_p()
    assert lib.lgt_create(ctypes.byref(g), None, ctypes.byref(ctx)) == _lib.LGT_ERR_INVALID_ARGUMENT
    assert ctx.value is None
    assert lib.lgt_last_error(None)


def test_null_context_is_rejected():
    from paper_2602_20516_amd import _lib
    lib = _lib.load()
    assert lib.lgt_dslash(None, None, None, None, 0.1, 0) == _lib.LGT_ERR_INVALID_ARGUMENT
    assert lib.lgt_md_step(None, None, None, None, 1.0, 0.1, 0.1, 1, None, None, None) == \
        _lib.LGT_ERR_INVALID_ARGUMENT
    assert lib.lgt_volume(None) == 0
    assert lib.lgt_destroy(None) == _lib.LGT_OK
