"""MI355X (gfx950) Wilson-fermion HMC hot path: HIP kernels behind a C ABI.

The computation lives in ``liblgt.so`` (sources in ``csrc/``, ABI in
``include/lgt.h``); this package is its Python binding.  Importing it loads
the library and fails loudly if it has not been built
(``python paper_2602_20516_amd/build.py``).
"""
from . import _lib

_lib.load()

from .api import (Batch, Lattice, LGTError, LGTNonFinite, LGTNotConverged, Params,  # noqa: E402
                  lgt_action, lgt_bilinear_force, lgt_cg_solve, lgt_cg_solve_batch, lgt_create, lgt_dslash,
                  lgt_dslash_noalloc,
                  lgt_fermion_force, lgt_gauge_force, lgt_hop_benchmark, lgt_hop_benchmark_mrhs, lgt_kinetic,
                  lgt_link_update,
                  lgt_md_step, lgt_md_step_eo, lgt_md_step_smeared, lgt_md_step_sw, lgt_schur_dslash,
                  lgt_fermion_force_eo, lgt_smeared_force, lgt_stout_backprop, lgt_stout_smear,
                  lgt_cg_solve_multishift, lgt_rational_force_eo, stout_schedule)
from .autograd import LatticeAction, lattice_action  # noqa: E402

__all__ = [
    "Batch", "Lattice", "Params", "LGTError", "LGTNotConverged", "LGTNonFinite", "lgt_cg_solve_batch",
    "lgt_create", "lgt_dslash", "lgt_dslash_noalloc", "lgt_cg_solve", "lgt_action", "lgt_fermion_force",
    "lgt_bilinear_force", "lgt_gauge_force", "lgt_link_update", "lgt_kinetic", "lgt_md_step",
    "lgt_hop_benchmark", "lgt_hop_benchmark_mrhs", "lgt_stout_smear", "lgt_stout_backprop", "lgt_smeared_force", "lgt_md_step_smeared", "lgt_md_step_sw",
    "lgt_schur_dslash", "lgt_fermion_force_eo", "lgt_md_step_eo", "lgt_cg_solve_multishift", "lgt_rational_force_eo", "stout_schedule",
    "LatticeAction", "lattice_action",
]
