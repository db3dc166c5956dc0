"""ctypes declarations of the C ABI in include/lgt.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblgt.so")

LGT_OK = 0
LGT_ERR_INVALID_ARGUMENT = 1
LGT_ERR_NOT_CONVERGED = 2
LGT_ERR_NONFINITE = 3
LGT_ERR_OUT_OF_MEMORY = 4
LGT_ERR_DEVICE = 5
LGT_ERR_UNSUPPORTED = 6

STATUS_NAMES = {
    0: "LGT_OK", 1: "LGT_ERR_INVALID_ARGUMENT", 2: "LGT_ERR_NOT_CONVERGED", 3: "LGT_ERR_NONFINITE",
    4: "LGT_ERR_OUT_OF_MEMORY", 5: "LGT_ERR_DEVICE", 6: "LGT_ERR_UNSUPPORTED",
}

LGT_FP64 = 0
LGT_MIXED_FP32 = 1
LGT_MIXED_BF16 = 2

LGT_OUT_FORCE = 0
LGT_OUT_GRAD = 1
LGT_OUT_MOMENTUM = 2


class Geom(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("fermion_t_bc", ctypes.c_int32)]


class SolverParams(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("even_odd", ctypes.c_int32), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int32), ("reliable_delta", ctypes.c_double),
                ("first_pass_factor", ctypes.c_double)]


class BatchItem(ctypes.Structure):
    _fields_ = [("ctx", ctypes.c_void_p), ("U", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("X", ctypes.c_void_p),
                ("Y_or_null", ctypes.c_void_p), ("kappa", ctypes.c_double)]


class SolverStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("reliable_updates", ctypes.c_int32),
                ("true_rel_residual", ctypes.c_double), ("ms", ctypes.c_double),
                ("corrections", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"iters": self.iters, "reliable_updates": self.reliable_updates,
                "true_rel_residual": self.true_rel_residual, "ms": self.ms, "corrections": self.corrections}


_vp = ctypes.c_void_p
_d = ctypes.c_double
_i = ctypes.c_int32
_st = ctypes.c_int

# name -> (restype, argtypes); mirrors include/lgt.h
PROTOTYPES = {
    "lgt_create": (_st, [ctypes.POINTER(Geom), _vp, ctypes.POINTER(_vp)]),
    "lgt_destroy": (_st, [_vp]),
    "lgt_last_error": (ctypes.c_char_p, [_vp]),
    "lgt_set_stream": (_st, [_vp, _vp]),
    "lgt_volume": (ctypes.c_int64, [_vp]),
    "lgt_dslash": (_st, [_vp, _vp, _vp, _vp, _d, _i]),
    "lgt_dslash_noalloc": (_st, [ctypes.POINTER(Geom), _vp, _vp, _vp, _vp, _d, _i]),
    "lgt_cg_solve": (_st, [_vp, _vp, _vp, _vp, _vp, _d, ctypes.POINTER(SolverParams),
                           ctypes.POINTER(SolverStats)]),
    "lgt_action": (_st, [_vp, _vp, _vp, _d, _d, ctypes.POINTER(SolverParams), ctypes.POINTER(_d),
                         ctypes.POINTER(_d), ctypes.POINTER(SolverStats)]),
    "lgt_fermion_force": (_st, [_vp, _vp, _vp, _d, ctypes.POINTER(SolverParams), _i, _d, _vp,
                                ctypes.POINTER(SolverStats)]),
    "lgt_bilinear_force": (_st, [_vp, _vp, _vp, _vp, _d, _d, _i, _d, _vp]),
    "lgt_gauge_force": (_st, [_vp, _vp, _d, _i, _d, _vp]),
    "lgt_link_update": (_st, [_vp, _vp, _vp, _d]),
    "lgt_kinetic": (_st, [_vp, _vp, ctypes.POINTER(_d)]),
    "lgt_momenta_from_normals": (_st, [_vp, _vp, _vp]),
    "lgt_md_step": (_st, [_vp, _vp, _vp, _vp, _d, _d, _d, _i, ctypes.POINTER(SolverParams),
                          ctypes.POINTER(_d), ctypes.POINTER(SolverStats)]),
    "lgt_hop_benchmark": (_st, [_vp, _vp, _vp, _i, _i, ctypes.POINTER(_d)]),
    "lgt_hop_benchmark_mrhs": (_st, [_vp, _vp, _vp, _i, _i, _i, ctypes.POINTER(_d)]),
    "lgt_batch_create": (_st, [_vp, ctypes.POINTER(_vp)]),
    "lgt_batch_destroy": (_st, [_vp]),
    "lgt_batch_last_error": (ctypes.c_char_p, [_vp]),
    "lgt_batch_set_stream": (_st, [_vp, _vp]),
    "lgt_cg_solve_batch": (_st, [_vp, _i, ctypes.POINTER(BatchItem), ctypes.POINTER(SolverParams),
                                 ctypes.POINTER(SolverStats)]),
    "lgt_stout_smear": (_st, [_vp, _vp, _vp, _d, _i]),
    "lgt_stout_backprop": (_st, [_vp, _vp, _vp, _d, _i, _vp]),
    "lgt_smeared_force": (_st, [_vp, _vp, _vp, _d, _d, _d, _i, ctypes.POINTER(SolverParams), _i, _d, _vp,
                                ctypes.POINTER(_d), ctypes.POINTER(SolverStats)]),
    "lgt_md_step_smeared": (_st, [_vp, _vp, _vp, _vp, _d, _d, _d, _i, _d, _i, ctypes.POINTER(SolverParams),
                                  ctypes.POINTER(_d), ctypes.POINTER(SolverStats)]),
    "lgt_md_step_sw": (_st, [_vp, _vp, _vp, _vp, _d, _d, _d, _i, _d, _i, _i, ctypes.POINTER(SolverParams),
                             ctypes.POINTER(_d), ctypes.POINTER(SolverStats)]),
    "lgt_schur_dslash": (_st, [_vp, _vp, _vp, _vp, _d, _i]),
    "lgt_fermion_force_eo": (_st, [_vp, _vp, _vp, _d, ctypes.POINTER(SolverParams), _i, _d, _vp,
                                   ctypes.POINTER(_d), ctypes.POINTER(SolverStats)]),
    "lgt_md_step_eo": (_st, [_vp, _vp, _vp, _vp, _d, _d, _d, _i, _i, ctypes.POINTER(SolverParams),
                             ctypes.POINTER(_d), ctypes.POINTER(SolverStats)]),
    "lgt_set_stout_checkpoints": (_st, [_vp, _i]),
    "lgt_set_hop_block_sites": (_st, [_vp, _i]),
    "lgt_set_hop_block_order": (_st, [_vp, _i]),
    "lgt_set_batch_hop_kernel": (_st, [_vp, _i]),
    "lgt_dslash_batch": (_st, [_vp, _vp, _i, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_d), _i, _i]),
    "lgt_stout_last_schedule": (_st, [_vp, ctypes.POINTER(_i), ctypes.POINTER(ctypes.c_int64)]),
    "lgt_stout_schedule": (_st, [_i, _i, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(_i), ctypes.POINTER(_i)]),
    "lgt_rational_force_eo": (_st, [_vp, _vp, _vp, _d, _i, ctypes.POINTER(_d), ctypes.POINTER(_d), _d,
                                    ctypes.POINTER(SolverParams), _i, _d, _vp, ctypes.POINTER(_d),
                                    ctypes.POINTER(SolverStats)]),
    "lgt_cg_solve_multishift": (_st, [_vp, _vp, _vp, _d, _i, ctypes.POINTER(_d), ctypes.POINTER(_vp),
                                      ctypes.POINTER(SolverParams), ctypes.POINTER(SolverStats)]),
}

_LIB = None


def load() -> ctypes.CDLL:
    """Load the in-tree liblgt.so; raises if it has not been built."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build the gfx950 library first "
            "(python paper_2602_20516_amd/build.py)")
    # PyTorch ships its own ROCm runtime libraries.  Loaded first, they also
    # satisfy this library's HIP dependency, so the process holds one HIP
    # runtime; loaded after this library, they bring a second runtime, and
    # whichever of the two initialises later finds no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib
