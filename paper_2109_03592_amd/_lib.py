"""ctypes declarations of the C ABI in include/sem.h (argument marshalling only).

Loads the in-tree ``libsem.so``; there is no fallback: if the library is not
built, importing this module raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsem.so")

SEM_OK, SEM_EINVAL, SEM_ENOMEM, SEM_EHIP, SEM_ENOCONV, SEM_EBREAKDOWN, SEM_EBUDGET, SEM_EUNSUPPORTED = range(8)
STATUS_NAMES = {0: "SEM_OK", 1: "SEM_EINVAL", 2: "SEM_ENOMEM", 3: "SEM_EHIP", 4: "SEM_ENOCONV",
                5: "SEM_EBREAKDOWN", 6: "SEM_EBUDGET", 7: "SEM_EUNSUPPORTED"}
SEM_MAP_BOX, SEM_MAP_PIPE_SQ2DISK = 0, 1
SEM_FP64, SEM_FP32 = 0, 1
SEM_PREC_FP64, SEM_PREC_MIXED = 0, 1
SEM_WITH_FP32 = 1
SEM_MAX_ORDER = 17


class MeshDesc(C.Structure):
    _fields_ = [("N", C.c_int), ("nel", C.c_int * 3), ("periodic", C.c_int * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("mapping", C.c_int),
                ("vertices", C.POINTER(C.c_double)), ("dirichlet_faces", C.c_int),
                ("precision_flags", C.c_int)]


class MeshInfo(C.Structure):
    _fields_ = [("N", C.c_int), ("E", C.c_int64), ("n_local", C.c_int64), ("n_global", C.c_int64),
                ("n_shared_local", C.c_int64), ("n_shared_global", C.c_int64),
                ("n_masked_global", C.c_int64), ("n_unmasked_global", C.c_int64),
                ("gs_plan_ids", C.c_int64), ("gs_plan_sum_ids", C.c_int64), ("gs_plan_len", C.c_int64),
                ("device_bytes", C.c_size_t)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int), ("precision", C.c_int),
                ("inner_tol", C.c_double), ("inner_max_iter", C.c_int), ("poll_every", C.c_int),
                ("use_graph", C.c_int), ("fixed_iters", C.c_int), ("x0_given", C.c_int),
                ("profile", C.c_int)]


class SolveStats(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("outer_iterations", C.c_int),
                ("rel_residual", C.c_double), ("bnorm", C.c_double), ("seconds", C.c_double),
                ("ms_operator", C.c_double), ("ms_gather_scatter", C.c_double), ("ms_update", C.c_double),
                ("operator_launches", C.c_int)]


class CoarseInfo(C.Structure):
    _fields_ = [("n_vertices", C.c_int64), ("n_coarse", C.c_int64), ("nnz", C.c_int64),
                ("chebyshev_steps", C.c_int), ("a", C.c_double), ("b", C.c_double)]


class AxgsInfo(C.Structure):
    _fields_ = [("enabled", C.c_int), ("epw", C.c_int), ("lines_per_wg", C.c_int), ("y_onchip", C.c_int),
                ("grid", C.c_int64), ("residual_ids", C.c_int64), ("residual_copies", C.c_int64)]


# name -> (restype, argtypes); kept in step with include/sem.h
_vp, _i, _d = C.c_void_p, C.c_int, C.c_double
SIGNATURES = {
    "sem_last_error": (C.c_char_p, []),
    "sem_version": (C.c_char_p, []),
    "sem_setup": (_i, [C.POINTER(MeshDesc), _vp, C.POINTER(_vp)]),
    "sem_free": (_i, [_vp]),
    "sem_info": (_i, [_vp, C.POINTER(MeshInfo)]),
    "sem_export_gll": (_i, [_i, _vp, _vp, _vp]),
    "sem_export_maps": (_i, [_vp, _vp, _vp, _vp]),
    "sem_export_geom": (_i, [_vp, _vp, _vp, _vp]),
    "sem_export_coords": (_i, [_vp, _vp]),
    "sem_host_setup": (_i, [C.POINTER(MeshDesc), C.POINTER(MeshInfo), _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "sem_load_geometry": (_i, [_vp, _vp, _vp, _vp]),
    "sem_set_operator_config": (_i, [_vp, _i, _i]),
    "sem_get_operator_config": (_i, [_vp, C.POINTER(_i), C.POINTER(_i)]),
    "sem_set_helmholtz": (_i, [_vp, _vp, _vp, _vp]),
    "sem_set_coarse": (_i, [_vp, _i, _d, _vp]),
    "sem_get_coarse_info": (_i, [_vp, C.POINTER(CoarseInfo)]),
    "sem_precond_apply": (_i, [_vp, _vp, _vp, _vp]),
    "sem_set_schwarz": (_i, [_vp, _i, _vp]),
    "sem_get_schwarz_info": (_i, [_vp, C.POINTER(_i), C.POINTER(C.c_int64)]),
    "sem_host_fdm_1d": (_i, [_i, _d, _i, _i, _vp, _vp, C.POINTER(_i), C.POINTER(_i)]),
    "sem_set_gs_config": (_i, [_vp, _i]),
    "sem_get_gs_config": (_i, [_vp, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "sem_set_axgs_config": (_i, [_vp, _i, _i, _i]),
    "sem_get_axgs_info": (_i, [_vp, _i, C.POINTER(AxgsInfo)]),
    "sem_host_axgs_residual": (_i, [C.POINTER(MeshDesc), _i, _i, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                    _vp, _vp]),
    "sem_proj_create": (_i, [_vp, _i, C.POINTER(_vp)]),
    "sem_proj_free": (_i, [_vp]),
    "sem_proj_reset": (_i, [_vp]),
    "sem_proj_size": (_i, [_vp, C.POINTER(_i)]),
    "sem_proj_project": (_i, [_vp, _vp, _vp, _vp]),
    "sem_proj_add": (_i, [_vp, _vp, C.POINTER(_i), _vp]),
    "sem_proj_solve": (_i, [_vp, _vp, _vp, C.POINTER(SolveOpts), C.POINTER(SolveStats), _vp]),
    "sem_ax": (_i, [_vp, _i, _vp, _vp, _vp, _vp]),
    "sem_gs": (_i, [_vp, _i, _vp, _vp]),
    "sem_ax_noalloc": (_i, [_vp, _i, _vp, _vp, _vp, _vp]),
    "sem_axgs": (_i, [_vp, _i, _vp, _vp, _vp]),
    "sem_mass": (_i, [_vp, _vp, _vp, _vp]),
    "sem_scatter": (_i, [_vp, _vp, _vp, _vp]),
    "sem_batch_create": (_i, [_i, C.c_size_t, _vp, C.POINTER(_vp)]),
    "sem_batch_free": (_i, [_vp]),
    "sem_batch_tune": (_i, [_vp, C.POINTER(_vp), _i, _vp]),
    "sem_batch_set_epw": (_i, [_vp, _i, _i]),
    "sem_batch_get_epw": (_i, [_vp, _i, _i, C.POINTER(_i)]),
    "sem_batch_set_grid": (_i, [_vp, _i, _i]),
    "sem_batch_get_grid": (_i, [_vp, C.POINTER(_i), C.POINTER(_i)]),
    "sem_batch_solve": (_i, [_vp, C.POINTER(_vp), _i, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(SolveOpts),
                             _vp, _vp]),
    "sem_batch_admit": (_i, [_vp, _vp, _vp, _vp, C.POINTER(SolveOpts), C.POINTER(_i), _vp]),
    "sem_batch_step": (_i, [_vp, _i, _i, _vp, C.POINTER(_i)]),
    "sem_batch_finished": (_i, [_vp, C.POINTER(_i), _i, C.POINTER(_i)]),
    "sem_batch_retire": (_i, [_vp, _i, C.POINTER(SolveStats)]),
    "sem_batch_slot_layout": (_i, [C.c_int64, _i, _vp, C.POINTER(C.c_size_t)]),
    "sem_solve_opts_default": (None, [C.POINTER(SolveOpts)]),
    "sem_pcg_solve": (_i, [_vp, _vp, _vp, C.POINTER(SolveOpts), C.POINTER(SolveStats), _vp]),
}

_lib = None


def load():
    """Load libsem.so and declare every entry point; raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2109_03592_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class SemError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = load().sem_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, where: str):
    if status != SEM_OK:
        raise SemError(status, where)
