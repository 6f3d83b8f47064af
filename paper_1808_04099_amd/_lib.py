"""ctypes declarations of the C ABI in include/bcm.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int8, c_int32, c_int64, c_size_t, \
    c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libbcm.so")

BCM_OK, BCM_NOT_CONVERGED, BCM_STAGNATED = 0, 1, 2
BCM_FP64, BCM_MIXED, BCM_MIXED_F32FIELDS = 0, 1, 2
PRECISIONS = {"fp64": BCM_FP64, "mixed": BCM_MIXED, "mixed_f32fields": BCM_MIXED_F32FIELDS}


class MeshDesc(ctypes.Structure):
    _fields_ = [("n_cubes", c_int32), ("n", c_int32), ("origin", POINTER(c_double)),
                ("level", POINTER(c_int8)), ("root_edge", c_double), ("nbr", POINTER(c_int32)),
                ("face_bc", POINTER(c_int8))]


class SolverOpts(ctypes.Structure):
    _fields_ = [("precision", c_int32), ("tol", c_double), ("max_iter", c_int32),
                ("max_outer", c_int32), ("inner_tol", c_double), ("pre_sweeps", c_int32),
                ("post_sweeps", c_int32), ("coarse_iters", c_int32), ("krylov", c_int32),
                ("coarse_solver", c_int32), ("coarse_cycles", c_int32),
                ("graph_split", c_int32), ("prolong", c_int32), ("check_every", c_int32)]


class Report(ctypes.Structure):
    _fields_ = [("status", c_int32), ("n_outer", c_int32), ("n_inner", c_int32),
                ("final_rel_res", c_double), ("history", POINTER(c_double)),
                ("history_cap", c_int32), ("history_len", c_int32)]


class ProjectIn(ctypes.Structure):
    _fields_ = [("u", c_void_p * 3), ("alpha", c_void_p), ("us", c_void_p * 3),
                ("us_const", c_double * 3), ("U_in", c_double), ("dt", c_double),
                ("rho", c_double), ("p0", c_void_p)]


class ProjectOut(ctypes.Structure):
    _fields_ = [("u_new", c_void_p * 3), ("p", c_void_p), ("face_u", c_void_p * 3),
                ("b", c_void_p)]


class AdjointIn(ctypes.Structure):
    _fields_ = [("u", c_void_p * 3), ("alpha", c_void_p), ("us", c_void_p * 3),
                ("us_const", c_double * 3), ("U_in", c_double), ("dt", c_double),
                ("rho", c_double), ("g_u_new", c_void_p * 3), ("g_p", c_void_p)]


class AdjointOut(ctypes.Structure):
    _fields_ = [("g_u", c_void_p * 3), ("g_alpha", c_void_p), ("g_U_in", c_double),
                ("lambda_", c_void_p), ("accumulate", c_int32)]


class MomentumIn(ctypes.Structure):
    _fields_ = [("u", c_void_p * 3), ("h_prev", c_void_p * 3), ("U_in", c_double),
                ("dt", c_double), ("nu", c_double), ("scheme", c_int32), ("cn_tol", c_double),
                ("cn_max_iter", c_int32)]


class MomentumOut(ctypes.Structure):
    _fields_ = [("u_tilde", c_void_p * 3), ("h", c_void_p * 3)]


SCHEMES = {"euler": 0, "ab2": 1, "cn": 2}


class Particles(ctypes.Structure):
    _fields_ = [("n", c_int32), ("X", c_void_p), ("dV", c_void_p), ("Us", c_void_p),
                ("us_const", c_double * 3)]

EXPORTS = {
    "bcm_default_opts": (None, [POINTER(SolverOpts)]),
    "bcm_mesh_create": (c_int, [POINTER(MeshDesc), POINTER(c_void_p)]),
    "bcm_mesh_destroy": (None, [c_void_p]),
    "bcm_plan_create": (c_int, [c_void_p, POINTER(SolverOpts), POINTER(c_void_p),
                                POINTER(c_size_t)]),
    "bcm_plan_destroy": (None, [c_void_p]),
    "bcm_plan_bind": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p]),
    "bcm_project": (c_int, [c_void_p, POINTER(ProjectIn), POINTER(ProjectOut), POINTER(Report),
                            c_void_p]),
    "bcm_project_recompute": (c_int, [c_void_p, POINTER(ProjectIn), c_void_p,
                                      POINTER(ProjectOut), c_void_p]),
    "bcm_project_adjoint": (c_int, [c_void_p, POINTER(AdjointIn), POINTER(AdjointOut),
                                    POINTER(Report), c_void_p]),
    "bcm_poisson_solve": (c_int, [c_void_p, c_void_p, c_void_p, c_int, POINTER(Report),
                                  c_void_p]),
    "bcm_apply_laplacian": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "bcm_compress_bound": (c_int, [c_void_p, POINTER(c_size_t)]),
    "bcm_compress": (c_int, [c_void_p, c_void_p, c_double, c_void_p, c_size_t, POINTER(c_size_t),
                             c_void_p]),
    "bcm_decompress": (c_int, [c_void_p, c_void_p, c_size_t, c_void_p, c_void_p]),
    "bcm_ib_force": (c_int, [c_void_p, POINTER(Particles), POINTER(c_void_p), POINTER(c_void_p),
                             c_double, c_double, c_void_p, c_void_p, c_void_p]),
    "bcm_momentum": (c_int, [c_void_p, POINTER(MomentumIn), POINTER(MomentumOut),
                             POINTER(Report), c_void_p]),
    "bcm_kinetic_energy": (c_int, [c_void_p, POINTER(c_void_p), c_double, c_double,
                                   POINTER(c_double), POINTER(c_void_p), c_void_p]),
    "bcm_kinetic_energy_noalloc": (c_int, [c_void_p, POINTER(c_void_p), c_double, c_double,
                                           POINTER(c_double), POINTER(c_void_p), c_void_p]),
    "bcm_timing_enable": (c_int, [c_void_p, c_char_p]),
    "bcm_timing_sample": (c_int, [c_void_p, c_int32]),
    "bcm_timing_read": (c_int, [c_void_p, POINTER(c_int64), POINTER(c_double)]),
    "bcm_timing_name": (c_char_p, [c_int]),
    "bcm_mesh_cells": (c_int64, [c_void_p]),
    "bcm_status_string": (c_char_p, [c_int]),
    "bcm_last_error": (c_char_p, []),
}

_lib = None


def load():
    """Load libbcm.so (built by paper_1808_04099_amd.build); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1808_04099_amd.build` (there is no fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
