"""ctypes declarations of the C ABI in include/mhdlbm.h (argument marshalling only).

The names, structs and constants mirror the header one to one. Loading fails loudly if the
built library is missing: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmhdlbm.so")

MHD_OK = 0
MHD_ERR_INVALID_ARG = -1
MHD_ERR_OOM = -2
MHD_ERR_HIP = -3
MHD_ERR_UNSTABLE = -4
MHD_ERR_STATE = -5
MHD_ERR_UNSUPPORTED = -6
STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "OOM", -3: "HIP", -4: "UNSTABLE", -5: "STATE",
                -6: "UNSUPPORTED"}

MHD_STORE_F32, MHD_STORE_F16, MHD_STORE_BF16, MHD_STORE_F16_SPLIT = 0, 1, 2, 3
MHD_BEXT_NONE, MHD_BEXT_UNIFORM_Y, MHD_BEXT_TANH_FRINGE_Y, MHD_BEXT_SIX_MAGNETS = 0, 1, 2, 3
MHD_FIELD_RHO, MHD_FIELD_U, MHD_FIELD_B_INDUCED = 0, 1, 2
(MHD_K_MAG_SWEEP, MHD_K_IB, MHD_K_LORENTZ, MHD_K_FLUID, MHD_K_BUDGET, MHD_K_CONTROL,
 MHD_K_COUNT) = range(7)

EXPORTS = ("mhd_last_error", "mhd_workspace_size", "mhd_create", "mhd_set_markers",
           "mhd_set_params", "mhd_set_field", "mhd_get_field", "mhd_get_time", "mhd_set_time",
           "mhd_step", "mhd_step_noalloc", "mhd_get_budgets", "mhd_record_budget", "mhd_set_profiling",
           "mhd_kernel_stats", "mhd_destroy", "mhd_get_tiles", "mhd_set_tiles",
           "mhd_set_graph", "mhd_tune", "mhd_mag_residual_curve", "mhd_choose_n_mag",
           "mhd_batch_workspace_size", "mhd_batch_create", "mhd_batch_pipe", "mhd_batch_tune",
           "mhd_batch_step", "mhd_batch_set_graph", "mhd_batch_set_profiling",
           "mhd_batch_kernel_stats", "mhd_batch_destroy")


class mhd_grid_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("rho_storage", C.c_int32), ("u_storage", C.c_int32), ("b_storage", C.c_int32),
                ("u_scale", C.c_double), ("b_scale", C.c_double)]


class mhd_pipe_desc(C.Structure):
    _fields_ = [("grid", mhd_grid_desc), ("n_markers", C.c_int64)]


class mhd_params(C.Structure):
    _fields_ = [("nu", C.c_double), ("eta", C.c_double), ("n_mag", C.c_int32),
                ("bext_kind", C.c_int32), ("lambda_u", C.c_double), ("lambda_b", C.c_double),
                ("G0", C.c_double), ("G1", C.c_double), ("period", C.c_double),
                ("B0", C.c_double), ("fringe_x0", C.c_double), ("fringe_w", C.c_double),
                ("yc", C.c_double), ("zc", C.c_double), ("avg_radius", C.c_double),
                ("flow_control", C.c_int32), ("lattice", C.c_int32),
                ("u_bulk_target", C.c_double), ("k_c", C.c_double), ("alpha", C.c_double),
                ("magnet_half_width", C.c_double), ("magnet_distance", C.c_double),
                ("gamma", C.c_double), ("omega_radius", C.c_double)]


class mhd_budget(C.Structure):
    _fields_ = [("step", C.c_int64), ("G", C.c_double), ("E_k", C.c_double), ("E_m", C.c_double),
                ("E_b", C.c_double), ("P_in", C.c_double), ("P_p", C.c_double),
                ("P_nu", C.c_double), ("P_L", C.c_double), ("M_eta", C.c_double),
                ("M_adv", C.c_double), ("joule", C.c_double), ("mass", C.c_double),
                ("Q", C.c_double), ("u_max", C.c_double), ("n_omega", C.c_double),
                ("res_mag", C.c_double), ("D_eta", C.c_double)]


_D = C.POINTER(C.c_double)
_lib = None


def lib() -> C.CDLL:
    """Load libmhdlbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(there is no non-HIP fallback)")
        L = C.CDLL(LIB_PATH)
        P = C.c_void_p
        L.mhd_last_error.restype = C.c_char_p
        L.mhd_last_error.argtypes = []
        L.mhd_workspace_size.argtypes = [C.POINTER(mhd_grid_desc), C.c_int64, C.POINTER(C.c_size_t)]
        L.mhd_create.argtypes = [C.POINTER(mhd_grid_desc), C.c_int64, C.c_void_p, C.c_size_t,
                                 C.c_void_p, C.POINTER(C.c_void_p)]
        L.mhd_set_markers.argtypes = [P, _D, C.c_int64, _D, _D]
        L.mhd_set_params.argtypes = [P, C.POINTER(mhd_params)]
        L.mhd_set_field.argtypes = [P, C.c_int32, _D]
        L.mhd_get_field.argtypes = [P, C.c_int32, _D]
        L.mhd_get_time.argtypes = [P, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.mhd_set_time.argtypes = [P, C.c_int64, C.c_double]
        L.mhd_step.argtypes = [P, C.c_int64, C.c_int32]
        L.mhd_step_noalloc.argtypes = [P, C.c_int64, C.c_int32]
        L.mhd_get_budgets.argtypes = [P, C.POINTER(mhd_budget), C.c_int64, C.POINTER(C.c_int64)]
        L.mhd_record_budget.argtypes = [P]
        L.mhd_set_profiling.argtypes = [P, C.c_int32]
        L.mhd_kernel_stats.argtypes = [P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]
        L.mhd_destroy.argtypes = [P]
        L.mhd_mag_residual_curve.argtypes = [P, C.c_int32, _D]
        L.mhd_choose_n_mag.argtypes = [P, C.c_double, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]
        I4 = C.c_int32 * 4
        L.mhd_get_tiles.argtypes = [P, I4]
        L.mhd_set_tiles.argtypes = [P, I4]
        L.mhd_set_graph.argtypes = [P, C.c_int32]
        L.mhd_tune.argtypes = [P, C.c_int32]
        PD = C.POINTER(mhd_pipe_desc)
        L.mhd_batch_workspace_size.argtypes = [PD, C.c_int32, C.POINTER(C.c_size_t)]
        L.mhd_batch_create.argtypes = [PD, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                       C.POINTER(C.c_void_p)]
        L.mhd_batch_pipe.argtypes = [P, C.c_int32, C.POINTER(C.c_void_p)]
        L.mhd_batch_tune.argtypes = [P, C.c_int32]
        L.mhd_batch_step.argtypes = [P, C.c_int64, C.c_int32]
        L.mhd_batch_set_graph.argtypes = [P, C.c_int32]
        L.mhd_batch_set_profiling.argtypes = [P, C.c_int32]
        L.mhd_batch_kernel_stats.argtypes = [P, C.c_int32, C.POINTER(C.c_int64),
                                             C.POINTER(C.c_double)]
        L.mhd_batch_destroy.argtypes = [P]
        for name in EXPORTS:
            if name != "mhd_last_error":
                getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


class MhdError(RuntimeError):
    def __init__(self, status: int, call: str, msg: str):
        super().__init__(f"{call}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def check(status: int, call: str) -> int:
    if status != MHD_OK:
        raise MhdError(status, call, lib().mhd_last_error().decode())
    return status
