"""ctypes declarations of libgpeps (include/gpeps.h), same names as the C ABI.

Loading fails loudly when the library has not been built: there is no
fallback implementation of any step.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgpeps.so")

GPEPS_OK = 0
STATUS_NAMES = {0: "GPEPS_OK", -1: "GPEPS_ERR_ARG", -2: "GPEPS_ERR_WORKSPACE", -3: "GPEPS_ERR_HIP",
                -4: "GPEPS_ERR_NUMERIC", -5: "GPEPS_ERR_STATE"}
GPEPS_C64_F64SVD, GPEPS_C128 = 0, 1
GPEPS_LAYER_RX, GPEPS_LAYER_RZZ, GPEPS_STEP, GPEPS_STEP_INVERSE, GPEPS_LAYER_REGAUGE = 0, 1, 2, 3, 4
GPEPS_MODE_BATCHED, GPEPS_MODE_PLAIN = 0, 1

# every symbol include/gpeps.h declares
EXPORTS = ("gpeps_workspace_size", "gpeps_init", "gpeps_reset", "gpeps_apply_layer", "gpeps_expect_z",
           "gpeps_bp_expect_z", "gpeps_bp_expect_z_noalloc",
           "gpeps_z_history", "gpeps_bond_dims", "gpeps_stats", "gpeps_set_angles", "gpeps_backward",
           "gpeps_mean_z", "gpeps_backward_mean_z", "gpeps_sync",
           "gpeps_time_kernels", "gpeps_time_backward", "gpeps_autotune", "gpeps_set_tiles", "gpeps_destroy", "gpeps_last_error")


class gpeps_graph(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_edges", ctypes.c_int32),
                ("edges", ctypes.POINTER(ctypes.c_int32)), ("colour", ctypes.POINTER(ctypes.c_int32))]


class gpeps_config(ctypes.Structure):
    _fields_ = [("d_max", ctypes.c_int32), ("precision", ctypes.c_int32), ("trunc_rel", ctypes.c_double),
                ("max_jacobi_sweeps", ctypes.c_int32), ("max_steps", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("adjoint", ctypes.c_int32)]


class GpepsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_LIB = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libgpeps.so and declare its prototypes (cached)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2309_15642_amd.build` "
                          "(the HIP library is required; there is no fallback)")
    lib = ctypes.CDLL(path)
    P = ctypes.POINTER
    c_i32, c_f64, c_sz, vp = ctypes.c_int32, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
    lib.gpeps_workspace_size.argtypes = [P(gpeps_graph), c_i32, P(c_i32), c_i32, P(gpeps_config), P(c_sz)]
    lib.gpeps_init.argtypes = [P(vp), P(gpeps_graph), c_i32, P(c_i32), c_i32, P(c_f64), P(c_f64),
                               P(gpeps_config), vp, c_sz, vp]
    lib.gpeps_reset.argtypes = [vp]
    lib.gpeps_apply_layer.argtypes = [vp, c_i32, c_i32]
    lib.gpeps_expect_z.argtypes = [vp, vp, c_i32]
    lib.gpeps_bp_expect_z.argtypes = [vp, c_i32, vp, c_i32, P(c_f64)]
    lib.gpeps_bp_expect_z_noalloc.argtypes = [vp, c_i32, vp, c_i32, P(c_f64)]
    lib.gpeps_z_history.argtypes = [vp, vp, c_i32, P(c_i32)]
    lib.gpeps_bond_dims.argtypes = [vp, P(c_i32)]
    lib.gpeps_stats.argtypes = [vp, P(ctypes.c_int64), c_i32]
    lib.gpeps_set_angles.argtypes = [vp, P(c_f64), P(c_f64)]
    lib.gpeps_backward.argtypes = [vp, vp, c_i32, P(c_f64), P(c_f64)]
    lib.gpeps_mean_z.argtypes = [vp, vp, c_i32]
    lib.gpeps_backward_mean_z.argtypes = [vp, P(c_f64), P(c_f64), P(c_f64)]
    lib.gpeps_sync.argtypes = [vp]
    lib.gpeps_time_kernels.argtypes = [vp, c_i32, c_i32, P(c_f64), P(ctypes.c_int64), P(ctypes.c_char_p)]
    lib.gpeps_time_backward.argtypes = [vp, P(c_f64), P(c_f64), P(c_f64), c_i32, P(c_f64), P(ctypes.c_int64),
                                        P(ctypes.c_char_p)]
    lib.gpeps_autotune.argtypes = [vp, c_i32, P(c_i32)]
    lib.gpeps_set_tiles.argtypes = [vp, P(c_i32)]
    lib.gpeps_destroy.argtypes = [vp]
    lib.gpeps_last_error.argtypes = [vp]
    lib.gpeps_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "gpeps_last_error":
            getattr(lib, name).restype = c_i32
    _LIB = lib
    return lib


def check(lib: ctypes.CDLL, status: int, ctx=None) -> None:
    if status != GPEPS_OK:
        msg = lib.gpeps_last_error(ctx)
        raise GpepsError(status, msg.decode() if msg else "")
