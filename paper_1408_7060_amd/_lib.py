"""ctypes declarations of the C ABI in include/etaim.h (marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_uint32, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libetaim.so")

OK, EINVAL, ENOMEM, EHIP, ENOCONV, ENONFINITE, EUNSTABLE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
FP64, FP32 = 0, 1
EFIE, CFIE = 0, 1
CPPIF, BLIF = 0, 1
F_CONTINUE_ON_NOCONV, F_FAIL_ON_UNSTABLE, F_GRAPH, F_IMPLICIT_STOP, F_RESIDUAL_CHECK, F_STEP_GRAPH = 1, 2, 4, 8, 16, 32
KERNEL_CLASSES = ["anterp_x", "yz_green", "fft_x_inv", "interp_near", "yz_delayed", "yz_commit", "krylov",
                  "ring_far"]


class Mesh(ctypes.Structure):
    _fields_ = [("nv", c_int32), ("xyz", POINTER(c_double)), ("nt", c_int32), ("tri", POINTER(c_int32))]


class Rwg(ctypes.Structure):
    _fields_ = [("ns", c_int32), ("idx", POINTER(c_int32))]


class Params(ctypes.Structure):
    _fields_ = [("fc", c_double), ("dt", c_double), ("beta", c_double), ("f_bw", c_double),
                ("nt_steps", c_int32), ("order", c_int32), ("grid", c_int32 * 3), ("d_near", c_double),
                ("ng", c_int32), ("precision", c_int32), ("batch", c_int32), ("tol", c_double),
                ("restart", c_int32), ("maxit", c_int32), ("flags", c_int32), ("sync_every", c_int32),
                ("formulation", c_int32), ("alpha", c_double), ("basis", c_int32), ("nsamp", c_int32),
                ("nomega", c_int32)]


class Derived(ctypes.Structure):
    _fields_ = [("dt", c_double), ("h", c_double), ("origin", c_double * 3), ("rmax", c_double),
                ("stencil_radius", c_double), ("ns", c_int32), ("ng", c_int32), ("mn", c_int32),
                ("nnz", c_int32), ("batch", c_int32), ("precision", c_int32), ("grid", c_int32 * 3),
                ("padded", c_int32 * 3), ("device_bytes", c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("steps_done", c_int32), ("total_iters", c_int32), ("max_iters", c_int32),
                ("first_noconv_step", c_int32), ("unstable_step", c_int32), ("ms_rhs", c_double),
                ("ms_solve", c_double), ("ms_commit", c_double), ("ms_total", c_double),
                ("max_rel_residual", c_double), ("iters_per_step", POINTER(c_int32)),
                ("residual_checks", c_int32), ("residual_worst_step", c_int32), ("max_residual64", c_double),
                ("graph_steps", c_int32), ("graph_halts", c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("radix", (c_int32 * 8) * 3), ("gather_rows", c_int32), ("lines_per_block", c_int32),
                ("interp_waves", c_int32), ("sync_every", c_int32), ("graph", c_int32), ("yz_engine", c_int32),
                ("x_engine", c_int32), ("guess_order", c_int32), ("precond", c_int32),
                ("delay_block", c_int32), ("interp_engine", c_int32),
                ("apply_ms", c_double),
                ("solve_ms", c_double)]


# name -> (restype, argtypes); every entry point the header declares
SIGNATURES = {
    "etaim_create": (c_int32, [POINTER(c_void_p), POINTER(Mesh), POINTER(Rwg), POINTER(Params), c_void_p]),
    "etaim_describe": (c_int32, [c_void_p, POINTER(Derived)]),
    "etaim_excitation_planewave": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double), c_double,
                                             c_double, c_void_p]),
    "etaim_excitation_planewave_noalloc": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double),
                                                     c_double, c_double, c_void_p]),
    "etaim_march": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, POINTER(Stats)]),
    "etaim_apply_z": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p]),
    "etaim_delayed_field": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "etaim_farfield": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_void_p, c_void_p]),
    "etaim_farfield_adjoint": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_void_p, c_void_p]),
    "etaim_adjoint_march": (c_int32, [c_void_p, c_void_p, c_void_p, POINTER(Stats)]),
    "etaim_march_continue": (c_int32, [c_void_p, c_void_p, c_void_p, c_int32, c_int32, POINTER(Stats)]),
    "etaim_state_size": (c_int32, [c_void_p, POINTER(c_size_t)]),
    "etaim_state_save": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "etaim_state_load": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "etaim_export": (c_int32, [c_void_p, c_int32, c_void_p, c_size_t]),
    "etaim_rcs": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_int32, POINTER(c_double), c_double, c_void_p,
                            c_void_p]),
    "etaim_db_error": (c_int32, [c_int32, POINTER(c_double), POINTER(c_double), POINTER(c_double), c_double,
                                 POINTER(c_double)]),
    "etaim_set_profiling": (c_int32, [c_void_p, c_int32]),
    "etaim_set_profiling_mask": (c_int32, [c_void_p, c_uint32]),
    "etaim_set_delay_mode": (c_int32, [c_void_p, c_int32]),
    "etaim_get_delay_mode": (c_int32, [c_void_p, POINTER(c_int32)]),
    "etaim_kernel_stats": (c_int32, [c_void_p, c_int32, POINTER(c_double), POINTER(c_double), POINTER(c_int64)]),
    "etaim_autotune": (c_int32, [c_void_p, c_int32, c_char_p, POINTER(Tuning)]),
    "etaim_get_tuning": (c_int32, [c_void_p, POINTER(Tuning)]),
    "etaim_set_tuning": (c_int32, [c_void_p, POINTER(Tuning)]),
    "etaim_last_error": (c_char_p, []),
    "etaim_destroy": (None, [c_void_p]),
}

_LIB = None


def load() -> ctypes.CDLL:
    """Load libetaim.so; raises if it has not been built (there is no fallback)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1408_7060_amd.build` "
                              "(the ET-AIM path has no CPU fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


class EtaimError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"etaim error {code}: {msg}")
        self.code = code


def check(code: int) -> None:
    if code != OK:
        raise EtaimError(code, load().etaim_last_error().decode(errors="replace"))
