"""ctypes declarations of the C ABI in include/eigenwave.h (marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int64, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeigenwave.so")

EW_OK = 0
STATUS_NAMES = {
    0: "EW_OK", -1: "EW_ERR_INVALID_ARG", -2: "EW_ERR_OOM", -3: "EW_ERR_HIP",
    -4: "EW_ERR_MG_NOT_CONVERGED", -5: "EW_ERR_NONFINITE", -6: "EW_ERR_NOT_CONVERGED",
    -7: "EW_ERR_UNSUPPORTED",
}
TS = {"explicit": 0, "implicit": 1}
FILTER = {"alpha_d": 0, "quarter": 1}
PRECISION = {"fp64": 0, "mixed": 1}
PREDICTOR = {"zero": 0, "scaled": 1, "cnn": 2, "extrap": 3, "proj": 4}
WALL_DIRICHLET, WALL_NEUMANN = 0, 1
CNN_PARAMS = 3057
CNN_HALO = 3


class GridDesc(ctypes.Structure):
    _fields_ = [("dim", c_int), ("n", c_int64 * 3), ("len", c_double * 3), ("order", c_int),
                ("walls", (c_int * 2) * 3)]


class OpDesc(ctypes.Structure):
    _fields_ = [("omega", c_double), ("ts", c_int), ("cfl", c_double), ("n_its", c_int), ("n_p", c_int),
                ("adjust_omega", c_int), ("filter_const", c_int), ("precision", c_int), ("mg_tol", c_double),
                ("mg_nu1", c_int), ("mg_nu2", c_int), ("mg_max_cycles", c_int), ("mg_coarse_sweeps", c_int),
                ("mg_coarse_points", c_int), ("predictor", c_int), ("proj_window", c_int),
                ("mg_max_levels", c_int), ("mg_relax", c_double), ("mg_relax_coarse", c_double)]


class OpInfo(ctypes.Structure):
    _fields_ = [("n_active", c_int64), ("n_t", c_int), ("dt", c_double), ("omega_used", c_double),
                ("t_final", c_double), ("alpha_d", c_double), ("mg_levels", c_int),
                ("mg_relax", c_double), ("mg_relax_coarse", c_double)]


class OpStats(ctypes.Structure):
    _fields_ = [("wave_solves", c_int64), ("time_steps", c_int64), ("pt_updates", c_int64),
                ("mg_solves", c_int64), ("mg_cycles", c_int64), ("laplacian_applies", c_int64),
                ("cnn_guesses", c_int64), ("guess_probes", c_int64), ("base_rel_res_sum", c_double),
                ("guess_rel_res_sum", c_double)]


class EigsDesc(ctypes.Structure):
    _fields_ = [("k", c_int), ("m", c_int), ("tol_ritz", c_double), ("tol_res", c_double),
                ("max_wave_solves", c_int64), ("seed", c_uint64), ("v0_dev", c_void_p), ("n_keep", c_int),
                ("max_probes", c_int)]


class EigsStats(ctypes.Structure):
    _fields_ = [("n_conv", c_int), ("n_returned", c_int), ("wave_solves", c_int64), ("restarts", c_int64),
                ("probes", c_int64), ("time_steps", c_int64), ("pt_updates", c_int64), ("mg_cycles", c_int64),
                ("seconds", c_double), ("max_res", c_double)]


class KernelProfile(ctypes.Structure):
    _fields_ = [("launches", c_int64), ("total_ms", c_double), ("bytes_alg", c_double)]


KCLASS = {"leapfrog": 0, "smooth": 1, "restrict": 2, "prolong": 3, "resnorm": 4, "update": 5, "coarse": 6,
          "smooth_zero": 7}


class BatchInfo(ctypes.Structure):
    _fields_ = [("nprob", c_int), ("n_small", c_int), ("n_large", c_int), ("max_steps_large", c_int),
                ("step_rows_per_thread", c_int), ("tune_us", c_double * 4), ("total_steps", c_int64),
                ("pt_updates_per_wave_solve", c_int64), ("state_fp64", c_int), ("steps_per_launch", c_int)]


class CnnTrainDesc(ctypes.Structure):
    _fields_ = [("steps", c_int), ("batch", c_int), ("lr", c_double), ("beta1", c_double), ("beta2", c_double),
                ("eps", c_double), ("seed", c_uint64)]


class CnnTrainStats(ctypes.Structure):
    _fields_ = [("steps", c_int), ("first_loss", c_double), ("last_loss", c_double), ("seconds", c_double)]


# name -> (restype, argtypes); every symbol include/eigenwave.h declares.
# ew_alloc_fn(bytes, device, stream, ctx) -> device pointer; ew_free_fn(ptr, ctx)
ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, ctypes.c_size_t, c_int, c_void_p, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_void_p)

SIGNATURES = {
    "ew_op_create": (c_int, [POINTER(GridDesc), POINTER(OpDesc), c_void_p, POINTER(c_void_p)]),
    "ew_op_create_mapped": (c_int, [POINTER(GridDesc), POINTER(OpDesc), POINTER(c_double), c_void_p,
                                    POINTER(c_void_p)]),
    "ew_op_mapped_rho": (c_int, [c_void_p, POINTER(c_double)]),
    "ew_op_destroy": (None, [c_void_p]),
    "ew_op_get_info": (c_int, [c_void_p, POINTER(OpInfo)]),
    "ew_op_get_stats": (c_int, [c_void_p, POINTER(OpStats)]),
    "ew_op_reset_stats": (c_int, [c_void_p]),
    "ew_op_probe_guesses": (c_int, [c_void_p, c_int]),
    "ew_op_apply_filter": (c_int, [c_void_p, c_void_p, c_void_p]),
    "ew_op_apply_laplacian": (c_int, [c_void_p, c_void_p, c_void_p]),
    "ew_apply_filter_noalloc": (c_int, [POINTER(GridDesc), POINTER(OpDesc), c_void_p, c_void_p, c_void_p]),
    "ew_op_mg_solve": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(c_int), POINTER(c_double)]),
    "ew_op_mg_vcycle": (c_int, [c_void_p, c_void_p, c_void_p]),
    "ew_op_mg_half_sweep": (c_int, [c_void_p, c_void_p, c_void_p, c_int]),
    "ew_eigs": (c_int, [c_void_p, POINTER(EigsDesc), c_int, POINTER(c_double), POINTER(c_double),
                        POINTER(c_double), c_void_p, POINTER(EigsStats)]),
    "ew_op_profile_begin": (c_int, [c_void_p, c_int, c_int]),
    "ew_op_profile_end": (c_int, [c_void_p, POINTER(KernelProfile)]),
    "ew_choose_periods": (c_int, [POINTER(GridDesc), POINTER(OpDesc), c_int, c_double, c_int, POINTER(c_int),
                                  POINTER(c_int)]),
    "ew_batch_create": (c_int, [c_int, POINTER(GridDesc), POINTER(OpDesc), c_void_p, POINTER(c_void_p)]),
    "ew_batch_destroy": (None, [c_void_p]),
    "ew_batch_get_info": (c_int, [c_void_p, POINTER(BatchInfo)]),
    "ew_batch_n_active": (c_int, [c_void_p, c_int, POINTER(c_int64), POINTER(c_int)]),
    "ew_batch_apply_filter": (c_int, [c_void_p, POINTER(c_void_p), POINTER(c_void_p)]),
    "ew_batch_eigs": (c_int, [c_void_p, POINTER(EigsDesc), c_int, POINTER(c_double), POINTER(c_double),
                              POINTER(c_double), POINTER(c_int), POINTER(c_void_p), POINTER(EigsStats)]),
    "ew_cnn_create": (c_int, [c_uint64, c_void_p, POINTER(c_void_p)]),
    "ew_cnn_destroy": (None, [c_void_p]),
    "ew_cnn_set_params": (c_int, [c_void_p, POINTER(ctypes.c_float)]),
    "ew_cnn_get_params": (c_int, [c_void_p, POINTER(ctypes.c_float)]),
    "ew_cnn_data_create": (c_int, [c_int, c_int, c_int, POINTER(c_void_p)]),
    "ew_cnn_data_destroy": (None, [c_void_p]),
    "ew_cnn_data_count": (c_int, [c_void_p, POINTER(c_int)]),
    "ew_cnn_data_append": (c_int, [c_void_p, c_int, c_void_p, c_void_p, POINTER(ctypes.c_float), POINTER(c_int)]),
    "ew_cnn_data_read": (c_int, [c_void_p, c_int, c_int, c_void_p, c_void_p, POINTER(ctypes.c_float),
                                 POINTER(c_int)]),
    "ew_cnn_data_collect": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_uint64]),
    "ew_cnn_forward": (c_int, [c_void_p, c_void_p, c_int, c_int, c_void_p]),
    "ew_cnn_loss_grad": (c_int, [c_void_p, c_void_p, c_int, c_int, POINTER(c_double), c_void_p]),
    "ew_cnn_train": (c_int, [c_void_p, c_void_p, POINTER(CnnTrainDesc), POINTER(CnnTrainStats)]),
    "ew_op_set_cnn": (c_int, [c_void_p, c_void_p]),
    "ew_op_cnn_guess": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "ew_fill_uniform": (c_int, [c_void_p, c_int64, c_uint64, c_void_p]),
    "ew_sym_eig": (c_int, [c_int, c_void_p, c_void_p, c_void_p]),
    "ew_set_allocator": (c_int, [c_void_p, c_void_p, c_void_p]),   # ALLOC_FN, FREE_FN cast to pointers
    "ew_last_error": (c_char_p, []),
    "ew_version": (c_char_p, []),
}

_lib = None


class EigenwaveError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def load() -> ctypes.CDLL:
    """Load libeigenwave.so from the package directory; raise if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime (soname libamdhip64.so.7).  Importing
    # it first makes the library's dependency on that soname resolve to the
    # same copy, so one HIP runtime serves both (two runtimes in one process
    # do not share devices, streams or memory).
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_2507_18282_amd.build` "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != EW_OK:
        msg = load().ew_last_error()
        raise EigenwaveError(status, msg.decode() if msg else "")
