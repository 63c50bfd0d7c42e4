"""ctypes declarations of the C ABI in include/afqmc.h (argument marshalling only)."""

from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libafqmc.so")

AFQMC_FP64, AFQMC_FP32, AFQMC_BF16X3 = 0, 1, 2
FLAG_HYBRID, FLAG_FREE_PROJECTION, FLAG_MEAN_FIELD, FLAG_CLOSED_SHELL = 0x1, 0x2, 0x4, 0x8
WEIGHT_MODES = {"phaseless": 0, "hybrid": FLAG_HYBRID, "free": FLAG_FREE_PROJECTION}
PRECISIONS = {"fp64": AFQMC_FP64, "fp32": AFQMC_FP32, "bf16x3": AFQMC_BF16X3}

STATUS_BITS = {0x1: "nonfinite", 0x2: "singular", 0x4: "ecap", 0x8: "wcap", 0x10: "fbcap",
               0x20: "phase"}

KERNEL_GROUPS = ["contract", "overlap", "fields", "abuild", "propagate", "qr", "weights", "comb",
                 "assemble", "guard"]

EXPORTS = ["afqmc_setup", "afqmc_workspace_bytes", "afqmc_get_info", "afqmc_walkers_init",
           "afqmc_measure", "afqmc_step", "afqmc_fields_draw", "afqmc_energy", "afqmc_get_status",
           "afqmc_kernel_timing", "afqmc_kernel_time", "afqmc_destroy", "afqmc_error_string",
           "afqmc_mcd_workspace_bytes", "afqmc_modified_cholesky", "afqmc_setup_multidet",
           "afqmc_batch_create", "afqmc_batch_step", "afqmc_batch_destroy", "afqmc_autotune",
           "afqmc_set_tile", "afqmc_get_tile", "afqmc_energy_enqueue", "afqmc_footprint_bytes",
           "afqmc_mfma_peak", "afqmc_get_growth", "afqmc_get_bound_counts",
           "afqmc_modified_cholesky_noalloc", "afqmc_batch_set_mode"]

TILES = {"default": 0, "w4": 1, "w2": 2, "wide": 3, "flat": 4, "stack": 5, "pp": 6, "bx": 7, "bx8": 8}
MFMA_PEAK_BYTES = 16384   # AFQMC_MFMA_PEAK_BYTES


class Params(C.Structure):
    _fields_ = [("M", C.c_int32), ("n_up", C.c_int32), ("n_dn", C.c_int32), ("n_chol", C.c_int32),
                ("dtau", C.c_double), ("e_trial", C.c_double), ("n_taylor", C.c_int32),
                ("qr_period", C.c_int32), ("pop_period", C.c_int32), ("precision", C.c_int32),
                ("el_cap_C", C.c_double), ("w_max", C.c_double), ("fb_cap", C.c_double),
                ("flags", C.c_uint32), ("n_growth", C.c_int32), ("theta_guard", C.c_double)]


class WalkersC(C.Structure):
    _fields_ = [("n_walkers", C.c_int32), ("reserved", C.c_int32), ("U", C.c_void_p),
                ("weight", C.c_void_p), ("arg_ovlp", C.c_void_p), ("log_ovlp", C.c_void_p),
                ("e_loc", C.c_void_p), ("phase", C.c_void_p), ("walker_id", C.c_void_p),
                ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t), ("step", C.c_int64)]


class FieldsC(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("job_id", C.c_uint64), ("x", C.c_void_p),
                ("u_comb", C.c_double)]


class InfoC(C.Structure):
    _fields_ = [("e_trial", C.c_double), ("e_hf", C.c_double), ("device_bytes", C.c_size_t)]


class AfqmcError(RuntimeError):
    pass


_lib = None


def load(path: str | None = None) -> C.CDLL:
    """Load libafqmc.so; raises if it has not been built (there is no fallback path)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise AfqmcError(f"{p} is missing: build it with `python -m paper_1711_02242_amd.build`")
    # torch ships its own HIP runtime (soname libamdhip64.so.7) and loads it by file name: loaded
    # first, it is the one the library binds to.  Loaded after the library, it would come in as
    # a second HIP runtime, and the streams and memory torch hands over would be foreign to ours.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(p)
    P = C.POINTER
    sig = {
        "afqmc_setup": ([P(Params), C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                         C.c_void_p, P(C.c_void_p)], C.c_int),
        "afqmc_setup_multidet": ([P(Params), C.c_double, C.c_void_p, C.c_void_p, C.c_int32,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, P(C.c_void_p)],
                                 C.c_int),
        "afqmc_workspace_bytes": ([C.c_void_p, C.c_int32, P(C.c_size_t)], C.c_int),
        "afqmc_get_info": ([C.c_void_p, P(InfoC)], C.c_int),
        "afqmc_walkers_init": ([C.c_void_p, P(WalkersC)], C.c_int),
        "afqmc_measure": ([C.c_void_p, P(WalkersC)], C.c_int),
        "afqmc_step": ([C.c_void_p, P(WalkersC), P(FieldsC)], C.c_int),
        "afqmc_fields_draw": ([C.c_void_p, P(WalkersC), P(FieldsC), C.c_void_p], C.c_int),
        "afqmc_energy": ([C.c_void_p, P(WalkersC), P(C.c_double)], C.c_int),
        "afqmc_get_status": ([C.c_void_p, P(C.c_uint32), C.c_int], C.c_int),
        "afqmc_get_growth": ([C.c_void_p, P(WalkersC), P(C.c_double)], C.c_int),
        "afqmc_get_bound_counts": ([C.c_void_p, P(C.c_uint64), C.c_int], C.c_int),
        "afqmc_kernel_timing": ([C.c_void_p, C.c_int], C.c_int),
        "afqmc_kernel_time": ([C.c_void_p, C.c_int, P(C.c_double), P(C.c_int64)], C.c_int),
        "afqmc_destroy": ([C.c_void_p], C.c_int),
        "afqmc_batch_create": ([C.c_int32, P(C.c_void_p), P(P(WalkersC)), C.c_void_p,
                                P(C.c_void_p)], C.c_int),
        "afqmc_batch_step": ([C.c_void_p, P(FieldsC)], C.c_int),
        "afqmc_batch_destroy": ([C.c_void_p], C.c_int),
        "afqmc_batch_set_mode": ([C.c_void_p, C.c_int32], C.c_int),
        "afqmc_autotune": ([C.c_void_p, P(WalkersC), C.c_int32, P(C.c_int32), P(C.c_double)],
                           C.c_int),
        "afqmc_set_tile": ([C.c_void_p, C.c_int32], C.c_int),
        "afqmc_energy_enqueue": ([C.c_void_p, P(WalkersC), C.c_void_p], C.c_int),
        "afqmc_mfma_peak": ([C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p, P(C.c_double)],
                            C.c_int),
        "afqmc_footprint_bytes": ([P(Params), C.c_int32, C.c_int32, P(C.c_size_t),
                                   P(C.c_size_t)], C.c_int),
        "afqmc_get_tile": ([C.c_void_p, P(C.c_int32)], C.c_int),
        "afqmc_error_string": ([C.c_int], C.c_char_p),
        "afqmc_mcd_workspace_bytes": ([C.c_int32, P(C.c_size_t)], C.c_int),
        "afqmc_modified_cholesky": ([C.c_void_p, C.c_int32, C.c_double, C.c_int32, C.c_void_p,
                                     P(C.c_int32), P(C.c_int32), C.c_void_p, C.c_size_t,
                                     C.c_void_p], C.c_int),
        "afqmc_modified_cholesky_noalloc": ([C.c_void_p, C.c_int32, C.c_double, C.c_int32,
                                             C.c_void_p, P(C.c_int32), P(C.c_int32),
                                             C.c_void_p], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    if path is None:
        _lib = lib
    return lib


def check(rc: int, what: str) -> None:
    if rc != 0:
        msg = load().afqmc_error_string(rc).decode()
        raise AfqmcError(f"{what}: {msg} ({rc})")
