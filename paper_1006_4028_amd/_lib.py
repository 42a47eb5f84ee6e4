"""ctypes declarations of the C ABI in ``include/dp.h`` (argument marshalling only).

The library is ``paper_1006_4028_amd/libdp.so`` built in-tree by
``paper_1006_4028_amd.build``.  There is no fallback: if the library is
missing or fails to load, importing the binding raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdp.so")

DP_OK = 0
DP_ERR_INVALID_ARG = -1
DP_ERR_OOM = -2
DP_ERR_DEVICE = -3
DP_ERR_NOT_CONVERGED = -4
DP_ERR_BREAKDOWN = -5
DP_ERR_NONFINITE = -6
DP_ERR_BAD_STATE = -7
DP_ERR_FULL = -8

DP_PREC = {"f64": 0, "f32": 1, "f16": 2, "f32single": 3}
DP_SOLVER = {"bicgstab": 0, "cgnr": 1}

DP_PRECOND, DP_DAGGER, DP_HOP_ONLY = 1, 2, 4
DP_NOALLOC_SCRATCH_BYTES, DP_NOALLOC_MAX_RHS = 128 << 20, 64
# test hooks of dp_apply (documented in include/dp.h)
DP_APPLY_SCHUR, DP_APPLY_F32, DP_APPLY_F16 = 8, 16, 32

EXPORTED = [
    "dp_create", "dp_destroy", "dp_last_error", "dp_set_gauge", "dp_set_gauge_dev", "dp_set_gauge_sf",
    "dp_sf_wall_sources", "dp_set_clover",
    "dp_set_clover_field", "dp_set_mass", "dp_set_kappa", "dp_set_alpha", "dp_set_alpha_space", "dp_apply",
    "dp_apply_dev", "dp_apply_dev_slots", "dp_apply_dev_noalloc", "dp_point_sources", "dp_solve", "dp_solve_sap",
    "dp_solve_sap_dev", "dp_sap_precondition", "dp_solve_dev", "dp_footprint_bytes", "dp_set_timing", "dp_get_timing", "dp_get_timing_samples",
    "dp_batch_open", "dp_batch_close",
    "dp_batch_admit", "dp_batch_step", "dp_batch_harvest", "dp_batch_status", "dp_batch_device_bytes",
]


class dp_sap_params(ctypes.Structure):
    _fields_ = [("r", ctypes.c_double), ("block", ctypes.c_int * 4), ("ncy", ctypes.c_int), ("nmr", ctypes.c_int),
                ("nkv", ctypes.c_int), ("precision", ctypes.c_int), ("max_iter", ctypes.c_int)]


class dp_params(ctypes.Structure):
    _fields_ = [("r", ctypes.c_double), ("solver", ctypes.c_int), ("precision", ctypes.c_int),
                ("max_iter", ctypes.c_int), ("delta", ctypes.c_double), ("x0_src", ctypes.c_int),
                ("ncols_group", ctypes.c_int)]


class dp_info(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("outer", ctypes.c_int),
                ("hop_calls", ctypes.c_int), ("restarts", ctypes.c_int), ("true_res", ctypes.c_double),
                ("seconds", ctypes.c_double), ("fallback", ctypes.c_int)]


class dp_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_longlong), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("flops", ctypes.c_double)]


class dp_batch_result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_longlong), ("slot", ctypes.c_int), ("info", dp_info)]


class DPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libdp error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1006_4028_amd.build` "
                          "(hipcc, gfx950); there is no CPU fallback")
    # torch bundles its own HIP runtime under the same soname as the system one
    # libdp.so links; whichever loads first serves the whole process, and torch
    # cannot initialise the GPU on a runtime newer than its own.  Loading torch
    # first makes both use torch's runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)
    L.dp_create.argtypes = [ip, ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]
    L.dp_destroy.argtypes = [vp]
    L.dp_destroy.restype = None
    L.dp_last_error.argtypes = [vp]
    L.dp_last_error.restype = ctypes.c_char_p
    L.dp_set_gauge.argtypes = [vp, dp]
    L.dp_set_gauge_dev.argtypes = [vp, vp, vp]
    L.dp_set_gauge_sf.argtypes = [vp, dp, ctypes.c_double]
    L.dp_sf_wall_sources.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp]
    L.dp_set_clover.argtypes = [vp, ctypes.c_double]
    L.dp_set_clover_field.argtypes = [vp, dp]
    L.dp_set_mass.argtypes = [vp, ctypes.c_double]
    L.dp_set_kappa.argtypes = [vp, ctypes.c_double]
    L.dp_set_alpha.argtypes = [vp, dp]
    L.dp_set_alpha_space.argtypes = [vp, dp, dp, dp]
    L.dp_solve_sap.argtypes = [vp, dp, ctypes.POINTER(dp_sap_params), dp, dp, ctypes.POINTER(dp_info)]
    L.dp_sap_precondition.argtypes = [vp, dp, ctypes.POINTER(dp_sap_params), dp]
    L.dp_solve_sap_dev.argtypes = [vp, vp, ctypes.POINTER(dp_sap_params), vp, dp, ctypes.POINTER(dp_info), vp]
    L.dp_apply.argtypes = [vp, dp, dp, ctypes.c_int]
    L.dp_apply_dev.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
    L.dp_apply_dev_slots.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, dp, dp, vp]
    L.dp_apply_dev_noalloc.argtypes = [vp, vp, vp, ctypes.c_int, ctypes.c_int, vp]
    L.dp_point_sources.argtypes = [vp, ip, ctypes.c_int, ctypes.c_int, vp, vp]
    L.dp_solve.argtypes = [vp, dp, ctypes.c_int, ctypes.POINTER(dp_params), dp, dp, ctypes.POINTER(dp_info)]
    L.dp_solve_dev.argtypes = [vp, vp, ctypes.c_int, ctypes.POINTER(dp_params), vp, dp,
                               ctypes.POINTER(dp_info), vp]
    L.dp_footprint_bytes.argtypes = [ip, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.dp_footprint_bytes.restype = ctypes.c_longlong
    L.dp_set_timing.argtypes = [vp, ctypes.c_int]
    L.dp_get_timing.argtypes = [vp, ctypes.POINTER(dp_kernel_stat), ctypes.c_int, ip]
    L.dp_get_timing_samples.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_float), ctypes.c_int, ip]
    L.dp_batch_open.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(vp)]
    L.dp_batch_close.argtypes = [vp]
    L.dp_batch_close.restype = None
    L.dp_batch_admit.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_double, dp, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_int, ctypes.c_longlong, ip]
    L.dp_batch_step.argtypes = [vp, ctypes.c_int, ip]
    L.dp_batch_harvest.argtypes = [vp, ctypes.POINTER(dp_batch_result), dp, ctypes.c_int, ip]
    L.dp_batch_status.argtypes = [vp, ip, ip, ip]
    L.dp_batch_device_bytes.argtypes = [vp]
    L.dp_batch_device_bytes.restype = ctypes.c_longlong
    _lib = L
    return L
