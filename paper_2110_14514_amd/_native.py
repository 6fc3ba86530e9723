"""ctypes declarations of the gcpstream C ABI (include/gcpstream.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Loading fails loudly when the library has not been built; there is
no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_char_p, c_double, c_int32, c_int64,
                    c_size_t, c_uint32, c_uint64, c_void_p)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgcpstream.so")

ABI_VERSION = 2
MAX_WINDOW = 64
MAX_RANK = 64

# gcp_status
OK, E_ARG, E_SHAPE, E_ALIGN, E_STATE, E_WORKSPACE, E_DEVICE, E_NUMERIC, E_UNSUPPORTED = range(9)
STATUS_NAMES = ["GCP_OK", "GCP_E_ARG", "GCP_E_SHAPE", "GCP_E_ALIGN", "GCP_E_STATE",
                "GCP_E_WORKSPACE", "GCP_E_DEVICE", "GCP_E_NUMERIC", "GCP_E_UNSUPPORTED"]

LOSS_IDS = {"gaussian": 0, "poisson_log": 1, "bernoulli_logit": 2, "poisson_id": 3, "bernoulli_odds": 4}
F32, F64 = 0, 1
SLICE_DENSE, SLICE_COO, SLICE_BITS = 0, 1, 2
WANT_LOSS, WANT_GRAD, IMPL_PLAIN = 1, 2, 256
FLAG_PLAIN_SCRATCH = 1
FLAG_KERNEL_VALU = 2
FLAG_KERNEL_MFMA = 4
FLAG_SAMPLED_ATOMIC = 8
FLAG_GAUSS_IDENTITY = 16
HIST_SLICES = 0
HIST_MODEL = 1
TSOLVE_LS = 0
TSOLVE_SGD = 1


class GcpParams(Structure):
    _fields_ = [
        ("abi_version", c_uint32), ("d", c_int32), ("dims", c_int64 * 4),
        ("rank", c_int32), ("window", c_int32), ("loss", c_int32),
        ("dtype", c_int32), ("slice_kind", c_int32), ("flags", c_int32),
        ("w", c_double), ("theta", c_double), ("lam", c_double), ("mu", c_double),
        ("lower", c_double), ("alpha_f", c_double), ("beta1", c_double),
        ("beta2", c_double), ("adam_eps", c_double), ("tau_f", c_int32),
        ("hist", c_int32), ("max_nnz", c_int64), ("p", c_int64),
        ("q", c_int64), ("seed", c_uint64), ("tsolve", c_int32),
        ("tau_w", c_int32), ("kappa_w", c_int32), ("kappa_f", c_int32),
        ("alpha_w", c_double), ("tol_w", c_double), ("tol_f", c_double),
        ("p_est", c_int64), ("q_est", c_int64),
    ]


class GcpSlice(Structure):
    _fields_ = [("kind", c_int32), ("reserved", c_int32), ("vals", c_void_p),
                ("coords", c_void_p), ("nnz", c_int64)]


class GcpBatchIO(Structure):
    _fields_ = [("X_t", c_void_p), ("s_t", c_void_p), ("loss", c_void_p),
                ("G", c_void_p * 3), ("g_s", c_void_p)]


# name -> (restype, argtypes), in header order
SIGNATURES = {
    "gcp_params_default": (None, [POINTER(GcpParams)]),
    "gcp_workspace_size": (c_int32, [POINTER(GcpParams), POINTER(c_size_t)]),
    "gcp_stream_init": (c_int32, [POINTER(GcpParams), POINTER(c_void_p), c_int32,
                                  POINTER(GcpSlice), c_void_p, POINTER(c_int64),
                                  c_void_p, c_size_t, c_void_p, POINTER(c_void_p)]),
    "gcp_loss_grad": (c_int32, [c_void_p, POINTER(GcpSlice), POINTER(c_void_p), c_void_p,
                                c_uint32, c_void_p, POINTER(c_void_p), c_void_p]),
    "gcp_loss_grad_scaled": (c_int32, [c_void_p, POINTER(GcpSlice), POINTER(c_void_p), c_void_p,
                                       c_uint32, c_void_p, c_void_p, POINTER(c_void_p), c_void_p]),
    "gcp_solve_st": (c_int32, [c_void_p, POINTER(GcpSlice), c_void_p]),
    "gcp_solve_st_info": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_int64),
                                    POINTER(c_int32), POINTER(c_uint64)]),
    "gcp_update_factors": (c_int32, [c_void_p, POINTER(GcpSlice), c_void_p]),
    "gcp_factor_info": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_double), POINTER(c_int64),
                                  POINTER(c_int32), POINTER(c_uint64)]),
    "gcp_slice_loss": (c_int32, [c_void_p, POINTER(GcpSlice), c_void_p, POINTER(c_double), POINTER(c_double)]),
    "gcp_local_loss": (c_int32, [c_void_p, POINTER(GcpSlice), c_void_p, POINTER(c_double)]),
    "gcp_ktensor_score": (c_int32, [c_void_p, c_void_p, POINTER(c_void_p), c_void_p, c_int32, POINTER(c_double)]),
    "gcp_get_factors": (c_int32, [c_void_p, POINTER(c_void_p)]),
    "gcp_factor_ptr": (c_int32, [c_void_p, c_int32, POINTER(c_void_p)]),
    "gcp_stream_info": (c_int32, [c_void_p, POINTER(c_int64), POINTER(c_int32),
                                  POINTER(c_int64), POINTER(c_int64), POINTER(c_int64)]),
    "gcp_stream_sync": (c_int32, [c_void_p]),
    "gcp_stream_destroy": (c_int32, [c_void_p]),
    "gcp_autotune": (c_int32, [c_void_p, POINTER(GcpSlice), c_char_p, POINTER(c_int32)]),
    "gcp_loss_grad_static": (c_int32, [POINTER(GcpParams), POINTER(GcpSlice), c_int32, c_void_p, c_void_p,
                                       POINTER(c_int64), c_int64, POINTER(c_void_p), c_void_p, c_uint32,
                                       c_void_p, POINTER(c_void_p), c_void_p, c_void_p]),
    "gcp_probe_gather": (c_int32, [c_void_p, c_void_p, c_void_p, c_int64, c_int64, c_int64, c_int32, c_int64,
                                   c_uint64, c_void_p, c_void_p]),
    "gcp_batch_autotune": (c_int32, [POINTER(c_void_p), POINTER(GcpBatchIO), c_int32, c_char_p,
                                     POINTER(c_int32)]),
    "gcp_batch_workspace_size": (c_int32, [POINTER(c_void_p), c_int32, POINTER(c_size_t)]),
    "gcp_batch_create": (c_int32, [POINTER(c_void_p), POINTER(GcpBatchIO), c_int32, c_void_p,
                                   c_size_t, c_void_p, POINTER(c_void_p)]),
    "gcp_batch_loss_grad": (c_int32, [c_void_p, c_uint32]),
    "gcp_batch_update_factors": (c_int32, [c_void_p]),
    "gcp_batch_solve_st": (c_int32, [c_void_p]),
    "gcp_batch_step": (c_int32, [c_void_p]),
    "gcp_batch_sync_streams": (c_int32, [c_void_p]),
    "gcp_batch_destroy": (c_int32, [c_void_p]),
    "gcp_kernel_timing": (c_int32, [c_void_p, c_int32, c_int32]),
    "gcp_kernel_time": (c_int32, [c_void_p, POINTER(c_double), POINTER(c_int64)]),
    "gcp_dump_samples": (c_int32, [c_void_p, POINTER(GcpSlice), c_int32, c_int64, c_void_p, c_void_p,
                                   c_int64, POINTER(c_int64)]),
    "gcp_status_string": (c_char_p, [c_int32]),
}

_lib = None


class GcpError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        name = STATUS_NAMES[status] if 0 <= status < len(STATUS_NAMES) else str(status)
        super().__init__(f"{where}: {name}")


def load(path: str = LIB_PATH):
    """Loads the HIP library and declares every exported call.  Raises if the
    library is missing: build it first (python -m paper_2110_14514_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"gcpstream HIP library not found at {path}; build it with "
            "`python -m paper_2110_14514_amd.build` (there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int, where: str):
    if status != OK:
        raise GcpError(status, where)
