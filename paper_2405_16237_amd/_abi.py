"""ctypes mirror of include/nbvh.h and loader of the in-tree libnbvh.so.

Argument marshalling only: every step of the neural query and the training
step runs in the library's HIP kernels. Importing this module fails loudly
when the shared library has not been built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnbvh.so")

NBVH_OK, NBVH_ERR_INVALID_ARG, NBVH_ERR_CAPACITY, NBVH_ERR_NOT_BOUND, NBVH_ERR_HIP, NBVH_ERR_UNSUPPORTED = range(6)
NBVH_FP32, NBVH_BF16, NBVH_FP8 = 0, 1, 2
NBVH_FLAG_CAPACITY, NBVH_FLAG_NONFINITE = 1, 2
NBVH_MAX_LEVELS = 32
NBVH_MISS = 0xFFFFFFFF
NBVH_INSIDE_CLIP, NBVH_INSIDE_REVERSE = 0, 1
NBVH_SEG_INSIDE = 0x80000000
(NBVH_BUF_PARAMS, NBVH_BUF_PARAMS_LP, NBVH_BUF_ADAM_M, NBVH_BUF_ADAM_V, NBVH_BUF_GRAD, NBVH_BUF_STATE,
 NBVH_BUF_AUX) = range(7)

STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "CAPACITY", 3: "NOT_BOUND", 4: "HIP", 5: "UNSUPPORTED"}


class NbvhConfig(ctypes.Structure):
    _fields_ = [
        ("n_levels", ctypes.c_int32), ("n_features", ctypes.c_int32), ("log2_T", ctypes.c_int32),
        ("n_samples", ctypes.c_int32), ("level_res", ctypes.c_int32 * NBVH_MAX_LEVELS),
        ("mlp_width", ctypes.c_int32), ("mlp_hidden", ctypes.c_int32), ("n_out", ctypes.c_int32),
        ("precision", ctypes.c_int32), ("scene_lo", ctypes.c_float * 3), ("scene_side", ctypes.c_float),
        ("w_hit", ctypes.c_float), ("w_t", ctypes.c_float), ("w_normal", ctypes.c_float), ("w_albedo", ctypes.c_float),
        ("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
        ("loss_scale", ctypes.c_float), ("inside_rule", ctypes.c_int32),
    ]


class NbvhParams(ctypes.Structure):
    _fields_ = [("params_dev", ctypes.c_void_p), ("params_lp_dev", ctypes.c_void_p), ("adam_m_dev", ctypes.c_void_p),
                ("adam_v_dev", ctypes.c_void_p), ("grad_dev", ctypes.c_void_p), ("state_dev", ctypes.c_void_p),
                ("aux_dev", ctypes.c_void_p)]


NBVH_K_COUNT = 9
KERNEL_GROUPS = ["traverse", "query_eval", "forward", "train_tile", "wgrad", "scatter", "optimizer", "scatter_sort",
                 "scatter_reduce"]


class NbvhProfile(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * NBVH_K_COUNT), ("calls", ctypes.c_int64 * NBVH_K_COUNT)]


class NbvhTuning(ctypes.Structure):
    _fields_ = [("query_waves", ctypes.c_int32), ("query_unroll", ctypes.c_int32), ("query_wgs_per_cu", ctypes.c_int32),
                ("train_waves", ctypes.c_int32), ("wgrad_splits", ctypes.c_int32), ("scatter_lds_kb", ctypes.c_int32),
                ("scatter_binned", ctypes.c_int32), ("scatter_hash_levels", ctypes.c_int32),
                ("query_pairs", ctypes.c_int32), ("query_lds_kb", ctypes.c_int32),
                ("traverse_mode", ctypes.c_int32), ("query_order", ctypes.c_int32)]


class NbvhQueryTrace(ctypes.Structure):
    _fields_ = [("seg_offsets_dev", ctypes.c_void_p), ("segs_dev", ctypes.c_void_p), ("z_dev", ctypes.c_void_p),
                ("u_dev", ctypes.c_void_p)]


class NbvhStateHost(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("skipped", ctypes.c_int64), ("loss_scale", ctypes.c_float),
                ("flags", ctypes.c_uint32), ("last_loss", ctypes.c_float * 4), ("last_n_segments", ctypes.c_uint64),
                ("n_evaluated", ctypes.c_uint64)]


# every entry point declared in include/nbvh.h
EXPORTS = [
    "nbvh_param_count", "nbvh_param_layout", "nbvh_aux_bytes", "nbvh_nodes_bytes", "nbvh_state_bytes", "nbvh_build",
    "nbvh_bind_params", "nbvh_reset_optimizer", "nbvh_sync_shadow", "nbvh_calibrate_fp8", "nbvh_workspace_bytes",
    "nbvh_traverse",
    "nbvh_query", "nbvh_query_noalloc", "nbvh_query_traced", "nbvh_query_segments", "nbvh_first_hits", "nbvh_group_ws_bytes", "nbvh_group_by_leaf", "nbvh_leaf_loss", "nbvh_node_rank", "nbvh_acceptance", "nbvh_encode", "nbvh_forward", "nbvh_backward", "nbvh_optimizer_step",
    "nbvh_train_step", "nbvh_loss", "nbvh_batch_desc_bytes", "nbvh_batch_create", "nbvh_batch_workspace_bytes",
    "nbvh_batch_query", "nbvh_batch_destroy", "nbvh_get_tuning", "nbvh_set_tuning", "nbvh_profile_begin", "nbvh_profile_end", "nbvh_read_state", "nbvh_device_status", "nbvh_param_bytes", "nbvh_unscaled_grad", "nbvh_clear_flags", "nbvh_last_error", "nbvh_version",
    "nbvh_destroy",
]

_lib = None


class NbvhError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("nbvh error %s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def load(path: str = LIB_PATH):
    """Load libnbvh.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libnbvh.so is not built (%s); run paper_2405_16237_amd/build.py" % path)
    L = ctypes.CDLL(path)
    P, U64, SZ, I = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_int
    st = ctypes.c_int
    sig = {
        "nbvh_param_count": (st, [P, P, P]),
        "nbvh_param_layout": (st, [P, P]),
        "nbvh_aux_bytes": (SZ, [P]),
        "nbvh_nodes_bytes": (SZ, [ctypes.c_uint32]),
        "nbvh_state_bytes": (SZ, []),
        "nbvh_build": (st, [P, P, ctypes.c_uint32, P, SZ, P, P]),
        "nbvh_bind_params": (st, [P, P]),
        "nbvh_reset_optimizer": (st, [P, P]),
        "nbvh_sync_shadow": (st, [P, P]),
        "nbvh_calibrate_fp8": (st, [P, P, U64, P]),
        "nbvh_workspace_bytes": (SZ, [P, U64, U64, U64]),
        "nbvh_traverse": (st, [P, P, U64, P, P, U64, P, SZ, P]),
        "nbvh_query": (st, [P, P, U64, P, U64, P, SZ, P]),
        "nbvh_query_traced": (st, [P, P, U64, P, U64, P, SZ, P, P]),
        "nbvh_query_noalloc": (st, [P, P, U64, P, U64, P]),
        "nbvh_query_segments": (st, [P, P, U64, P, P, P, P, SZ, P]),
        "nbvh_encode": (st, [P, P, U64, P, P]),
        "nbvh_first_hits": (st, [P, P, U64, P, P, P, P, P, P, P]),
        "nbvh_group_ws_bytes": (SZ, [U64]),
        "nbvh_group_by_leaf": (st, [P, P, P, U64, P, P, P, SZ, P]),
        "nbvh_leaf_loss": (st, [P, P, P, P, U64, P, P, P, SZ, P]),
        "nbvh_node_rank": (st, [P, P, P, ctypes.c_uint32, U64, P, P]),
        "nbvh_acceptance": (st, [P, ctypes.c_uint32, ctypes.c_float, P, P]),
        "nbvh_forward": (st, [P, P, U64, P, P, SZ, P]),
        "nbvh_backward": (st, [P, P, U64, P, P, SZ, P]),
        "nbvh_optimizer_step": (st, [P, P]),
        "nbvh_train_step": (st, [P, P, P, U64, P, P, SZ, P]),
        "nbvh_loss": (st, [P, P, P, U64, P, P, P, SZ, P]),
        "nbvh_batch_desc_bytes": (SZ, [ctypes.c_uint32]),
        "nbvh_batch_create": (st, [P, ctypes.c_uint32, P, SZ, P, P]),
        "nbvh_batch_workspace_bytes": (SZ, [P, U64, U64]),
        "nbvh_batch_query": (st, [P, P, U64, P, U64, P, SZ, P]),
        "nbvh_batch_destroy": (None, [P]),
        "nbvh_get_tuning": (st, [P, P]),
        "nbvh_set_tuning": (st, [P, P]),
        "nbvh_profile_begin": (st, [P]),
        "nbvh_profile_end": (st, [P, P]),
        "nbvh_read_state": (st, [P, P, P]),
        "nbvh_clear_flags": (st, [P, P]),
        "nbvh_device_status": (st, [P, P, P]),
        "nbvh_param_bytes": (SZ, [P, ctypes.c_int]),
        "nbvh_unscaled_grad": (st, [P, P, ctypes.c_int, P]),
        "nbvh_last_error": (ctypes.c_char_p, []),
        "nbvh_version": (ctypes.c_char_p, []),
        "nbvh_destroy": (None, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status: int):
    if status != NBVH_OK:
        raise NbvhError(status, _lib.nbvh_last_error().decode())
