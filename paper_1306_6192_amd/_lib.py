"""ctypes binding of ``libmi355gemm.so`` (argument marshalling only).

Every entry point of ``include/mi355gemm.h`` is bound here under the same
name; the arithmetic all happens in the library's gfx950 kernels.  If the
library has not been built, :func:`load` raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import (POINTER, Structure, c_char_p, c_float, c_int32, c_int64, c_uint64, c_uint8,
                    c_void_p, c_double)

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libmi355gemm.so")
TUNING_TABLE = os.path.join(PKG, "tuning", "mi355x.jsonl")

GEMM_OK = 0
GEMM_PENDING = 1
GEMM_EINVAL = -1
GEMM_EUNSUPPORTED = -2
GEMM_ENOMEM = -3
GEMM_EHIP = -4
GEMM_EBUSY = -5
GEMM_ENOTFOUND = -6
GEMM_EINTERNAL = -7
NOALLOC_SCRATCH_BYTES = 64 << 20   # GEMM_NOALLOC_SCRATCH_BYTES

MODE_F32 = 0
MODE_BF16 = 1
MODE_F16 = 2
MODE_F8E4M3 = 3
MODE_SPLIT_BF16X3 = 4
MODE_F64 = 5   # kernel family of gemm_plain_f64 (not a problem mode)
MODE_C32 = 6   # kernel family of gemm_plain_c32 (not a problem mode)
NUM_MODES = 5
NUM_KERNEL_FAMILIES = 7
MODE_NAMES = {MODE_F32: "f32", MODE_BF16: "bf16", MODE_F16: "f16", MODE_F8E4M3: "e4m3",
              MODE_SPLIT_BF16X3: "split_bf16x3", MODE_F64: "f64", MODE_C32: "c32"}
ELEM_SIZE = {MODE_F32: 4, MODE_BF16: 2, MODE_F16: 2, MODE_F8E4M3: 1, MODE_SPLIT_BF16X3: 4}


class GemmProblem(Structure):
    _fields_ = [("mode", c_int32), ("flags", c_int32),
                ("m", c_int64), ("n", c_int64), ("k", c_int64),
                ("A", c_void_p), ("lda", c_int64),
                ("B", c_void_p), ("ldb", c_int64),
                ("C", c_void_p), ("ldc", c_int64),
                ("scale_a", c_float), ("scale_b", c_float)]


class ServeConfig(Structure):
    _fields_ = [("hbm_budget_bytes", c_uint64), ("max_inflight", c_int32), ("num_streams", c_int32),
                ("max_batch", c_int32), ("queue_capacity", c_int32), ("executor", c_int32),
                ("fake_fail_every", c_int32)]


class ServeResult(Structure):
    _fields_ = [("status", c_int32), ("batch_size", c_int32),
                ("t_arrival_ns", c_uint64), ("t_admit_ns", c_uint64),
                ("t_launch_ns", c_uint64), ("t_done_ns", c_uint64)]


class ServeStats(Structure):
    _fields_ = [("submitted", c_uint64), ("completed", c_uint64), ("failed", c_uint64),
                ("batches", c_uint64), ("inflight_bytes", c_uint64), ("peak_inflight_bytes", c_uint64),
                ("queued", c_int32), ("inflight", c_int32)]


class GemmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_P = POINTER(GemmProblem)
_SIGS = {
    "gemm_plain": (c_int32, [_P, c_void_p]),
    "gemm_plain_cfg": (c_int32, [_P, c_int32, c_int32, c_void_p]),
    "gemm_plain_workspace_bytes": (c_int32, [_P, POINTER(c_uint64)]),
    "gemm_plain_noalloc": (c_int32, [_P, c_void_p]),
    "gemm_ablation": (c_int32, [_P, c_int32, c_void_p]),
    "gemm_plain_f64": (c_int32, [c_int64, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_int64, c_void_p,
                                 c_int64, c_void_p]),
    "gemm_plain_f64_cfg": (c_int32, [c_int64, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_int64, c_void_p,
                                     c_int64, c_int32, c_void_p]),
    "gemm_plain_c32": (c_int32, [c_int64, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_int64, c_void_p,
                                 c_int64, c_void_p]),
    "gemm_plain_c32_cfg": (c_int32, [c_int64, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_int64, c_void_p,
                                     c_int64, c_int32, c_void_p]),
    "gemm_add": (c_int32, [c_int32, c_int32, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_int64, c_void_p,
                           c_int64, c_void_p]),
    "gemm_num_configs": (c_int32, [c_int32]),
    "gemm_config_info": (c_int32, [c_int32, c_int32, POINTER(c_int32)]),
    "gemm_config_chunk": (c_int32, [c_int32, c_int32]),
    "gemm_convert_f32": (c_int32, [c_void_p, c_int64, c_int32, c_void_p, c_void_p]),
    "gemm_quantize_e4m3": (c_int32, [c_void_p, c_int64, c_void_p, c_void_p, c_void_p]),
    "gemm_errnorm": (c_int32, [c_void_p, c_int64, c_void_p, c_int64, c_int64, c_int64, c_void_p, c_void_p]),
    "gemm_grouped": (c_int32, [_P, c_int32, c_void_p]),
    "gemm_grouped_graph_create": (c_int32, [_P, c_int32, POINTER(c_void_p)]),
    "gemm_grouped_info": (c_int32, [c_int32, POINTER(c_int32)]),
    "gemm_grouped_lookup": (c_int32, [c_int32, c_int64, c_int64, c_int64, POINTER(c_int32)]),
    "gemm_grouped_plan": (c_int32, [_P, c_int32, POINTER(c_int32)]),
    "gemm_grouped_schedule": (c_int32, [_P, c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                        POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)]),
    "gemm_graph_launch": (c_int32, [c_void_p, c_void_p]),
    "gemm_graph_destroy": (c_int32, [c_void_p]),
    "gemm_tune": (c_int32, [c_int32, c_int64, c_int64, c_int64, c_void_p]),
    "gemm_tune_bucket": (c_int32, [c_int32, c_int64, c_int64, c_int64, c_void_p]),
    "gemm_tune_grouped": (c_int32, [c_int32, c_int64, c_int64, c_int64, c_void_p]),
    "gemm_tune_grouped_mix": (c_int32, [_P, c_int32, c_void_p]),
    "gemm_tuner_lookup": (c_int32, [c_int32, c_int64, c_int64, c_int64, POINTER(c_int32), POINTER(c_int32)]),
    "gemm_tuner_load": (c_int32, [c_char_p]),
    "gemm_tuner_save": (c_int32, [c_char_p]),
    "gemm_serve_footprint": (c_int32, [_P, POINTER(c_uint64)]),
    "gemm_serve_create": (c_int32, [POINTER(ServeConfig), POINTER(c_void_p)]),
    "gemm_serve_submit": (c_int32, [c_void_p, _P, c_uint64, POINTER(c_uint64)]),
    "gemm_serve_poll": (c_int32, [c_void_p, c_uint64, POINTER(ServeResult)]),
    "gemm_serve_drain": (c_int32, [c_void_p]),
    "gemm_serve_replay": (c_int32, [c_void_p, _P, POINTER(c_uint64), c_int32, POINTER(c_uint64)]),
    "gemm_serve_stats": (c_int32, [c_void_p, POINTER(ServeStats)]),
    "gemm_serve_destroy": (c_int32, [c_void_p]),
    "gemm_now_ns": (c_uint64, []),
    "gemm_last_error": (c_char_p, []),
    "gemm_version": (c_int32, []),
}

_lib = None


def load():
    """Load the built library (raises if it is missing: no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                              "or python paper_1306_6192_amd/build.py")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        # the measured tuning table shipped with the package (MI355X), unless
        # the environment names another one
        table = os.environ.get("MI355GEMM_TUNE_FILE") or TUNING_TABLE
        if os.path.exists(table):
            lib.gemm_tuner_load(table.encode())
        _lib = lib
    return _lib


def last_error() -> str:
    return (load().gemm_last_error() or b"").decode(errors="replace")


def check(rc: int) -> int:
    if rc < 0:
        raise GemmError(rc, last_error())
    return rc


def problem(mode, m, n, k, A, lda, B, ldb, C, ldc, scale_a=1.0, scale_b=1.0, flags=0) -> GemmProblem:
    return GemmProblem(int(mode), int(flags), int(m), int(n), int(k), A, int(lda), B, int(ldb), C, int(ldc),
                       float(scale_a), float(scale_b))


def problems_array(probs):
    arr = (GemmProblem * max(1, len(probs)))()
    for i, p in enumerate(probs):
        arr[i] = p
    return arr
