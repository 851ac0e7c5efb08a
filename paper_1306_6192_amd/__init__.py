"""mi355gemm: dense C = A*B on AMD Instinct MI355X (gfx950).

A thin Python layer over the C-ABI library ``libmi355gemm.so``: it checks
tensor shapes, fills the problem structs and passes device pointers and the
current HIP stream.  All arithmetic runs in the library's HIP kernels;
PyTorch only provides device memory and streams.
"""
from __future__ import annotations

import ctypes

from . import _lib
from ._lib import (GEMM_EBUSY, GEMM_EINVAL, GEMM_ENOMEM, GEMM_EUNSUPPORTED, GEMM_OK, GEMM_PENDING,
                   MODE_BF16, MODE_C32, MODE_F8E4M3, MODE_F16, MODE_F32, MODE_F64, MODE_NAMES, MODE_SPLIT_BF16X3,
                   GemmError, check, load)

__all__ = ["gemm", "gemm_f64", "gemm_c32", "add", "convert", "quantize_e4m3", "errnorm", "grouped", "ProblemBatch",
           "GroupedGraph", "Server", "tune",
           "tuner_lookup", "config_info", "num_configs", "GemmError", "MODE_F32", "MODE_BF16", "MODE_F16",
           "MODE_F8E4M3", "MODE_SPLIT_BF16X3", "MODE_F64", "MODE_C32", "MODE_NAMES", "load"]


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dtype_ok(t, mode) -> bool:
    torch = _torch()
    want = {MODE_F32: (torch.float32,), MODE_SPLIT_BF16X3: (torch.float32,),
            MODE_BF16: (torch.bfloat16, torch.int16, torch.uint16),
            MODE_F16: (torch.float16, torch.int16, torch.uint16),
            MODE_F8E4M3: (torch.float8_e4m3fn, torch.uint8, torch.int8)}[mode]
    return t.dtype in want


def _check_mat(t, name, mode=None):
    if t.dim() != 2:
        raise ValueError(f"{name} must be 2-D")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.size(0) > 0 and t.size(1) > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must be row-major (unit column stride)")
    if mode is not None and not _dtype_ok(t, mode):
        raise TypeError(f"{name} has dtype {t.dtype}, not valid for mode {MODE_NAMES[mode]}")


def _ld(t):
    return max(1, t.stride(0) if t.size(0) > 1 else t.size(1))


def make_problem(A, B, C, mode=MODE_F32, scale_a=1.0, scale_b=1.0):
    m, k = A.shape
    n = B.shape[1]
    return _lib.problem(mode, m, n, k, A.data_ptr() or None, _ld(A), B.data_ptr() or None, _ld(B),
                        C.data_ptr() or None, _ld(C), scale_a, scale_b)


def gemm(A, B, out=None, mode=MODE_F32, scale_a=1.0, scale_b=1.0, cfg=None, split_k=None, stream=None):
    """C = A @ B (float32 result) for device matrices A (m x k) and B (k x n).

    ``mode`` selects the arithmetic form; A and B must hold the matching
    element type (float32, bfloat16, float16 or E4M3 codes).  ``cfg`` and
    ``split_k`` override the tuning table."""
    torch = _torch()
    _check_mat(A, "A", mode)
    _check_mat(B, "B", mode)
    if A.shape[1] != B.shape[0]:
        raise ValueError(f"inner dimensions differ: {tuple(A.shape)} @ {tuple(B.shape)}")
    m, n = A.shape[0], B.shape[1]
    if out is None:
        out = torch.empty((m, n), dtype=torch.float32, device=A.device)
    _check_mat(out, "out")
    if out.dtype != torch.float32 or tuple(out.shape) != (m, n):
        raise ValueError("out must be float32 of shape (m, n)")
    p = make_problem(A, B, out, mode, scale_a, scale_b)
    lib = load()
    if cfg is None and split_k is None:
        check(lib.gemm_plain(ctypes.byref(p), _stream_ptr(stream)))
    else:
        if cfg is None or split_k is None:
            c, s = tuner_lookup(mode, m, n, A.shape[1])
            cfg = c if cfg is None else cfg
            split_k = s if split_k is None else split_k
        check(lib.gemm_plain_cfg(ctypes.byref(p), int(cfg), int(split_k), _stream_ptr(stream)))
    return out


def _gemm_same_type(A, B, out, dtype, entry, cfg, stream):
    torch = _torch()
    for t, name in ((A, "A"), (B, "B")):
        _check_mat(t, name)
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if A.shape[1] != B.shape[0]:
        raise ValueError(f"inner dimensions differ: {tuple(A.shape)} @ {tuple(B.shape)}")
    m, k = A.shape
    n = B.shape[1]
    if out is None:
        out = torch.empty((m, n), dtype=dtype, device=A.device)
    _check_mat(out, "out")
    if out.dtype != dtype or tuple(out.shape) != (m, n):
        raise ValueError(f"out must be {dtype} of shape (m, n)")
    lib = load()
    args = (m, n, k, A.data_ptr() or None, _ld(A), B.data_ptr() or None, _ld(B), out.data_ptr() or None, _ld(out))
    if cfg is None:
        check(getattr(lib, entry)(*args, _stream_ptr(stream)))
    else:
        check(getattr(lib, entry + "_cfg")(*args, int(cfg), _stream_ptr(stream)))
    return out


def gemm_f64(A, B, out=None, cfg=None, stream=None):
    """C = A @ B in binary64 for float64 device matrices (gemm_plain_f64)."""
    return _gemm_same_type(A, B, out, _torch().float64, "gemm_plain_f64", cfg, stream)


def gemm_c32(A, B, out=None, cfg=None, stream=None):
    """C = A @ B over complex float for complex64 device matrices
    (gemm_plain_c32; four real float32 products per complex term)."""
    return _gemm_same_type(A, B, out, _torch().complex64, "gemm_plain_c32", cfg, stream)


def add(A, B, out=None, subtract=False, stream=None):
    """C = A + B (or A - B) element-wise for float32 or float64 device
    matrices (gemm_add); ``out`` may be A or B for an in-place update."""
    torch = _torch()
    for t, name in ((A, "A"), (B, "B")):
        _check_mat(t, name)
    if A.dtype != B.dtype or A.dtype not in (torch.float32, torch.float64):
        raise TypeError("A and B must both be float32 or both float64")
    if A.shape != B.shape:
        raise ValueError(f"shapes differ: {tuple(A.shape)} vs {tuple(B.shape)}")
    if out is None:
        out = torch.empty_like(A)
    _check_mat(out, "out")
    if out.dtype != A.dtype or out.shape != A.shape:
        raise ValueError("out must match A in dtype and shape")
    m, n = A.shape
    dtype = MODE_F64 if A.dtype == torch.float64 else MODE_F32
    check(load().gemm_add(dtype, 1 if subtract else 0, m, n, A.data_ptr() or None, _ld(A), B.data_ptr() or None,
                          _ld(B), out.data_ptr() or None, _ld(out), _stream_ptr(stream)))
    return out


def paper_kernel(A, B, out=None, variant=1, stream=None):
    """C = A @ B (float32) with the paper's kernels rebuilt for gfx950:
    variant 0 = global-memory thread-per-element, 1 = 16x16 LDS tiles."""
    torch = _torch()
    _check_mat(A, "A", MODE_F32)
    _check_mat(B, "B", MODE_F32)
    if A.shape[1] != B.shape[0]:
        raise ValueError("inner dimensions differ")
    m, n = A.shape[0], B.shape[1]
    if out is None:
        out = torch.empty((m, n), dtype=torch.float32, device=A.device)
    p = make_problem(A, B, out, MODE_F32)
    check(load().gemm_ablation(ctypes.byref(p), int(variant), _stream_ptr(stream)))
    return out


def convert(x, mode, stream=None):
    """float32 -> bfloat16 / float16 codes (RNE), as a tensor of that dtype."""
    torch = _torch()
    if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous float32 device tensor")
    dt = {MODE_BF16: torch.bfloat16, MODE_F16: torch.float16}[mode]
    out = torch.empty(x.shape, dtype=dt, device=x.device)
    check(load().gemm_convert_f32(x.data_ptr() or None, x.numel(), mode, out.data_ptr() or None,
                                  _stream_ptr(stream)))
    return out


def quantize_e4m3(x, stream=None):
    """Per-tensor E4M3 quantisation: returns (codes uint8, scale float32 device tensor of 1)."""
    torch = _torch()
    if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous float32 device tensor")
    q = torch.empty(x.shape, dtype=torch.uint8, device=x.device)
    s = torch.empty(1, dtype=torch.float32, device=x.device)
    check(load().gemm_quantize_e4m3(x.data_ptr() or None, x.numel(), q.data_ptr() or None, s.data_ptr(),
                                    _stream_ptr(stream)))
    return q, s


def errnorm(C, R, stream=None):
    """(sum (C-R)^2, sum R^2, max|C-R|) in binary64, computed on the device.
    Returns a float64 device tensor of 3."""
    torch = _torch()
    _check_mat(C, "C")
    _check_mat(R, "R")
    if C.dtype != torch.float32 or R.dtype != torch.float64 or C.shape != R.shape:
        raise ValueError("C float32 and R float64 of equal shape expected")
    out = torch.empty(3, dtype=torch.float64, device=C.device)
    m, n = C.shape
    check(load().gemm_errnorm(C.data_ptr() or None, _ld(C), R.data_ptr() or None, _ld(R), m, n,
                              out.data_ptr(), _stream_ptr(stream)))
    return out


def num_configs(mode) -> int:
    return check(load().gemm_num_configs(mode))


def config_info(mode, cfg) -> dict:
    info = (ctypes.c_int32 * 6)()
    check(load().gemm_config_info(mode, cfg, info))
    return dict(zip(("BM", "BN", "BK", "waves", "lds_bytes", "mfma_k"), list(info)))


def config_chunk(mode, cfg) -> int:
    """Elements per 16-byte chunk a configuration copies straight into LDS,
    or 0 for a register-staged configuration (gemm_config_chunk)."""
    return check(load().gemm_config_chunk(mode, cfg))


def tuner_lookup(mode, m, n, k):
    c = ctypes.c_int32()
    s = ctypes.c_int32()
    check(load().gemm_tuner_lookup(mode, m, n, k, ctypes.byref(c), ctypes.byref(s)))
    return c.value, s.value


def tune(mode, m, n, k, stream=None):
    check(load().gemm_tune(mode, m, n, k, _stream_ptr(stream)))
    return tuner_lookup(mode, m, n, k)


def grouped(problems, mode=MODE_F32, stream=None):
    """Run many products in one persistent launch.  ``problems`` is a list of
    (A, B, C) device tensors (all of one mode); FP8 entries may be
    (A, B, C, scale_a, scale_b), or a :class:`ProblemBatch` built once."""
    batch = problems if isinstance(problems, ProblemBatch) else ProblemBatch(problems, mode)
    batch.run(stream)


class ProblemBatch:
    """A list of (A, B, C) device tensors turned once into the C-ABI problem
    array, so that repeated grouped launches of the same problems pay no
    per-problem Python cost (the tensors are kept alive with it)."""

    def __init__(self, problems, mode=MODE_F32):
        probs = [make_problem(t[0], t[1], t[2], mode, *(t[3:5] if len(t) >= 5 else (1.0, 1.0)))
                 for t in problems]
        self._keep = problems
        self.count = len(probs)
        self.array = _lib.problems_array(probs)

    def run(self, stream=None):
        check(load().gemm_grouped(self.array, self.count, _stream_ptr(stream)))


class GroupedGraph:
    """A captured grouped launch, replayed with :meth:`launch`."""

    def __init__(self, problems, mode=MODE_F32):
        probs = [make_problem(t[0], t[1], t[2], mode, *(t[3:5] if len(t) >= 5 else (1.0, 1.0)))
                 for t in problems]
        self._keep = problems          # the graph holds raw pointers into these tensors
        arr = _lib.problems_array(probs)
        h = ctypes.c_void_p()
        check(load().gemm_grouped_graph_create(arr, len(probs), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        check(load().gemm_graph_launch(self._h, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(load().gemm_graph_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching product server (see gemm_serve_* in the header)."""

    def __init__(self, hbm_budget_bytes=8 << 30, max_inflight=256, num_streams=4, max_batch=64,
                 queue_capacity=100000, executor=0, fake_fail_every=0):
        cfg = _lib.ServeConfig(hbm_budget_bytes, max_inflight, num_streams, max_batch, queue_capacity,
                               executor, fake_fail_every)
        h = ctypes.c_void_p()
        check(load().gemm_serve_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h

    def submit(self, prob, t_arrival_ns=0):
        t = ctypes.c_uint64()
        rc = load().gemm_serve_submit(self._h, ctypes.byref(prob), int(t_arrival_ns), ctypes.byref(t))
        return rc, t.value

    def poll(self, ticket):
        r = _lib.ServeResult()
        rc = load().gemm_serve_poll(self._h, int(ticket), ctypes.byref(r))
        return rc, r

    def drain(self):
        check(load().gemm_serve_drain(self._h))

    def stats(self):
        s = _lib.ServeStats()
        check(load().gemm_serve_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in _lib.ServeStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(load().gemm_serve_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def now_ns() -> int:
    return int(load().gemm_now_ns())
