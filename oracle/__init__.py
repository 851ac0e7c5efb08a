"""The oracle: a plain, slow, obviously correct CPU implementation of what the
GPU library computes.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  The product library (the HIP
kernels and their C-ABI) never calls it, links it or shares code with it.

Contents, each following the paper or a public definition:

* :func:`gemm` -- c_ij = sum_r a_ir b_rj in binary64 (Implementation section,
  the product equation; summation order of Listing 1), by the C loop in
  ``gemm_f64.c``.  Inputs are promoted exactly to binary64.
* :func:`gemm_sampled` -- the same definition for selected (i, j) only.
* :func:`gemm_fp8` / :func:`gemm_split_bf16x3` -- the products the reduced
  precision forms compute, on their quantised operands, in binary64.
* :func:`gemm_dot2` -- the same definition evaluated with the compensated dot
  product (twice binary64 precision, then rounded): the reference for a
  binary64 product.
* :func:`gemm_c128` -- the complex product (Results section, Table 2's
  complex column) on interleaved (re, im) binary64 pairs.
* :func:`add` -- the element-wise sum or difference of two matrices (Results
  section, the addition/subtraction algorithm of Fig. 9).
* :func:`relerr` -- the normwise relative error ||C - R||_F / ||R||_F.
* ``formats`` -- RNE conversions to bfloat16, binary16 and OCP E4M3.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import formats  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_gemm_f64.so")
_lib = None

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int64)


def default_threads() -> int:
    return len(os.sched_getaffinity(0))


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.oracle_gemm_f64.argtypes = [_i64, _i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64, ctypes.c_int]
        lib.oracle_gemm_f64.restype = None
        lib.oracle_gemm_f64_sampled.argtypes = [_i64, _ip, _ip, _i64, _dp, _i64, _dp, _i64, _dp, ctypes.c_int]
        lib.oracle_gemm_f64_sampled.restype = None
        for name in ("oracle_gemm_dot2", "oracle_gemm_c128"):
            getattr(lib, name).argtypes = [_i64, _i64, _i64, _dp, _i64, _dp, _i64, _dp, _i64, ctypes.c_int]
            getattr(lib, name).restype = None
        for name in ("oracle_gemm_dot2_sampled", "oracle_gemm_c128_sampled"):
            getattr(lib, name).argtypes = [_i64, _ip, _ip, _i64, _dp, _i64, _dp, _i64, _dp, ctypes.c_int]
            getattr(lib, name).restype = None
        _lib = lib
    return _lib


def _as_f64(x) -> np.ndarray:
    x = np.asarray(x)
    if x.dtype not in (np.float64, np.float32, np.float16) and not np.issubdtype(x.dtype, np.integer):
        raise TypeError(f"oracle takes float or integer arrays, got {x.dtype}")
    return np.ascontiguousarray(x, dtype=np.float64)


def gemm(A, B, threads: int | None = None) -> np.ndarray:
    """C = A @ B by the definition, every c_ij summed in ascending r in binary64."""
    A = _as_f64(A)
    B = _as_f64(B)
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError(f"shape mismatch {A.shape} @ {B.shape}")
    m, k = A.shape
    n = B.shape[1]
    C = np.empty((m, n), dtype=np.float64)
    if m and n:
        _load().oracle_gemm_f64(m, n, k,
                                A.ctypes.data_as(_dp), max(k, 1),
                                B.ctypes.data_as(_dp), max(n, 1),
                                C.ctypes.data_as(_dp), n,
                                threads or default_threads())
    return C


def gemm_sampled(A, B, rows, cols, threads: int | None = None) -> np.ndarray:
    """c_ij for the listed (rows[t], cols[t]) pairs, same definition and order."""
    A = _as_f64(A)
    B = _as_f64(B)
    m, k = A.shape
    n = B.shape[1]
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    if rows.shape != cols.shape or rows.ndim != 1:
        raise ValueError("rows and cols must be 1-D and of equal length")
    if rows.size and (rows.min() < 0 or rows.max() >= m or cols.min() < 0 or cols.max() >= n):
        raise IndexError("sample index out of range")
    out = np.empty(rows.size, dtype=np.float64)
    if rows.size:
        _load().oracle_gemm_f64_sampled(rows.size, rows.ctypes.data_as(_ip), cols.ctypes.data_as(_ip), k,
                                        A.ctypes.data_as(_dp), max(k, 1),
                                        B.ctypes.data_as(_dp), max(n, 1),
                                        out.ctypes.data_as(_dp), threads or default_threads())
    return out


def _check_pair(A, B):
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError(f"shape mismatch {A.shape} @ {B.shape}")


def _check_samples(rows, cols, m, n):
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    if rows.shape != cols.shape or rows.ndim != 1:
        raise ValueError("rows and cols must be 1-D and of equal length")
    if rows.size and (rows.min() < 0 or rows.max() >= m or cols.min() < 0 or cols.max() >= n):
        raise IndexError("sample index out of range")
    return rows, cols


def gemm_dot2(A, B, threads: int | None = None) -> np.ndarray:
    """C = A @ B by the definition (ascending r), each c_ij evaluated with the
    compensated dot product Dot2 (Ogita, Rump, Oishi 2005): as accurate as a
    sum in twice binary64 precision, rounded once to binary64."""
    A = _as_f64(A)
    B = _as_f64(B)
    _check_pair(A, B)
    m, k = A.shape
    n = B.shape[1]
    C = np.empty((m, n), dtype=np.float64)
    if m and n:
        _load().oracle_gemm_dot2(m, n, k, A.ctypes.data_as(_dp), max(k, 1), B.ctypes.data_as(_dp), max(n, 1),
                                 C.ctypes.data_as(_dp), n, threads or default_threads())
    return C


def gemm_dot2_sampled(A, B, rows, cols, threads: int | None = None) -> np.ndarray:
    """Dot2 values of c_ij for the listed (rows[t], cols[t]) pairs."""
    A = _as_f64(A)
    B = _as_f64(B)
    _check_pair(A, B)
    m, k = A.shape
    n = B.shape[1]
    rows, cols = _check_samples(rows, cols, m, n)
    out = np.empty(rows.size, dtype=np.float64)
    if rows.size:
        _load().oracle_gemm_dot2_sampled(rows.size, rows.ctypes.data_as(_ip), cols.ctypes.data_as(_ip), k,
                                         A.ctypes.data_as(_dp), max(k, 1), B.ctypes.data_as(_dp), max(n, 1),
                                         out.ctypes.data_as(_dp), threads or default_threads())
    return out


def _as_c128(x) -> np.ndarray:
    x = np.asarray(x)
    if not np.iscomplexobj(x):
        raise TypeError(f"complex oracle takes complex arrays, got {x.dtype}")
    return np.ascontiguousarray(x, dtype=np.complex128)


def gemm_c128(A, B, threads: int | None = None) -> np.ndarray:
    """Complex C = A @ B: every term (ar br - ai bi) + i (ar bi + ai br) and
    every partial sum rounded to binary64, accumulated in ascending r."""
    A = _as_c128(A)
    B = _as_c128(B)
    _check_pair(A, B)
    m, k = A.shape
    n = B.shape[1]
    C = np.empty((m, n), dtype=np.complex128)
    if m and n:
        _load().oracle_gemm_c128(m, n, k, A.ctypes.data_as(_dp), max(k, 1), B.ctypes.data_as(_dp), max(n, 1),
                                 C.ctypes.data_as(_dp), n, threads or default_threads())
    return C


def gemm_c128_sampled(A, B, rows, cols, threads: int | None = None) -> np.ndarray:
    """Complex c_ij for the listed (rows[t], cols[t]) pairs, same order."""
    A = _as_c128(A)
    B = _as_c128(B)
    _check_pair(A, B)
    m, k = A.shape
    n = B.shape[1]
    rows, cols = _check_samples(rows, cols, m, n)
    out = np.empty(rows.size, dtype=np.complex128)
    if rows.size:
        _load().oracle_gemm_c128_sampled(rows.size, rows.ctypes.data_as(_ip), cols.ctypes.data_as(_ip), k,
                                         A.ctypes.data_as(_dp), max(k, 1), B.ctypes.data_as(_dp), max(n, 1),
                                         out.ctypes.data_as(_dp), threads or default_threads())
    return out


def add(A, B, subtract: bool = False) -> np.ndarray:
    """c_ij = a_ij + b_ij (or a_ij - b_ij), element by element, in binary64.

    For binary32 operands the binary64 sum rounded to binary32 is the
    correctly rounded binary32 sum (double rounding is harmless when the wider
    format has at least 2p + 2 bits, 53 >= 2*24 + 2)."""
    A = _as_f64(A)
    B = _as_f64(B)
    if A.shape != B.shape:
        raise ValueError(f"shape mismatch {A.shape} vs {B.shape}")
    return A - B if subtract else A + B


def gemm_rows(A, B, rows, threads: int | None = None) -> np.ndarray:
    """Full rows ``rows`` of C = A @ B (the same loop on the selected rows of A)."""
    A = _as_f64(A)
    return gemm(A[np.asarray(rows, dtype=np.int64)], B, threads)


def dequant(bits, fmt: str) -> np.ndarray:
    """Exact binary64 values of bfloat16 / binary16 / E4M3 codes."""
    return formats.decode(bits, fmt)


def gemm_fp8(qa_bits, qb_bits, scale_a, scale_b, threads=None) -> np.ndarray:
    """C = (s_a * s_b) * sum_r qa_ir qb_rj: the E4M3 product with the per-tensor
    scales applied after the sum (all in binary64)."""
    s = float(np.float64(np.float32(scale_a)) * np.float64(np.float32(scale_b)))
    return gemm(dequant(qa_bits, "e4m3"), dequant(qb_bits, "e4m3"), threads) * s


def gemm_split_bf16x3(A_f32, B_f32, threads=None) -> np.ndarray:
    """sum_r (hi_a hi_b + hi_a lo_b + lo_a hi_b) in binary64, with (hi, lo) the
    bfloat16 split of each float32 operand; the lo*lo term is not part of the
    compensated form."""
    ah, al = (dequant(b, "bf16") for b in formats.split_bf16(A_f32))
    bh, bl = (dequant(b, "bf16") for b in formats.split_bf16(B_f32))
    return gemm(ah, bh, threads) + gemm(ah, bl, threads) + gemm(al, bh, threads)


def relerr(C, R) -> float:
    """Normwise relative error ||C - R||_F / ||R||_F in binary64.

    If ||R||_F == 0 the value returned is ||C||_F (which must then be 0)."""
    C = np.asarray(C, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    if C.shape != R.shape:
        raise ValueError(f"shape mismatch {C.shape} vs {R.shape}")
    d = np.sqrt(np.sum((C - R) ** 2))
    r = np.sqrt(np.sum(R ** 2))
    return float(d / r) if r > 0 else float(np.sqrt(np.sum(C ** 2)))


def errnorm_terms(C, R):
    """(sum (C-R)^2, sum R^2, max |C-R|) in binary64: the three reductions the
    relative error is made of."""
    C = np.asarray(C, dtype=np.float64)
    R = np.asarray(R, dtype=np.float64)
    d = C - R
    return float(np.sum(d * d)), float(np.sum(R * R)), float(np.max(np.abs(d))) if d.size else 0.0
