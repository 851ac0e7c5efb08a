"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks.

This module holds no arithmetic of the product itself: it only draws numbers.
Every generator is ``numpy.random.default_rng(seed)``-based so a (shape,
distribution, seed) triple names one input exactly.  Values are drawn in
binary64 and rounded to float32 (RNE, numpy's cast); ``draw64``/``pair64``
keep the binary64 values and ``draw_c64``/``pair_c64`` give complex64
matrices (real parts drawn before imaginary parts).

Distributions (the paper prints no input values; these are the workloads'
stated recipes):

* ``uniform``  -- i.i.d. uniform[-1, 1].
* ``normal``   -- i.i.d. N(0, 1).
* ``wide``     -- sign * 2**u with u ~ uniform[-8, 8] (continuous) and a fair
  random sign; ``wide_int`` draws integer u, so every entry is a power of two.
* ``integers`` -- i.i.d. integers in [-R, R] (exact in every format when small).
* ``loguniform_dims`` -- d = round(exp(U(ln lo, ln hi))) clamped to [lo, hi],
  drawn per problem in the order m, n, k.
* ``poisson_arrivals`` -- cumulative exponential inter-arrival gaps at rate
  ``lam`` per second, first arrival at t = 0.
* ``dtype_mix`` -- per-request mode draw with the given probabilities.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def draw64(g: np.random.Generator, shape, dist: str = "uniform", R: int = 16) -> np.ndarray:
    """One binary64 matrix from generator ``g`` (advances ``g``), not rounded."""
    if dist == "uniform":
        x = g.uniform(-1.0, 1.0, size=shape)
    elif dist == "normal":
        x = g.standard_normal(size=shape)
    elif dist == "wide":
        u = g.uniform(-8.0, 8.0, size=shape)
        s = np.where(g.random(size=shape) < 0.5, -1.0, 1.0)
        x = s * np.exp2(u)
    elif dist == "wide_int":
        u = g.integers(-8, 9, size=shape)
        s = np.where(g.random(size=shape) < 0.5, -1.0, 1.0)
        x = s * np.exp2(u.astype(np.float64))
    elif dist == "integers":
        x = g.integers(-R, R + 1, size=shape).astype(np.float64)
    else:
        raise ValueError(f"unknown distribution {dist!r}")
    return x.astype(np.float64)


def draw(g: np.random.Generator, shape, dist: str = "uniform", R: int = 16) -> np.ndarray:
    """One float32 matrix from generator ``g`` (advances ``g``): draw64 rounded
    to float32."""
    return draw64(g, shape, dist, R).astype(np.float32)


def draw_c64(g: np.random.Generator, shape, dist: str = "uniform", R: int = 16) -> np.ndarray:
    """One complex64 matrix: the real parts are drawn first, then the
    imaginary parts, each as ``draw``."""
    re = draw(g, shape, dist, R)
    im = draw(g, shape, dist, R)
    out = np.empty(shape, dtype=np.complex64)
    out.real = re
    out.imag = im
    return out


def pair(m: int, n: int, k: int, seed: int = 0, dist: str = "uniform", R: int = 16):
    """(A, B): A is m x k, drawn first, then B (k x n), from one seeded stream."""
    g = rng(seed)
    A = draw(g, (m, k), dist, R)
    B = draw(g, (k, n), dist, R)
    return A, B


def pair64(m: int, n: int, k: int, seed: int = 0, dist: str = "uniform", R: int = 16):
    """(A, B) in binary64 (A first), for the double-precision product."""
    g = rng(seed)
    return draw64(g, (m, k), dist, R), draw64(g, (k, n), dist, R)


def pair_c64(m: int, n: int, k: int, seed: int = 0, dist: str = "uniform", R: int = 16):
    """(A, B) complex64 (A first), for the complex-float product."""
    g = rng(seed)
    return draw_c64(g, (m, k), dist, R), draw_c64(g, (k, n), dist, R)


def loguniform_dims(count: int, lo: int, hi: int, seed: int = 0) -> np.ndarray:
    """(count, 3) int64 array of (m, n, k), each log-uniform in [lo, hi]."""
    g = rng(seed)
    u = g.uniform(np.log(lo), np.log(hi), size=(count, 3))
    d = np.rint(np.exp(u)).astype(np.int64)
    return np.clip(d, lo, hi)


def grouped_problems(count: int = 512, lo: int = 32, hi: int = 1024, seed: int = 0,
                     dist: str = "uniform"):
    """[(A_i, B_i)] for ``count`` problems with log-uniform dims; the dims are
    drawn first, then A_i and B_i in problem order from one stream."""
    dims = loguniform_dims(count, lo, hi, seed)
    g = rng(seed + 1)
    out = []
    for m, n, k in dims:
        A = draw(g, (int(m), int(k)), dist)
        B = draw(g, (int(k), int(n)), dist)
        out.append((A, B))
    return out


def poisson_arrivals(count: int, lam: float, seed: int = 0) -> np.ndarray:
    """Arrival times in seconds (float64), first at 0."""
    g = rng(seed)
    gaps = g.exponential(1.0 / lam, size=count)
    t = np.cumsum(gaps)
    return t - t[0]


def dtype_mix(count: int, probs=(0.5, 0.35, 0.15), seed: int = 0) -> np.ndarray:
    """Index into the mode list per request (default: FP32 / BF16 / E4M3)."""
    g = rng(seed)
    return g.choice(len(probs), size=count, p=np.asarray(probs) / np.sum(probs))
