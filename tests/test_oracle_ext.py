"""Pins for the oracle's binary64-checking, complex and addition functions
(CPU only).

* ``gemm_dot2`` (compensated product, the reference for a binary64 GPU
  product) is pinned to exact rational arithmetic, to cancellation cases
  whose exact value plain binary64 loses, and to bitwise agreement with the
  plain loop where every partial sum is exact.  A dropped TwoProduct error
  term fails the squared-(1 + 2^-30) case; a dropped TwoSum error term fails
  the 2^60 cancellation case.
* ``gemm_c128`` (complex product, Table 2's complex column) is pinned to
  Gaussian-integer products computed exactly in integers, to a complex
  diagonal closed form, to exact rational arithmetic within the a-priori
  bound and to the conjugation identity.  A sign slip in either component
  fails the Gaussian-integer case; a transposed operand fails it on
  non-square shapes.
* ``add`` (the matrix addition/subtraction of the Results section, Fig. 9)
  is pinned to IEEE binary32 arithmetic (numpy's float32 add), to A - A = 0
  and to Sterbenz-exact differences.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

U = 2.0 ** -53


def gamma(k: int) -> float:
    return k * U / (1 - k * U)


def exact_dot(a, b) -> Fraction:
    return sum((Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b)), Fraction(0))


# ---------------------------------------------------------------- Dot2

def test_dot2_recovers_cancelled_sum():
    """[2^60, 1, -2^60] . [1, 1, 1] = 1: the plain loop returns 0, the
    compensated sum must return 1 exactly (the TwoSum error term)."""
    A = np.array([[2.0 ** 60, 1.0, -2.0 ** 60]])
    B = np.ones((3, 1))
    assert oracle.gemm(A, B)[0, 0] == 0.0
    assert oracle.gemm_dot2(A, B)[0, 0] == 1.0


def test_dot2_recovers_product_error():
    """x = 1 + 2^-30: x*x - (1 + 2^-29) = 2^-60 exactly.  The binary64 product
    rounds 2^-60 away; the compensated product keeps it (the TwoProduct error
    term)."""
    x = 1.0 + 2.0 ** -30
    A = np.array([[x, -1.0]])
    B = np.array([[x], [1.0 + 2.0 ** -29]])
    assert oracle.gemm(A, B)[0, 0] == 0.0
    assert oracle.gemm_dot2(A, B)[0, 0] == 2.0 ** -60


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (3, 4, 5), (5, 3, 8), (2, 7, 16)])
def test_dot2_vs_rational_error_bound(m, n, k):
    """|res - c| <= u |c| + gamma_k^2 sum |a b| (Ogita, Rump, Oishi 2005,
    Proposition 3.5), on binary64 inputs with full 53-bit significands."""
    g = np.random.default_rng(11)
    A = g.uniform(-1, 1, (m, k))
    B = g.uniform(-1, 1, (k, n))
    C = oracle.gemm_dot2(A, B)
    for i in range(m):
        for j in range(n):
            ex = exact_dot(A[i], B[:, j])
            s = float(np.sum(np.abs(A[i]) * np.abs(B[:, j])))
            err = abs(Fraction(float(C[i, j])) - ex)
            assert err <= Fraction(U) * abs(ex) + Fraction(gamma(k) ** 2 * s) * (1 + Fraction(1, 2 ** 40))


def test_dot2_ill_conditioned_vs_rational():
    """Dot products with cancellation down from 2^60: the plain loop is off by
    far more than one ulp of the result, the compensated one stays inside the
    twice-precision bound."""
    g = np.random.default_rng(12)
    k = 12
    rows = []
    for _ in range(6):
        a = g.uniform(1, 2, k) * np.exp2(g.integers(0, 60, k))
        a[k // 2:] = -a[: k // 2] * (1 + g.uniform(-1, 1, k // 2) * 2.0 ** -40)
        rows.append(a)
    A = np.array(rows)
    B = np.ones((k, 1))
    Cd = oracle.gemm_dot2(A, B)
    Cp = oracle.gemm(A, B)
    worst_plain = 0.0
    for i in range(A.shape[0]):
        ex = exact_dot(A[i], B[:, 0])
        s = float(np.sum(np.abs(A[i])))
        err = abs(Fraction(float(Cd[i, 0])) - ex)
        assert err <= Fraction(U) * abs(ex) + Fraction(gamma(k) ** 2 * s) * 2
        if ex != 0:
            worst_plain = max(worst_plain, float(abs(Fraction(float(Cp[i, 0])) - ex) / abs(ex)))
    assert worst_plain > 1e-10   # the case really is beyond plain binary64


@pytest.mark.parametrize("m,n,k", [(4, 5, 6), (17, 9, 33)])
def test_dot2_equals_plain_on_exact_inputs(m, n, k):
    """Integer entries with |partial sums| < 2^53: both loops are exact."""
    g = np.random.default_rng(13)
    A = g.integers(-1000, 1001, (m, k)).astype(np.float64)
    B = g.integers(-1000, 1001, (k, n)).astype(np.float64)
    assert np.array_equal(oracle.gemm_dot2(A, B), oracle.gemm(A, B))
    assert np.array_equal(oracle.gemm_dot2(A, B), (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float64))


def test_dot2_sampled_matches_full_and_empty():
    g = np.random.default_rng(14)
    A = g.uniform(-1, 1, (9, 13))
    B = g.uniform(-1, 1, (13, 7))
    C = oracle.gemm_dot2(A, B)
    rows = np.array([0, 8, 3, 5])
    cols = np.array([6, 0, 2, 2])
    assert np.array_equal(oracle.gemm_dot2_sampled(A, B, rows, cols), C[rows, cols])
    assert np.array_equal(oracle.gemm_dot2(np.zeros((3, 0)), np.zeros((0, 4))), np.zeros((3, 4)))


# ---------------------------------------------------------------- complex

def gaussian_ints(g, shape, r=50):
    return (g.integers(-r, r + 1, shape) + 1j * g.integers(-r, r + 1, shape)).astype(np.complex128)


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (3, 5, 7), (7, 3, 5), (16, 9, 33)])
def test_complex_gaussian_integers_exact(m, n, k):
    """Re C = Ar Br - Ai Bi, Im C = Ar Bi + Ai Br, computed in int64."""
    g = np.random.default_rng(21)
    A = gaussian_ints(g, (m, k))
    B = gaussian_ints(g, (k, n))
    Ar, Ai = A.real.astype(np.int64), A.imag.astype(np.int64)
    Br, Bi = B.real.astype(np.int64), B.imag.astype(np.int64)
    C = oracle.gemm_c128(A, B)
    assert np.array_equal(C.real, (Ar @ Br - Ai @ Bi).astype(np.float64))
    assert np.array_equal(C.imag, (Ar @ Bi + Ai @ Br).astype(np.float64))


def test_complex_diagonal_and_rotation():
    """(D B)_ij = d_i b_ij; multiplying by i I maps b to i b = -Im b + i Re b."""
    g = np.random.default_rng(22)
    d = (g.standard_normal(6) + 1j * g.standard_normal(6)).astype(np.complex64).astype(np.complex128)
    B = (g.standard_normal((6, 4)) + 1j * g.standard_normal((6, 4))).astype(np.complex64).astype(np.complex128)
    C = oracle.gemm_c128(np.diag(d), B)
    # one nonzero term per element; products of float32 values are exact in binary64
    ref = (d.real[:, None] * B.real - d.imag[:, None] * B.imag) + 1j * (
        d.real[:, None] * B.imag + d.imag[:, None] * B.real)
    assert np.array_equal(C, ref)
    R = oracle.gemm_c128(1j * np.eye(6), B)
    assert np.array_equal(R.real, -B.imag)
    assert np.array_equal(R.imag, B.real)


@pytest.mark.parametrize("m,n,k", [(2, 3, 4), (4, 4, 8)])
def test_complex_vs_rational_bound(m, n, k):
    """Each component within gamma_{k+2} sum(|ar br| + |ai bi|) of the exact
    value (one rounding per product and per partial sum)."""
    g = np.random.default_rng(23)
    A = g.uniform(-1, 1, (m, k)) + 1j * g.uniform(-1, 1, (m, k))
    B = g.uniform(-1, 1, (k, n)) + 1j * g.uniform(-1, 1, (k, n))
    C = oracle.gemm_c128(A, B)
    for i in range(m):
        for j in range(n):
            a, b = A[i], B[:, j]
            er = exact_dot(a.real, b.real) - exact_dot(a.imag, b.imag)
            ei = exact_dot(a.real, b.imag) + exact_dot(a.imag, b.real)
            sr = float(np.sum(np.abs(a.real * b.real) + np.abs(a.imag * b.imag)))
            si = float(np.sum(np.abs(a.real * b.imag) + np.abs(a.imag * b.real)))
            assert abs(Fraction(float(C[i, j].real)) - er) <= Fraction(gamma(k + 2) * sr)
            assert abs(Fraction(float(C[i, j].imag)) - ei) <= Fraction(gamma(k + 2) * si)


def test_complex_conjugation_bitwise_and_library():
    """conj(A) conj(B) = conj(A B) bit for bit (negation is exact), and numpy's
    complex128 product agrees within 2 gamma_{k+2} (|A| |B|)."""
    g = np.random.default_rng(24)
    A = g.standard_normal((11, 19)) + 1j * g.standard_normal((11, 19))
    B = g.standard_normal((19, 6)) + 1j * g.standard_normal((19, 6))
    C = oracle.gemm_c128(A, B)
    assert np.array_equal(oracle.gemm_c128(np.conj(A), np.conj(B)), np.conj(C))
    bound = 2 * gamma(21) * 2 * (np.abs(A) @ np.abs(B))
    assert np.all(np.abs(C - A @ B) <= bound)
    rows, cols = np.array([0, 10, 4]), np.array([5, 0, 3])
    assert np.array_equal(oracle.gemm_c128_sampled(A, B, rows, cols), C[rows, cols])


def test_complex_rejects_real_input():
    with pytest.raises(TypeError):
        oracle.gemm_c128(np.ones((2, 2)), np.ones((2, 2)))


# ---------------------------------------------------------------- addition

@pytest.mark.parametrize("dist", ["uniform", "normal", "wide"])
def test_add_matches_ieee_binary32(dist):
    """float32(binary64 a +- b) = the IEEE binary32 sum/difference."""
    g = synth.rng(31)
    A = synth.draw(g, (64, 96), dist)
    B = synth.draw(g, (64, 96), dist)
    assert np.array_equal(oracle.add(A, B).astype(np.float32), A + B)
    assert np.array_equal(oracle.add(A, B, subtract=True).astype(np.float32), A - B)


def test_add_identities():
    g = synth.rng(32)
    A = synth.draw(g, (33, 17), "normal")
    assert np.array_equal(oracle.add(A, A, subtract=True), np.zeros((33, 17)))
    assert np.array_equal(oracle.add(A, np.zeros_like(A)), A.astype(np.float64))
    # Sterbenz: y/2 <= x <= 2y  =>  x - y is exact in binary32
    x = np.float32(1.75) * np.abs(A) + np.float32(1.0)
    y = np.float32(1.0) + np.abs(A)
    d = oracle.add(x, y, subtract=True)
    assert np.array_equal(d.astype(np.float32).astype(np.float64), d)
