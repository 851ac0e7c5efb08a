"""Pins for the binary64 reference product (the oracle), CPU only.

Each test checks the oracle against something other than itself: closed
forms, exact rational arithmetic, algebraic identities that hold bit for bit,
and a library routine within the a-priori error bound.  A dropped term, a sign
or index slip, a transposed operand, a wrong summation order or a fused
multiply-add each fails at least one of them.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth

SHAPES = [(1, 1, 1), (3, 5, 7), (7, 3, 5), (17, 9, 33), (64, 48, 40)]


def gamma(k: int) -> float:
    """gamma_k = k u / (1 - k u), u = 2^-53 (Higham, Accuracy and Stability
    of Numerical Algorithms, sec. 3.1) bounds the relative error of a
    length-k recursive dot product."""
    u = 2.0 ** -53
    return k * u / (1 - k * u)


@pytest.mark.parametrize("m,n,k", SHAPES)
def test_identity_both_sides(m, n, k):
    A, B = synth.pair(m, n, k, seed=1)
    assert np.array_equal(oracle.gemm(A, np.eye(k)), A.astype(np.float64))
    assert np.array_equal(oracle.gemm(np.eye(m), A), A.astype(np.float64))
    assert np.array_equal(oracle.gemm(np.eye(k), B), B.astype(np.float64))


@pytest.mark.parametrize("m,n", [(1, 1), (5, 9), (33, 17)])
def test_diagonal_closed_form(m, n):
    """(D B)_ij = d_i b_ij and (B D)_ij = b_ij d_j: the paper's O(n) special
    case (Implementation section).  Exact in binary64 for float32 inputs."""
    g = synth.rng(2)
    d = synth.draw(g, (m,), "normal")
    B = synth.draw(g, (m, n), "normal")
    C = oracle.gemm(np.diag(d), B)
    assert np.array_equal(C, d.astype(np.float64)[:, None] * B.astype(np.float64))
    e = synth.draw(g, (n,), "normal")
    C2 = oracle.gemm(B, np.diag(e))
    assert np.array_equal(C2, B.astype(np.float64) * e.astype(np.float64)[None, :])


@pytest.mark.parametrize("m,n,k", SHAPES)
def test_rank1_closed_form(m, n, k):
    """A = u v^T, B = w z^T  =>  C = (v . w) u z^T, exact for small integers."""
    g = synth.rng(3)
    u, v, w, z = (g.integers(-9, 10, size=s).astype(np.float64) for s in (m, k, k, n))
    C = oracle.gemm(np.outer(u, v), np.outer(w, z))
    assert np.array_equal(C, float(np.dot(v, w)) * np.outer(u, z))


def test_index_closed_form():
    """a_ir = i + 1, b_rj = r + j  =>  c_ij = (i + 1) (k (k - 1) / 2 + k j)."""
    m, n, k = 6, 11, 13
    A = np.add.outer(np.arange(m), np.zeros(k)) + 1
    B = np.add.outer(np.arange(k), np.arange(n)).astype(np.float64)
    i = np.arange(m)[:, None]
    j = np.arange(n)[None, :]
    expect = (i + 1) * (k * (k - 1) / 2 + k * j)
    assert np.array_equal(oracle.gemm(A, B), expect.astype(np.float64))


@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (2, 3, 4), (5, 4, 8), (8, 8, 8)])
def test_integer_exact_vs_rational(m, n, k):
    A, B = synth.pair(m, n, k, seed=4, dist="integers", R=1000)
    exact = [[sum(Fraction(int(A[i, r])) * Fraction(int(B[r, j])) for r in range(k))
              for j in range(n)] for i in range(m)]
    assert np.array_equal(oracle.gemm(A, B), np.array(exact, dtype=np.float64))


@pytest.mark.parametrize("m,n,k", [(3, 4, 5), (8, 8, 8), (2, 7, 8)])
def test_rational_brute_force_error_bound(m, n, k):
    """|R - exact| <= gamma_k (|A| |B|) elementwise, with exact rational AB."""
    A, B = synth.pair(m, n, k, seed=5, dist="normal")
    R = oracle.gemm(A, B)
    absAB = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))
    for i in range(m):
        for j in range(n):
            ex = sum(Fraction(float(A[i, r])) * Fraction(float(B[r, j])) for r in range(k))
            assert abs(Fraction(R[i, j]) - ex) <= Fraction(gamma(k) * absAB[i, j] * (1 + 1e-12))


def test_transpose_identity_bitwise():
    """(A B)^T = B^T A^T bit for bit: the same products, in the same order."""
    A, B = synth.pair(23, 31, 19, seed=6, dist="normal")
    C = oracle.gemm(A, B)
    Ct = oracle.gemm(np.ascontiguousarray(B.T), np.ascontiguousarray(A.T))
    assert np.array_equal(C.T, Ct)


def test_block_structure_bitwise():
    """Row blocks of A give row blocks of C; column blocks of B give column
    blocks of C (every c_ij depends only on row i of A and column j of B)."""
    A, B = synth.pair(20, 24, 15, seed=7)
    C = oracle.gemm(A, B)
    assert np.array_equal(C[:7], oracle.gemm(A[:7], B))
    assert np.array_equal(C[7:], oracle.gemm(A[7:], B))
    assert np.array_equal(C[:, 5:13], oracle.gemm(A, B[:, 5:13]))


def test_summation_order_ascending_r():
    """[1, 2^-53, 2^-53] . [1, 1, 1]: ascending r gives exactly 1 (each tiny
    term ties to even and vanishes); any other order starting from the small
    terms would give 1 + 2^-52.  Listing 1's loop runs r upward from c = 0."""
    A = np.array([[1.0, 2.0 ** -53, 2.0 ** -53]])
    B = np.ones((3, 1))
    assert oracle.gemm(A, B)[0, 0] == 1.0
    A2 = np.array([[2.0 ** -53, 2.0 ** -53, 1.0]])
    assert oracle.gemm(A2, B)[0, 0] == 1.0 + 2.0 ** -52


def test_no_fused_multiply_add():
    """s = -(1 + 2^-29); (1 + 2^-30)^2 rounds to 1 + 2^-29, so separate
    rounding gives exactly 0, whereas a fused multiply-add would keep 2^-60."""
    a1 = 1.0 + 2.0 ** -30
    A = np.array([[-(1.0 + 2.0 ** -29), a1]])
    B = np.array([[1.0], [a1]])
    assert oracle.gemm(A, B)[0, 0] == 0.0


def test_empty_shapes():
    A, B = synth.pair(4, 5, 0, seed=8)
    assert np.array_equal(oracle.gemm(A, B), np.zeros((4, 5)))
    assert oracle.gemm(np.zeros((0, 3)), np.zeros((3, 5))).shape == (0, 5)
    assert oracle.gemm(np.zeros((4, 3)), np.zeros((3, 0))).shape == (4, 0)
    with pytest.raises(ValueError):
        oracle.gemm(np.zeros((4, 3)), np.zeros((2, 5)))


def test_thread_count_invariance():
    A, B = synth.pair(37, 29, 301, seed=9, dist="normal")
    C1 = oracle.gemm(A, B, threads=1)
    for t in (2, 3, 8):
        assert np.array_equal(C1, oracle.gemm(A, B, threads=t))


@pytest.mark.parametrize("m,n,k", [(64, 64, 64), (33, 70, 513), (5, 3, 4097)])
def test_library_routine_within_bound(m, n, k):
    """numpy's binary64 product agrees within 2 gamma_k normwise (both are
    within gamma_k of the exact product)."""
    A, B = synth.pair(m, n, k, seed=10, dist="normal")
    R = oracle.gemm(A, B)
    L = A.astype(np.float64) @ B.astype(np.float64)
    absAB = np.abs(A.astype(np.float64)) @ np.abs(B.astype(np.float64))
    assert np.all(np.abs(R - L) <= 2 * gamma(k) * absAB * (1 + 1e-9))


def test_sampled_and_rows_match_full():
    A, B = synth.pair(41, 37, 53, seed=11, dist="normal")
    C = oracle.gemm(A, B)
    g = synth.rng(12)
    rows = g.integers(0, 41, size=50)
    cols = g.integers(0, 37, size=50)
    assert np.array_equal(oracle.gemm_sampled(A, B, rows, cols), C[rows, cols])
    assert np.array_equal(oracle.gemm_rows(A, B, [0, 40, 7]), C[[0, 40, 7]])
    with pytest.raises(IndexError):
        oracle.gemm_sampled(A, B, [41], [0])


def test_relerr_definition():
    R = np.array([[3.0, 0.0], [0.0, 4.0]])
    C = np.array([[3.0, 0.0], [0.0, 4.0 + 0.5]])
    assert oracle.relerr(C, R) == pytest.approx(0.5 / 5.0, rel=0, abs=1e-16)
    assert oracle.relerr(np.zeros((2, 2)), np.zeros((2, 2))) == 0.0
    assert oracle.relerr(np.ones((1, 1)), np.zeros((1, 1))) == 1.0
    s, r, mx = oracle.errnorm_terms(C, R)
    assert (s, r, mx) == (0.25, 25.0, 0.5)


def test_split_bf16x3_drops_exactly_the_lo_lo_term():
    """Operands built as hi + lo with hi = 256 k (|k| in [65, 127], exact in
    bfloat16) and |lo| <= 63 (below half an ulp of hi, and hi + lo stays in
    hi's binade [2^14, 2^15)): the bfloat16 split of each float32 value is
    exactly (hi, lo), so the compensated product must be
    the exact integer product minus sum_r lo_a lo_b -- checked in int64.
    Dropping a cross term, or keeping lo*lo, fails."""
    g = synth.rng(77)

    def operand(shape):
        k = g.integers(65, 128, shape) * g.choice([-1, 1], shape)
        lo = g.integers(-63, 64, shape)
        return (256 * k + lo).astype(np.int64), lo.astype(np.int64)

    A, LA = operand((9, 14))
    B, LB = operand((14, 11))
    got = oracle.gemm_split_bf16x3(A.astype(np.float32), B.astype(np.float32))
    want = A @ B - LA @ LB
    assert np.array_equal(got, want.astype(np.float64))
    # bfloat16-exact operands (lo = 0): the plain product
    Ah, Bh = (A - LA).astype(np.float32), (B - LB).astype(np.float32)
    assert np.array_equal(oracle.gemm_split_bf16x3(Ah, Bh), oracle.gemm(Ah, Bh))


def test_fp8_product_applies_both_scales_after_the_sum():
    """E4M3 codes from the OCP table written out by hand (0x38 = 1, 0x40 = 2,
    0x44 = 3, 0x48 = 4, 0x30 = 0.5, sign bit 0x80), so the pin does not lean on
    the oracle's own encoder: C = s_a s_b sum_r qa qb in binary64."""
    val = {0x38: 1.0, 0x40: 2.0, 0x44: 3.0, 0x48: 4.0, 0x30: 0.5,
           0xB8: -1.0, 0xC0: -2.0, 0xC4: -3.0, 0xC8: -4.0, 0xB0: -0.5, 0x00: 0.0}
    codes = np.array(sorted(val), dtype=np.uint8)
    g = synth.rng(78)
    qa = g.choice(codes, (6, 10)).astype(np.uint8)
    qb = g.choice(codes, (10, 5)).astype(np.uint8)
    va = np.vectorize(val.get)(qa).astype(np.float64)
    vb = np.vectorize(val.get)(qb).astype(np.float64)
    got = oracle.gemm_fp8(qa, qb, 3.0, 0.25)
    assert np.array_equal(got, (va @ vb) * 0.75)   # small dyadic values: every step exact
    assert np.array_equal(oracle.dequant(qa, "e4m3"), va)
