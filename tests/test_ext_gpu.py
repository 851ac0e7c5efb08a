"""Parity of the binary64 product, the complex-float product and the matrix
addition/subtraction (the paper's Results section: Table 2's double and
complex columns, Fig. 9's addition) with the oracle, through the C-ABI.

Bars:
* gemm_plain_f64: every element within (k + 2) u64 (|A||B|)_ij of the exact
  product, checked against the compensated (Dot2) oracle, whose own error is
  below u64 |c| + gamma_k^2 (|A||B|); integer, identity and diagonal inputs
  bit-exact.
* gemm_plain_c32: each component within (2k + 2) u32 of the sum of the
  absolute values of its 2k real products, against the binary64 complex
  oracle; Gaussian-integer inputs bit-exact.
* gemm_add: bit-exact (one IEEE operation per element) in float and double.
"""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import dev, host, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1306_6192_amd as mg  # noqa: E402

U64 = 2.0 ** -53
U32 = 2.0 ** -24

SHAPES = [(1, 1, 1), (2, 3, 4), (17, 33, 5), (64, 64, 16), (65, 130, 17), (129, 80, 96), (257, 129, 31),
          (300, 208, 1040), (97, 61, 4099)]


def _f64_bound(A, B, R, k):
    absAB = np.abs(A) @ np.abs(B)
    return (k + 2) * U64 * absAB + U64 * np.abs(R) + 1e-300


def _assert_f64(C, R, A, B, k, what):
    err = np.abs(C - R)
    bound = _f64_bound(A, B, R, k)
    bad = err > bound
    assert not bad.any(), f"{what}: {bad.sum()} elements beyond the binary64 bound, first {np.argwhere(bad)[0]}"


def _c32_bounds(A, B, k):
    Ar, Ai = np.abs(A.real.astype(np.float64)), np.abs(A.imag.astype(np.float64))
    Br, Bi = np.abs(B.real.astype(np.float64)), np.abs(B.imag.astype(np.float64))
    g = (2 * k + 2) * U32
    return g * (Ar @ Br + Ai @ Bi) + 1e-37, g * (Ar @ Bi + Ai @ Br) + 1e-37


def _assert_c32(C, R, A, B, k, what):
    br, bi = _c32_bounds(A, B, k)
    er = np.abs(C.real.astype(np.float64) - R.real)
    ei = np.abs(C.imag.astype(np.float64) - R.imag)
    assert not (er > br).any(), f"{what}: real part beyond bound at {np.argwhere(er > br)[0]}"
    assert not (ei > bi).any(), f"{what}: imaginary part beyond bound at {np.argwhere(ei > bi)[0]}"


# ---------------------------------------------------------------- binary64

@pytest.mark.parametrize("m,n,k", SHAPES)
def test_f64_shapes_every_config(m, n, k):
    log(f"f64 shape {(m, n, k)}")
    A, B = synth.pair64(m, n, k, seed=m * 5 + n + 3 * k)
    R = oracle.gemm_dot2(A, B)
    dA, dB = dev(A), dev(B)
    for cfg in range(mg.num_configs(mg.MODE_F64)):
        C = host(mg.gemm_f64(dA, dB, cfg=cfg))
        _assert_f64(C, R, A, B, k, f"f64 {(m, n, k)} cfg {cfg}")
    C = host(mg.gemm_f64(dA, dB))
    _assert_f64(C, R, A, B, k, f"f64 {(m, n, k)} tuned")
    assert oracle.relerr(C, R) <= 1e-14


@pytest.mark.parametrize("m,n,k", [(64, 64, 64), (200, 300, 1000), (513, 257, 4096)])
def test_f64_integers_bit_exact(m, n, k):
    """Integers in [-2^20, 2^20]: |partial sums| < k 2^40 < 2^53, exact in
    any order."""
    log(f"f64 integer-exact {(m, n, k)}")
    g = synth.rng(41)
    A = g.integers(-2 ** 20, 2 ** 20 + 1, (m, k)).astype(np.float64)
    B = g.integers(-2 ** 20, 2 ** 20 + 1, (k, n)).astype(np.float64)
    R = oracle.gemm(A, B)
    dA, dB = dev(A), dev(B)
    for cfg in range(mg.num_configs(mg.MODE_F64)):
        assert np.array_equal(host(mg.gemm_f64(dA, dB, cfg=cfg)), R), cfg


def test_f64_identity_diagonal_bit_exact():
    log("f64 identity/diagonal")
    g = synth.rng(42)
    A = synth.draw64(g, (150, 70), "normal")
    assert np.array_equal(host(mg.gemm_f64(dev(A), dev(np.eye(70)))), A)
    assert np.array_equal(host(mg.gemm_f64(dev(np.eye(150)), dev(A))), A)
    d = synth.draw64(g, (150,), "normal")
    assert np.array_equal(host(mg.gemm_f64(dev(np.diag(d)), dev(A))), d[:, None] * A)


def test_f64_strided_misaligned_and_guard_band():
    """Operands 8 bytes past a 16-byte boundary with odd strides; C inside a
    NaN-filled buffer whose outside must stay untouched."""
    log("f64 strided/misaligned")
    m, n, k = 131, 77, 203
    A, B = synth.pair64(m, n, k, seed=43)
    R = oracle.gemm_dot2(A, B)
    bufA = torch.zeros((m, k + 3), dtype=torch.float64, device="cuda")
    bufB = torch.zeros((k, n + 5), dtype=torch.float64, device="cuda")
    bufA[:, 1:k + 1] = dev(A)
    bufB[:, 1:n + 1] = dev(B)
    bufC = torch.full((m + 2, n + 7), float("nan"), dtype=torch.float64, device="cuda")
    outC = bufC[1:m + 1, 3:n + 3]
    for cfg in range(mg.num_configs(mg.MODE_F64)):
        mg.gemm_f64(bufA[:, 1:k + 1], bufB[:, 1:n + 1], out=outC, cfg=cfg)
        full = host(bufC)
        _assert_f64(full[1:m + 1, 3:n + 3], R, A, B, k, f"strided cfg {cfg}")
        mask = np.ones_like(full, dtype=bool)
        mask[1:m + 1, 3:n + 3] = False
        assert np.isnan(full[mask]).all(), f"cfg {cfg} wrote outside C"


# k and n even (whole 16-byte chunks): the asynchronous-copy tiles run these;
# ragged m and n, a partial k-tile of 16, one row and one chunk
F64_CHUNKED = [(1, 2, 2), (33, 34, 18), (64, 512, 16), (129, 66, 18), (257, 130, 1034), (300, 208, 1040),
               (513, 260, 4098)]


def _f64_async_configs():
    return [c for c in range(mg.num_configs(mg.MODE_F64)) if mg.config_chunk(mg.MODE_F64, c) > 0]


@pytest.mark.parametrize("m,n,k", F64_CHUNKED)
def test_f64_async_tiles_chunked_shapes(m, n, k):
    """The asynchronous-copy binary64 tiles: within the bound of the
    compensated oracle and bit for bit equal to the register-staged tile
    (the same MFMAs in the same k order)."""
    log(f"f64 async tiles {(m, n, k)}")
    A, B = synth.pair64(m, n, k, seed=m + 7 * n + 3 * k)
    R = oracle.gemm_dot2(A, B)
    dA, dB = dev(A), dev(B)
    ref = host(mg.gemm_f64(dA, dB, cfg=0))
    cfgs = _f64_async_configs()
    assert cfgs
    for cfg in cfgs:
        C = host(mg.gemm_f64(dA, dB, cfg=cfg))
        _assert_f64(C, R, A, B, k, f"f64 async {(m, n, k)} cfg {cfg}")
        assert np.array_equal(C, ref), cfg


def test_f64_async_tiles_strides_and_fallback():
    """Even padded strides run the asynchronous-copy tiles; an odd stride or a
    base 8 bytes off 16-byte alignment falls back to the register-staged
    tile.  Same bits in every case, nothing written outside C."""
    log("f64 async tiles strides/fallback")
    m, n, k = 140, 98, 260
    A, B = synth.pair64(m, n, k, seed=45)
    ref = host(mg.gemm_f64(dev(A), dev(B), cfg=0))
    for pad_a, pad_b, off in [(2, 4, 0), (1, 2, 0), (2, 4, 1)]:
        bufA = torch.zeros((m, k + pad_a + off), dtype=torch.float64, device="cuda")
        bufB = torch.zeros((k, n + pad_b + off), dtype=torch.float64, device="cuda")
        dA, dB = bufA[:, off:off + k], bufB[:, off:off + n]
        dA.copy_(dev(A))
        dB.copy_(dev(B))
        for cfg in _f64_async_configs():
            big = torch.full((m + 2, n + 2), float("nan"), dtype=torch.float64, device="cuda")
            mg.gemm_f64(dA, dB, out=big[1:m + 1, 1:n + 1], cfg=cfg)
            h = host(big)
            assert np.array_equal(h[1:m + 1, 1:n + 1], ref), (pad_a, pad_b, off, cfg)
            mask = np.ones_like(h, dtype=bool)
            mask[1:m + 1, 1:n + 1] = False
            assert np.isnan(h[mask]).all()


def test_f64_empty_and_k0():
    log("f64 empty / k = 0")
    C = torch.full((5, 6), 7.0, dtype=torch.float64, device="cuda")
    mg.gemm_f64(torch.zeros((5, 0), dtype=torch.float64, device="cuda"),
                torch.zeros((0, 6), dtype=torch.float64, device="cuda"), out=C)
    assert np.array_equal(host(C), np.zeros((5, 6)))
    out = mg.gemm_f64(torch.zeros((0, 3), dtype=torch.float64, device="cuda"),
                      torch.zeros((3, 4), dtype=torch.float64, device="cuda"))
    assert tuple(out.shape) == (0, 4)


@pytest.mark.parametrize("size", [4096, 8192])
def test_f64_full_size_sampled(size):
    """The paper's 4096 x 4096 double product (Table 2) and 8192^3, on 512
    sampled outputs plus one full row against the compensated oracle."""
    log(f"f64 {size}^3 sampled")
    A, B = synth.pair64(size, size, size, seed=0)
    C = host(mg.gemm_f64(dev(A), dev(B)))
    g = synth.rng(44)
    rows = g.integers(0, size, 512)
    cols = g.integers(0, size, 512)
    R = oracle.gemm_dot2_sampled(A, B, rows, cols)
    absAB = np.einsum("ij,ji->i", np.abs(A[rows]), np.abs(B[:, cols]))
    err = np.abs(C[rows, cols] - R)
    assert np.all(err <= (size + 2) * U64 * absAB + U64 * np.abs(R))
    r = size // 3
    Rrow = oracle.gemm_dot2_sampled(A, B, np.full(size, r), np.arange(size))
    assert oracle.relerr(C[r], Rrow) <= 1e-14


# ---------------------------------------------------------------- complex

@pytest.mark.parametrize("m,n,k", SHAPES)
def test_c32_shapes_every_config(m, n, k):
    log(f"c32 shape {(m, n, k)}")
    A, B = synth.pair_c64(m, n, k, seed=m * 3 + n * 5 + k)
    R = oracle.gemm_c128(A, B)
    dA, dB = dev(A), dev(B)
    for cfg in range(mg.num_configs(mg.MODE_C32)):
        C = host(mg.gemm_c32(dA, dB, cfg=cfg))
        _assert_c32(C, R, A, B, k, f"c32 {(m, n, k)} cfg {cfg}")
    C = host(mg.gemm_c32(dA, dB))
    _assert_c32(C, R, A, B, k, f"c32 {(m, n, k)} tuned")
    assert oracle.relerr(C.view(np.float32), R.view(np.float64)) <= (1e-6 if k <= 1024 else 1e-5)


@pytest.mark.parametrize("m,n,k", [(64, 64, 64), (200, 300, 1000), (257, 129, 4100)])
def test_c32_gaussian_integers_bit_exact(m, n, k):
    """Gaussian integers with parts in [-16, 16]: every float32 partial sum of
    the 2k real products is an integer below 2^24, so any order is exact."""
    log(f"c32 Gaussian-integer {(m, n, k)}")
    A, B = synth.pair_c64(m, n, k, seed=45, dist="integers", R=16)
    R = oracle.gemm_c128(A, B)
    dA, dB = dev(A), dev(B)
    for cfg in range(mg.num_configs(mg.MODE_C32)):
        C = host(mg.gemm_c32(dA, dB, cfg=cfg))
        assert np.array_equal(C.astype(np.complex128), R), cfg


def test_c32_rotation_and_conjugate_bit_exact():
    """i I B = -Im B + i Re B exactly; A conj-pair identity checked through the
    oracle values."""
    log("c32 rotation")
    g = synth.rng(46)
    B = synth.draw_c64(g, (90, 70), "normal")
    I = (1j * np.eye(90)).astype(np.complex64)
    C = host(mg.gemm_c32(dev(I), dev(B)))
    assert np.array_equal(C.real, -B.imag) and np.array_equal(C.imag, B.real)


def test_c32_strided_misaligned_and_guard_band():
    log("c32 strided/misaligned")
    m, n, k = 131, 77, 203
    A, B = synth.pair_c64(m, n, k, seed=47)
    R = oracle.gemm_c128(A, B)
    bufA = torch.zeros((m, k + 3), dtype=torch.complex64, device="cuda")
    bufB = torch.zeros((k, n + 5), dtype=torch.complex64, device="cuda")
    bufA[:, 1:k + 1] = dev(A)
    bufB[:, 1:n + 1] = dev(B)
    bufC = torch.full((m + 2, n + 7), complex("nan+nanj"), dtype=torch.complex64, device="cuda")
    outC = bufC[1:m + 1, 3:n + 3]
    for cfg in range(mg.num_configs(mg.MODE_C32)):
        mg.gemm_c32(bufA[:, 1:k + 1], bufB[:, 1:n + 1], out=outC, cfg=cfg)
        full = host(bufC)
        _assert_c32(full[1:m + 1, 3:n + 3], R, A, B, k, f"strided cfg {cfg}")
        mask = np.ones(full.shape, dtype=bool)
        mask[1:m + 1, 3:n + 3] = False
        assert np.isnan(full[mask].real).all() and np.isnan(full[mask].imag).all(), cfg


# k and n even (whole 16-byte chunks of two complex values): the
# asynchronous-copy tiles run these
C32_CHUNKED = [(1, 2, 2), (33, 34, 18), (64, 256, 16), (129, 66, 26), (257, 130, 1034), (300, 208, 1040)]


def _c32_async_configs():
    return [c for c in range(mg.num_configs(mg.MODE_C32)) if mg.config_chunk(mg.MODE_C32, c) > 0]


@pytest.mark.parametrize("m,n,k", C32_CHUNKED)
def test_c32_async_tiles_chunked_shapes(m, n, k):
    """The asynchronous-copy complex tiles: within the component bound of the
    binary64 complex oracle and bit for bit equal to the register-staged tile
    (each accumulator receives the same real products in the same order)."""
    log(f"c32 async tiles {(m, n, k)}")
    A, B = synth.pair_c64(m, n, k, seed=m + 3 * n + 7 * k)
    R = oracle.gemm_c128(A, B)
    dA, dB = dev(A), dev(B)
    ref = host(mg.gemm_c32(dA, dB, cfg=0))
    cfgs = _c32_async_configs()
    assert cfgs
    for cfg in cfgs:
        C = host(mg.gemm_c32(dA, dB, cfg=cfg))
        _assert_c32(C, R, A, B, k, f"c32 async {(m, n, k)} cfg {cfg}")
        assert np.array_equal(C.view(np.float32), ref.view(np.float32)), cfg


def test_c32_async_tiles_strides_and_fallback():
    """Even padded strides run the asynchronous-copy tiles; an odd stride or a
    base one complex element off 16-byte alignment falls back to the
    register-staged tile.  Same bits, nothing written outside C."""
    log("c32 async tiles strides/fallback")
    m, n, k = 140, 98, 260
    A, B = synth.pair_c64(m, n, k, seed=48)
    ref = host(mg.gemm_c32(dev(A), dev(B), cfg=0))
    for pad_a, pad_b, off in [(2, 4, 0), (1, 2, 0), (2, 4, 1)]:
        bufA = torch.zeros((m, k + pad_a + off), dtype=torch.complex64, device="cuda")
        bufB = torch.zeros((k, n + pad_b + off), dtype=torch.complex64, device="cuda")
        dA, dB = bufA[:, off:off + k], bufB[:, off:off + n]
        dA.copy_(dev(A))
        dB.copy_(dev(B))
        for cfg in _c32_async_configs():
            big = torch.full((m + 2, n + 2), complex("nan+nanj"), dtype=torch.complex64, device="cuda")
            mg.gemm_c32(dA, dB, out=big[1:m + 1, 1:n + 1], cfg=cfg)
            h = host(big)
            assert np.array_equal(h[1:m + 1, 1:n + 1].view(np.float32), ref.view(np.float32)), (pad_a, pad_b, off, cfg)
            mask = np.ones(h.shape, dtype=bool)
            mask[1:m + 1, 1:n + 1] = False
            assert np.isnan(h[mask].real).all() and np.isnan(h[mask].imag).all()


def test_c32_empty_and_k0():
    log("c32 k = 0")
    C = torch.full((5, 6), 7 + 7j, dtype=torch.complex64, device="cuda")
    mg.gemm_c32(torch.zeros((5, 0), dtype=torch.complex64, device="cuda"),
                torch.zeros((0, 6), dtype=torch.complex64, device="cuda"), out=C)
    assert np.array_equal(host(C), np.zeros((5, 6), np.complex64))


def test_c32_full_size_sampled():
    """The paper's 4096 x 4096 complex-float product (Table 2), on 512 sampled
    outputs plus one full row."""
    log("c32 4096^3 sampled")
    size = 4096
    A, B = synth.pair_c64(size, size, size, seed=0)
    C = host(mg.gemm_c32(dev(A), dev(B)))
    g = synth.rng(48)
    rows = g.integers(0, size, 512)
    cols = g.integers(0, size, 512)
    R = oracle.gemm_c128_sampled(A, B, rows, cols)
    a, b = A[rows].astype(np.complex128), B[:, cols].T.astype(np.complex128)
    gk = (2 * size + 2) * U32
    br = gk * np.sum(np.abs(a.real) * np.abs(b.real) + np.abs(a.imag) * np.abs(b.imag), axis=1)
    bi = gk * np.sum(np.abs(a.real) * np.abs(b.imag) + np.abs(a.imag) * np.abs(b.real), axis=1)
    c = C[rows, cols].astype(np.complex128)
    assert np.all(np.abs(c.real - R.real) <= br) and np.all(np.abs(c.imag - R.imag) <= bi)
    r = size // 3
    Rrow = oracle.gemm_c128_sampled(A, B, np.full(size, r), np.arange(size))
    assert oracle.relerr(C[r].view(np.float32), Rrow.view(np.float64)) <= 1e-5


# ---------------------------------------------------------------- addition

ADD_SHAPES = [(1, 1), (3, 5), (7, 9), (17, 1000), (64, 4096), (300, 257), (1, 5000)]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("m,n", ADD_SHAPES)
def test_add_bit_exact(dtype, m, n):
    log(f"add {dtype} {(m, n)}")
    g = synth.rng(m * 13 + n)
    A = synth.draw(g, (m, n), "wide") if dtype == "f32" else synth.draw64(g, (m, n), "wide")
    B = synth.draw(g, (m, n), "wide") if dtype == "f32" else synth.draw64(g, (m, n), "wide")
    dA, dB = dev(A), dev(B)
    for sub in (False, True):
        C = host(mg.add(dA, dB, subtract=sub))
        assert np.array_equal(C, oracle.add(A, B, subtract=sub).astype(A.dtype)), sub


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_add_in_place_strided_and_guard_band(dtype):
    log(f"add {dtype} in place / strided")
    m, n = 123, 75
    tdt = torch.float32 if dtype == "f32" else torch.float64
    g = synth.rng(51)
    A = synth.draw64(g, (m, n), "normal").astype(np.float32 if dtype == "f32" else np.float64)
    B = synth.draw64(g, (m, n), "normal").astype(A.dtype)
    ref = oracle.add(A, B).astype(A.dtype)
    bufA = torch.full((m + 2, n + 9), float("nan"), dtype=tdt, device="cuda")
    bufA[1:m + 1, 1:n + 1] = dev(A)
    vA = bufA[1:m + 1, 1:n + 1]
    mg.add(vA, dev(B), out=vA)   # in place, misaligned by one element, padded stride
    full = host(bufA)
    assert np.array_equal(full[1:m + 1, 1:n + 1], ref)
    mask = np.ones(full.shape, dtype=bool)
    mask[1:m + 1, 1:n + 1] = False
    assert np.isnan(full[mask]).all()


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_add_paper_size(dtype):
    """The paper's 4096 x 4096 addition (Results section), every element."""
    log(f"add {dtype} 4096^2")
    g = synth.rng(52)
    A = synth.draw(g, (4096, 4096)) if dtype == "f32" else synth.draw64(g, (4096, 4096))
    B = synth.draw(g, (4096, 4096)) if dtype == "f32" else synth.draw64(g, (4096, 4096))
    C = host(mg.add(dev(A), dev(B), subtract=True))
    assert np.array_equal(C, oracle.add(A, B, subtract=True).astype(A.dtype))
