"""Parity of the FP32 product (gemm_plain / gemm_plain_cfg) with the binary64
oracle, through the C-ABI.  Tolerance: every element within the float32
worst-case bound (k + 2) u32 (|A||B|)_ij, and the normwise relative error
within 1e-6 at m = n = k = 512 and 1e-5 at the large shapes.  Integer-valued,
identity and diagonal inputs, whose every partial sum is exact, must match
bit for bit."""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import abs_product, assert_within_bound, dev, host, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1306_6192_amd as mg  # noqa: E402

EDGE_SHAPES = [(1, 1, 1), (2, 3, 4), (7, 5, 3), (31, 33, 17), (32, 32, 32), (33, 31, 65), (64, 64, 64),
               (127, 129, 255), (128, 128, 128), (129, 257, 100), (255, 3, 513), (3, 255, 1000),
               (257, 129, 31), (300, 200, 1), (97, 61, 4099)]


def _configs():
    return list(range(mg.num_configs(mg.MODE_F32)))


def test_c1_512_cube_seed0():
    log("plain f32 512^3 seed 0")
    A, B = synth.pair(512, 512, 512, seed=0)
    R = oracle.gemm(A, B)
    C = host(mg.gemm(dev(A), dev(B)))
    assert oracle.relerr(C, R) <= 1e-6
    assert_within_bound(C, R, abs_product(A, B), 512, "512^3")


@pytest.mark.parametrize("m,n,k", EDGE_SHAPES)
def test_edge_shapes_every_config(m, n, k):
    log(f"plain f32 edge shape {(m, n, k)}")
    A, B = synth.pair(m, n, k, seed=m * 7 + n * 3 + k)
    R = oracle.gemm(A, B)
    absAB = abs_product(A, B)
    dA, dB = dev(A), dev(B)
    for cfg in _configs():
        for split in (1, 3):
            C = host(mg.gemm(dA, dB, cfg=cfg, split_k=split))
            assert_within_bound(C, R, absAB, k, f"shape {(m, n, k)} cfg {cfg} split {split}")
            # normwise: 1e-6 up to k = 1024 (the 512^3 workload's bound), 1e-5 beyond
            assert oracle.relerr(C, R) <= (1e-6 if k <= 1024 else 1e-5)


@pytest.mark.parametrize("m,n,k", [(64, 64, 64), (200, 300, 1000), (513, 257, 4096)])
def test_integer_inputs_bit_exact(m, n, k):
    """Entries in [-16, 16] with k * 16^2 < 2^24: every float32 partial sum is
    an exactly representable integer, so any summation order is exact."""
    log(f"plain f32 integer-exact {(m, n, k)}")
    A, B = synth.pair(m, n, k, seed=21, dist="integers", R=16)
    R = oracle.gemm(A, B)
    dA, dB = dev(A), dev(B)
    for cfg in _configs():
        for split in (1, 2, 5):
            C = host(mg.gemm(dA, dB, cfg=cfg, split_k=split))
            assert np.array_equal(C.astype(np.float64), R), (cfg, split)


def test_identity_and_diagonal_bit_exact():
    log("plain f32 identity/diagonal")
    g = synth.rng(22)
    A = synth.draw(g, (150, 70), "normal")
    C = host(mg.gemm(dev(A), dev(np.eye(70, dtype=np.float32))))
    assert np.array_equal(C, A)
    C = host(mg.gemm(dev(np.eye(150, dtype=np.float32)), dev(A)))
    assert np.array_equal(C, A)
    d = synth.draw(g, (150,), "normal")
    C = host(mg.gemm(dev(np.diag(d).astype(np.float32)), dev(A)))
    assert np.array_equal(C, (d[:, None] * A).astype(np.float32))   # RN32(d_i a_ij)
    # the oracle value is the exact product here, rounded once to float32
    assert np.array_equal(C, oracle.gemm(np.diag(d), A).astype(np.float32))


def test_padded_and_misaligned_strides():
    """Row strides that are not multiples of 4 elements and base pointers off
    16-byte alignment take the element-wise load/store paths."""
    log("plain f32 padded/misaligned strides")
    m, n, k = 133, 77, 301
    A, B = synth.pair(m, n, k, seed=23)
    R = oracle.gemm(A, B)
    absAB = abs_product(A, B)
    bigA = torch.zeros((m, k + 3 + 1), device="cuda")
    bigB = torch.zeros((k, n + 5 + 1), device="cuda")
    dA = bigA[:, 1:k + 1]
    dB = bigB[:, 1:n + 1]
    dA.copy_(dev(A))
    dB.copy_(dev(B))
    bigC = torch.full((m, n + 7), 7.0, device="cuda")
    out = bigC[:, 1:n + 1]
    for cfg in _configs():
        mg.gemm(dA, dB, out=out, cfg=cfg, split_k=1)
        C = host(out)
        assert_within_bound(C, R, absAB, k, f"padded cfg {cfg}")
    h = host(bigC)
    assert np.all(h[:, 0] == 7.0) and np.all(h[:, n + 1:] == 7.0)


def test_guard_band_canaries():
    """Writes stay inside C: a frame of sentinel rows/columns around the output
    is untouched for every configuration and split."""
    log("plain f32 guard band")
    m, n, k = 97, 101, 203
    A, B = synth.pair(m, n, k, seed=24)
    dA, dB = dev(A), dev(B)
    G = 16
    for cfg in _configs():
        for split in (1, 4):
            big = torch.full((m + 2 * G, n + 2 * G), -12345.0, device="cuda")
            out = big[G:G + m, G:G + n]
            mg.gemm(dA, dB, out=out, cfg=cfg, split_k=split)
            h = host(big)
            frame = np.ones(h.shape, bool)
            frame[G:G + m, G:G + n] = False
            assert np.all(h[frame] == -12345.0), (cfg, split)


def test_repeat_and_cross_config_bitwise():
    """Same inputs -> same bits on a re-run; without split-K every tile
    configuration sums each element in the same order, so all agree bitwise."""
    log("plain f32 determinism")
    A, B = synth.pair(300, 260, 777, seed=25, dist="normal")
    dA, dB = dev(A), dev(B)
    ref = host(mg.gemm(dA, dB, cfg=0, split_k=1))
    assert np.array_equal(ref, host(mg.gemm(dA, dB, cfg=0, split_k=1)))
    for cfg in _configs():
        assert np.array_equal(ref, host(mg.gemm(dA, dB, cfg=cfg, split_k=1))), cfg
    s3 = host(mg.gemm(dA, dB, cfg=3, split_k=3))
    assert np.array_equal(s3, host(mg.gemm(dA, dB, cfg=3, split_k=3)))


# k and n whole 16-byte chunks (multiples of 4 floats): the asynchronous-copy
# tiles run these; ragged m, n not a multiple of the tile, k with a partial
# k-tile of 16, one-row and one-chunk extremes
CHUNKED_SHAPES = [(1, 4, 4), (33, 36, 20), (64, 512, 16), (129, 388, 8), (257, 132, 1036), (300, 208, 1040),
                  (513, 260, 4100)]


def _chunked_configs():
    return [c for c in _configs() if mg.config_chunk(mg.MODE_F32, c) > 0]


@pytest.mark.parametrize("m,n,k", CHUNKED_SHAPES)
def test_async_tiles_chunked_shapes(m, n, k):
    """The asynchronous-copy FP32 tiles on shapes they accept: within the
    float32 bound of the oracle, and bit for bit equal to the register-staged
    tile (same MFMA sequence per element), with and without split-K."""
    log(f"plain f32 async tiles {(m, n, k)}")
    A, B = synth.pair(m, n, k, seed=m + 5 * n + 11 * k, dist="normal")
    R = oracle.gemm(A, B)
    absAB = abs_product(A, B)
    dA, dB = dev(A), dev(B)
    assert _chunked_configs()
    for split in (1, 3):
        ref = host(mg.gemm(dA, dB, cfg=0, split_k=split))
        for cfg in _chunked_configs():
            C = host(mg.gemm(dA, dB, cfg=cfg, split_k=split))
            assert_within_bound(C, R, absAB, k, f"shape {(m, n, k)} cfg {cfg} split {split}")
            assert np.array_equal(C, ref), (cfg, split)


def test_async_tiles_strides_and_fallback():
    """Padded row strides that stay whole chunks run the asynchronous-copy
    tiles; a base pointer off 16-byte alignment or a stride that is not a
    whole chunk falls back to the register-staged tile of the same size.  All
    give the same bits and leave the frame around C untouched."""
    log("plain f32 async tiles strides/fallback")
    m, n, k = 200, 132, 520
    A, B = synth.pair(m, n, k, seed=31, dist="normal")
    ref = host(mg.gemm(dev(A), dev(B), cfg=0, split_k=1))
    for pad_a, pad_b, off in [(4, 8, 0), (3, 4, 0), (4, 8, 1)]:
        bigA = torch.zeros((m, k + pad_a + off), device="cuda")
        bigB = torch.zeros((k, n + pad_b + off), device="cuda")
        dA = bigA[:, off:off + k]
        dB = bigB[:, off:off + n]
        dA.copy_(dev(A))
        dB.copy_(dev(B))
        for cfg in _chunked_configs():
            big = torch.full((m + 2, n + 2), -7.0, device="cuda")
            mg.gemm(dA, dB, out=big[1:m + 1, 1:n + 1], cfg=cfg, split_k=1)
            h = host(big)
            assert np.array_equal(h[1:m + 1, 1:n + 1], ref), (pad_a, pad_b, off, cfg)
            frame = np.ones(h.shape, bool)
            frame[1:m + 1, 1:n + 1] = False
            assert np.all(h[frame] == -7.0)


def test_empty_and_k_zero():
    log("plain f32 empty/k=0")
    out = torch.full((5, 7), 3.0, device="cuda")
    mg.gemm(torch.zeros((5, 0), device="cuda"), torch.zeros((0, 7), device="cuda"), out=out)
    assert np.all(host(out) == 0.0)
    o2 = torch.empty((0, 7), device="cuda")
    mg.gemm(torch.zeros((0, 4), device="cuda"), torch.zeros((4, 7), device="cuda"), out=o2)


LARGE = [(2048, 2048, 2048), (4096, 4096, 4096), (8192, 8192, 8192), (8192, 1024, 4096), (128, 8192, 8192)]


@pytest.mark.parametrize("m,n,k", LARGE)
def test_large_shapes_sampled(m, n, k):
    """The plain FP32 workloads at full size, launched as the benchmark
    launches them (tuning-table choice), checked on 1024 sampled outputs plus
    two full rows against the oracle."""
    log(f"plain f32 large {(m, n, k)}")
    A, B = synth.pair(m, n, k, seed=0)
    C = host(mg.gemm(dev(A), dev(B)))
    g = synth.rng(99)
    rows = g.integers(0, m, size=1024)
    cols = g.integers(0, n, size=1024)
    R = oracle.gemm_sampled(A, B, rows, cols)
    absAB = np.array([np.abs(A[i].astype(np.float64)) @ np.abs(B[:, j].astype(np.float64))
                      for i, j in zip(rows, cols)])
    assert_within_bound(C[rows, cols], R, absAB, k, f"large {(m, n, k)}")
    assert oracle.relerr(C[rows, cols], R) <= 1e-5
    full_rows = [0, m - 1]
    Rr = oracle.gemm_rows(A, B, full_rows)
    assert oracle.relerr(C[full_rows], Rr) <= 1e-5
