"""Outputs and operands past 2^31 elements, through the C-ABI.

Every kernel family forms its global addresses in 64 bits; these products put
rows of C (and, in two cases, rows of A or B) beyond element 2^31 of their
allocation.  Inputs are integer-valued (|x| <= 16, every partial sum an exact
integer in the kernel's arithmetic), so the sampled rows must equal the
oracle's bit for bit.  C starts as NaN with padding columns: afterwards no
output may be NaN (every one was written) and every padding element must be
(nothing was written beyond column n)."""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import dev, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1306_6192_amd as mg  # noqa: E402

TWO31 = 2 ** 31


def _sample_rows(m, ld):
    """Both ends, the rows around the first one that starts past element
    2^31 of a buffer with row stride ld, and eight drawn ones."""
    far = -(-TWO31 // ld)
    rows = {0, 1, far - 1, far, far + 1, m - 2, m - 1}
    rows |= set(synth.rng(m + ld).integers(0, m, 8).tolist())
    return sorted(r for r in rows if 0 <= r < m)


def _padded_out(m, n, pad, dtype):
    nan = complex(float("nan"), float("nan")) if dtype == torch.complex64 else float("nan")
    buf = torch.full((m, n + pad), nan, dtype=dtype, device="cuda")
    return buf, buf[:, :n]


def _check(buf, n, rows, R, what):
    torch.cuda.synchronize()
    assert not torch.isnan(buf[:, :n]).any().item(), f"{what}: an output was not written"
    if buf.shape[1] > n:
        assert torch.isnan(buf[:, n:]).all().item(), f"{what}: a write beyond column n"
    got = buf[torch.as_tensor(rows, device="cuda"), :n].cpu().numpy()
    assert np.array_equal(got.astype(R.dtype), R), f"{what}: sampled rows differ from the oracle"


def _free():
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


# (m, n, k, A row padding, C row padding, cfg, split); None = tuning table
F32_CASES = [
    (50001, 45003, 20, 0, 5, None, None),      # ragged, tuned choice
    (50001, 45003, 20, 0, 5, 0, 1),            # register-staged 256x256
    (50000, 45056, 32, 45024, 8, 20, 1),       # asynchronous copy, k-tiles of 32; A is 9 GB (lda 45056)
    (50000, 45056, 32, 0, 8, 13, 1),           # asynchronous copy, k-tiles of 16
    (33001, 33003, 96, 0, 5, 3, 3),            # split-K: the third partial slab starts past 2^31
    (33000, 33004, 96, 0, 8, 15, 3),           # the same on an asynchronous-copy tile
    (50001, 45003, 20, 45011, 5, 25, 1),       # asynchronous copy with 4-byte loads, ragged; A is 9 GB
    (33001, 33003, 96, 0, 5, 26, 3),           # the same (64 x 64), split-K slab past 2^31
]


@pytest.mark.parametrize("m,n,k,pad_a,pad_c,cfg,split", F32_CASES)
def test_f32_past_2_31(m, n, k, pad_a, pad_c, cfg, split):
    log(f"limits f32 {(m, n, k)} lda pad {pad_a} ldc pad {pad_c} cfg {cfg} split {split}")
    A, B = synth.pair(m, n, k, seed=m + n + k, dist="integers", R=16)
    if pad_a:
        abuf = torch.empty((m, k + pad_a), dtype=torch.float32, device="cuda")
        dA = abuf[:, :k]
        dA.copy_(dev(A))
    else:
        dA = dev(A)
    buf, C = _padded_out(m, n, pad_c, torch.float32)
    mg.gemm(dA, dev(B), out=C, cfg=cfg, split_k=split)
    rows = _sample_rows(m, n + pad_c)
    _check(buf, n, rows, oracle.gemm(A[rows], B), f"f32 {(m, n, k)} cfg {cfg} split {split}")
    del buf, C, dA
    _free()


@pytest.mark.parametrize("cfg", [None, 20, 25])
def test_f32_b_rows_past_2_31(cfg):
    """B rows 2^26 + 64 elements apart: row 32 onwards starts past element
    2^31 of B's allocation (12.9 GB)."""
    m, n, k, ldb = 4096, 4100, 48, 2 ** 26 + 64
    log(f"limits f32 B stride {ldb} cfg {cfg}")
    A, B = synth.pair(m, n, k, seed=5, dist="integers", R=16)
    bbuf = torch.empty((k, ldb), dtype=torch.float32, device="cuda")
    dB = bbuf[:, :n]
    dB.copy_(dev(B))
    buf, C = _padded_out(m, n, 4, torch.float32)
    mg.gemm(dev(A), dB, out=C, cfg=cfg, split_k=None if cfg is None else 1)
    rows = _sample_rows(m, n + 4)
    _check(buf, n, rows, oracle.gemm(A[rows], B), f"f32 B stride {ldb} cfg {cfg}")
    del buf, C, dB, bbuf
    _free()


@pytest.mark.parametrize("m,n,k,pad_c", [(50001, 45003, 32, 5), (50000, 45056, 64, 8)])
def test_bf16_past_2_31(m, n, k, pad_c):
    log(f"limits bf16 {(m, n, k)}")
    A, B = synth.pair(m, n, k, seed=m + k, dist="integers", R=16)
    qa, qb = mg.convert(dev(A), mg.MODE_BF16), mg.convert(dev(B), mg.MODE_BF16)
    buf, C = _padded_out(m, n, pad_c, torch.float32)
    mg.gemm(qa, qb, out=C, mode=mg.MODE_BF16)
    rows = _sample_rows(m, n + pad_c)
    _check(buf, n, rows, oracle.gemm(A[rows], B), f"bf16 {(m, n, k)}")
    del buf, C, qa, qb
    _free()


def _family_cases(mode):
    async_cfgs = [c for c in range(mg.num_configs(mode)) if mg.config_chunk(mode, c) > 0]
    return [((46341, 46343), None), ((46341, 46343), 0)] + [((46342, 46344), c) for c in async_cfgs]


@pytest.mark.parametrize("case", range(4))
def test_f64_past_2_31(case):
    """C of 2.15·10⁹ doubles (17.2 GB): register-staged (odd n) and every
    asynchronous-copy tile (even n)."""
    cases = _family_cases(mg.MODE_F64)
    if case >= len(cases):
        pytest.skip("fewer asynchronous-copy binary64 tiles")
    (m, n), cfg = cases[case]
    k = 16
    log(f"limits f64 {(m, n, k)} cfg {cfg}")
    A, B = synth.pair64(m, n, k, seed=m + n, dist="integers", R=16)
    buf, C = _padded_out(m, n, 2, torch.float64)
    mg.gemm_f64(dev(A), dev(B), out=C, cfg=cfg)
    rows = _sample_rows(m, n + 2)
    _check(buf, n, rows, oracle.gemm(A[rows], B), f"f64 {(m, n, k)} cfg {cfg}")
    del buf, C
    _free()


@pytest.mark.parametrize("case", range(4))
def test_c32_past_2_31(case):
    """C of 2.15·10⁹ complex floats (17.2 GB), Gaussian-integer inputs."""
    cases = _family_cases(mg.MODE_C32)
    if case >= len(cases):
        pytest.skip("fewer asynchronous-copy complex tiles")
    (m, n), cfg = cases[case]
    k = 8
    log(f"limits c32 {(m, n, k)} cfg {cfg}")
    A, B = synth.pair_c64(m, n, k, seed=m + n + 1, dist="integers", R=16)
    buf, C = _padded_out(m, n, 2, torch.complex64)
    mg.gemm_c32(dev(A), dev(B), out=C, cfg=cfg)
    rows = _sample_rows(m, n + 2)
    R = oracle.gemm_c128(A[rows], B)
    _check(buf, n, rows, R, f"c32 {(m, n, k)} cfg {cfg}")
    del buf, C
    _free()
