"""A seeded sweep of random problems through gemm_plain_cfg: every mode of a
gemm_problem_t, random m, n, k (log-uniform in [1, 600]), row strides
padded by 0-9 elements, operands starting 0-3 elements into their buffers
(so 16-byte alignment comes and goes; every fourth case keeps k, n, strides
and bases in whole 16-byte chunks, so the asynchronous-copy configurations
run as drawn), a random tile configuration and split-K factor.  Each output
is checked against the oracle of the operands the kernel sees (the binary64
product; for the reduced-precision forms the exact product of the quantised
operands) within the float32 accumulation bound, and C sits in a NaN-filled
buffer whose border must stay NaN."""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import abs_product, log
from tests.test_precision_gpu import check_bound, quantise_host, secondary

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1306_6192_amd as mg  # noqa: E402

MODES = [mg.MODE_F32, mg.MODE_BF16, mg.MODE_F16, mg.MODE_F8E4M3, mg.MODE_SPLIT_BF16X3]
CASES = 40


def _case(mode, i):
    g = synth.rng(1000 * mode + i)
    m, n, k = (int(x) for x in np.exp(g.uniform(0, np.log(600), 3)).round().clip(1, 600))
    pads = [int(x) for x in g.integers(0, 10, 3)]
    offs = [int(x) for x in g.integers(0, 4, 2)]
    if i % 4 == 0:
        # k, n, strides and bases whole 16-byte chunks: the asynchronous-copy
        # configurations run as drawn instead of falling back
        n, k = -(-n // 16) * 16, -(-k // 16) * 16
        pads[0], pads[1] = 16 * (pads[0] % 2), 16 * (pads[1] % 2)
        offs = [0, 0]
    cfg = int(g.integers(0, mg.num_configs(mode)))
    split = int(g.integers(1, 5))
    dist = "normal" if i % 2 else "uniform"
    return m, n, k, pads, offs, cfg, split, dist


def _placed(codes, pad, off, dtype):
    """`codes` (rows x cols, numpy) placed in a wider device buffer: a view
    with row stride cols + pad + off starting `off` elements in."""
    rows, cols = codes.shape
    buf = torch.zeros((rows, cols + pad + off), dtype=dtype, device="cuda")
    view = buf[:, off:off + cols]
    view.copy_(torch.from_numpy(np.ascontiguousarray(codes)).to(dtype).cuda())
    return view


@pytest.mark.parametrize("mode", MODES)
def test_random_problems(mode):
    for i in range(CASES):
        m, n, k, pads, offs, cfg, split, dist = _case(mode, i)
        what = f"{mg.MODE_NAMES[mode]} case {i}: {(m, n, k)} pads {pads} offsets {offs} cfg {cfg} split {split}"
        log(what)
        A, B = synth.pair(m, n, k, seed=7000 + 100 * mode + i, dist=dist)
        sa = sb = 1.0
        if mode in (mg.MODE_F32, mg.MODE_SPLIT_BF16X3):
            dA = _placed(A, pads[0], offs[0], torch.float32)
            dB = _placed(B, pads[1], offs[1], torch.float32)
        else:
            qa, _, sa = quantise_host(A, mode)
            qb, _, sb = quantise_host(B, mode)
            dt = torch.uint8 if mode == mg.MODE_F8E4M3 else torch.int16
            dA = _placed(qa.view(np.int16) if dt == torch.int16 else qa, pads[0], offs[0], dt)
            dB = _placed(qb.view(np.int16) if dt == torch.int16 else qb, pads[1], offs[1], dt)
        buf = torch.full((m + 2, n + pads[2] + 2), float("nan"), device="cuda")
        C = buf[1:m + 1, 1:n + 1]
        mg.gemm(dA, dB, out=C, mode=mode, scale_a=sa, scale_b=sb, cfg=cfg, split_k=split)
        h = buf.cpu().numpy()
        got = h[1:m + 1, 1:n + 1]
        border = np.ones_like(h, dtype=bool)
        border[1:m + 1, 1:n + 1] = False
        assert np.isnan(h[border]).all(), f"{what}: a write outside C"
        if mode == mg.MODE_F32:
            check_bound(got, oracle.gemm(A, B), abs_product(A, B), k, what)
        else:
            R, W, terms, extra = secondary(A, B, mode)
            check_bound(got, R, W, terms, what, extra)
