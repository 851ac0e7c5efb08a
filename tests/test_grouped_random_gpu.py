"""A seeded sweep of random problems through one grouped launch per mode:
m, n, k log-uniform in [1, 600], row strides padded by 0-9 elements and
operands starting 0-3 elements into their buffers (so rows start at any
element alignment), each C inside a NaN-filled buffer.  Every grouped result
must equal the plain launch of the same problem bit for bit (the plain
launch is pinned to the oracle by the random-shape and precision tests), and
no write may land outside C.  Exercises the grouped stream's edge handling:
k and n tails, the last rows' clamped chunks, and problems below one 16-byte
chunk of k or n."""
import numpy as np
import pytest

import synth
from tests._gpu import host, log
from tests.test_precision_gpu import quantise_host
from tests.test_random_shapes_gpu import _placed

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1306_6192_amd as mg  # noqa: E402

MODES = [mg.MODE_F32, mg.MODE_BF16, mg.MODE_F16, mg.MODE_F8E4M3, mg.MODE_SPLIT_BF16X3]
COUNT = 60


@pytest.mark.parametrize("mode", MODES)
def test_grouped_random_problems_match_plain(mode):
    log(f"grouped random {mg.MODE_NAMES[mode]}")
    g = synth.rng(5000 + mode)
    cases = []
    for i in range(COUNT):
        m, n, k = (int(x) for x in np.exp(g.uniform(0, np.log(600), 3)).round().clip(1, 600))
        pads = [int(x) for x in g.integers(0, 10, 3)]
        offs = [int(x) for x in g.integers(0, 4, 2)]
        A, B = synth.pair(m, n, k, seed=9000 + 100 * mode + i, dist="normal")
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
        cases.append(((m, n, k), pads, offs, dA, dB, buf, buf[1:m + 1, 1:n + 1], sa, sb))
    ops = [(c[3], c[4], c[6], c[7], c[8]) if mode == mg.MODE_F8E4M3 else (c[3], c[4], c[6]) for c in cases]
    mg.grouped(ops, mode=mode)
    for i, (shape, pads, offs, dA, dB, buf, C, sa, sb) in enumerate(cases):
        what = f"{mg.MODE_NAMES[mode]} problem {i}: {shape} pads {pads} offsets {offs}"
        h = host(buf)
        border = np.ones_like(h, dtype=bool)
        border[1:shape[0] + 1, 1:shape[1] + 1] = False
        assert np.isnan(h[border]).all(), f"{what}: a write outside C"
        ref = host(mg.gemm(dA, dB, mode=mode, scale_a=sa, scale_b=sb, cfg=0, split_k=1))
        got = h[1:shape[0] + 1, 1:shape[1] + 1]
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), what
