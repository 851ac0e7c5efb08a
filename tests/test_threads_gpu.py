"""Two host threads enqueueing products on the same stream.  The library's
split-K workspace belongs to the (device, stream) pair and grows on demand;
each caller holds the stream's workspace lock from the buffer's growth to
the enqueue of the kernels that use it, so neither thread's kernels can
run on a buffer the other thread has just replaced.  Every product must
match the same product computed alone, bit for bit."""
import threading

import numpy as np
import pytest

import synth
from tests._gpu import dev, host, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1306_6192_amd as mg  # noqa: E402


def test_two_threads_on_one_stream():
    log("two host threads, one stream, growing split-K workspace")
    shapes = [(48 * i, 80 * i, 640) for i in range(1, 11)]       # 4-way split-K slabs grow with m n
    ops = []
    for i, (m, n, k) in enumerate(shapes):
        A, B = synth.pair(m, n, k, seed=300 + i)
        ops.append((dev(A), dev(B)))
    cfg = 3   # a register-staged 128 x 128 tile: any shape
    ref = [host(mg.gemm(a, b, cfg=cfg, split_k=4)) for a, b in ops]
    torch.cuda.synchronize()
    outs = {}
    errors = []

    def run(tid, rep, stream):
        try:
            for i in range(tid, len(ops)):       # both threads grow the fresh stream's workspace
                a, b = ops[i]
                outs[(tid, rep, i)] = mg.gemm(a, b, cfg=cfg, split_k=4, stream=stream)
        except Exception as e:   # reported after join
            errors.append(e)

    for rep in range(4):
        stream = torch.cuda.Stream()             # a new stream starts with an empty workspace
        threads = [threading.Thread(target=run, args=(t, rep, stream)) for t in range(2)]
        for t in threads:
            t.start()
        for t in threads:
            t.join(timeout=120)
        assert not any(t.is_alive() for t in threads), "a thread did not finish"
        stream.synchronize()
    assert not errors, errors
    torch.cuda.synchronize()
    assert len(outs) == 4 * (2 * len(ops) - 1)
    for (tid, rep, i), C in outs.items():
        assert np.array_equal(host(C), ref[i]), (tid, rep, shapes[i])
