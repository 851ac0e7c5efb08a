"""Grouped product (one persistent launch over many problems) and its graph
replay, through the C-ABI.  Every grouped result must equal the plain launch
of the same problem bit for bit (same tiles, same summation order), and the
plain launch is pinned to the oracle by the plain and precision tests; a
sample of problems is also checked against the oracle directly."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from paper_1306_6192_amd import _lib
from tests._gpu import abs_product, assert_within_bound, dev, host, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1306_6192_amd as mg  # noqa: E402


def _operands(A, B, mode):
    if mode == mg.MODE_F32:
        return dev(A), dev(B)
    return mg.convert(dev(A), mode), mg.convert(dev(B), mode)


def _group(count, lo, hi, seed, mode):
    probs = synth.grouped_problems(count, lo, hi, seed)
    ops = []
    for A, B in probs:
        a, b = _operands(A, B, mode)
        C = torch.full((A.shape[0], B.shape[1]), np.nan, device="cuda")
        ops.append((a, b, C))
    return probs, ops


@pytest.mark.parametrize("mode", [mg.MODE_F32, mg.MODE_BF16])
def test_grouped_512_matches_plain_bitwise(mode):
    """The grouped workload: 512 problems, m, n, k log-uniform in [32, 1024],
    seed 0; FP32, and BF16 inputs with float32 output."""
    log(f"grouped 512 {mg.MODE_NAMES[mode]}")
    probs, ops = _group(512, 32, 1024, 0, mode)
    mg.grouped(ops, mode=mode)
    got = [host(C) for (_, _, C) in ops]
    for i, (a, b, _) in enumerate(ops):
        ref = host(mg.gemm(a, b, mode=mode, cfg=3, split_k=1))
        assert np.array_equal(got[i], ref), f"problem {i} shape {a.shape}x{b.shape}"
    # a sample of problems against the oracle
    for i in range(0, 512, 37):
        A, B = probs[i]
        if mode == mg.MODE_F32:
            R, W = oracle.gemm(A, B), abs_product(A, B)
        else:
            from oracle import formats as F
            va, vb = F.decode(F.to_bf16_bits(A), "bf16"), F.decode(F.to_bf16_bits(B), "bf16")
            R, W = oracle.gemm(va, vb), abs_product(va, vb)
        assert_within_bound(got[i], R, W, A.shape[1], f"grouped problem {i}")


@pytest.mark.parametrize("mode", [mg.MODE_F32, mg.MODE_F16, mg.MODE_F8E4M3, mg.MODE_SPLIT_BF16X3])
def test_grouped_small_every_mode(mode):
    log(f"grouped small {mg.MODE_NAMES[mode]}")
    probs = synth.grouped_problems(40, 1, 300, seed=5)
    ops = []
    for A, B in probs:
        if mode == mg.MODE_F8E4M3:
            qa, sa = mg.quantize_e4m3(dev(A))
            qb, sb = mg.quantize_e4m3(dev(B))
            ops.append((qa, qb, torch.empty((A.shape[0], B.shape[1]), device="cuda"),
                        float(host(sa)[0]), float(host(sb)[0])))
        else:
            a, b = _operands(A, B, mode) if mode != mg.MODE_SPLIT_BF16X3 else (dev(A), dev(B))
            ops.append((a, b, torch.empty((A.shape[0], B.shape[1]), device="cuda")))
    mg.grouped(ops, mode=mode)
    for i, t in enumerate(ops):
        extra = dict(scale_a=t[3], scale_b=t[4]) if len(t) == 5 else {}
        ref = host(mg.gemm(t[0], t[1], mode=mode, cfg=0, split_k=1,
                           **extra))
        assert np.array_equal(host(t[2]), ref), i


def test_graph_replay_matches_direct_launch():
    """Captured once, replayed several times with eager work in between; every
    replay must reproduce the direct grouped launch bit for bit."""
    log("grouped graph replay")
    probs, ops = _group(64, 16, 512, 3, mg.MODE_F32)
    mg.grouped(ops)
    direct = [host(C).copy() for (_, _, C) in ops]
    graph = mg.GroupedGraph(ops)
    for rep in range(3):
        for (_, _, C) in ops:
            C.fill_(float("nan"))
        torch.cuda.synchronize()
        graph.launch()
        torch.cuda.synchronize()
        for i, (_, _, C) in enumerate(ops):
            assert np.array_equal(host(C), direct[i]), (rep, i)
        # unrelated eager work between replays
        x = torch.randn(1000, 1000, device="cuda")
        (x @ x).sum().item()
    graph.close()


def test_grouped_edge_cases():
    log("grouped edge cases")
    lib = _lib.load()
    # empty list, empty outputs, and k = 0 problems (zeros)
    assert lib.gemm_grouped(None, 0, None) == 0
    a = torch.zeros((5, 0), device="cuda")
    b = torch.zeros((0, 7), device="cuda")
    c = torch.full((5, 7), 3.0, device="cuda")
    e = torch.empty((0, 7), device="cuda")
    A, B = synth.pair(33, 17, 9, seed=1)
    c2 = torch.empty((33, 17), device="cuda")
    mg.grouped([(a, b, c), (torch.zeros((0, 4), device="cuda"), torch.zeros((4, 7), device="cuda"), e),
                (dev(A), dev(B), c2)])
    assert np.all(host(c) == 0.0)
    assert_within_bound(host(c2), oracle.gemm(A, B), abs_product(A, B), 9, "grouped tiny")
    # mixed modes are rejected
    p0 = mg.make_problem(dev(A), dev(B), c2, mg.MODE_F32)
    ab = mg.convert(dev(A), mg.MODE_BF16)
    bb = mg.convert(dev(B), mg.MODE_BF16)
    p1 = mg.make_problem(ab, bb, c2, mg.MODE_BF16)
    arr = _lib.problems_array([p0, p1])
    assert lib.gemm_grouped(arr, 2, None) == _lib.GEMM_EINVAL
    assert "mode" in _lib.last_error()
    h = ctypes.c_void_p()
    assert lib.gemm_grouped_graph_create(arr, 2, ctypes.byref(h)) == _lib.GEMM_EINVAL


def test_problem_batch_repeated_launches():
    """A ProblemBatch (problem array built once) launched repeatedly on one
    stream -- the descriptor uploads cycle through the pinned staging ring --
    gives the list form's bits every time."""
    log("grouped problem batch x6")
    probs, ops = _group(48, 32, 300, 7, mg.MODE_F32)
    mg.grouped(ops)
    want = [host(c).copy() for _, _, c in ops]
    batch = mg.ProblemBatch(ops)
    for rep in range(6):
        for _, _, c in ops:
            c.fill_(float("nan"))
        batch.run()
        for i, (_, _, c) in enumerate(ops):
            assert np.array_equal(host(c), want[i]), (rep, i)


@pytest.mark.parametrize("mode", [mg.MODE_F32, mg.MODE_BF16, mg.MODE_F16, mg.MODE_F8E4M3, mg.MODE_SPLIT_BF16X3])
def test_grouped_variant1_matches_plain_bitwise(mode, tmp_path):
    """The two-tile grouped kernel (variant 1, selected through the tuning
    table) gives the same bits as the plain launch too, on the grouped
    workload (FP32, BF16, F16) or a mixed batch (E4M3, split-BF16x3)."""
    import os
    log(f"grouped variant 1 {mg.MODE_NAMES[mode]}")
    lib = _lib.load()
    f = tmp_path / "v.jsonl"
    f.write_text('{"grouped_eff": %d, "eff": 0.600, "variant": 1}\n' % mode)
    _lib.check(lib.gemm_tuner_load(str(f).encode()))
    try:
        info = (ctypes.c_int32 * 7)()
        _lib.check(lib.gemm_grouped_info(mode, info))
        assert info[6] == 1 and info[0] != info[1]
        if mode == mg.MODE_F8E4M3:
            probs = synth.grouped_problems(200, 16, 1024, seed=11)
            ops = []
            for A, B in probs:
                qa, sa = mg.quantize_e4m3(dev(A))
                qb, sb = mg.quantize_e4m3(dev(B))
                ops.append((qa, qb, torch.empty((A.shape[0], B.shape[1]), device="cuda"),
                            float(host(sa)[0]), float(host(sb)[0])))
        elif mode == mg.MODE_SPLIT_BF16X3:
            probs = synth.grouped_problems(200, 16, 1024, seed=12)
            ops = [(dev(A), dev(B), torch.empty((A.shape[0], B.shape[1]), device="cuda")) for A, B in probs]
        else:
            probs, ops = _group(512, 32, 1024, 0, mode)
        cfgs = (ctypes.c_int32 * len(ops))()
        arr = _lib.problems_array([mg.make_problem(t[0], t[1], t[2], mode, *t[3:]) for t in ops])
        _lib.check(lib.gemm_grouped_plan(arr, len(ops), cfgs))
        assert {info[0], info[1]} <= set(cfgs) | {-1}, "both tiles are used"
        mg.grouped(ops, mode=mode)
        for i, t in enumerate(ops):
            extra = dict(scale_a=t[3], scale_b=t[4]) if len(t) == 5 else {}
            ref = host(mg.gemm(t[0], t[1], mode=mode, cfg=3, split_k=1, **extra))
            assert np.array_equal(host(t[2]), ref), f"problem {i}"
    finally:
        f.write_text('{"grouped_eff": %d, "eff": 0.600, "variant": 0}\n' % mode)
        _lib.check(lib.gemm_tuner_load(str(f).encode()))
        shipped = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                               "paper_1306_6192_amd", "tuning", "mi355x.jsonl")
        if os.path.exists(shipped):
            _lib.check(lib.gemm_tuner_load(shipped.encode()))


def test_tune_grouped_mix_records_a_variant(tmp_path):
    """gemm_tune_grouped_mix times the grouped kernel variants on a mixed
    batch and records one for the mode (the launch results stay the plain
    launch's bits whichever it picks); the shipped table is restored after."""
    import os
    log("grouped mix tuning")
    lib = _lib.load()
    mode = mg.MODE_BF16
    probs, ops = _group(60, 32, 600, 21, mode)
    arr = _lib.problems_array([mg.make_problem(a, b, c, mode) for a, b, c in ops])
    stream = torch.cuda.current_stream().cuda_stream
    try:
        _lib.check(lib.gemm_tune_grouped_mix(arr, len(ops), stream))
        info = (ctypes.c_int32 * 7)()
        _lib.check(lib.gemm_grouped_info(mode, info))
        assert info[6] in (0, 1)
        f = tmp_path / "t.jsonl"
        _lib.check(lib.gemm_tuner_save(str(f).encode()))
        assert any(ln.startswith('{"grouped_eff": %d,' % mode) for ln in f.read_text().splitlines())
        mg.grouped(ops, mode=mode)
        for i, (a, b, c) in enumerate(ops):
            assert np.array_equal(host(c), host(mg.gemm(a, b, mode=mode, cfg=3, split_k=1))), i
    finally:
        g = tmp_path / "r.jsonl"
        g.write_text('{"grouped_eff": %d, "eff": 0.600, "variant": 0}\n' % mode)
        _lib.check(lib.gemm_tuner_load(str(g).encode()))
        shipped = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                               "paper_1306_6192_amd", "tuning", "mi355x.jsonl")
        if os.path.exists(shipped):
            _lib.check(lib.gemm_tuner_load(shipped.encode()))
