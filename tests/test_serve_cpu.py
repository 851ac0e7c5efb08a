"""Serving runtime on the host fake executor (no GPU): admission, ordering,
back-pressure, failure isolation and latency accounting."""
import ctypes

import numpy as np
import pytest

import synth
from paper_1306_6192_amd import _lib

FAKE_BASE = 0x100000000


def fake_problem(i, m, n, k, mode=0):
    """A problem with distinct fake device addresses (never dereferenced)."""
    base = FAKE_BASE + i * (1 << 40)
    return _lib.problem(mode, m, n, k, base, k, base + (1 << 37), n, base + (2 << 37), n)


def make_server(**kw):
    cfg = dict(hbm_budget_bytes=1 << 30, max_inflight=64, num_streams=4, max_batch=16, queue_capacity=10000,
               executor=1, fake_fail_every=0)
    cfg.update(kw)
    h = ctypes.c_void_p()
    rc = _lib.load().gemm_serve_create(ctypes.byref(_lib.ServeConfig(**cfg)), ctypes.byref(h))
    assert rc == 0, _lib.last_error()
    return h


def submit(h, p, t=0):
    t_out = ctypes.c_uint64()
    rc = _lib.load().gemm_serve_submit(h, ctypes.byref(p), t, ctypes.byref(t_out))
    return rc, t_out.value


def poll(h, ticket):
    r = _lib.ServeResult()
    rc = _lib.load().gemm_serve_poll(h, ticket, ctypes.byref(r))
    return rc, r


def stats(h):
    s = _lib.ServeStats()
    assert _lib.load().gemm_serve_stats(h, ctypes.byref(s)) == 0
    return s


def footprint(p):
    f = ctypes.c_uint64()
    assert _lib.load().gemm_serve_footprint(ctypes.byref(p), ctypes.byref(f)) == 0
    return f.value


def test_footprint_definition():
    p = fake_problem(0, 100, 200, 300)
    assert footprint(p) == 4 * (100 * 300 + 300 * 200 + 100 * 200)
    p = fake_problem(0, 100, 200, 300, mode=1)
    assert footprint(p) == 2 * (100 * 300 + 300 * 200) + 4 * 100 * 200
    p = fake_problem(0, 100, 200, 300, mode=3)
    assert footprint(p) == (100 * 300 + 300 * 200) + 4 * 100 * 200


def test_admission_budget_fifo_and_completion():
    lib = _lib.load()
    dims = synth.loguniform_dims(300, 16, 512, seed=3)
    probs = [fake_problem(i, *map(int, d)) for i, d in enumerate(dims)]
    fps = [footprint(p) for p in probs]
    budget = max(fps) * 3
    h = make_server(hbm_budget_bytes=budget, max_inflight=8, num_streams=2, max_batch=4)
    tickets = []
    for p in probs:
        rc, t = submit(h, p)
        assert rc == 0
        tickets.append(t)
    assert tickets == sorted(tickets) and len(set(tickets)) == len(tickets)     # monotonic tickets
    assert lib.gemm_serve_drain(h) == 0
    s = stats(h)
    assert s.completed == 300 and s.failed == 0 and s.queued == 0 and s.inflight == 0
    assert s.inflight_bytes == 0
    assert 0 < s.peak_inflight_bytes <= budget
    res = []
    for t in tickets:
        rc, r = poll(h, t)
        assert rc == 0 and r.status == 0
        assert r.t_arrival_ns <= r.t_admit_ns <= r.t_launch_ns <= r.t_done_ns
        assert 1 <= r.batch_size <= 4
        res.append(r)
    admits = [r.t_admit_ns for r in res]
    assert admits == sorted(admits)                                             # FIFO admission
    # a polled ticket is gone
    rc, _ = poll(h, tickets[0])
    assert rc == _lib.GEMM_ENOTFOUND
    assert lib.gemm_serve_destroy(h) == 0


def test_over_budget_and_queue_full():
    lib = _lib.load()
    # 8192^3 keeps the fake executor busy for ~1.1 ms per request (1 us per
    # GFLOP), far longer than 50 submissions take
    p_small = fake_problem(0, 8192, 8192, 8192)
    p_big = fake_problem(1, 65536, 65536, 65536)
    h = make_server(hbm_budget_bytes=footprint(p_small) * 10, queue_capacity=3, max_inflight=1, num_streams=1,
                    max_batch=1)
    rc, _ = submit(h, p_big)
    assert rc == _lib.GEMM_ENOMEM and "budget" in _lib.last_error()
    # a queue of capacity 3 behind one in-flight slot fills up
    codes = [submit(h, p_small)[0] for _ in range(50)]
    assert _lib.GEMM_EBUSY in codes
    assert lib.gemm_serve_drain(h) == 0
    assert lib.gemm_serve_destroy(h) == 0


def test_injected_failure_fails_only_that_batch():
    lib = _lib.load()
    h = make_server(max_batch=1, num_streams=1, fake_fail_every=3)
    tickets = [submit(h, fake_problem(i, 32, 32, 32))[1] for i in range(12)]
    assert lib.gemm_serve_drain(h) == 0
    outcomes = []
    for t in tickets:
        rc, r = poll(h, t)
        outcomes.append(rc)
        assert (rc == 0) == (r.status == 0)
    assert outcomes.count(_lib.GEMM_EINTERNAL) == 4 and outcomes.count(0) == 8
    s = stats(h)
    assert s.failed == 4 and s.completed == 8
    # the server keeps serving after failures
    rc, t = submit(h, fake_problem(99, 8, 8, 8))
    assert rc == 0
    assert lib.gemm_serve_drain(h) == 0
    assert lib.gemm_serve_destroy(h) == 0


def test_replay_latency_from_scheduled_arrival():
    """Open-loop replay: every arrival stamp is the scheduled time, so the
    measured latency counts the time a request waited to be submitted."""
    lib = _lib.load()
    n = 200
    offs = (synth.poisson_arrivals(n, 20000.0, seed=1) * 1e9).astype(np.uint64)
    probs = _lib.problems_array([fake_problem(i, 64, 64, 64) for i in range(n)])
    h = make_server()
    tickets = (ctypes.c_uint64 * n)()
    t0 = lib.gemm_now_ns()
    rc = lib.gemm_serve_replay(h, probs, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), n, tickets)
    assert rc == 0
    assert lib.gemm_serve_drain(h) == 0
    arr = []
    for i in range(n):
        rc, r = poll(h, tickets[i])
        assert rc == 0
        arr.append(r.t_arrival_ns)
        assert r.t_done_ns >= r.t_arrival_ns
    arr = np.array(arr, dtype=np.int64) - int(t0)
    # arrival stamps follow the schedule (t0 is read just before the call)
    assert np.all(np.abs(np.diff(arr) - np.diff(offs.astype(np.int64))) < 1_000_000)
    assert lib.gemm_serve_destroy(h) == 0


def test_bad_configs_and_arguments():
    lib = _lib.load()
    h = ctypes.c_void_p()
    for bad in (dict(max_inflight=0), dict(num_streams=0), dict(num_streams=17), dict(max_batch=0),
                dict(queue_capacity=0), dict(hbm_budget_bytes=0), dict(executor=5), dict(fake_fail_every=-1)):
        cfg = dict(hbm_budget_bytes=1 << 30, max_inflight=4, num_streams=1, max_batch=1, queue_capacity=4,
                   executor=1, fake_fail_every=0)
        cfg.update(bad)
        assert lib.gemm_serve_create(ctypes.byref(_lib.ServeConfig(**cfg)), ctypes.byref(h)) == _lib.GEMM_EINVAL
    s = make_server()
    bad = fake_problem(0, 4, 4, 4)
    bad.lda = 1
    assert submit(s, bad)[0] == _lib.GEMM_EINVAL
    assert poll(s, 12345)[0] == _lib.GEMM_ENOTFOUND
    assert lib.gemm_serve_destroy(s) == 0
