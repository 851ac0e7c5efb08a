"""The grouped launch's static schedule, without a GPU (gemm_grouped_schedule
builds it on the host from fake device addresses that nothing
dereferences): every output tile of every problem appears exactly once, the
lists fit the launch, a workgroup's tiles are its XCD's (workgroup w runs on
XCD w mod 8, which holds whole problems where the balance allows), and the
work is balanced over the workgroups."""
import ctypes

import numpy as np
import pytest

import synth
from paper_1306_6192_amd import _lib

STRIDE = 1 << 32


def problems(mode, shapes):
    out = []
    for i, (m, n, k) in enumerate(shapes):
        base = (1 << 40) + 3 * i * STRIDE
        out.append(_lib.problem(mode, m, n, k, base, max(1, k), base + STRIDE, max(1, n), base + 2 * STRIDE,
                                max(1, n)))
    return out


def schedule(mode, shapes):
    lib = _lib.load()
    ps = problems(mode, shapes)
    arr = _lib.problems_array(ps)
    nwg, nt = ctypes.c_int32(), ctypes.c_int32()
    _lib.check(lib.gemm_grouped_schedule(arr, len(ps), ctypes.byref(nwg), ctypes.byref(nt), None, None, None, None))
    first = (ctypes.c_int32 * (nwg.value + 1))()
    tp, m0, n0 = ((ctypes.c_int32 * max(1, nt.value))() for _ in range(3))
    _lib.check(lib.gemm_grouped_schedule(arr, len(ps), ctypes.byref(nwg), ctypes.byref(nt), first, tp, m0, n0))
    cfg = (ctypes.c_int32 * max(1, len(ps)))()
    _lib.check(lib.gemm_grouped_plan(arr, len(ps), cfg))
    n = nt.value
    return (nwg.value, np.array(first[:nwg.value + 1]), np.array(tp[:n]), np.array(m0[:n]), np.array(n0[:n]),
            np.array(cfg[:len(ps)]))


def tile_dims(mode, cfg):
    info = (ctypes.c_int32 * 6)()
    _lib.check(_lib.load().gemm_config_info(mode, int(cfg), info))
    return info[0], info[1], info[2]


def grouped_shapes(count, lo, hi, seed):
    return [(A.shape[0], B.shape[1], A.shape[1]) for A, B in synth.grouped_problems(count, lo, hi, seed)]


CASES = [
    (_lib.MODE_BF16, grouped_shapes(512, 32, 1024, 0)),
    (_lib.MODE_F32, grouped_shapes(512, 32, 1024, 0)),
    (_lib.MODE_F8E4M3, grouped_shapes(60, 64, 4096, 3)),
    (_lib.MODE_F32, [(5, 7, 3), (0, 9, 9), (300, 200, 0), (1, 1, 1), (129, 257, 33)]),
]


@pytest.mark.parametrize("mode,shapes", CASES, ids=["bf16-512", "f32-512", "e4m3-60", "f32-edge"])
def test_every_tile_once(mode, shapes):
    nwg, first, tp, m0, n0, cfg = schedule(mode, shapes)
    assert first[0] == 0 and first[-1] == len(tp) and np.all(np.diff(first) >= 0)
    want = set()
    for i, (m, n, k) in enumerate(shapes):
        if m == 0 or n == 0:
            assert cfg[i] == -1
            continue
        bm, bn, _ = tile_dims(mode, cfg[i])
        want |= {(i, a, b) for a in range(0, m, bm) for b in range(0, n, bn)}
    got = list(zip(tp.tolist(), m0.tolist(), n0.tolist()))
    assert len(got) == len(set(got)), "a tile is scheduled twice"
    assert set(got) == want
    assert 0 < nwg <= 256 * 4 or len(want) == 0


def test_xcd_locality_and_balance():
    """The grouped workload (BF16): most problems stay on one XCD, and no
    workgroup carries much more than the mean work (tile area times k)."""
    mode, shapes = CASES[0]
    nwg, first, tp, m0, n0, cfg = schedule(mode, shapes)
    xcd = np.zeros(len(tp), dtype=int)
    for w in range(nwg):
        xcd[first[w]:first[w + 1]] = w % 8
    one_xcd = sum(len(set(xcd[tp == i].tolist())) == 1 for i in range(len(shapes)))
    assert one_xcd >= 0.9 * len(shapes), one_xcd
    work = np.zeros(nwg)
    for w in range(nwg):
        for t in range(first[w], first[w + 1]):
            m, n, k = shapes[tp[t]]
            bm, bn, bk = tile_dims(mode, cfg[tp[t]])
            work[w] += bm * bn * (-(-k // bk) * bk)
    assert work.max() <= 1.5 * work.mean(), (work.max(), work.mean())
