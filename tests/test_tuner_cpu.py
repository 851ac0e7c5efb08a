"""Host logic of the autotuner, the grouped planner and the workspace
accounting, without a GPU: table lookups (exact, bucket, grouped), the
planner taking the table's calibrated efficiency and alone choices, the grouped kernels' occupancy plan
against the LDS they allocate, and the workspace a plain launch needs."""
import ctypes
import os
import re

import pytest

from paper_1306_6192_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RESOURCES = os.path.join(ROOT, "paper_1306_6192_amd", "_build", "kernel_resources.txt")
LDS_PER_CU = 160 * 1024

# Fake device addresses: nothing here dereferences them.
A_PTR, B_PTR, C_PTR = 1 << 40, 1 << 41, 1 << 42


def prob(mode, m, n, k, A=A_PTR, B=B_PTR, C=C_PTR):
    return _lib.problem(mode, m, n, k, A, max(1, k), B, max(1, n), C, max(1, n))


def lookup(mode, m, n, k):
    c, s = ctypes.c_int32(), ctypes.c_int32()
    _lib.check(_lib.load().gemm_tuner_lookup(mode, m, n, k, ctypes.byref(c), ctypes.byref(s)))
    return c.value, s.value


def grouped_info(mode):
    info = (ctypes.c_int32 * 7)()
    _lib.check(_lib.load().gemm_grouped_info(mode, info))
    return list(info)


def grouped_lookup(mode, m, n, k):
    out = (ctypes.c_int32 * 3)()
    _lib.check(_lib.load().gemm_grouped_lookup(mode, m, n, k, out))
    return list(out)


def workspace(p):
    w = ctypes.c_uint64()
    _lib.check(_lib.load().gemm_plain_workspace_bytes(ctypes.byref(p), ctypes.byref(w)))
    return w.value


def config_info(mode, cfg):
    info = (ctypes.c_int32 * 6)()
    _lib.check(_lib.load().gemm_config_info(mode, cfg, info))
    return list(info)


def bucket(d):
    return max(0, int(d).bit_length() - 1)


MODES = [_lib.MODE_F32, _lib.MODE_BF16, _lib.MODE_F16, _lib.MODE_F8E4M3, _lib.MODE_SPLIT_BF16X3]


@pytest.mark.parametrize("mode", MODES)
def test_grouped_occupancy_plan_fits_lds(mode):
    """The planner's resident workgroups per CU times the kernel's LDS fits the
    CU, and (when the build's resource report is present) matches the
    occupancy the compiler reports for that kernel."""
    cfg0, cfg1, wg_per_cu, lds, alone0, alone1, variant = grouped_info(mode)
    assert wg_per_cu >= 1
    assert wg_per_cu * lds <= LDS_PER_CU, (mode, wg_per_cu, lds)
    # the kernel's LDS is two stages of the larger tile (the plain
    # configurations' two-stage LDS)
    assert lds == max(config_info(mode, cfg0)[4], config_info(mode, cfg1)[4])
    if os.path.exists(RESOURCES):
        waves = config_info(mode, cfg0)[3]
        found = False
        for line in open(RESOURCES):
            if not line.startswith("_Z26gemm_grouped_stream_kernel"):
                continue
            name = line.split()[0]
            # the kernel's occupancy bound and ring depth are its last two
            # template arguments: (3, 2) for variant 0, (2, 4) for variant 1
            tail = re.search(r"Li(\d+)ELi(\d+)EEvPK9GroupDesc", name)
            if not tail or (int(tail.group(1)), int(tail.group(2))) != ((3, 2), (2, 4))[variant]:
                continue
            lds_m = re.search(r"LDS Size \[bytes/block\]=(\d+)", line)
            occ_m = re.search(r"Occupancy \[waves/SIMD\]=(\d+)", line)
            if not (lds_m and occ_m) or int(lds_m.group(1)) != lds:
                continue
            # the mode is the first template argument of the first tile
            tmode = re.search(r"CfgILi(\d+)E", name)
            is_f32 = "F32Cfg" in name.split("S0_")[0]
            if (mode == _lib.MODE_F32) != is_f32 or (not is_f32 and int(tmode.group(1)) != mode):
                continue
            found = True
            # four SIMDs per CU; a workgroup of `waves` waves puts waves/4 on each
            assert int(occ_m.group(1)) * 4 // waves >= wg_per_cu, line
        assert found, f"no resource line for the grouped kernel of mode {mode}"


def test_plain_workspace_accounting():
    # split-K slabs: split * m * n float32 (slab stride rounded to 4 elements)
    m, n, k = 128, 8192, 8192
    cfg, split = lookup(_lib.MODE_F32, m, n, k)
    assert split > 1
    assert workspace(prob(_lib.MODE_F32, m, n, k)) == split * m * n * 4
    # a product without split-K needs none
    assert workspace(prob(_lib.MODE_F32, 8192, 8192, 8192)) == 0
    # empty products need none
    assert workspace(prob(_lib.MODE_F32, 5, 0, 7)) == 0
    assert workspace(prob(_lib.MODE_F32, 5, 6, 0)) == 0


def test_presplit_not_taken_when_3k16_exceeds_int32():
    """The pre-split split-BF16x3 path indexes an inner dimension of 3 k16 in
    32 bits: at k = 2^30 its configurations fall back to the register-staged
    split tile, which needs no operand copies (only split-K slabs)."""
    mode = _lib.MODE_SPLIT_BF16X3
    m, n = 1, 8
    for k in (1 << 30, (1 << 30) - 5):
        p = prob(mode, m, n, k)
        cfg, split = lookup(mode, m, n, k)
        ws = workspace(p)
        k16 = (k + 15) // 16 * 16
        copies = 6 * k16 * (m + n)
        assert ws < copies, (k, ws)
        slabs = (split * ((m * n + 3) // 4 * 4) * 4 + 255) // 256 * 256 if split > 1 else 0
        assert ws <= slabs


def test_bucket_entry_serves_unmeasured_shapes(tmp_path):
    mode = _lib.MODE_F16
    m, n, k = 3001, 211, 77777          # buckets 11, 7, 16: no exact entry
    f = tmp_path / "t.jsonl"
    f.write_text('{"bucket": "plain", "mode": %d, "bm": %d, "bn": %d, "bk": %d, "cfg": 4, "split": 2}\n'
                 % (mode, bucket(m), bucket(n), bucket(k)))
    _lib.check(_lib.load().gemm_tuner_load(str(f).encode()))
    assert lookup(mode, m, n, k) == (4, 2)
    # every shape of the bucket takes it; a neighbouring bucket does not
    assert lookup(mode, 2048, 128, 65536) == (4, 2)
    assert lookup(mode, 4095, 255, 131071) == (4, 2)
    # an exact entry still wins over its bucket
    f.write_text('{"mode": %d, "m": %d, "n": %d, "k": %d, "cfg": 1, "split": 1}\n' % (mode, m, n, k))
    _lib.check(_lib.load().gemm_tuner_load(str(f).encode()))
    assert lookup(mode, m, n, k) == (1, 1)
    assert lookup(mode, 2048, 128, 65536) == (4, 2)


def test_grouped_planner_takes_the_table_choice(tmp_path):
    """In a batch every problem runs on the stream's tile (for a two-tile
    stream, the cost model's pick under the small-tile efficiency the table
    holds for the mode); alone it takes the bucket's measured configuration
    between the two gemm_grouped_info lists.  Every configuration gives the
    same bits, so only the speed depends on these entries."""
    mode = _lib.MODE_F16
    cfg0, cfg1, wg_per_cu, _, alone0, alone1, _ = grouped_info(mode)
    area = lambda c: config_info(mode, c)[0] * config_info(mode, c)[1]
    assert area(alone1) < area(alone0)
    m, n, k = 3000, 2900, 40000          # k outside every tuned bucket
    before = grouped_lookup(mode, m, n, k)
    assert before[2] == 0
    f = tmp_path / "g.jsonl"
    lib = _lib.load()
    probs = [prob(mode, m, n, k, A=A_PTR + i * (1 << 34), B=B_PTR + i * (1 << 34), C=C_PTR + i * (1 << 34))
             for i in range(3)]
    other = prob(mode, 700, 900, 300, A=A_PTR + 5 * (1 << 34), B=B_PTR + 5 * (1 << 34), C=C_PTR + 5 * (1 << 34))
    empty = prob(mode, 0, 900, 300, A=A_PTR + 6 * (1 << 34), B=B_PTR + 6 * (1 << 34), C=C_PTR + 6 * (1 << 34))
    arr = _lib.problems_array(probs + [other, empty])
    try:
        if cfg0 == cfg1:
            effs = ((4.0, cfg0), (0.05, cfg0))
        else:
            # padded area: 2162 small tiles of 64x64 against 552 large of
            # 128x128; at efficiency 4 the small tile costs a quarter, at
            # 0.05 twenty times
            small = cfg1 if area(cfg1) < area(cfg0) else cfg0
            effs = ((4.0, small), (0.05, cfg0 + cfg1 - small))
        for eff, want in effs:
            f.write_text('{"grouped_eff": %d, "eff": %.3f}\n' % (mode, eff))
            _lib.check(lib.gemm_tuner_load(str(f).encode()))
            assert grouped_lookup(mode, m, n, k)[0] == want, eff
            out = (ctypes.c_int32 * 5)()
            _lib.check(lib.gemm_grouped_plan(arr, 5, out))
            assert list(out[:3]) == [want] * 3, eff
            assert out[3] == grouped_lookup(mode, 700, 900, 300)[0]
            assert out[4] == -1
        large = effs[1][1]
        # an efficiency outside (0, 4] is not loaded
        f.write_text('{"grouped_eff": %d, "eff": 9.0}\n' % mode)
        _lib.check(lib.gemm_tuner_load(str(f).encode()))
        assert grouped_lookup(mode, m, n, k)[0] == large
        # alone: the bucket's measured configuration, in the current form and
        # in the older form that also carried an in-batch tile (ignored now)
        for flip, line in ((0, '"alone": %d'), (1, '"tile": 0, "alone": %d'), (0, '"tile": 1, "alone": %d')):
            f.write_text(('{"bucket": "grouped", "mode": %d, "bm": %d, "bn": %d, "bk": %d, ' + line + '}\n')
                         % (mode, bucket(m), bucket(n), bucket(k), flip))
            _lib.check(lib.gemm_tuner_load(str(f).encode()))
            after = grouped_lookup(mode, m, n, k)
            assert after[1] == (alone0, alone1)[flip] and after[2] == 1
            assert after[0] == large
    finally:
        # back to the default efficiency, then the shipped table's entries
        f.write_text('{"grouped_eff": %d, "eff": 0.600, "variant": 0}\n' % mode)
        _lib.check(lib.gemm_tuner_load(str(f).encode()))
        shipped = os.path.join(ROOT, "paper_1306_6192_amd", "tuning", "mi355x.jsonl")
        if os.path.exists(shipped):
            _lib.check(lib.gemm_tuner_load(shipped.encode()))


def test_grouped_lookup_and_plan_validate():
    lib = _lib.load()
    out = (ctypes.c_int32 * 3)()
    assert lib.gemm_grouped_lookup(9, 1, 1, 1, out) == _lib.GEMM_EINVAL
    assert lib.gemm_grouped_lookup(0, -1, 1, 1, out) == _lib.GEMM_EINVAL
    info = (ctypes.c_int32 * 7)()
    assert lib.gemm_grouped_info(5, info) == _lib.GEMM_EINVAL
    bad = _lib.problems_array([prob(0, 4, 4, 4), prob(1, 4, 4, 4, A=A_PTR + 4096, B=B_PTR + 4096, C=C_PTR + 4096)])
    cfgs = (ctypes.c_int32 * 2)()
    assert lib.gemm_grouped_plan(bad, 2, cfgs) == _lib.GEMM_EINVAL
    assert "one mode" in _lib.last_error()
    assert lib.gemm_tune_grouped(0, 0, 4, 4, None) == _lib.GEMM_EINVAL
    assert lib.gemm_tune_bucket(9, 4, 4, 4, None) == _lib.GEMM_EINVAL


@pytest.mark.parametrize("mode", [_lib.MODE_F32, _lib.MODE_BF16, _lib.MODE_F8E4M3])
def test_grouped_variant_from_the_table(mode, tmp_path):
    """A "variant" in the mode's grouped_eff line selects the grouped kernel:
    variant 1 runs two tiles (a 128x128 and a 64x64 configuration, two or
    three workgroups per CU) and its cost model gives small problems the
    small tile; variant 0 runs one 128x128 tile at three per CU.  A line without a
    variant means variant 0."""
    lib = _lib.load()
    f = tmp_path / "v.jsonl"
    shapes = [(32, 40, 64), (900, 1000, 300), (100, 80, 500)]
    probs = [prob(mode, m, n, k, A=A_PTR + i * (1 << 34), B=B_PTR + i * (1 << 34), C=C_PTR + i * (1 << 34))
             for i, (m, n, k) in enumerate(shapes * 200)]
    arr = _lib.problems_array(probs)
    try:
        f.write_text('{"grouped_eff": %d, "eff": 0.600, "variant": 1}\n' % mode)
        _lib.check(lib.gemm_tuner_load(str(f).encode()))
        cfg0, cfg1, wg, lds, a0, a1, v = grouped_info(mode)
        assert v == 1 and cfg0 != cfg1 and wg >= 2 and wg * lds <= LDS_PER_CU
        assert config_info(mode, cfg0)[:2] == [128, 128] and config_info(mode, cfg1)[:2] == [64, 64]
        out = (ctypes.c_int32 * len(probs))()
        _lib.check(lib.gemm_grouped_plan(arr, len(probs), out))
        assert out[0] == cfg1 and out[1] == cfg0      # the 32x40 problem on 64x64, 900x1000 on 128x128
        f.write_text('{"grouped_eff": %d, "eff": 0.600}\n' % mode)
        _lib.check(lib.gemm_tuner_load(str(f).encode()))
        cfg0, cfg1, wg, lds, a0, a1, v = grouped_info(mode)
        assert v == 0 and cfg0 == cfg1 and wg == 3 and wg * lds <= LDS_PER_CU
        assert config_info(mode, cfg0)[:2] == [128, 128]
        _lib.check(lib.gemm_grouped_plan(arr, len(probs), out))
        assert set(out) == {cfg0}
        # a variant the kernels do not have is not taken from a table: the
        # line is skipped and the mode keeps the kernel it had
        f.write_text('{"grouped_eff": %d, "eff": 0.600, "variant": 1}\n' % mode)
        _lib.check(lib.gemm_tuner_load(str(f).encode()))
        f.write_text('{"grouped_eff": %d, "eff": 0.600, "variant": 7}\n' % mode)
        assert lib.gemm_tuner_load(str(f).encode()) == 0
        assert grouped_info(mode)[6] == 1
    finally:
        f.write_text('{"grouped_eff": %d, "eff": 0.600, "variant": 0}\n' % mode)
        _lib.check(lib.gemm_tuner_load(str(f).encode()))
        shipped = os.path.join(ROOT, "paper_1306_6192_amd", "tuning", "mi355x.jsonl")
        if os.path.exists(shipped):
            _lib.check(lib.gemm_tuner_load(shipped.encode()))


def test_grouped_variant_survives_save_and_load(tmp_path):
    """gemm_tuner_save writes the mode's grouped variant and efficiency, and
    loading the saved table restores them (the form tune.py ships)."""
    lib = _lib.load()
    mode = _lib.MODE_F16
    f, g = tmp_path / "in.jsonl", tmp_path / "out.jsonl"
    try:
        f.write_text('{"grouped_eff": %d, "eff": 0.900, "variant": 1}\n' % mode)
        _lib.check(lib.gemm_tuner_load(str(f).encode()))
        _lib.check(lib.gemm_tuner_save(str(g).encode()))
        lines = [ln for ln in g.read_text().splitlines() if ln.startswith('{"grouped_eff": %d,' % mode)]
        assert lines == ['{"grouped_eff": %d, "eff": 0.900, "variant": 1}' % mode]
        f.write_text('{"grouped_eff": %d, "eff": 0.600, "variant": 0}\n' % mode)
        _lib.check(lib.gemm_tuner_load(str(f).encode()))
        assert grouped_info(mode)[6] == 0
        _lib.check(lib.gemm_tuner_load(str(g).encode()))
        assert grouped_info(mode)[6] == 1
    finally:
        f.write_text('{"grouped_eff": %d, "eff": 0.600, "variant": 0}\n' % mode)
        _lib.check(lib.gemm_tuner_load(str(f).encode()))
        shipped = os.path.join(ROOT, "paper_1306_6192_amd", "tuning", "mi355x.jsonl")
        if os.path.exists(shipped):
            _lib.check(lib.gemm_tuner_load(shipped.encode()))
