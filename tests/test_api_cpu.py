"""The C-ABI library without a GPU: it loads, exports every declared entry
point, and rejects bad arguments before making any HIP call."""
import ctypes
import os
import re

import pytest

from paper_1306_6192_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mi355gemm.h")

# Fake device addresses: validation never dereferences them.
A_PTR, B_PTR, C_PTR = 0x10000000, 0x20000000, 0x30000000


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gemm_\w+)\s*\(", text)))


def test_library_loads_without_gpu():
    lib = _lib.load()
    assert lib.gemm_version() >= 1


def test_every_declared_symbol_is_exported():
    lib = _lib.load()
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding covers every one of them
    assert set(names) <= set(_lib._SIGS), set(names) - set(_lib._SIGS)


def _prob(**kw):
    d = dict(mode=0, m=4, n=5, k=6, A=A_PTR, lda=6, B=B_PTR, ldb=5, C=C_PTR, ldc=5)
    d.update(kw)
    return _lib.problem(d["mode"], d["m"], d["n"], d["k"], d["A"], d["lda"], d["B"], d["ldb"], d["C"], d["ldc"],
                        d.get("scale_a", 1.0), d.get("scale_b", 1.0), d.get("flags", 0))


BAD = [
    (dict(m=-1), "negative"),
    (dict(k=-2), "negative"),
    (dict(lda=5), "lda"),
    (dict(ldb=4), "ldb"),
    (dict(ldc=4), "ldc"),
    (dict(mode=7), "mode"),
    (dict(mode=5), "mode"),   # binary64 and complex have entry points of their own
    (dict(mode=6), "mode"),
    (dict(mode=-1), "mode"),
    (dict(flags=1), "flags"),
    (dict(C=None), "C is NULL"),
    (dict(A=None), "NULL"),
    (dict(B=None), "NULL"),
    (dict(mode=3, scale_a=0.0), "scale"),
    (dict(mode=3, scale_b=float("inf")), "scale"),
    (dict(mode=3, scale_a=-1.0), "scale"),
    (dict(C=A_PTR + 8), "overlap"),
    (dict(C=B_PTR - 16), "overlap"),
]


@pytest.mark.parametrize("kw,msg", BAD)
def test_plain_rejects_bad_arguments(kw, msg):
    lib = _lib.load()
    p = _prob(**kw)
    rc = lib.gemm_plain(ctypes.byref(p), None)
    assert rc == _lib.GEMM_EINVAL
    assert msg.lower() in _lib.last_error().lower()
    rc = lib.gemm_plain_cfg(ctypes.byref(p), 0, 1, None)
    assert rc == _lib.GEMM_EINVAL


def test_plain_cfg_rejects_bad_config_and_split():
    lib = _lib.load()
    p = _prob()
    assert lib.gemm_plain_cfg(ctypes.byref(p), 0, 0, None) == _lib.GEMM_EINVAL
    assert lib.gemm_plain_cfg(ctypes.byref(p), 999, 1, None) == _lib.GEMM_EINVAL
    assert lib.gemm_plain_cfg(ctypes.byref(p), -1, 1, None) == _lib.GEMM_EINVAL


def test_empty_output_is_a_noop_without_gpu():
    lib = _lib.load()
    for kw in (dict(m=0, A=None, C=None), dict(n=0, ldb=1, ldc=1, B=None, C=None)):
        p = _prob(**kw)
        assert lib.gemm_plain(ctypes.byref(p), None) == _lib.GEMM_OK, _lib.last_error()


def test_null_problem_pointer():
    lib = _lib.load()
    assert lib.gemm_plain(None, None) == _lib.GEMM_EINVAL


def test_config_tables():
    lib = _lib.load()
    n = lib.gemm_num_configs(0)
    assert n >= 4
    info = (ctypes.c_int32 * 6)()
    seen = set()
    for c in range(n):
        assert lib.gemm_config_info(0, c, info) == 0
        bm, bn, bk, waves, lds, mk = list(info)
        # register-staged tiles take k-tiles of 32, asynchronous-copy ones 16
        assert bm % 32 == 0 and bn % 32 == 0 and bk in (16, 32) and waves in (4, 8) and 0 < lds <= 160 * 1024
        assert mk == 2
        seen.add((bm, bn, bk, waves))
    # tiles of one size and wave count differ in their wave grid or pipeline
    # (one barrier per k-tile or per two), so only the distinct sizes count
    assert len(seen) >= 8
    assert lib.gemm_config_info(0, n, info) == _lib.GEMM_EINVAL
    assert lib.gemm_num_configs(9) == _lib.GEMM_EINVAL


def test_k_tiles_divide_the_split_grain():
    """Split-K hands each split whole grains of k (32 for FP32 and
    split-BF16x3, 64 for BF16/F16, 128 for FP8); a k-tile that does not divide
    the grain would straddle two splits."""
    lib = _lib.load()
    info = (ctypes.c_int32 * 6)()
    for mode, grain in {0: 32, 1: 64, 2: 64, 3: 128, 4: 32}.items():
        for c in range(lib.gemm_num_configs(mode)):
            assert lib.gemm_config_info(mode, c, info) == 0
            assert grain % info[2] == 0, (mode, c, info[2])


def test_config_chunk():
    """Chunked (asynchronous-copy) configurations report 16 bytes of their
    element type; register-staged ones 0; each family has both kinds."""
    lib = _lib.load()
    elems = {0: 4, 1: 8, 2: 8, 3: 16, _lib.MODE_F64: 2, _lib.MODE_C32: 2}
    for mode, ce in elems.items():
        chunks = [lib.gemm_config_chunk(mode, c) for c in range(lib.gemm_num_configs(mode))]
        assert set(chunks) == {0, ce}, (mode, chunks)
    assert lib.gemm_config_chunk(0, lib.gemm_num_configs(0)) == _lib.GEMM_EINVAL
    assert lib.gemm_config_chunk(-1, 0) == _lib.GEMM_EINVAL


def test_tuner_lookup_is_a_pure_function_of_shape(tmp_path):
    lib = _lib.load()
    c1, s1, c2, s2 = (ctypes.c_int32() for _ in range(4))
    assert lib.gemm_tuner_lookup(0, 8192, 8192, 8192, ctypes.byref(c1), ctypes.byref(s1)) == 0
    assert lib.gemm_tuner_lookup(0, 8192, 8192, 8192, ctypes.byref(c2), ctypes.byref(s2)) == 0
    assert (c1.value, s1.value) == (c2.value, s2.value)
    assert s1.value == 1
    # a skinny shape with few output tiles asks for split-K or small tiles
    assert lib.gemm_tuner_lookup(0, 128, 8192, 8192, ctypes.byref(c1), ctypes.byref(s1)) == 0
    info = (ctypes.c_int32 * 6)()
    lib.gemm_config_info(0, c1.value, info)
    tiles = -(-128 // info[0]) * -(-8192 // info[1]) * s1.value
    assert tiles >= 128
    # save/load round trip of an (empty or filled) table
    path = str(tmp_path / "tune.jsonl").encode()
    assert lib.gemm_tuner_save(path) == 0
    assert lib.gemm_tuner_load(path) == 0
    assert lib.gemm_tuner_load(b"/nonexistent/file") == _lib.GEMM_ENOTFOUND


def test_tuner_file_entries_override(tmp_path):
    lib = _lib.load()
    path = tmp_path / "t.jsonl"
    path.write_text('{"mode": 0, "m": 333, "n": 444, "k": 555, "cfg": 3, "split": 2}\n'
                    'garbage line\n'
                    '{"mode": 0, "m": 1, "n": 1, "k": 1, "cfg": 999, "split": 1}\n')
    assert lib.gemm_tuner_load(str(path).encode()) == 0
    c, s = ctypes.c_int32(), ctypes.c_int32()
    lib.gemm_tuner_lookup(0, 333, 444, 555, ctypes.byref(c), ctypes.byref(s))
    assert (c.value, s.value) == (3, 2)


def test_misc_entry_points_validate():
    lib = _lib.load()
    assert lib.gemm_convert_f32(None, -1, 1, None, None) == _lib.GEMM_EINVAL
    assert lib.gemm_convert_f32(A_PTR, 10, 0, B_PTR, None) == _lib.GEMM_EINVAL
    assert lib.gemm_convert_f32(A_PTR, 10, 1, A_PTR + 8, None) == _lib.GEMM_EINVAL
    assert lib.gemm_convert_f32(None, 0, 1, None, None) == _lib.GEMM_OK
    assert lib.gemm_quantize_e4m3(A_PTR, 10, B_PTR, None, None) == _lib.GEMM_EINVAL
    assert lib.gemm_errnorm(A_PTR, 3, B_PTR, 3, 2, 4, C_PTR, None) == _lib.GEMM_EINVAL
    assert lib.gemm_errnorm(A_PTR, 4, B_PTR, 4, 2, 4, None, None) == _lib.GEMM_EINVAL


EXT = ["gemm_plain_f64", "gemm_plain_c32"]


def _ext_args(**kw):
    d = dict(m=4, n=5, k=6, A=A_PTR, lda=6, B=B_PTR, ldb=5, C=C_PTR, ldc=5)
    d.update(kw)
    return [d["m"], d["n"], d["k"], d["A"], d["lda"], d["B"], d["ldb"], d["C"], d["ldc"]]


EXT_BAD = [
    (dict(m=-1), "negative"),
    (dict(lda=5), "lda"),
    (dict(ldb=4), "ldb"),
    (dict(ldc=4), "ldc"),
    (dict(C=None), "C is NULL"),
    (dict(A=None), "NULL"),
    (dict(C=A_PTR + 8), "overlap"),
    (dict(C=B_PTR - 16), "overlap"),
]


@pytest.mark.parametrize("entry", EXT)
@pytest.mark.parametrize("kw,msg", EXT_BAD)
def test_f64_c32_reject_bad_arguments(entry, kw, msg):
    lib = _lib.load()
    assert getattr(lib, entry)(*_ext_args(**kw), None) == _lib.GEMM_EINVAL
    assert msg.lower() in _lib.last_error().lower()
    assert getattr(lib, entry + "_cfg")(*_ext_args(**kw), 0, None) == _lib.GEMM_EINVAL


@pytest.mark.parametrize("entry", EXT)
def test_f64_c32_empty_output_and_bad_config(entry):
    lib = _lib.load()
    assert getattr(lib, entry)(*_ext_args(m=0, A=None, C=None), None) == _lib.GEMM_OK
    assert getattr(lib, entry + "_cfg")(*_ext_args(), -1, None) == _lib.GEMM_EINVAL
    assert getattr(lib, entry + "_cfg")(*_ext_args(), 99, None) == _lib.GEMM_EINVAL


def test_f64_c32_config_tables():
    lib = _lib.load()
    info = (ctypes.c_int32 * 6)()
    for mode, mk in ((_lib.MODE_F64, 4), (_lib.MODE_C32, 2)):
        n = lib.gemm_num_configs(mode)
        assert n >= 2
        for c in range(n):
            assert lib.gemm_config_info(mode, c, info) == 0
            assert info[2] == 16 and info[3] in (4, 8) and info[5] == mk and 0 < info[4] <= 160 * 1024
    assert lib.gemm_num_configs(_lib.NUM_KERNEL_FAMILIES) == _lib.GEMM_EINVAL
    c, s = ctypes.c_int32(), ctypes.c_int32()
    assert lib.gemm_tuner_lookup(_lib.MODE_F64, 4096, 4096, 4096, ctypes.byref(c), ctypes.byref(s)) == \
        _lib.GEMM_EINVAL   # no gemm_problem_t mode: the lookup is for problem modes


def test_add_validates():
    lib = _lib.load()
    F32, F64 = _lib.MODE_F32, _lib.MODE_F64
    assert lib.gemm_add(1, 0, 4, 5, A_PTR, 5, B_PTR, 5, C_PTR, 5, None) == _lib.GEMM_EUNSUPPORTED
    assert lib.gemm_add(F32, 0, -1, 5, A_PTR, 5, B_PTR, 5, C_PTR, 5, None) == _lib.GEMM_EINVAL
    assert lib.gemm_add(F32, 0, 4, 5, A_PTR, 4, B_PTR, 5, C_PTR, 5, None) == _lib.GEMM_EINVAL
    assert lib.gemm_add(F64, 0, 4, 5, A_PTR, 5, None, 5, C_PTR, 5, None) == _lib.GEMM_EINVAL
    # partial overlap is rejected, exact aliasing (in place) passes validation
    assert lib.gemm_add(F32, 0, 4, 5, A_PTR, 5, B_PTR, 5, A_PTR + 4, 5, None) == _lib.GEMM_EINVAL
    assert lib.gemm_add(F64, 1, 4, 5, A_PTR, 5, B_PTR, 5, B_PTR, 6, None) == _lib.GEMM_EINVAL
    assert lib.gemm_add(F32, 0, 0, 5, None, 5, None, 5, None, 5, None) == _lib.GEMM_OK


@pytest.mark.parametrize("dim", ["m", "n", "k"])
def test_dimensions_above_2_30_are_unsupported(dim):
    """Tile indices and per-dimension counters are 32-bit: a dimension above
    2^30 is refused before any HIP call (offsets themselves are 64-bit)."""
    lib = _lib.load()
    big = (1 << 30) + 1
    kw = {dim: big}
    if dim == "k":
        kw["lda"] = big
    if dim == "n":
        kw.update(ldb=big, ldc=big)
    p = _prob(**kw)
    assert lib.gemm_plain(ctypes.byref(p), None) == _lib.GEMM_EUNSUPPORTED
    assert "2^30" in _lib.last_error()
