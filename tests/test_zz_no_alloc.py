"""The allocation-free plain product (gemm_plain_noalloc) against gemm_plain.

gemm_plain_noalloc runs gemm_plain's plan with its workspace in a fixed
device array, so on the same inputs the two give the same bits.  Each case
makes two calls in a row through the C-ABI, the second on a smaller product
than the first (the array still holds the first call's partial sums), and
compares every output element with gemm_plain's; the smaller product is also
checked normwise against the oracle.  A product that needs more workspace than
the array holds is refused before any device work (a CPU test)."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from paper_1306_6192_amd import _lib
from tests._gpu import dev, host, log


def _problem(mode, A, B, C, scale_a=1.0, scale_b=1.0):
    m, k = A.shape
    n = B.shape[1]
    return _lib.problem(mode, m, n, k, A.data_ptr(), A.stride(0), B.data_ptr(), B.stride(0), C.data_ptr(),
                        C.stride(0), scale_a, scale_b)


def _operands(torch, mode, m, n, k, seed):
    A, B = synth.pair(m, n, k, seed=seed)
    dA, dB = dev(A), dev(B)
    if mode == _lib.MODE_BF16:
        import paper_1306_6192_amd as mg
        dA, dB = mg.convert(dA, mode), mg.convert(dB, mode)
    return A, B, dA, dB


# (mode, first (larger) shape, second (smaller) shape); every shape here runs
# split-K or the split-BF16x3 operand copies, so it uses the scratch array
CASES = [
    (_lib.MODE_F32, (128, 8192, 8192), (512, 512, 512)),
    (_lib.MODE_SPLIT_BF16X3, (1024, 1024, 1024), (512, 512, 512)),
    (_lib.MODE_BF16, (128, 8192, 8192), (100, 3000, 5000)),
]


@pytest.mark.gpu
@pytest.mark.parametrize("mode,first,second", CASES, ids=[_lib.MODE_NAMES[c[0]] for c in CASES])
def test_noalloc_equals_plain_two_calls(mode, first, second):
    torch = pytest.importorskip("torch")
    lib = _lib.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for i, (m, n, k) in enumerate((first, second)):
        log(f"noalloc {_lib.MODE_NAMES[mode]} call {i + 1}: {m}x{n}x{k}")
        p0 = _lib.problem(mode, m, n, k, 1 << 40, k, 2 << 40, n, 3 << 40, n)
        ws = ctypes.c_uint64()
        _lib.check(lib.gemm_plain_workspace_bytes(ctypes.byref(p0), ctypes.byref(ws)))
        assert 0 < ws.value <= _lib.NOALLOC_SCRATCH_BYTES, ws.value
        A, B, dA, dB = _operands(torch, mode, m, n, k, seed=10 + i)
        ref = torch.full((m, n), float("nan"), dtype=torch.float32, device="cuda")
        out = torch.full((m, n), float("nan"), dtype=torch.float32, device="cuda")
        _lib.check(lib.gemm_plain(ctypes.byref(_problem(mode, dA, dB, ref)), stream))
        _lib.check(lib.gemm_plain_noalloc(ctypes.byref(_problem(mode, dA, dB, out)), stream))
        C, R = host(out), host(ref)
        assert np.array_equal(C.view(np.uint32), R.view(np.uint32)), \
            f"{int((C.view(np.uint32) != R.view(np.uint32)).sum())} elements differ from gemm_plain"
        if i == 1 and mode != _lib.MODE_BF16:
            err = oracle.relerr(C, oracle.gemm(A, B))
            log(f"  relerr vs oracle {err:.3e}")
            assert err <= 1e-5, err


def test_noalloc_refuses_a_workspace_beyond_the_array():
    """split-BF16x3 at 4096^3 takes the pre-split path (192 MiB of operand
    copies): refused with GEMM_EINVAL before any device call (fake pointers,
    never dereferenced)."""
    lib = _lib.load()
    p = _lib.problem(_lib.MODE_SPLIT_BF16X3, 4096, 4096, 4096, 1 << 40, 4096, 2 << 40, 4096, 3 << 40, 4096)
    ws = ctypes.c_uint64()
    _lib.check(lib.gemm_plain_workspace_bytes(ctypes.byref(p), ctypes.byref(ws)))
    assert ws.value > _lib.NOALLOC_SCRATCH_BYTES
    rc = lib.gemm_plain_noalloc(ctypes.byref(p), None)
    assert rc == _lib.GEMM_EINVAL
    assert "gemm_plain_noalloc holds at most" in _lib.last_error()
