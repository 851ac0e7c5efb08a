"""Operand preparation (conversions, E4M3 quantisation) and the binary64
comparison reduction on the GPU, against the oracle.  Conversions are integer
(code) results: bit-exact.  The reduction is binary64 arithmetic in another
order: within 1e-12 relative."""
import numpy as np
import pytest

import oracle
import synth
from oracle import formats as F
from tests._gpu import dev, host, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1306_6192_amd as mg  # noqa: E402


def _values(seed, n=300_001):
    g = synth.rng(seed)
    x = np.concatenate([synth.draw(g, (n,), "normal"), synth.draw(g, (n,), "wide"),
                        (synth.draw(g, (n,), "normal") * np.float32(1e-39)).astype(np.float32),
                        np.array([0.0, -0.0, 65504.0, 65520.0, 1e30, -1e30, 3.0e38], np.float32)])
    return x.astype(np.float32)


@pytest.mark.parametrize("mode,fmt", [(1, "bf16"), (2, "f16")])
def test_convert_bit_exact(mode, fmt):
    log(f"convert f32 -> {fmt}")
    x = _values(30 + mode)
    got = host(mg.convert(dev(x), mode).view(torch.int16)).view(np.uint16)
    want = F.to_bf16_bits(x) if fmt == "bf16" else F.to_f16_bits(x)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("dist", ["normal", "wide", "uniform"])
def test_quantize_e4m3_bit_exact(dist):
    log(f"quantize e4m3 {dist}")
    g = synth.rng(40)
    x = synth.draw(g, (1000, 777), dist)
    q, s = mg.quantize_e4m3(dev(x))
    s_host = np.float32(host(s)[0])
    assert s_host == F.e4m3_scale(x)
    assert np.array_equal(host(q), F.to_e4m3_bits(x, s_host))


def test_quantize_e4m3_zero_and_empty():
    log("quantize e4m3 zeros")
    q, s = mg.quantize_e4m3(dev(np.zeros((3, 5), np.float32)))
    assert host(s)[0] == 1.0 and np.all(host(q) == 0)
    q, s = mg.quantize_e4m3(torch.zeros((0,), device="cuda"))
    assert host(s)[0] == 1.0


@pytest.mark.parametrize("m,n", [(1, 1), (37, 53), (1000, 3000)])
def test_errnorm_matches_oracle_terms(m, n):
    log(f"errnorm {(m, n)}")
    g = synth.rng(41)
    R = g.standard_normal((m, n))
    C = (R + 1e-3 * g.standard_normal((m, n))).astype(np.float32)
    out = host(mg.errnorm(dev(C), dev(R)))
    sd, sr, mx = oracle.errnorm_terms(C, R)
    assert out[0] == pytest.approx(sd, rel=1e-12)
    assert out[1] == pytest.approx(sr, rel=1e-12)
    assert out[2] == mx
    assert np.sqrt(out[0] / out[1]) == pytest.approx(oracle.relerr(C, R), rel=1e-12)


@pytest.mark.parametrize("mode", [0, 1, 3])
def test_tune_records_a_legal_choice(mode):
    """gemm_tune times every legal choice on its own non-zero operands and
    records one: the lookup returns it, it is a valid configuration and split,
    and gemm_plain then computes the shape with it (integer inputs: exact)."""
    m, n, k = 300, 208, 1040
    log(f"tune mode {mode} {(m, n, k)}")
    cfg, split = mg.tune(mode, m, n, k)
    assert 0 <= cfg < mg.num_configs(mode) and split >= 1
    assert mg.tuner_lookup(mode, m, n, k) == (cfg, split)
    A, B = synth.pair(m, n, k, seed=61, dist="integers", R=4)
    dA, dB = dev(A), dev(B)
    if mode in (1, 2):
        dA, dB = mg.convert(dA, mode), mg.convert(dB, mode)
    elif mode == 3:   # integers of magnitude <= 4 are exact E4M3 values
        dA, dB = dA.to(torch.float8_e4m3fn), dB.to(torch.float8_e4m3fn)
    C = host(mg.gemm(dA, dB, mode=mode))
    assert np.array_equal(C.astype(np.float64), oracle.gemm(A, B))
