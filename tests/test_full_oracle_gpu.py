"""Whole-output parity at the full workload sizes: the 8192^3 products the
benchmark times (same inputs, same tuned launches) against the oracle's full
binary64 product, normwise over every element, taken on the device by the
comparison reduction (gemm_errnorm).

Bars: the float32 product within 1e-5 on uniform[-1, 1] inputs; the
split-BF16x3 product within 1e-5 on N(0, 1) and on the wide-range inputs;
BF16, F16 and E4M3 within their format bands on N(0, 1) (the same bands as
the sampled precision tests)."""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import dev, host, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1306_6192_amd as mg  # noqa: E402

N = 8192
BAND = {mg.MODE_F32: 1e-5, mg.MODE_SPLIT_BF16X3: 1e-5, mg.MODE_BF16: 8e-3, mg.MODE_F16: 1e-3,
        mg.MODE_F8E4M3: 8e-2}


def full_error(dC, dR):
    e = host(mg.errnorm(dC, dR))
    return float(np.sqrt(e[0] / e[1]))


def operands(dA, dB, mode):
    if mode in (mg.MODE_BF16, mg.MODE_F16):
        return mg.convert(dA, mode), mg.convert(dB, mode), 1.0, 1.0
    if mode == mg.MODE_F8E4M3:
        qa, sa = mg.quantize_e4m3(dA)
        qb, sb = mg.quantize_e4m3(dB)
        return qa, qb, float(host(sa)[0]), float(host(sb)[0])
    return dA, dB, 1.0, 1.0


CASES = [("uniform", [mg.MODE_F32]),
         ("normal", [mg.MODE_SPLIT_BF16X3, mg.MODE_F32, mg.MODE_BF16, mg.MODE_F16, mg.MODE_F8E4M3]),
         ("wide", [mg.MODE_SPLIT_BF16X3])]


@pytest.mark.parametrize("dist,modes", CASES, ids=[c[0] for c in CASES])
def test_8192_whole_output_against_oracle(dist, modes):
    log(f"full oracle 8192^3 {dist}: computing the binary64 product")
    A, B = synth.pair(N, N, N, seed=0, dist=dist)
    R = oracle.gemm(A, B)
    dR = torch.from_numpy(R).cuda()
    del R
    dA, dB = dev(A), dev(B)
    del A, B
    for mode in modes:
        log(f"full oracle 8192^3 {dist} {mg.MODE_NAMES[mode]}")
        a, b, sa, sb = operands(dA, dB, mode)
        C = mg.gemm(a, b, mode=mode, scale_a=sa, scale_b=sb)
        err = full_error(C, dR)
        log(f"  relerr {err:.3e} (bar {BAND[mode]:.0e})")
        assert err <= BAND[mode], (dist, mg.MODE_NAMES[mode], err)
        del a, b, C
    del dR, dA, dB
    torch.cuda.empty_cache()


def test_512_whole_output_against_oracle():
    """The 512^3 correctness workload: normwise error at most 1e-6."""
    A, B = synth.pair(512, 512, 512, seed=0)
    C = mg.gemm(dev(A), dev(B))
    err = full_error(C, dev(oracle.gemm(A, B)))
    assert err <= 1e-6, err
