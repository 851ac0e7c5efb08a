"""The paper's two GPU kernels rebuilt for gfx950 (global-memory and 16x16
LDS tiles), checked against the oracle like the matrix-core path."""
import numpy as np
import pytest

import oracle
import synth
from tests._gpu import abs_product, assert_within_bound, dev, host, log

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1306_6192_amd as mg  # noqa: E402


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (7, 5, 3), (16, 16, 16), (33, 47, 129), (300, 200, 511)])
def test_paper_kernels_within_bound(variant, m, n, k):
    log(f"ablation variant {variant} {(m, n, k)}")
    A, B = synth.pair(m, n, k, seed=50 + m + n + k, dist="normal")
    C = host(mg.paper_kernel(dev(A), dev(B), variant=variant))
    assert_within_bound(C, oracle.gemm(A, B), abs_product(A, B), k, f"variant {variant}")


@pytest.mark.parametrize("variant", [0, 1])
def test_paper_kernels_integer_exact_and_equal(variant):
    log(f"ablation variant {variant} integer")
    A, B = synth.pair(130, 90, 1000, seed=51, dist="integers", R=16)
    C = host(mg.paper_kernel(dev(A), dev(B), variant=variant))
    assert np.array_equal(C.astype(np.float64), oracle.gemm(A, B))


def test_paper_kernels_same_order():
    """Both kernels add the products of each c_ij in ascending r with fused
    multiply-adds, so they agree bit for bit on any input."""
    log("ablation variants bitwise")
    A, B = synth.pair(77, 65, 300, seed=52, dist="normal")
    dA, dB = dev(A), dev(B)
    assert np.array_equal(host(mg.paper_kernel(dA, dB, variant=0)), host(mg.paper_kernel(dA, dB, variant=1)))
