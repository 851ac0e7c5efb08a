"""Helpers shared by the GPU tests (device transfer and error bounds)."""
import sys

import numpy as np

U32 = 2.0 ** -24   # unit roundoff of binary32


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def abs_product(A, B):
    """(|A| |B|) in binary64 (numpy; only the error bound uses it)."""
    return np.abs(np.asarray(A, np.float64)) @ np.abs(np.asarray(B, np.float64))


def fp32_bound(k: int, absAB, extra_ulps: float = 2.0):
    """Worst-case error of a float32 sum of k float32 products in any order:
    (k + extra) * u32 * (|A||B|)_ij (each product and each addition adds at
    most one rounding of relative size u32)."""
    return (k + extra_ulps) * U32 * absAB


def assert_within_bound(C, R, absAB, k, what=""):
    err = np.abs(np.asarray(C, np.float64) - R)
    bound = fp32_bound(k, absAB) + 1e-30
    bad = err > bound
    if bad.any():
        i = np.argwhere(bad)[0]
        raise AssertionError(f"{what}: {bad.sum()} elements beyond the float32 bound; first at {tuple(i)}: "
                             f"C={C[tuple(i)]!r} R={R[tuple(i)]!r} bound={bound[tuple(i)]!r}")
