"""Measure tile configurations on the current GPU and write the tuning table
the library loads at start-up.

    python -m paper_1306_6192_amd.tune [--out PATH] [--what exact,plain-buckets,grouped]

Three kinds of entries (each chosen by the library's own timing):

* ``exact``: the configuration and split-K factor of each benchmark shape
  (``gemm_tune``: every legal configuration and split-K factor, timed with
  HIP events on non-zero operands; the near-ties are re-timed and the fastest
  kept), keyed by (mode, m, n, k);
* ``plain-buckets``: the same measurement on one representative shape per
  log2 bucket of (m, n, k) (``gemm_tune_bucket``), consulted for every shape
  without an exact entry;
* ``grouped``: the plain tile (128x128 or 64x64) per bucket for a problem
  launched alone (``gemm_tune_grouped``), and per mode the grouped kernel
  variant (one tile at three workgroups per CU, or two tiles with a cost
  model) and the small-tile efficiency of that cost model, measured on a
  mixed batch of seeded synthetic problems (``gemm_tune_grouped_mix``): 512 problems with m, n, k
  log-uniform in [32, 1024] (the grouped workload's distribution, another
  seed) for FP32, BF16, F16 and split-BF16x3, and 48 problems with m, n, k
  log-uniform in [64, 4096] (a serving batch) for E4M3.

Buckets cover the grouped workload (dims log-uniform in [32, 1024], FP32 and
BF16) and the serving workload (dims log-uniform in [64, 4096], FP32, BF16
and E4M3).  The representative shape of bucket b is the geometric mean of
the part of [2^b, 2^(b+1)) the workloads cover.  The table is saved after
every mode, so an interrupted run keeps what it measured.
"""
from __future__ import annotations

import argparse
import itertools
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning", "mi355x.jsonl")

PLAIN_F32 = [(2048, 2048, 2048), (4096, 4096, 4096), (8192, 8192, 8192), (8192, 1024, 4096), (128, 8192, 8192),
             (512, 512, 512)]
SQUARES = [(2048, 2048, 2048), (4096, 4096, 4096), (8192, 8192, 8192)]

# dimension ranges of the workloads whose shapes are tuned per bucket
GROUPED_RANGE = (32, 1024)
SERVING_RANGE = (64, 4096)


def exact_shapes(mg):
    out = [(mg.MODE_F32, s) for s in PLAIN_F32]
    for mode in (mg.MODE_BF16, mg.MODE_F16, mg.MODE_F8E4M3, mg.MODE_SPLIT_BF16X3):
        out += [(mode, s) for s in SQUARES]
    return out


def bucket_reps(lo: int, hi: int):
    """(bucket, representative dimension) of every log2 bucket meeting [lo, hi]."""
    out = []
    for b in range(int(math.log2(lo)), int(math.log2(hi)) + 1):
        a, z = max(lo, 1 << b), min(hi, (1 << (b + 1)) - 1)
        if a <= z:
            out.append((b, int(round(math.sqrt(a * z)))))
    return out


def bucket_shapes(mg):
    """{mode: [representative (m, n, k)]} over the grouped and serving ranges."""
    ranges = {mg.MODE_F32: [GROUPED_RANGE, SERVING_RANGE], mg.MODE_BF16: [GROUPED_RANGE, SERVING_RANGE],
              mg.MODE_F8E4M3: [SERVING_RANGE]}
    out = {}
    for mode, rs in ranges.items():
        reps = {}
        for lo, hi in rs:
            for b, d in bucket_reps(lo, hi):
                reps.setdefault(b, []).append(d)
        # one representative per bucket (the lower one where both ranges
        # cover it: the grouped range ends at 1024)
        dims = [(b, sorted(ds)[(len(ds) - 1) // 2]) for b, ds in sorted(reps.items())]
        out[mode] = [(m, n, k) for (_, m), (_, n), (_, k) in itertools.product(dims, dims, dims)]
    return out


def calibrate_mix(mg, _lib, lib, torch, mode, count, lo, hi, stream):
    """gemm_tune_grouped_mix on `count` seeded problems with dims log-uniform
    in [lo, hi] (seed 100, not the benchmark's), operands uniform[-1, 1]
    on the device in the mode's element type."""
    # the seeded input generators live beside the package, at the
    # repository root
    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import synth
    g = torch.Generator(device="cuda").manual_seed(100)
    ops = []
    for m, n, k in synth.loguniform_dims(count, lo, hi, seed=100).tolist():
        a = torch.rand((m, k), device="cuda", generator=g) * 2 - 1
        b = torch.rand((k, n), device="cuda", generator=g) * 2 - 1
        if mode in (mg.MODE_BF16, mg.MODE_F16):
            a, b = mg.convert(a, mode), mg.convert(b, mode)
        elif mode == mg.MODE_F8E4M3:
            a, _ = mg.quantize_e4m3(a)
            b, _ = mg.quantize_e4m3(b)
        ops.append((a, b, torch.empty((m, n), device="cuda")))
    probs = [mg.make_problem(a, b, c, mode) for a, b, c in ops]
    torch.cuda.synchronize()
    _lib.check(lib.gemm_tune_grouped_mix(_lib.problems_array(probs), len(probs), stream))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--what", default="exact,plain-buckets,grouped")
    ap.add_argument("--modes", default="", help="comma-separated mode names to tune (default: all)")
    args = ap.parse_args(argv)
    what = set(args.what.split(","))
    import torch

    import paper_1306_6192_amd as mg
    from paper_1306_6192_amd import _lib
    torch.cuda.set_device(0)
    lib = mg.load()
    stream = torch.cuda.current_stream().cuda_stream
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)

    def save():
        _lib.check(lib.gemm_tuner_save(args.out.encode()))

    keep = {mode for mode, name in mg.MODE_NAMES.items() if not args.modes or name in args.modes.split(",")}
    if "exact" in what:
        for mode, (m, n, k) in exact_shapes(mg):
            if mode not in keep:
                continue
            cfg, split = mg.tune(mode, m, n, k)
            info = mg.config_info(mode, cfg)
            print(f"{mg.MODE_NAMES[mode]:>13} {m}x{n}x{k}: cfg {cfg} ({info['BM']}x{info['BN']}x{info['BK']}) "
                  f"split {split}", flush=True)
        save()
    if "grouped" in what:
        mixes = {mg.MODE_F32: (512, 32, 1024), mg.MODE_BF16: (512, 32, 1024), mg.MODE_F16: (512, 32, 1024),
                 mg.MODE_SPLIT_BF16X3: (512, 32, 1024), mg.MODE_F8E4M3: (48, 64, 4096)}
        for mode, (count, lo, hi) in mixes.items():
            if mode not in keep:
                continue
            calibrate_mix(mg, _lib, lib, torch, mode, count, lo, hi, stream)
            print(f"grouped mix {mg.MODE_NAMES[mode]}: kernel variant and small-tile efficiency measured", flush=True)
        save()
    buckets = bucket_shapes(mg)
    for kind, entry in (("plain-buckets", lib.gemm_tune_bucket), ("grouped", lib.gemm_tune_grouped)):
        if kind not in what:
            continue
        for mode, shapes in buckets.items():
            if mode not in keep:
                continue
            t0 = time.time()
            for i, (m, n, k) in enumerate(shapes):
                _lib.check(entry(mode, m, n, k, stream))
                if i % 64 == 63:
                    print(f"{kind} {mg.MODE_NAMES[mode]}: {i + 1}/{len(shapes)} ({time.time() - t0:.0f} s)",
                          flush=True)
            save()
            print(f"{kind} {mg.MODE_NAMES[mode]}: {len(shapes)} buckets in {time.time() - t0:.0f} s", flush=True)
    print(f"wrote {args.out}")


if __name__ == "__main__":
    sys.exit(main())
