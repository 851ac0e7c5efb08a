"""Benchmark of the plain FP32 product on one MI355X.

One step = one product of each plain FP32 workload shape, (m, n, k) in
{2048^3, 4096^3, 8192^3, (8192, 1024, 4096), (128, 8192, 8192)}, entries
uniform[-1, 1] from seed 0, inputs resident in HBM before the timed region.
The line printed reports aggregate TFLOP/s over the step (2mnk flops per
product), the roofline of the dominant launch (the 8192^3 product, timed with
HIP events on the stream it runs on), the sampled normwise error of every
shape against the binary64 oracle, and the oracle itself timed on the host's
cores on a bounded sample (some rows of the 8192^3 product).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SHAPES = [(2048, 2048, 2048), (4096, 4096, 4096), (8192, 8192, 8192), (8192, 1024, 4096), (128, 8192, 8192)]
DOMINANT = (8192, 8192, 8192)
PEAK_FP32_MFMA_TFLOPS = 157.3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target length of the oracle sample")
    ap.add_argument("--samples", type=int, default=512, help="sampled outputs per shape for the error")
    return ap.parse_args()


def cpu_baseline(A, B, target_s: float):
    """The oracle (binary64 loop, all host threads) on whole rows of the
    8192^3 product, enough rows for about `target_s` seconds."""
    import oracle
    threads = oracle.default_threads()
    B64 = np.ascontiguousarray(B, dtype=np.float64)
    m, k = A.shape
    n = B.shape[1]
    rows = threads
    t0 = time.perf_counter()
    oracle.gemm(A[:rows].astype(np.float64), B64, threads)
    dt = time.perf_counter() - t0
    total_rows = rows
    total_t = dt
    more = int(max(0, (target_s - dt) / max(dt, 1e-9) * rows))
    more = min(more, m - rows) // threads * threads
    if more > 0:
        t0 = time.perf_counter()
        oracle.gemm(A[rows:rows + more].astype(np.float64), B64, threads)
        total_t += time.perf_counter() - t0
        total_rows += more
    flops = 2.0 * total_rows * n * k
    return {"value": flops / total_t / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"{total_rows} full rows of the {m}x{n}x{k} product (binary64 loop), {total_t:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus above 1 is not supported"}))
        sys.exit(2)
    import torch

    import paper_1306_6192_amd as mg
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    mg.load()

    # inputs, resident in HBM
    data = []
    for (m, n, k) in SHAPES:
        A, B = synth.pair(m, n, k, seed=0)
        dA = torch.from_numpy(A).to(dev)
        dB = torch.from_numpy(B).to(dev)
        dC = torch.empty((m, n), dtype=torch.float32, device=dev)
        data.append((A, B, dA, dB, dC))
    stream = torch.cuda.current_stream()

    def step(events=None):
        for i, (_, _, dA, dB, dC) in enumerate(data):
            if events is not None:
                events[i][0].record(stream)
            mg.gemm(dA, dB, out=dC, stream=stream)
            if events is not None:
                events[i][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in SHAPES] for _ in range(args.steps)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record(stream)
    for s in range(args.steps):
        step(evs[s])
    t_end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t_start.elapsed_time(t_end)

    flops_step = sum(2.0 * m * n * k for (m, n, k) in SHAPES)
    value = flops_step * args.steps / (total_ms / 1e3) / 1e12
    per_shape = []
    dom = None
    for i, (m, n, k) in enumerate(SHAPES):
        ms = [evs[s][i][0].elapsed_time(evs[s][i][1]) for s in range(args.steps)]
        avg = float(np.mean(ms))
        tf = 2.0 * m * n * k / (avg / 1e3) / 1e12
        cfg, split = mg.tuner_lookup(mg.MODE_F32, m, n, k)
        per_shape.append({"m": m, "n": n, "k": k, "ms_avg": round(avg, 4), "ms_min": round(float(np.min(ms)), 4),
                          "tflops": round(tf, 2), "frac_peak": round(tf / PEAK_FP32_MFMA_TFLOPS, 4),
                          "cfg": mg.config_info(mg.MODE_F32, cfg), "split_k": split})
        if (m, n, k) == DOMINANT:
            dom = (avg, tf)

    # sampled normwise error of every shape against the binary64 oracle
    import oracle
    g = synth.rng(1234)
    for i, (m, n, k) in enumerate(SHAPES):
        A, B, _, _, dC = data[i]
        C = dC.cpu().numpy()
        rows = g.integers(0, m, size=args.samples)
        cols = g.integers(0, n, size=args.samples)
        R = oracle.gemm_sampled(A, B, rows, cols)
        per_shape[i]["rel_err_sampled"] = float(oracle.relerr(C[rows, cols], R))

    achieved = dom[1]
    line = {
        "metric": "GEMM TFLOP/s (fp32, plain) and % MFMA peak at stated error",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: uniform[-1,1] float32, numpy default_rng seed 0 (A then B)",
        "config": {"workload": "plain fp32 gemm, one product each of (m,n,k) = 2048^3, 4096^3, 8192^3, "
                               "(8192,1024,4096), (128,8192,8192), row-major",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": PEAK_FP32_MFMA_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_MFMA_TFLOPS, 4), "traffic": None,
                     "kernel": "gemm_f32_plain_kernel, 8192^3", "avg_launch_ms": round(dom[0], 4)},
        "per_shape": per_shape,
        "max_rel_err_sampled": max(p["rel_err_sampled"] for p in per_shape),
        "wall_s_timed": round(wall, 3),
    }
    if not args.no_cpu_baseline:
        A, B = data[SHAPES.index(DOMINANT)][:2]
        line["cpu_baseline"] = cpu_baseline(A, B, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
