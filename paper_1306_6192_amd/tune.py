"""Measure the tile configuration and split-K factor of the benchmark shapes on
the current GPU and write the tuning table the library loads at start-up.

    python -m paper_1306_6192_amd.tune [--out PATH]

Every entry is chosen by `gemm_tune` (the library times each legal
configuration and split-K factor with HIP events on non-zero operands,
re-times the near-ties and keeps the fastest); the table is keyed by
(mode, m, n, k) only.
"""
from __future__ import annotations

import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning", "mi355x.jsonl")

PLAIN_F32 = [(2048, 2048, 2048), (4096, 4096, 4096), (8192, 8192, 8192), (8192, 1024, 4096), (128, 8192, 8192),
             (512, 512, 512)]
SQUARES = [(2048, 2048, 2048), (4096, 4096, 4096), (8192, 8192, 8192)]


def shapes():
    import paper_1306_6192_amd as mg
    out = [(mg.MODE_F32, s) for s in PLAIN_F32]
    for mode in (mg.MODE_BF16, mg.MODE_F16, mg.MODE_F8E4M3, mg.MODE_SPLIT_BF16X3):
        out += [(mode, s) for s in SQUARES]
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    args = ap.parse_args(argv)
    import torch

    import paper_1306_6192_amd as mg
    from paper_1306_6192_amd import _lib
    torch.cuda.set_device(0)
    mg.load()
    for mode, (m, n, k) in shapes():
        cfg, split = mg.tune(mode, m, n, k)
        info = mg.config_info(mode, cfg)
        print(f"{mg.MODE_NAMES[mode]:>13} {m}x{n}x{k}: cfg {cfg} ({info['BM']}x{info['BN']}x{info['BK']}) "
              f"split {split}", flush=True)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    _lib.check(_lib.load().gemm_tuner_save(args.out.encode()))
    print(f"wrote {args.out}")


if __name__ == "__main__":
    sys.exit(main())
