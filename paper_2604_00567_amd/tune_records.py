"""Generates tuning records for this device: runs the library's autotuner
(fft_tune: every compiled configuration timed with HIP events, only outputs
bit-identical to the first configuration that runs, normally the default,
accepted) for N = 2^1 .. 2^20 in
each precision and appends the winners to --out (the DSFFT_TUNE_FILE
format).  Copy the file beside libdsfft.so as tuning_records.txt to make the
records the library's defaults.

    python -m paper_2604_00567_amd.tune_records --out tuning_records.txt
"""
from __future__ import annotations

import argparse
import json
import os
import sys


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--bytes", type=float, default=float(1 << 28),
                    help="input bytes per timed execute (256 MiB: the batched workloads' size)")
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--log-min", type=int, default=1)
    ap.add_argument("--log-max", type=int, default=20)
    ap.add_argument("--dtypes", default="f16,f32,f16f32",
                    help="comma-separated: f16, f32, f16f32 (binary16 storage, binary32 butterflies)")
    args = ap.parse_args()
    os.environ["DSFFT_TUNE_FILE"] = os.path.abspath(args.out)
    from paper_2604_00567_amd import binding

    ap_dtypes = args.dtypes.split(",")
    for dtype in ap_dtypes:
        eb = 8 if dtype == "f32" else 4
        for m in range(args.log_min, args.log_max + 1):
            n = 1 << m
            batch = max(1, int(args.bytes // (n * eb)))
            rep = binding.fft_tune(n, batch, dtype, "dual_select", reps=args.reps)
            best = max(rep, key=lambda c: c["GBs"])
            print(json.dumps({"n": n, "dtype": dtype, "batch": batch, "best": best,
                              "candidates": [(c["variant"], c["GBs"], c["config"]) for c in rep]}),
                  flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
