"""Benchmark: lattice updates per second of the colour-gradient LB printing step.

Workload: the print-bed filament set-up, D3Q19, 512x256x128 (16.8M cells),
head moving at 0.01 along x, power-law ink n = 0.5, FP32 storage and
arithmetic, synthetic initial state (ink-filled nozzle in air).  One step is
one full time step of the method on every cell.

Prints one JSON line (MLUPS, HBM roofline fraction of the dominant kernel,
and the FP64 CPU oracle timed on a bounded sample of the same workload).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_LU = {"f64": 608, "f32": 304}


def cpu_baseline(seconds: float = 15.0):
    """The FP64 oracle on the 128x64x32 crop of the same set-up, as many steps
    as fit in about `seconds`, on all host threads."""
    import numpy as np  # noqa: F401

    from oracle import oracle as O
    from paper_2102_02655_amd import workloads as W

    cfg = W.print_bed(storage="f64", crop=True)
    ry, rb = W.nozzle_fields(cfg)
    s = O.OracleSim(cfg, ry, rb)
    s.step(1)
    cells = cfg["shape"][0] * cfg["shape"][1] * cfg["shape"][2]
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < seconds:
        s.step(2)
        steps += 2
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": cells * steps / dt / 1e6, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"128x64x32 crop of the print-bed set-up, {steps} steps after 1 warm-up, FP64"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2102_02655_amd import lbprint, workloads as W

    cfg = W.print_bed(n=0.5, storage=args.storage)
    ry, rb = W.nozzle_fields(cfg)
    nx, ny, nz = cfg["shape"]
    cells = nx * ny * nz
    sim = lbprint.Sim(cfg, ry, rb, device="cuda:0")
    sim.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _, _, _, cons = sim.moments(dtype="float32")
    mlups = cells * args.steps / dt / 1e6
    bpl = BYTES_PER_LU[args.storage]
    achieved = bpl * mlups * 1e6 / 1e9
    out = {
        "metric": "MLUPS",
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {"workload": f"print-bed filament D3Q19 {nx}x{ny}x{nz}, moving head, power-law n=0.5",
                   "cells": cells, "storage": args.storage},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "scope": "whole step, algorithmic bytes"},
        "mass": list(map(float, cons["mass"])),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
