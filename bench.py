"""Benchmark: lattice updates per second of the colour-gradient LB printing step.

Workload: the print-bed filament set-up, D3Q19, 512x256x128 (16.8M cells),
head moving at 0.01 along x, power-law ink n = 0.5, FP32 storage and
arithmetic, synthetic initial state (ink-filled nozzle in air).  One step is
one full time step of the method on every cell.

Prints one JSON line: whole-step MLUPS, the HBM roofline of the dominant
kernel (the fused step kernel, timed with HIP events on the library's stream
over the timed region; beside it the rate of a plain 1 GiB copy on the same
GPU) and the FP64 CPU oracle timed on a bounded sample of the same workload.

Other modes: --workload largest (the 1024x512x384 domain, BF16 deviations by
default), --workload print2d (the paper's 2-D printing set-up on D2Q9, swept
over the nozzle speed, with the Sec. IV observables) and --serve (the
parameter-sweep trace through the continuous-batching server and one request
at a time).
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per lattice update: each of the 2 x 19 populations read
# once and written once; the reduced forms also read and write the cell's
# five FP32 moments (2 x (38 x 2 + 5 x 4) B).
BYTES_PER_LU = {"f64": 608, "f32": 304, "bf16dev": 192, "f16dev": 192}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fused_pc_print_bed_512x256x128_{}_traffic.md")


def source_digest() -> str:
    """SHA-256 over the HIP sources and the C header (sorted by name)."""
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(ROOT, "paper_2102_02655_amd", "csrc", "*")))
    files.append(os.path.join(ROOT, "include", "lbprint.h"))
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(storage: str):
    """HBM bytes per launch of the fused kernel on the print bed from the
    committed PMC summary of this storage form, or None when there is none or
    the kernel sources changed since it was taken."""
    path = TRAFFIC_FILE.format(storage)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m_sha = re.search(r"source_sha256:\s*([0-9a-f]{64})", txt)
    m_b = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if not (m_sha and m_b) or m_sha.group(1) != source_digest():
        return None
    return float(m_b.group(1))


def host_cpu():
    """CPU model, logical CPUs and physical cores of this host (from
    /proc/cpuinfo: distinct (physical id, core id) pairs)."""
    model, cores, logical = None, set(), 0
    phys = core = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "processor":
                    logical += 1
                elif k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None:
            cores.add((phys, core))
    except OSError:
        pass
    return {"cpu_model": model, "logical_cpus": logical or os.cpu_count(), "physical_cores": len(cores) or None}


def cpu_baseline(seconds: float = 15.0, full_box: bool = False):
    """The FP64 oracle on the 128x64x32 crop of the same set-up: three timed
    runs of about seconds/4 each on all the oracle's threads (median
    reported), then a single-thread run; with full_box, also 20 steps of the
    whole 512x256x128 box (about 15 GB of host memory, a minute of CPU)."""
    from oracle import oracle as O
    from paper_2102_02655_amd import workloads as W

    cfg = W.print_bed(storage="f64", crop=True)
    ry, rb = W.nozzle_fields(cfg)
    s = O.OracleSim(cfg, ry, rb)
    s.step(1)
    cells = cfg["shape"][0] * cfg["shape"][1] * cfg["shape"][2]
    threads = O.threads()

    def timed(budget):
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < budget:
            s.step(2)
            steps += 2
        return cells * steps / (time.perf_counter() - t0) / 1e6, steps

    runs = [timed(seconds / 4) for _ in range(3)]
    rates = sorted(r for r, _ in runs)
    O.set_threads(1)
    one, one_steps = timed(seconds / 4)
    O.set_threads(threads)
    out = {"value": rates[1], "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"128x64x32 crop of the print-bed set-up, FP64, median of 3 runs of "
                     f"{'/'.join(str(n) for _, n in runs)} steps on {threads} threads after 1 warm-up step",
           "runs_MLUPS": [r for r, _ in runs], "one_thread_MLUPS": one, "one_thread_steps": one_steps}
    out.update(host_cpu())
    del s
    if full_box:
        cfg = W.print_bed(storage="f64")
        ry, rb = W.nozzle_fields(cfg)
        s = O.OracleSim(cfg, ry, rb)
        s.step(1)
        t0 = time.perf_counter()
        s.step(20)
        dt = time.perf_counter() - t0
        out["full_box_MLUPS"] = 512 * 256 * 128 * 20 / dt / 1e6
        out["full_box_sample"] = "20 steps of the 512x256x128 print bed after 1 warm-up step"
    return out


def copy_probe(nbytes: int = 1 << 30, reps: int = 3):
    """A plain elementwise copy of known size (read nbytes, write nbytes),
    used to scale the PMC byte counters."""
    import torch

    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    print(f"copy probe: {reps} x torch.neg over {nbytes} B (read {nbytes} B + write {nbytes} B per launch)",
          file=sys.stderr, flush=True)


def copy_rate(nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Attainable HBM rate of a plain elementwise copy (read nbytes, write
    nbytes per launch), GB/s, timed with events on the current stream."""
    import torch

    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.neg(a, out=b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.neg(a, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * nbytes / (ms * 1e-3) / 1e9


def serve(args):
    """Serving sweep: the parameter-sweep trace through the continuous-batching
    server, then through one-at-a-time plain stepping, on the same GPU."""
    import numpy as np
    import torch

    from paper_2102_02655_amd import lbprint as LB
    from paper_2102_02655_amd import serving as S

    st = args.serve_storage
    reqs = S.make_requests(count=args.serve_count, seed=4, rate=args.serve_rate, steps=args.serve_steps, storage=st)
    log = (lambda m: print(m, file=sys.stderr, flush=True)) if args.verbose else None
    warm = S.make_requests(count=2, seed=99, rate=1000.0, lmin=32, lmax=40, steps=4)
    S.Server(8 << 30, chunk=2).run(warm)  # library load, first captures
    torch.cuda.synchronize()
    batched = S.Server(int(args.serve_budget_gb * 1e9), chunk=args.serve_chunk, keep_fields=False,
                       lanes=args.serve_lanes).run(reqs, log=log)
    # the baseline is plain FP32 served one request at a time
    seq = None
    if not args.serve_skip_sequential:
        base = reqs if st == "f32" else S.make_requests(count=args.serve_count, seed=4, rate=args.serve_rate,
                                                        steps=args.serve_steps, storage="f32")
        seq = S.run_sequential(base, log=log)
    # spot check: a few requests rerun alone reproduce the served masses bit for bit
    same = True
    by_id = {r.id: r for r in batched.results}
    for req in reqs[:3]:
        sim = LB.Sim(req.cfg, req.ry, req.rb)
        sim.step(req.steps)
        _, _, _, cons = sim.moments(dtype=np.float64)
        same &= bool(np.array_equal(cons["mass"], by_id[req.id].mass))
        sim.close()
    b, q = batched.summary(), (seq.summary() if seq is not None else None)
    out = {
        "metric": "sweep sims/hour",
        "value": b["sims_per_hour"],
        "unit": "sims/hour",
        "n_gpus": 1,
        "higher_is_better": True,
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"parameter sweep: {args.serve_count} printing simulations, cubic boxes L~U{{32..160}}, "
                               f"{args.serve_steps} steps each, Poisson arrivals {args.serve_rate}/s",
                   "storage": st, "budget_GB": args.serve_budget_gb, "chunk": args.serve_chunk,
                   "lanes": args.serve_lanes},
        "batched": b,
        "sequential": q,
        "mix_equals_alone": same,
    }
    print(json.dumps(out), flush=True)


def largest(args):
    """The largest single domain, 1024x512x384 (201M cells): footprint, MLUPS,
    the HBM roofline of the fused kernel and the FP64 mass ledger over the run."""
    import torch

    from paper_2102_02655_amd import lbprint, workloads as W

    st = args.storage or "bf16dev"
    cfg = W.largest_domain(storage=st)
    nx, ny, nz = cfg["shape"]
    cells = nx * ny * nz
    ry, rb = W.nozzle_fields(cfg)
    sim = lbprint.Sim(cfg, ry, rb, device="cuda:0")
    del ry, rb
    c0 = sim.moments_device(None, None, None)
    print(f"largest domain {nx}x{ny}x{nz} {st}: created, footprint {sim.nbytes / 1e9:.2f} GB", file=sys.stderr,
          flush=True)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    sim.timing(True)
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sim.timing(False)
    tm = sim.timing_read()
    c1 = sim.moments_device(None, None, None)
    mlups = cells * args.steps / dt / 1e6
    bpl = BYTES_PER_LU[st]
    k_ms = tm["step_ms"] / max(tm["steps"], 1)
    achieved = bpl * cells / (k_ms * 1e-3) / 1e9
    # mass ledger since creation: change = wall + open-face + created - deleted
    resid = []
    for k in range(2):
        lhs = c1["mass"][k] - c0["mass"][k]
        rhs = c1["mass_wall"][k] + c1["mass_open"][k] + c1["mass_created"][k] - c1["mass_deleted"][k]
        resid.append(abs(lhs - rhs) / c1["mass"][1])
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
        "dtype": "f64" if st == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"largest single domain, D3Q19 {nx}x{ny}x{nz}, moving head u=0.01, r_in 24, "
                               f"power-law n=0.5", "cells": cells, "storage": st},
        "footprint_GB": sim.nbytes / 1e9,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "kb_fused_pc", "kernel_ms": k_ms,
                     "algorithmic_bytes": bpl * cells, "prep_ms": tm["prep_ms"] / max(tm["steps"], 1)},
        "mass": list(map(float, c1["mass"])),
        "mass_ledger_residual_rel": resid,
        "cpu_baseline": None,
    }
    sim.close()
    print(json.dumps(out), flush=True)


def print2d(args):
    """The paper's 2-D printing set-up (Sec. III, 880 x 240 D2Q9, one Table I
    ink) swept over the nozzle speed v_nozzle = ratio * v_ink: each run lets
    the ink cross the gap to the substrate and the nozzle travel `travel`
    nozzle widths, then reads the Sec. IV observables of the thread behind
    the nozzle (lb_observe) and forms the POI, normalised over the sweep."""
    import math

    import torch

    from paper_2102_02655_amd import lbprint, workloads as W

    st = args.storage or "f32"
    d, gap, wall, nx, nz = 60.0, 60.0, 4.0, 880, 240
    v_ink = W.ink_speed_lb(args.ink)
    runs, total_lu, total_s = [], 0, 0.0
    for r in [float(v) for v in args.ratios.split(",")]:
        cfg = W.printing_2d(args.ink, v_ratio=r, nx=nx, nz=nz, d=d, gap=gap, wall=wall, storage=st)
        ry, rb = W.nozzle_fields(cfg)
        steps = int(math.ceil(gap / v_ink + args.travel * d / (r * v_ink)))
        sim = lbprint.Sim(cfg, ry, rb, device="cuda:0")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, chunk = 0, 20000
        while done < steps:
            k = min(chunk, steps - done)
            sim.step(k)
            done += k
            torch.cuda.synchronize()
            print(f"print2d {args.ink} v_nozzle = {r} v_ink: {done}/{steps} steps", file=sys.stderr, flush=True)
        dt = time.perf_counter() - t0
        # the thread: the ink deposited behind the nozzle (the head moves
        # towards -x), from half a nozzle width behind its trailing wall (the
        # ink still attached to the nozzle left out) back to its start, below
        # the tip
        x_start = cfg["nozzle"]["x0"][0]
        x_now = x_start - r * v_ink * steps
        lo = int(math.ceil(x_now + d + wall))
        length = int(math.ceil(x_start + d / 2.0 + wall)) - lo + 1
        obs = sim.observe(lo % nx, min(length, nx), int(gap))
        _, _, _, cons = sim.moments(dtype="float32")
        sim.close()
        poi = (obs["coverage"] * d / (obs["height"] * obs["dp_max"])
               if obs["height"] > 0 and obs["dp_max"] > 0 else 0.0)
        total_lu += nx * nz * steps
        total_s += dt
        runs.append({"v_ratio": r, "steps": steps, "seconds": dt, "MLUPS": nx * nz * steps / dt / 1e6,
                     "height": obs["height"], "coverage": obs["coverage"], "ink_area": obs["ink_area"],
                     "dp_max_over_p0": obs["dp_max"] / obs["p0"], "substrate_ink": obs["substrate_ink"],
                     "POI": poi, "mass": list(map(float, cons["mass"]))})
    top = max((x["POI"] for x in runs), default=0.0)
    for x in runs:
        x["POI_norm"] = x["POI"] / top if top > 0 else 0.0
    out = {"metric": "MLUPS", "value": total_lu / total_s / 1e6, "unit": "MLUPS", "n_gpus": 1,
           "higher_is_better": True, "vs_baseline": None, "dtype": "f64" if st == "f64" else "f32",
           "data": "synthetic",
           "config": {"workload": f"2-D printing sweep (Sec. III set-up), D2Q9 {nx}x{nz}, ink {args.ink}, "
                                  f"nozzle travel {args.travel} d after the ink crosses the gap",
                      "storage": st, "v_ink": v_ink},
           "runs": runs}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default=None, choices=["f32", "f64", "bf16dev", "f16dev"],
                    help="population storage (default: f32 on the print bed, bf16dev on the largest domain)")
    ap.add_argument("--workload", default="print_bed", choices=["print_bed", "largest", "print2d"],
                    help="print_bed: the 512x256x128 benchmark; largest: the 1024x512x384 domain; "
                         "print2d: the paper's 2-D printing sweep over the nozzle speed")
    ap.add_argument("--ink", default="1%-25C", help="print2d: Table I ink")
    ap.add_argument("--ratios", default="0.25,0.5,0.75,1.0,1.25,1.5,1.75",
                    help="print2d: nozzle speeds in units of the ink speed")
    ap.add_argument("--travel", type=float, default=3.0, help="print2d: nozzle travel in nozzle widths")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-full", action="store_true",
                    help="also time the oracle on 20 steps of the whole 512x256x128 box (about 15 GB of host memory)")
    ap.add_argument("--copy-probe", action="store_true", help="first run a plain copy of known size (PMC scaling)")
    ap.add_argument("--serve", action="store_true", help="run the serving sweep instead of the step benchmark")
    ap.add_argument("--serve-count", type=int, default=256)
    ap.add_argument("--serve-steps", type=int, default=2000)
    ap.add_argument("--serve-rate", type=float, default=4.0)
    ap.add_argument("--serve-budget-gb", type=float, default=32.0)
    ap.add_argument("--serve-chunk", type=int, default=20)
    ap.add_argument("--serve-lanes", type=int, default=2, help="batches on concurrent streams")
    ap.add_argument("--serve-storage", default="f32", choices=["f32", "bf16dev", "f16dev"])
    ap.add_argument("--serve-skip-sequential", action="store_true", help="skip the one-at-a-time FP32 baseline")
    ap.add_argument("--verbose", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.serve:
        serve(args)
        return
    if args.workload == "largest":
        largest(args)
        return
    if args.workload == "print2d":
        print2d(args)
        return
    if args.storage is None:
        args.storage = "f32"

    import torch

    from paper_2102_02655_amd import lbprint, workloads as W

    if args.copy_probe:
        copy_probe()
    cfg = W.print_bed(n=0.5, storage=args.storage)
    ry, rb = W.nozzle_fields(cfg)
    nx, ny, nz = cfg["shape"]
    cells = nx * ny * nz
    sim = lbprint.Sim(cfg, ry, rb, device="cuda:0")
    sim.step(args.warmup)
    torch.cuda.synchronize()
    sim.timing(True)
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    sim.timing(False)
    tm = sim.timing_read()
    _, _, _, cons = sim.moments(dtype="float32")
    mlups = cells * args.steps / dt / 1e6
    bpl = BYTES_PER_LU[args.storage]
    k_ms = tm["step_ms"] / max(tm["steps"], 1)
    alg_bytes = bpl * cells
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    traffic = measured_traffic(args.storage)
    copy_gbs = copy_rate()
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
        "dtype": "f64" if args.storage == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"print-bed filament, D3Q19 {nx}x{ny}x{nz}, moving head u=0.01, power-law n=0.5",
                   "cells": cells, "storage": args.storage},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "kb_fused_pc", "kernel_ms": k_ms, "algorithmic_bytes": alg_bytes,
                     "prep_ms": tm["prep_ms"] / max(tm["steps"], 1),
                     "whole_step_GBs": bpl * mlups * 1e6 / 1e9,
                     # the kernel's algorithmic rate against a plain copy's on this GPU
                     "copy_GBs": copy_gbs, "frac_of_copy": achieved / copy_gbs},
        "mass": list(map(float, cons["mass"])),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(full_box=args.cpu_full)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
