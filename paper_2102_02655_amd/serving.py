"""Continuous-batching server for parameter-sweep simulations.

Requests (a printing set-up, an initial state, a step count) arrive over
time.  The server keeps every admitted simulation's state resident on the
GPU, admits waiting requests in arrival order while their device footprint
(lb_footprint) fits the memory budget, and keeps every admitted simulation
stepping: each has a stream of its own with up to two chunks of steps queued
(each chunk one launch of its captured chain of steps), so their work
overlaps on the device; a simulation whose last chunk has completed is read
out and released at once, and requests that arrive while others run join as
memory frees up.

The comparison point ("sequential") serves the same trace one request at a
time with plain lb_step calls.

All work runs in the HIP library; this module is host-side scheduling only.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import lbprint as LB
from . import workloads as W


@dataclass
class Request:
    id: int
    arrival: float          # seconds after the start of the run
    cfg: dict
    steps: int
    ry: np.ndarray = None
    rb: np.ndarray = None


@dataclass
class Result:
    id: int
    arrival: float
    admitted: float
    done: float
    cells: int
    steps: int
    mass: np.ndarray = None
    fields: tuple = None    # (rho_Y, rho_B, u) if kept

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class RunStats:
    mode: str
    results: list = field(default_factory=list)
    wall: float = 0.0
    peak_bytes: int = 0
    launches: int = 0   # chunk launches (batched) or runs (sequential)

    def summary(self) -> dict:
        lat = np.array([r.latency for r in self.results])
        lups = sum(r.cells * r.steps for r in self.results)
        return {
            "mode": self.mode,
            "requests": len(self.results),
            "wall_s": self.wall,
            "sims_per_hour": len(self.results) / self.wall * 3600.0 if self.wall > 0 else None,
            "MLUPS": lups / self.wall / 1e6 if self.wall > 0 else None,
            "latency_p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "latency_p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "latency_mean_s": float(lat.mean()) if len(lat) else None,
            "peak_resident_GB": self.peak_bytes / 1e9,
            "launches": self.launches,
        }


def make_requests(count=256, seed=4, rate=4.0, lmin=32, lmax=160, steps=2000, storage="f32"):
    """The sweep trace: Poisson arrivals, cubic boxes of edge U{lmin..lmax},
    ink power-law n, extrusion and head speeds drawn per request."""
    reqs = []
    for r in W.serving_trace(count=count, seed=seed, rate=rate, lmin=lmin, lmax=lmax, steps=steps,
                             storage=storage):
        ry, rb = W.nozzle_fields(r["cfg"])
        reqs.append(Request(r["id"], r["arrival"], r["cfg"], r["steps"], ry, rb))
    return reqs


class Server:
    """Continuous batching over one GPU."""

    def __init__(self, budget_bytes: int, chunk: int = 20, device: str = "cuda:0", keep_fields: bool = False,
                 depth: int = 2):
        if chunk < 2:
            raise ValueError("chunk must be >= 2")
        if depth < 1:
            raise ValueError("depth must be >= 1")
        self.budget = int(budget_bytes)
        self.chunk = int(chunk)
        self.depth = int(depth)
        self.device = device
        self.keep_fields = keep_fields

    def run(self, requests, log=None) -> RunStats:
        """Serve `requests` in arrival order.  Every admitted simulation keeps
        up to `depth` chunks of `chunk` steps queued on its own stream (one
        lb_step_batch call each, a captured chain of steps); completion is
        polled per simulation with stream events, so the host never waits for
        the whole device and the GPU is not left idle while finished
        simulations are read out or new ones created."""
        import torch

        stats = RunStats("batched")
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        queue = collections.deque()
        active = []  # [req, sim, steps not yet launched, bytes, admitted_at, deque of chunk events]
        used = 0
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        while pending or queue or active:
            clock = now()
            while pending and pending[0].arrival <= clock:
                queue.append(pending.popleft())
            # admission in arrival order, by device footprint
            while queue:
                need = LB.footprint(queue[0].cfg)
                if need > self.budget:
                    raise RuntimeError(f"request {queue[0].id} needs {need} B, above the budget")
                if used + need > self.budget:
                    break
                req = queue.popleft()
                sim = LB.Sim(req.cfg, req.ry, req.rb, device=self.device, stream=torch.cuda.Stream(self.device))
                active.append([req, sim, req.steps, need, now(), collections.deque()])
                used += need
                stats.peak_bytes = max(stats.peak_bytes, used)
            progressed = False
            still = []
            for a in active:
                req, sim, left, need, admitted, inflight = a
                while inflight and inflight[0].query():
                    inflight.popleft()
                    progressed = True
                while left > 0 and len(inflight) < self.depth:
                    k = min(self.chunk, left)
                    LB.step_batch([sim], [k])
                    ev = torch.cuda.Event()
                    ev.record(sim.stream)
                    inflight.append(ev)
                    left -= k
                    stats.launches += 1
                    progressed = True
                a[2] = left
                if left > 0 or inflight:
                    still.append(a)
                    continue
                ry, rb, u, cons = sim.moments(dtype=np.float64)
                nx, ny, nz = req.cfg["shape"]
                res = Result(req.id, req.arrival, admitted, now(), nx * ny * nz, req.steps, cons["mass"],
                             (ry, rb, u) if self.keep_fields else None)
                stats.results.append(res)
                if log:
                    log(f"request {req.id} done: L={nx} latency {res.latency:.3f} s")
                sim.close()
                used -= need
                progressed = True
            active = still
            if not progressed:
                if active:
                    time.sleep(0.0002)
                elif pending:
                    wait = pending[0].arrival - now()
                    if wait > 0:
                        time.sleep(min(wait, 0.005))
        torch.cuda.synchronize(self.device)
        stats.wall = now()
        return stats


def run_sequential(requests, device: str = "cuda:0", keep_fields: bool = False, log=None) -> RunStats:
    """The same trace served one request at a time with lb_step."""
    import torch

    stats = RunStats("sequential")
    order = sorted(requests, key=lambda r: r.arrival)
    t0 = time.perf_counter()
    now = lambda: time.perf_counter() - t0  # noqa: E731
    for req in order:
        wait = req.arrival - now()
        if wait > 0:
            time.sleep(wait)
        admitted = now()
        sim = LB.Sim(req.cfg, req.ry, req.rb, device=device)
        stats.peak_bytes = max(stats.peak_bytes, LB.footprint(req.cfg))
        sim.step(req.steps)
        torch.cuda.synchronize(device)
        ry, rb, u, cons = sim.moments(dtype=np.float64)
        nx, ny, nz = req.cfg["shape"]
        res = Result(req.id, req.arrival, admitted, now(), nx * ny * nz, req.steps, cons["mass"],
                     (ry, rb, u) if keep_fields else None)
        stats.results.append(res)
        if log:
            log(f"request {req.id} done (sequential): L={nx} latency {res.latency:.3f} s")
        sim.close()
        stats.launches += 1
    stats.wall = now()
    return stats
