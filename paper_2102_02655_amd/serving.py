"""Continuous-batching server for parameter-sweep simulations.

Requests (a printing set-up, an initial state, a step count) arrive over
time.  The server keeps every admitted simulation's state resident on the
GPU and admits waiting requests in arrival order while their device
footprint (lb_footprint) fits the memory budget and a batch has a free
slot (lb_batch_step takes at most 64 members).  Admitted simulations are
members of `lanes` batches (lb_batch_*), each on a stream of its own; a new
member joins the batch with the fewest cells.  Every round is one
lb_batch_step call per batch that advances each member by up to `chunk`
steps, a replay of the batch's captured graph of batched kernels over its
device slot table; the batches' streams run concurrently, so one batch's
kernels fill the GPU while another's launch drains.  Up to `depth` rounds
are queued; when a round has run, the simulations it finished are read out
and released, and requests that arrived meanwhile join the next round.

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
                 depth: int = 2, lanes: int = 2):
        if chunk < 1:
            raise ValueError("chunk must be >= 1")
        if depth < 1:
            raise ValueError("depth must be >= 1")
        if lanes < 1:
            raise ValueError("lanes must be >= 1")
        self.budget = int(budget_bytes)
        self.chunk = int(chunk)
        self.depth = int(depth)
        self.lanes = int(lanes)
        self.device = device
        self.keep_fields = keep_fields

    def run(self, requests, log=None) -> RunStats:
        """Serve `requests` (one storage form) in arrival order."""
        import torch

        stats = RunStats("batched")
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        if not pending:
            return stats
        forms = {r.cfg.get("storage", "f32") for r in pending}
        if len(forms) != 1:
            raise ValueError(f"one storage form per server run, got {sorted(forms)}")
        form = forms.pop()
        batches = [LB.Batch(form, device=self.device) for _ in range(self.lanes)]
        cells = [0] * self.lanes      # cells of each batch's members
        queue = collections.deque()
        active = []                   # admitted members still to be read out
        rounds = collections.deque()  # (events, members this round finished)
        used = 0
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731

        while pending or queue or active:
            clock = now()
            while pending and pending[0].arrival <= clock:
                queue.append(pending.popleft())
            # admission in arrival order, by device footprint (each simulation
            # is created on a stream of its own, so its upload overlaps the
            # queued rounds)
            while queue and len(active) < self.lanes * LB.Batch.MAX_MEMBERS:
                need = LB.footprint(queue[0].cfg)
                if need > self.budget:
                    raise RuntimeError(f"request {queue[0].id} needs {need} B, above the budget")
                if used + need > self.budget:
                    break
                open_lanes = [i for i in range(self.lanes)
                              if sum(m.lane == i for m in active) < LB.Batch.MAX_MEMBERS]
                lane = min(open_lanes, key=lambda i: cells[i])
                req = queue.popleft()
                sim = LB.Sim(req.cfg, req.ry, req.rb, device=self.device, stream=torch.cuda.Stream(self.device))
                nx, ny, nz = req.cfg["shape"]
                active.append(_Member(req, sim, need, now(), lane, nx * ny * nz))
                cells[lane] += nx * ny * nz
                used += need
                stats.peak_bytes = max(stats.peak_bytes, used)
            progressed = False
            # one more round of every member that still has steps to launch
            members = [m for m in active if m.left > 0]
            if members and len(rounds) < self.depth:
                events = []
                for i, batch in enumerate(batches):
                    mine = [m for m in members if m.lane == i]
                    if not mine:
                        continue
                    ks = [min(self.chunk, m.left) for m in mine]
                    batch.step([m.sim for m in mine], ks)
                    ev = torch.cuda.Event()
                    ev.record(batch.stream)
                    events.append(ev)
                    for m, k in zip(mine, ks):
                        m.left -= k
                    stats.launches += 1
                rounds.append((events, [m for m in members if m.left == 0]))
                progressed = True
            # read out and release what the rounds that have run finished
            while rounds and all(ev.query() for ev in rounds[0][0]):
                _, finished = rounds.popleft()
                done = {id(m) for m in finished}
                for m in finished:
                    ry, rb, u, cons = m.sim.moments(dtype=np.float64)
                    nx, ny, nz = m.req.cfg["shape"]
                    res = Result(m.req.id, m.req.arrival, m.admitted, now(), nx * ny * nz, m.req.steps, cons["mass"],
                                 (ry, rb, u) if self.keep_fields else None)
                    stats.results.append(res)
                    if log:
                        log(f"request {m.req.id} done: L={nx} latency {res.latency:.3f} s")
                    m.sim.close()
                    used -= m.need
                    cells[m.lane] -= m.cells
                active = [m for m in active if id(m) not in done]
                progressed = True
            if not progressed:
                if rounds:
                    # the queue waits for memory or the next round for a slot:
                    # wait for the oldest round, unless an arrival is due first
                    if pending and not queue and pending[0].arrival - now() < 0.002:
                        time.sleep(max(pending[0].arrival - now(), 0.0))
                    else:
                        for ev in rounds[0][0]:
                            ev.synchronize()
                elif pending:
                    time.sleep(min(max(pending[0].arrival - now(), 0.0), 0.005))
        torch.cuda.synchronize(self.device)
        stats.wall = now()
        for batch in batches:
            batch.close()
        return stats


class _Member:
    """An admitted request: its simulation, the steps not yet launched, its
    device bytes, admission time, batch and cell count."""

    def __init__(self, req, sim, need, admitted, lane, cells):
        self.req = req
        self.sim = sim
        self.left = req.steps
        self.need = need
        self.admitted = admitted
        self.lane = lane
        self.cells = cells


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
