"""Online re-planning: solves arrive over time and are served in batches.

The paper asks the planner to be fast enough for online re-planning
(criterion (iv) of Sect. 1; re-planning is named again in Sect. 5). This module
serves a stream of plan requests on one GPU:

* requests wait in arrival order; each time the GPU is free the scheduler
  admits the waiting requests first come, first served, while the device
  footprint of the batch (swarm state + distance matrix + distance-builder
  workspace) stays within a budget; a request whose footprint alone exceeds
  the budget can never run and is rejected (status ``E_ADMIT``), so the head
  of the queue always fits and every admission round admits at least one;
* the admitted requests run as one batch (`dpso_run_batch`), distance
  matrices of scenes already resident are reused (re-planning on a known
  scene skips the distance build);
* latency is completion time minus arrival time.

The scheduler is independent of the executor, so admission and accounting
are tested on the CPU with a stub executor and a fake clock.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np

from . import scenes


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the stream
    scene: "scenes.Scene"
    params: dict
    key: str = ""           # scene identity for the distance-matrix cache

    @property
    def n(self) -> int:
        return self.scene.n


E_ADMIT = -6   # rejected at admission: footprint above the whole budget


@dataclasses.dataclass
class Record:
    rid: int
    n: int
    arrival: float
    start: float
    done: float
    cost: int
    batch: int
    status: int = 0   # 0 served, E_ADMIT rejected

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def poisson_requests(count, rate, seed=5, n_lo=50, n_hi=800, swarm=512, generations=300):
    """Arrivals of a Poisson process of the given rate; request r has n
    log-uniform in [n_lo, n_hi], alternates facade and bridge scenes, and uses
    scene seed r."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for r in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        if r % 2 == 0:
            h = int(round(math.sqrt(0.9e6 * n)))
            sc = scenes.facade(n, int(round(h * 10 / 3)), h, int(round(n / 50)), seed=r)
        else:
            sc = scenes.bridge(n, int(round(40_000 * n / 200)), max(1, int(round(6 * n / 200))), seed=r)
        prm = scenes.swarm_params(swarm, generations, seed=0, instance=r)
        reqs.append(Request(r, float(arrivals[r]), sc, prm, key=f"scene{r}"))
    return reqs


class Scheduler:
    """First come, first served admission under a device-memory budget.
    Requests that exceed the budget on their own are moved to `rejected`."""

    def __init__(self, budget_bytes: int, footprint, max_batch: int = 1024):
        self.budget = int(budget_bytes)
        self.footprint = footprint
        self.max_batch = int(max_batch)
        self.rejected = []

    def admit(self, queue: collections.deque) -> list:
        batch, used = [], 0
        while queue and len(batch) < self.max_batch:
            need = self.footprint(queue[0])
            if need > self.budget:
                self.rejected.append(queue.popleft())
                continue
            if used + need > self.budget:
                break
            batch.append(queue.popleft())
            used += need
        return batch


def serve(requests, executor, scheduler: Scheduler, clock=time.perf_counter, sleep=time.sleep):
    """Serves `requests` (sorted by arrival) in real time; returns Records."""
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    queue = collections.deque()
    records, nbatch = [], 0
    t0 = clock()
    while pending or queue:
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            queue.append(pending.popleft())
        if not queue:
            sleep(max(0.0, pending[0].arrival - now))
            continue
        batch = scheduler.admit(queue)
        for req in scheduler.rejected:
            now = clock() - t0
            records.append(Record(req.rid, req.n, req.arrival, now, now, -1, -1, E_ADMIT))
        scheduler.rejected.clear()
        if not batch:
            continue
        start = clock() - t0
        costs = executor.solve(batch)
        done = clock() - t0
        for req, cost in zip(batch, costs):
            records.append(Record(req.rid, req.n, req.arrival, start, done, int(cost), nbatch))
        nbatch += 1
    return records


def summary(records, warmup: int = 0) -> dict:
    """Latency percentiles and throughput over the served requests after
    `warmup` (rejected requests are counted, not timed)."""
    after = sorted(records, key=lambda r: r.rid)[warmup:]
    rs = [r for r in after if r.status == 0]
    if not rs:
        return {"requests": 0, "rejected": len(after)}
    lat = np.array([r.latency for r in rs])
    span = max(r.done for r in rs) - min(r.arrival for r in rs)
    return {"requests": len(rs), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3), "solves_per_s": len(rs) / span if span > 0 else 0.0,
            "batches": len({r.batch for r in rs}), "rejected": len(after) - len(rs),
            "mean_batch": len(rs) / max(1, len({r.batch for r in rs}))}


class GpuExecutor:
    """Runs an admitted batch with the batched C ABI; keeps distance matrices
    of recent scenes resident on the device (a bounded cache)."""

    def __init__(self, stream=None, cache_scenes: int = 64):
        import torch
        from . import dpso
        self.dpso, self.torch = dpso, torch
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.cache = collections.OrderedDict()
        self.cache_scenes = cache_scenes

    def footprint(self, req: Request) -> int:
        d = self.dpso
        n, p = req.n, req.params
        return (d.state_bytes(n, p["swarm_size"], p["max_generations"]) + 4 * n * n +
                d.dist_work_bytes(n, len(req.scene.boxes_mm)))

    def _dist(self, req: Request):
        D = self.cache.get(req.key)
        if D is None:
            D = self.dpso.build_dist(req.scene, stream=self.stream)
            self.cache[req.key] = D
            while len(self.cache) > self.cache_scenes:
                self.cache.popitem(last=False)
        else:
            self.cache.move_to_end(req.key)
        return D

    def solve(self, batch):
        d = self.dpso
        Ds = [self._dist(r) for r in batch]
        b = d.Batch([(D, r.params) for D, r in zip(Ds, batch)], stream=self.stream)
        # each swarm stops at its own max_generations
        b.init().run(max(r.params["max_generations"] for r in batch))
        return [d.get_best(st, self.stream)[1] for st in b.states]
