"""Online re-planning: plan requests arrive over time and are served in batches.

The paper asks the planner to be fast enough for online re-planning
(criterion (iv) of Sect. 1; re-planning is named again in Sect. 5). This module
serves a stream of plan requests on one GPU:

* a request names a site (a scene: viewpoints and obstacles) and its
  obstacle version; a site's distance matrix and swarm stay resident on the
  device between requests. A request on a resident site with unchanged
  obstacles resumes that swarm for its generations (re-planning from where
  the last plan left off); a changed obstacle rebuilds the distance matrix in
  place and restarts the swarm on it; a swarm whose trace capacity is spent
  restarts on the cached matrix; a site that is not resident is planned from
  scratch;
* requests wait in arrival order; each time the GPU is free the scheduler
  admits the waiting requests first come, first served while the device
  memory of the resident sites plus the new ones stays within a budget,
  evicting the least recently used sites that are not in the batch; a request
  whose own footprint exceeds the budget can never run and is rejected
  (status ``E_ADMIT``, decided by the library's ``dpso_request_footprint``),
  so the head of the queue always fits; a second request for a site already
  in the batch waits for the next one;
* the admitted requests run as one batch (`dpso_run_batch`); or, with
  continuous batching (`serve(..., chunk=k)`), the running requests' swarms
  advance together in rounds of at most k generations, each round one
  `dpso_run_batch` call that stops at the first request to finish; after a
  round the finished requests complete and waiting ones join, so a request
  waits for one round, not for a whole batch, before its swarm runs. A
  request's result is the same either way: a swarm run in parts equals the
  swarm run at once;
* latency is completion time minus arrival time.

The scheduler is independent of the executor, so admission, residency and
accounting are tested on the CPU with a stub executor and a fake clock.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time

import numpy as np

from . import scenes
from .dpso import E_ADMIT, OK   # status codes of the C ABI (DPSO_OK, DPSO_E_ADMIT)


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the stream
    scene: "scenes.Scene"
    params: dict            # swarm parameters; max_generations is the swarm's capacity
    key: str = ""           # site identity ("": a one-off scene, not kept resident)
    version: int = 0        # obstacle version of the site
    generations: int = 0    # generations this request runs (0: params["max_generations"])

    @property
    def n(self) -> int:
        return self.scene.n

    @property
    def run_generations(self) -> int:
        return self.generations or self.params["max_generations"]


@dataclasses.dataclass
class Record:
    rid: int
    n: int
    arrival: float
    start: float
    done: float
    cost: int
    batch: int
    status: int = OK        # OK served, E_ADMIT rejected
    action: str = ""        # plan, resume, rebuild, restart (see GpuExecutor.solve)
    generation: int = -1    # generations the swarm has completed
    tour: np.ndarray | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def poisson_requests(count, rate, seed=5, n_lo=50, n_hi=800, swarm=512, generations=300):
    """One-off plans: arrivals of a Poisson process of the given rate; request r
    has n log-uniform in [n_lo, n_hi], alternates facade and bridge scenes,
    and uses scene seed r."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for r in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        prm = scenes.swarm_params(swarm, generations, seed=0, instance=r)
        reqs.append(Request(r, float(arrivals[r]), _site_scene(r, n), prm))
    return reqs


def _site_scene(s: int, n: int) -> "scenes.Scene":
    if s % 2 == 0:
        h = int(round(math.sqrt(0.9e6 * n)))
        return scenes.facade(n, int(round(h * 10 / 3)), h, int(round(n / 50)), seed=s)
    return scenes.bridge(n, int(round(40_000 * n / 200)), max(1, int(round(6 * n / 200))), seed=s)


def replan_requests(count, rate, seed=5, sites=100, n_lo=50, n_hi=800, swarm=512, generations=300,
                    change_permille=200, capacity_runs=32):
    """Re-planning stream: Poisson arrivals at `rate`/s over `sites` sites.
    Site s has n log-uniform in [n_lo, n_hi] (drawn first, in site order) and
    alternates facade and bridge scenes with scene seed s. Request r picks a
    site uniformly; on a site seen before, with probability
    change_permille / 1000 one of its obstacles has moved since (a new
    obstacle version, `scenes.moved_box`). Every request runs `generations`
    generations; a swarm holds `capacity_runs` such runs before it restarts."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    arrivals = np.cumsum(gaps) - gaps[0]
    site_n = [int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))))) for _ in range(sites)]
    base, version, seen, current = {}, [0] * sites, set(), {}
    reqs = []
    for r in range(count):
        s = int(rng.integers(sites))
        if s in seen and int(rng.integers(1000)) < change_permille:
            version[s] += 1
        seen.add(s)
        if s not in base:
            base[s] = _site_scene(s, site_n[s])
            current[s] = (0, base[s])
        if current[s][0] != version[s]:
            current[s] = (version[s], scenes.moved_box(base[s], seed=1_000_003 * s + version[s]))
        prm = scenes.swarm_params(swarm, generations * capacity_runs, seed=0, instance=s)
        reqs.append(Request(r, float(arrivals[r]), current[s][1], prm, key=f"site{s}",
                            version=version[s], generations=generations))
    return reqs


class Scheduler:
    """First come, first served admission under a device-memory budget, with
    resident sites evicted least recently used first.

    footprint(req) -> (status, bytes): the bytes a request holds while
    resident, and E_ADMIT if they exceed the whole budget (such requests go to
    `rejected`). Evicted site keys collect in `evicted` for the executor."""

    def __init__(self, budget_bytes: int, footprint, max_batch: int = 1024):
        self.budget = int(budget_bytes)
        self.footprint = footprint
        self.max_batch = int(max_batch)
        self.rejected, self.evicted = [], []
        self.resident = collections.OrderedDict()   # site key -> bytes, least recent first
        self.n_evicted = 0

    def resident_bytes(self) -> int:
        return sum(self.resident.values())

    def admit(self, queue: collections.deque, busy=frozenset(), held: int = 0) -> list:
        """Admits from the head of the queue. `busy`: site keys whose swarm is
        running (never evicted; a request for one waits); `held`: bytes of
        running one-off scenes."""
        batch, keys, new = [], set(busy), held
        while queue and len(batch) < self.max_batch:
            req = queue[0]
            status, need = self.footprint(req)
            if status == E_ADMIT:
                self.rejected.append(queue.popleft())
                continue
            if req.key and req.key in keys:
                break                        # its swarm runs in this batch (or is running) already
            cost = 0 if req.key and req.key in self.resident else need
            while self.resident_bytes() + new + cost > self.budget:
                victim = next((k for k in self.resident if k not in keys), None)
                if victim is None:
                    break
                del self.resident[victim]
                self.evicted.append(victim)
                self.n_evicted += 1
            if self.resident_bytes() + new + cost > self.budget:
                break
            batch.append(queue.popleft())
            if req.key:                      # resident from now on, most recently used
                keys.add(req.key)
                self.resident[req.key] = self.resident.pop(req.key, need)
            else:                            # a one-off scene holds memory while it runs
                new += need
        return batch


def serve(requests, executor, scheduler: Scheduler, clock=time.perf_counter, sleep=time.sleep,
          chunk: int = 0):
    """Serves `requests` (sorted by arrival) in real time; returns Records.

    executor.solve(batch) returns one dict per request with "cost" and
    optionally "action", "generation" and "tour"; executor.evict(keys), if
    present, releases the sites the scheduler evicted. With chunk > 0 the
    requests are served by continuous batching (executor.start / step /
    finish, see `serve_continuous`)."""
    if chunk > 0:
        return serve_continuous(requests, executor, scheduler, chunk, clock, sleep)
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
            records.append(Record(req.rid, req.n, req.arrival, now, now, -1, -1, E_ADMIT, "rejected"))
        scheduler.rejected.clear()
        if scheduler.evicted:
            if hasattr(executor, "evict"):
                executor.evict(list(scheduler.evicted))
            scheduler.evicted.clear()
        if not batch:
            continue
        start = clock() - t0
        results = executor.solve(batch)
        done = clock() - t0
        for req, res in zip(batch, results):
            records.append(Record(req.rid, req.n, req.arrival, start, done, int(res["cost"]), nbatch,
                                  OK, res.get("action", ""), int(res.get("generation", -1)),
                                  res.get("tour")))
        nbatch += 1
    return records


def serve_continuous(requests, executor, scheduler: Scheduler, chunk: int, clock=time.perf_counter,
                     sleep=time.sleep):
    """Continuous batching. The running requests' swarms advance together,
    each round min(chunk, fewest generations any running request still
    needs) generations in one executor.step call; then the requests whose
    generations are done complete (executor.finish) and the scheduler admits
    waiting ones (executor.start), which join the next round. A record's
    `batch` is the round its request joined in.

    executor.start(batch) prepares the requests' swarms and returns one
    handle each; executor.step(handles, g) runs g generations of all of them;
    executor.finish(handle) returns the dict executor.solve would."""
    pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
    queue = collections.deque()
    running = []             # [request, handle, generations left, start, round joined]
    records, rounds = [], 0
    t0 = clock()
    while pending or queue or running:
        now = clock() - t0
        while pending and pending[0].arrival <= now:
            queue.append(pending.popleft())
        if not queue and not running:
            sleep(max(0.0, pending[0].arrival - now))
            continue
        if queue:
            busy = {r[0].key for r in running if r[0].key}
            held = sum(scheduler.footprint(r[0])[1] for r in running if not r[0].key)
            batch = scheduler.admit(queue, busy=busy, held=held)
            for req in scheduler.rejected:
                now = clock() - t0
                records.append(Record(req.rid, req.n, req.arrival, now, now, -1, -1, E_ADMIT, "rejected"))
            scheduler.rejected.clear()
            if scheduler.evicted:
                if hasattr(executor, "evict"):
                    executor.evict(list(scheduler.evicted))
                scheduler.evicted.clear()
            if batch:
                start = clock() - t0
                for req, h in zip(batch, executor.start(batch)):
                    running.append([req, h, req.run_generations, start, rounds])
        if not running:
            continue
        g = min(int(chunk), min(r[2] for r in running))
        executor.step([r[1] for r in running], g)
        rounds += 1
        left = []
        finished = []
        for r in running:
            r[2] -= g
            (finished if r[2] <= 0 else left).append(r)
        results = [executor.finish(r[1]) for r in finished]
        done = clock() - t0
        for (req, _, _, start, joined), res in zip(finished, results):
            records.append(Record(req.rid, req.n, req.arrival, start, done, int(res["cost"]), joined,
                                  OK, res.get("action", ""), int(res.get("generation", -1)),
                                  res.get("tour")))
        running = left
    return records


def summary(records, warmup: int = 0, scheduler: Scheduler | None = None) -> dict:
    """Latency percentiles, throughput and residency over the served requests
    after `warmup` (rejected requests are counted, not timed)."""
    after = sorted(records, key=lambda r: r.rid)[warmup:]
    rs = [r for r in after if r.status == OK]
    if not rs:
        return {"requests": 0, "rejected": len(after)}
    lat = np.array([r.latency for r in rs])
    span = max(r.done for r in rs) - min(r.arrival for r in rs)
    acts = collections.Counter(r.action for r in rs)
    out = {"requests": len(rs), "p50_ms": float(np.percentile(lat, 50) * 1e3),
           "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
           "max_ms": float(lat.max() * 1e3), "solves_per_s": len(rs) / span if span > 0 else 0.0,
           "batches": len({r.batch for r in rs}), "rejected": len(after) - len(rs),
           "mean_batch": len(rs) / max(1, len({r.batch for r in rs})),
           "actions": dict(sorted(acts.items())),
           # the swarm resumed from device memory / the distance matrix reused
           "state_hit_rate": acts["resume"] / len(rs),
           "dist_hit_rate": (acts["resume"] + acts["restart"]) / len(rs)}
    if scheduler is not None:
        out["evictions"] = scheduler.n_evicted
    return out


@dataclasses.dataclass
class _Site:
    version: int
    D: object               # device int32 [n][n]
    state: object           # device swarm state
    params: dict
    t: int = 0              # generations completed


class GpuExecutor:
    """Runs admitted batches with the batched C ABI (or, with `single`, each
    request on the plain single-instance path: dpso_init_nn, dpso_run). Sites
    keep their distance matrix and swarm state in device memory until
    evicted; distance matrices are built with the builder's static workspace
    (no allocation)."""

    def __init__(self, budget_bytes: int, stream=None, single: bool = False):
        import torch
        from . import dpso
        self.dpso, self.torch = dpso, torch
        self.budget = int(budget_bytes)
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.sites = {}
        self.work = None
        self.single = bool(single)

    def footprint(self, req: Request):
        return self.dpso.request_footprint(req.n, req.params, self.budget)

    def evict(self, keys):
        for k in keys:
            self.sites.pop(k, None)

    def _work(self, count):
        need = self.dpso.batch_work_bytes(count)
        if self.work is None or self.work.numel() < need:
            self.work = self.torch.empty(max(need, 1 << 16), dtype=self.torch.uint8, device="cuda")
        return self.work

    def _prepare(self, batch):
        """Each request's site and action: "plan" (site not resident: build the
        matrix, start a swarm), "rebuild" (obstacles changed: rebuild the matrix
        in place, restart the swarm), "restart" (the swarm's capacity is spent:
        restart it on the cached matrix), "resume" (run the resident swarm
        further). Returns (sites, actions, sites to initialise)."""
        d, torch = self.dpso, self.torch
        sites, actions, cold = [], [], []
        for req in batch:
            G = req.run_generations
            site = self.sites.get(req.key) if req.key else None
            if site is None:
                D = torch.empty((req.n, req.n), dtype=torch.int32, device="cuda")
                d.build_dist_noalloc(req.scene, out=D, stream=self.stream)
                site = _Site(req.version, D, d.new_state(req.n, req.params), dict(req.params))
                if req.key:
                    self.sites[req.key] = site
                act = "plan"
            elif site.version != req.version:
                d.build_dist_noalloc(req.scene, out=site.D, stream=self.stream)
                site.version = req.version
                act = "rebuild"
            elif site.t + G > site.params["max_generations"]:
                act = "restart"
            else:
                act = "resume"
            if act != "resume":
                cold.append(site)
                site.t = 0
            site.t += G
            sites.append(site)
            actions.append(act)
        return sites, actions, cold

    def _init(self, cold):
        if cold:
            self.dpso.Batch([(s.D, s.params) for s in cold], stream=self.stream,
                            states=[s.state for s in cold], work=self._work(len(cold))).init()

    def _result(self, site, act):
        tour, cost, gen, _ = self.dpso.get_best(site.state, self.stream)
        return {"cost": cost, "action": act, "generation": gen, "tour": tour}

    def start(self, batch):
        """Continuous batching: prepares the requests' swarms (as solve does)
        and returns one handle per request."""
        sites, actions, cold = self._prepare(batch)
        self._init(cold)
        return list(zip(sites, actions))

    def step(self, handles, generations):
        """Runs `generations` generations of the handles' swarms as one batch."""
        self.dpso.Batch([(s.D, s.params) for s, _ in handles], stream=self.stream,
                        states=[s.state for s, _ in handles], work=self._work(len(handles))).run(generations)

    def finish(self, handle):
        return self._result(*handle)

    def solve(self, batch):
        """Runs the batch's requests to completion (actions: see _prepare)."""
        d = self.dpso
        sites, actions, cold = self._prepare(batch)
        if self.single:
            for site, act, req in zip(sites, actions, batch):
                if act != "resume":
                    d.init_nn(site.D, site.params, site.state, stream=self.stream)
                d.run(site.D, site.params, site.state, req.run_generations, stream=self.stream)
        else:
            self._init(cold)
        for G in sorted({r.run_generations for r in batch}) if not self.single else ():
            group = [s for s, r in zip(sites, batch) if r.run_generations == G]
            d.Batch([(s.D, s.params) for s in group], stream=self.stream,
                    states=[s.state for s in group], work=self._work(len(group))).run(G)
        return [self._result(site, act) for site, act in zip(sites, actions)]
