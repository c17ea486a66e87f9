"""Scheduler and latency accounting of the re-planning server, on the CPU
with a stub executor and a fake clock (no GPU)."""
import collections

import numpy as np

from paper_1706_04399_amd import scenes, serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class StubExecutor:
    """Takes `per_request` seconds of fake time per request of a batch (plus
    `overhead`), returns n as the cost, and records the batches it saw."""

    def __init__(self, clock, per_request=0.01, overhead=0.005):
        self.clock, self.per, self.over = clock, per_request, overhead
        self.batches = []

    def solve(self, batch):
        self.batches.append([r.rid for r in batch])
        self.clock.t += self.over + self.per * len(batch)
        return [{"cost": r.n} for r in batch]


def _reqs(arrivals, n=10, keys=None):
    sc = scenes.line(list(range(n)))
    keys = keys or [""] * len(arrivals)
    return [serve.Request(i, a, sc, scenes.swarm_params(4, 3), key=k)
            for i, (a, k) in enumerate(zip(arrivals, keys))]


def fp(budget, size):
    """A footprint function as the executor's: (E_ADMIT if above the budget, bytes)."""
    def f(r):
        b = size(r) if callable(size) else size
        return (serve.E_ADMIT if b > budget else serve.OK), b
    return f


def test_admission_respects_budget_and_order():
    sched = serve.Scheduler(budget_bytes=250, footprint=fp(250, 100), max_batch=10)
    q = collections.deque(_reqs([0.0] * 5))
    assert [r.rid for r in sched.admit(q)] == [0, 1]
    assert [r.rid for r in sched.admit(q)] == [2, 3]
    assert [r.rid for r in sched.admit(q)] == [4]
    big = serve.Scheduler(budget_bytes=50, footprint=fp(50, 100))
    q = collections.deque(_reqs([0.0] * 2))
    assert big.admit(q) == [] and not q                  # can never fit: rejected
    assert [r.rid for r in big.rejected] == [0, 1]
    mixed = serve.Scheduler(budget_bytes=150, footprint=fp(150, lambda r: 200 if r.rid == 1 else 100))
    q = collections.deque(_reqs([0.0] * 4))
    assert [r.rid for r in mixed.admit(q)] == [0]        # 1 rejected, 2 does not fit beside 0
    assert [r.rid for r in mixed.rejected] == [1]
    assert [r.rid for r in mixed.admit(q)] == [2]
    capped = serve.Scheduler(budget_bytes=10 ** 9, footprint=fp(10 ** 9, 1), max_batch=3)
    q = collections.deque(_reqs([0.0] * 7))
    assert [len(capped.admit(q)) for _ in range(3)] == [3, 3, 1]


def test_serve_batches_waiting_requests_and_accounts_latency():
    clock = FakeClock()
    ex = StubExecutor(clock, per_request=0.01, overhead=0.005)
    sched = serve.Scheduler(budget_bytes=10 ** 9, footprint=fp(10 ** 9, 1))
    reqs = _reqs([0.0, 0.001, 0.002, 0.5, 0.5001])
    recs = serve.serve(reqs, ex, sched, clock=clock, sleep=clock.sleep)
    # request 0 runs alone; 1 and 2 arrived meanwhile and run together; the
    # late pair waits for its own arrival
    assert ex.batches == [[0], [1, 2], [3], [4]] or ex.batches == [[0], [1, 2], [3, 4]]
    by = {r.rid: r for r in recs}
    assert abs(by[0].done - 0.015) < 1e-9 and abs(by[0].latency - 0.015) < 1e-9
    assert abs(by[1].start - 0.015) < 1e-9 and abs(by[2].done - (0.015 + 0.025)) < 1e-9
    assert all(r.cost == 10 for r in recs)
    assert all(r.done >= r.start >= r.arrival for r in recs)


def test_summary_percentiles_and_warmup():
    recs = [serve.Record(i, 5, 0.0, 0.0, (i + 1) * 0.001, 0, i) for i in range(100)]
    s = serve.summary(recs, warmup=10)
    lat = np.arange(11, 101) * 0.001
    assert s["requests"] == 90
    assert abs(s["p50_ms"] - np.percentile(lat, 50) * 1e3) < 1e-9
    assert abs(s["p99_ms"] - np.percentile(lat, 99) * 1e3) < 1e-9
    assert s["batches"] == 90


def test_poisson_requests_shape():
    reqs = serve.poisson_requests(40, rate=50.0, seed=5, n_lo=50, n_hi=800)
    arr = np.array([r.arrival for r in reqs])
    assert arr[0] == 0.0 and (np.diff(arr) >= 0).all()
    assert all(50 <= r.n <= 800 for r in reqs)
    assert 0.2 < arr[-1] < 2.0                    # about 40 / 50 s
    assert {r.key for r in reqs} == {""}            # one-off scenes, never resident


def test_resident_sites_cost_nothing_and_evict_least_recent_first():
    sched = serve.Scheduler(budget_bytes=300, footprint=fp(300, 100))
    q = collections.deque(_reqs([0.0] * 3, keys=["a", "b", "c"]))
    assert [r.rid for r in sched.admit(q)] == [0, 1, 2]
    assert list(sched.resident) == ["a", "b", "c"] and sched.resident_bytes() == 300
    # a re-plan of a resident site needs no memory; "a" becomes most recent
    q = collections.deque(_reqs([0.0], keys=["a"]))
    assert [r.rid for r in sched.admit(q)] == [0] and not sched.evicted
    assert list(sched.resident) == ["b", "c", "a"]
    # a new site evicts the least recently used one that is not in the batch
    q = collections.deque(_reqs([0.0, 0.0], keys=["b", "d"]))
    assert [r.rid for r in sched.admit(q)] == [0, 1]
    assert sched.evicted == ["c"] and list(sched.resident) == ["a", "b", "d"]
    assert sched.n_evicted == 1


def test_second_request_for_a_site_waits_for_the_next_batch():
    sched = serve.Scheduler(budget_bytes=10 ** 6, footprint=fp(10 ** 6, 10))
    q = collections.deque(_reqs([0.0] * 4, keys=["a", "b", "a", "c"]))
    assert [r.rid for r in sched.admit(q)] == [0, 1]     # FCFS: stops at the second "a"
    assert [r.rid for r in sched.admit(q)] == [2, 3]


def test_sites_in_the_batch_are_never_evicted():
    sched = serve.Scheduler(budget_bytes=200, footprint=fp(200, 100))
    q = collections.deque(_reqs([0.0] * 3, keys=["a", "b", "c"]))
    assert [r.rid for r in sched.admit(q)] == [0, 1]     # "c" must wait: a and b are running
    assert not sched.evicted
    assert [r.rid for r in sched.admit(q)] == [2] and sched.evicted == ["a"]


def test_replan_requests_shape():
    reqs = serve.replan_requests(300, rate=50.0, seed=5, sites=20, n_lo=20, n_hi=60, swarm=8,
                                 generations=10, change_permille=300, capacity_runs=4)
    arr = np.array([r.arrival for r in reqs])
    assert arr[0] == 0.0 and (np.diff(arr) >= 0).all()
    by_site = {}
    for r in reqs:
        by_site.setdefault(r.key, []).append(r)
        assert r.generations == 10 and r.params["max_generations"] == 40
    assert len(by_site) == 20
    changes = 0
    for key, rs in by_site.items():
        assert len({r.n for r in rs}) == 1 and all(20 <= r.n <= 60 for r in rs)
        assert rs[0].version == 0
        for a, b in zip(rs, rs[1:]):
            assert b.version in (a.version, a.version + 1)
            same = np.array_equal(a.scene.boxes_mm, b.scene.boxes_mm)
            assert same or b.version != a.version          # obstacles change only with a new version
            assert np.array_equal(a.scene.vp_mm, b.scene.vp_mm)
            changes += b.version != a.version
    assert 0.2 < changes / (len(reqs) - 20) < 0.4


def test_moved_box_keeps_viewpoints_outside_and_moves_one_box():
    sc = scenes.facade(60, 20_000, 6_000, 4, seed=3)
    for seed in range(12):
        mv = scenes.moved_box(sc, seed)
        diff = (mv.boxes_mm != sc.boxes_mm).any(axis=1)
        assert diff.sum() <= 1 and np.array_equal(mv.vp_mm, sc.vp_mm)
        for p in mv.vp_mm:
            for b in mv.boxes_mm:
                c = mv.clearance_mm
                assert not all(b[a] - c < p[a] < b[a + 3] + c for a in range(3))


def test_rejected_requests_are_recorded_not_timed():
    clock = FakeClock()
    ex = StubExecutor(clock)
    sched = serve.Scheduler(budget_bytes=100, footprint=fp(100, lambda r: 1000 if r.rid % 2 else 10))
    recs = serve.serve(_reqs([0.0, 0.0, 0.1, 0.2]), ex, sched, clock=clock, sleep=clock.sleep)
    by = {r.rid: r for r in recs}
    assert by[1].status == serve.E_ADMIT and by[3].status == serve.E_ADMIT
    assert by[0].status == 0 and by[2].status == 0
    assert all(rid in (0, 2) for b in ex.batches for rid in b)
    s = serve.summary(recs)
    assert s["requests"] == 2 and s["rejected"] == 2


class RoundStub:
    """Continuous-batching executor: a round of g generations takes
    `per_gen` * g seconds of fake time; records (rids, g) per round and the
    generations each request ran."""

    def __init__(self, clock, per_gen=0.001):
        self.clock, self.per = clock, per_gen
        self.rounds, self.ran = [], collections.Counter()

    def start(self, batch):
        return [(r.rid, r.n) for r in batch]

    def step(self, handles, g):
        self.rounds.append(([rid for rid, _ in handles], g))
        for rid, _ in handles:
            self.ran[rid] += g
        self.clock.t += self.per * g

    def finish(self, handle):
        return {"cost": handle[1]}


def _gen_reqs(arrivals, gens, keys=None):
    sc = scenes.line(list(range(10)))
    keys = keys or [""] * len(arrivals)
    return [serve.Request(i, a, sc, scenes.swarm_params(4, 64), key=k, generations=g)
            for i, (a, g, k) in enumerate(zip(arrivals, gens, keys))]


def test_continuous_batching_joins_requests_between_rounds():
    clock = FakeClock()
    ex = RoundStub(clock, per_gen=0.001)
    sched = serve.Scheduler(budget_bytes=10 ** 9, footprint=fp(10 ** 9, 1))
    recs = serve.serve(_gen_reqs([0.0, 0.0015], [10, 10]), ex, sched, clock=clock, sleep=clock.sleep, chunk=4)
    # request 1 arrives during the first round and joins the second; rounds
    # stop at the first request to finish
    assert ex.rounds == [([0], 4), ([0, 1], 4), ([0, 1], 2), ([1], 4)]
    assert dict(ex.ran) == {0: 10, 1: 10}
    by = {r.rid: r for r in recs}
    assert abs(by[0].start - 0.0) < 1e-12 and abs(by[0].done - 0.010) < 1e-12
    assert abs(by[1].start - 0.004) < 1e-12 and abs(by[1].done - 0.014) < 1e-12
    assert (by[0].batch, by[1].batch) == (0, 1)     # the round each joined in
    assert all(r.cost == 10 for r in recs)


def test_continuous_batching_keeps_one_swarm_per_site():
    clock = FakeClock()
    ex = RoundStub(clock, per_gen=0.001)
    sched = serve.Scheduler(budget_bytes=10 ** 9, footprint=fp(10 ** 9, 1))
    reqs = _gen_reqs([0.0, 0.0, 0.0], [6, 6, 3], keys=["a", "a", "b"])
    recs = serve.serve(reqs, ex, sched, clock=clock, sleep=clock.sleep, chunk=100)
    # FCFS: the second "a" waits for the first; "b" is behind it in the queue
    assert ex.rounds == [([0], 6), ([1, 2], 3), ([1], 3)]
    by = {r.rid: r for r in recs}
    assert by[1].start >= by[0].done
    assert dict(ex.ran) == {0: 6, 1: 6, 2: 3}


def test_running_sites_are_never_evicted_and_one_offs_hold_memory():
    sched = serve.Scheduler(budget_bytes=200, footprint=fp(200, 100))
    q = collections.deque(_reqs([0.0, 0.0], keys=["a", "b"]))
    assert [r.rid for r in sched.admit(q)] == [0, 1]
    q = collections.deque(_reqs([0.0], keys=["c"]))
    assert [r.rid for r in sched.admit(q, busy={"a"})] == [0]
    assert sched.evicted == ["b"]                      # "a" is running: "b" goes
    q = collections.deque(_reqs([0.0], keys=["d"]))
    assert sched.admit(q, busy={"a", "c"}) == [] and len(q) == 1
    q = collections.deque(_reqs([0.0]))
    one_off = serve.Scheduler(budget_bytes=200, footprint=fp(200, 100))
    assert one_off.admit(q, held=150) == [] and len(q) == 1
