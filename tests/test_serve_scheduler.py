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
        return [r.n for r in batch]


def _reqs(arrivals, n=10):
    sc = scenes.line(list(range(n)))
    return [serve.Request(i, a, sc, scenes.swarm_params(4, 3)) for i, a in enumerate(arrivals)]


def test_admission_respects_budget_and_order():
    sched = serve.Scheduler(budget_bytes=250, footprint=lambda r: 100, max_batch=10)
    q = collections.deque(_reqs([0.0] * 5))
    assert [r.rid for r in sched.admit(q)] == [0, 1]
    assert [r.rid for r in sched.admit(q)] == [2, 3]
    assert [r.rid for r in sched.admit(q)] == [4]
    big = serve.Scheduler(budget_bytes=50, footprint=lambda r: 100)
    q = collections.deque(_reqs([0.0] * 2))
    assert big.admit(q) == [] and not q                  # can never fit: rejected
    assert [r.rid for r in big.rejected] == [0, 1]
    mixed = serve.Scheduler(budget_bytes=150, footprint=lambda r: 200 if r.rid == 1 else 100)
    q = collections.deque(_reqs([0.0] * 4))
    assert [r.rid for r in mixed.admit(q)] == [0]        # 1 rejected, 2 does not fit beside 0
    assert [r.rid for r in mixed.rejected] == [1]
    assert [r.rid for r in mixed.admit(q)] == [2]
    capped = serve.Scheduler(budget_bytes=10 ** 9, footprint=lambda r: 1, max_batch=3)
    q = collections.deque(_reqs([0.0] * 7))
    assert [len(capped.admit(q)) for _ in range(3)] == [3, 3, 1]


def test_serve_batches_waiting_requests_and_accounts_latency():
    clock = FakeClock()
    ex = StubExecutor(clock, per_request=0.01, overhead=0.005)
    sched = serve.Scheduler(budget_bytes=10 ** 9, footprint=lambda r: 1)
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
    assert len({r.key for r in reqs}) == 40


def test_rejected_requests_are_recorded_not_timed():
    clock = FakeClock()
    ex = StubExecutor(clock)
    sched = serve.Scheduler(budget_bytes=100, footprint=lambda r: 1000 if r.rid % 2 else 10)
    recs = serve.serve(_reqs([0.0, 0.0, 0.1, 0.2]), ex, sched, clock=clock, sleep=clock.sleep)
    by = {r.rid: r for r in recs}
    assert by[1].status == serve.E_ADMIT and by[3].status == serve.E_ADMIT
    assert by[0].status == 0 and by[2].status == 0
    assert all(rid in (0, 2) for b in ex.batches for rid in b)
    s = serve.summary(recs)
    assert s["requests"] == 2 and s["rejected"] == 2
