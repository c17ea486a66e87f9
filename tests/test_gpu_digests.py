"""The library against the oracle at the workloads' own sizes.

The oracle's end-of-run states are too slow to recompute inside a test (the
n = 1000 run evaluates about 4.1e12 exchanges), so `tests/golden/make_digests.py`
ran the oracle once and stored digests of its final states (every counter,
the global best and its trace in full, hashes of tours, personal bests,
velocities and costs). Here the library runs the same workloads from the same
seeded scenes and its exported states must give the same digests."""
import json
import os

import numpy as np
import pytest

import oracle
from paper_1706_04399_amd import scenes
from parity import digest_mismatches, library_digest, note

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _load(name):
    path = os.path.join(GOLDEN, f"digest_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} has not been written (tests/golden/make_digests.py {name})")
    with open(path) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def dp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1706_04399_amd import dpso
    dpso.lib()
    return dpso


def _dev(D):
    import torch
    return torch.from_numpy(np.ascontiguousarray(D, dtype=np.int32)).cuda()


def test_workload3_full_run_matches_oracle_digest(dp):
    """facade n = 1000, 20 boxes, swarm 4096, 2000 generations, exchange on
    every generation: the whole final swarm equals the oracle's."""
    want = _load("facade1000")
    sc, prm = scenes.workload(3)
    assert want["params"] == prm and want["n"] == sc.n
    D = oracle.build_dist(sc)
    Dg = _dev(D)
    note("facade1000: 2000 generations against the oracle digest")
    state = dp.init_nn(Dg, prm)
    dp.run(Dg, prm, state, prm["max_generations"])
    got = library_digest(dp, state, sc.n, prm["swarm_size"], full=True)
    bad = digest_mismatches(got, want["digest"])
    assert not bad, bad


def test_batch256_matches_oracle_digest(dp):
    """The batched workload (256 instances, n log-uniform in [20, 500], swarm
    256, 500 generations, exchange on stall) in one batched call on a side
    stream: every instance's final swarm equals the
    oracle's solve of that instance alone."""
    import torch
    want = _load("batch256")
    G = want["generations"]
    items, ns = [], []
    for rec in want["instances"]:
        i = rec["instance"]
        sc = scenes.batch_instance(i)
        assert sc.n == rec["n"]
        prm = scenes.swarm_params(256, G, seed=0, instance=i)
        items.append((_dev(oracle.build_dist(sc)), prm))
        ns.append(sc.n)
    stream = torch.cuda.Stream()
    note(f"batch of {len(items)} instances, {G} generations, against the oracle digests")
    b = dp.Batch(items, stream=stream).init()
    b.run(G)
    bad = []
    for rec, st, n in zip(want["instances"], b.states, ns):
        m = digest_mismatches(library_digest(dp, st, n, 256, stream), rec["digest"])
        if m:
            bad.append((rec["instance"], n, m[:3]))
    assert not bad, bad[:5]
