"""Launch configurations and the autotuner on the GPU: every entry the tuning
table can hold (threads per particle in the move, the edge exchange's row
form) gives the oracle's swarm bit for bit, single-instance and batched, and
dpso_autotune leaves the swarm as it found it."""
import numpy as np
import pytest

import oracle
from paper_1706_04399_amd import scenes
from parity import mismatches, note

pytestmark = pytest.mark.gpu

U16, I32, BLOCK, PAIR, QUAD = 1, 2, 3, 4, 5
CONFIGS = [(t, r) for t in (64, 128, 256, 512) for r in (U16, I32, BLOCK, PAIR, QUAD)]


@pytest.fixture(scope="module")
def dp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1706_04399_amd import dpso
    dpso.lib()
    yield dpso
    dpso.tuning_reset()


def _dev(D):
    import torch
    return torch.from_numpy(np.ascontiguousarray(D, dtype=np.int32)).cuda()


def _valid(n, tpb, rows):
    ns = (n + 63) // 64 * 64
    return ns <= 16 * tpb and (rows == BLOCK or (rows == I32 and n <= 1024) or
                               (rows == U16 and 8 <= n <= 1024) or (rows == PAIR and 128 < n <= 1024) or
                               (rows == QUAD and 256 < n <= 1024))


SIZES = [
    # (n, swarm, generations, overrides): every move width at EPT 1 .. 16 and
    # each row form on aligned, unaligned and padded n, mutation generations
    (9, 7, 6, dict(ee_trigger=2)),
    (30, 16, 6, {}),
    (100, 12, 5, dict(ee_trigger=2)),
    (200, 16, 5, dict(ee_trigger=2)),
    (264, 8, 4, dict(ee_trigger=2, mutation_swaps=3)),
    (517, 6, 3, dict(ee_trigger=2)),
    (1000, 6, 3, dict(ee_trigger=2)),
    (2000, 4, 2, dict(ee_trigger=2)),
]


@pytest.mark.parametrize("n,S,gens,kw", SIZES, ids=[f"n{c[0]}" for c in SIZES])
def test_every_configuration_matches_oracle(dp, n, S, gens, kw):
    sc = scenes.random_points(n, seed=n + 3, n_boxes=3)
    D = oracle.build_dist(sc)
    prm = scenes.swarm_params(S, gens, seed=41, instance=n, **kw)
    ref = oracle.new_state(D, prm)
    oracle.run(D, prm, ref, gens)
    Dg = _dev(D)
    tried = 0
    for tpb, rows in CONFIGS:
        if not _valid(n, tpb, rows):
            continue
        dp.tuning_set(n, S, {"move_threads": tpb, "exchange_rows": rows})
        # int32 rows of an n off 16 bytes resolve to 16-bit rows
        want = U16 if rows == I32 and n % 4 and 8 <= n <= 1024 else rows
        assert dp.tuning_get(n, S) == {"move_threads": tpb, "exchange_rows": want}
        note(f"tuning n={n} S={S}: {tpb} threads, rows {rows}")
        state = dp.init_nn(Dg, prm)
        dp.run(Dg, prm, state, gens)
        bad = mismatches(dp.export_state(state, n, S), ref)
        assert not bad, f"{tpb} threads, rows {rows}: {bad}"
        info = dp.get_info(state)
        assert (info["sweeps"], info["moves"], info["reshuffled"]) == (ref.n_sweeps, ref.n_moves, ref.n_reshuffled)
        tried += 1
    dp.tuning_set(n, S, None)
    assert tried == (3 if n > 1024 else 20 if n > 256 else 16 if n > 128 else 12)


def _force_everywhere(dp, tpb, rows):
    """Every bucket of the table set to (tpb, rows) where it can take it."""
    dp.tuning_reset()
    for b in range(1, 13):
        n = min(1 << b, 4096)
        for particles in (100, 500, 1000, 2000, 5000, 10000):
            for cfg in ((tpb, rows), (tpb, 0), (0, rows)):
                try:
                    dp.tuning_set(n, particles, {"move_threads": cfg[0], "exchange_rows": cfg[1]})
                    break
                except dp.DpsoError:
                    continue


BATCH = [
    (3, 5, {}), (30, 16, {}), (64, 8, dict(ee_trigger=2)), (65, 12, {}), (128, 6, dict(ee_trigger=2)),
    (200, 20, {}), (257, 7, dict(ee_trigger=2)), (515, 6, dict(ee_trigger=2)), (1000, 5, dict(ee_trigger=2)),
    (1030, 3, dict(ee_trigger=2)), (45, 10, dict(ee_neighbourhood=1, ee_trigger=2)),
    (77, 9, dict(velocity_cap=30, w=1.0, phi1=0.4, phi2=0.4)), (88, 12, dict(mutation_swaps=5)),
]


def test_batch_under_forced_tables_matches_oracle(dp):
    import torch
    gens = 5
    members, refs = [], []
    for k, (n, S, kw) in enumerate(BATCH):
        sc = scenes.random_points(n, seed=300 + k, n_boxes=2 if n > 3 else 0)
        D = oracle.build_dist(sc)
        prm = scenes.swarm_params(S, gens, seed=k, instance=k, **kw)
        ref = oracle.new_state(D, prm)
        oracle.run(D, prm, ref, gens)
        members.append((D, prm))
        refs.append(ref)
    stream = torch.cuda.Stream()
    for tpb, rows in [(64, U16), (128, I32), (256, BLOCK), (64, BLOCK), (256, PAIR), (256, QUAD)]:
        _force_everywhere(dp, tpb, rows)
        note(f"batch of {len(members)} under table ({tpb}, {rows})")
        b = dp.Batch([(_dev(D), p) for D, p in members], stream=stream).init()
        b.run(2)
        b.run(gens - 2)
        for k, ((D, prm), st, ref) in enumerate(zip(members, b.states, refs)):
            bad = mismatches(dp.export_state(st, D.shape[0], prm["swarm_size"], stream), ref)
            assert not bad, f"table ({tpb}, {rows}) instance {k} (n={D.shape[0]}): {bad}"
    dp.tuning_reset()


@pytest.mark.parametrize("n,S,kw", [(200, 64, dict(ee_trigger=2)), (30, 16, {}), (1500, 8, dict(ee_trigger=2))])
def test_autotune_leaves_swarm_and_records_pick(dp, n, S, kw):
    dp.tuning_reset()
    sc = scenes.random_points(n, seed=n, n_boxes=4)
    D = oracle.build_dist(sc)
    prm = scenes.swarm_params(S, 10, seed=3, instance=n, **kw)
    Dg = _dev(D)
    state = dp.init_nn(Dg, prm)
    dp.run(Dg, prm, state, 2)
    before = dp.export_state(state, n, S)
    note(f"autotune n={n} S={S}")
    out = dp.autotune(Dg, prm, state, 3)
    res = out["results"]
    assert len({r["digest"] for r in res}) == 1
    # 3 (or 2) move widths, then the row forms other than the default (int32
    # rows are not a separate candidate for an n off 16 bytes)
    assert len(res) == {200: 7, 30: 5, 1500: 3}[n]
    assert all(r["ms"] > 0 for r in res)
    after = dp.export_state(state, n, S)
    for k in ("X", "P", "V", "vlen", "F", "FP", "G", "trace"):
        assert np.array_equal(before[k], after[k]), k
    assert dp.tuning_get(n, S) == out["chosen"]
    # the run after it, under the pick, still equals the oracle
    dp.run(Dg, prm, state, 3)
    ref = oracle.new_state(D, prm)
    oracle.run(D, prm, ref, 5)
    bad = mismatches(dp.export_state(state, n, S), ref)
    assert not bad, bad
    dp.tuning_reset()


def test_autotune_refuses_a_run_past_max_generations(dp):
    sc = scenes.random_points(40, seed=1, n_boxes=1)
    D = oracle.build_dist(sc)
    prm = scenes.swarm_params(8, 4, seed=3, instance=1)
    Dg = _dev(D)
    state = dp.init_nn(Dg, prm)
    dp.run(Dg, prm, state, 2)
    with pytest.raises(dp.DpsoError) as e:
        dp.autotune(Dg, prm, state, 3)
    assert e.value.status == dp.E_RANGE


def test_batch_calls_in_a_row_match_oracle(dp):
    """dpso_run_batch on a side stream, called three times, with the
    program's own work and a synchronisation between calls, every call's
    states against the oracle at the same generation."""
    import torch
    members, refs = [], []
    for k, (n, S, kw) in enumerate(BATCH[:9]):
        sc = scenes.random_points(n, seed=500 + k, n_boxes=2 if n > 3 else 0)
        D = oracle.build_dist(sc)
        prm = scenes.swarm_params(S, 12, seed=k, instance=k, **kw)
        members.append((D, prm))
        refs.append(oracle.new_state(D, prm))
    dp.tuning_reset()
    stream = torch.cuda.Stream()
    b = dp.Batch([(_dev(D), p) for D, p in members], stream=stream).init()
    for call in range(3):
        note(f"batch calls in a row, call {call}")
        b.run(3)
        stream.synchronize()
        torch.zeros(1 << 20, device="cuda").sum().item()   # other work between the calls
        for k, ((D, prm), st, ref) in enumerate(zip(members, b.states, refs)):
            oracle.run(D, prm, ref, 3)
            bad = mismatches(dp.export_state(st, D.shape[0], prm["swarm_size"], stream), ref)
            assert not bad, f"call {call} instance {k} (n={D.shape[0]}): {bad}"


@pytest.mark.parametrize("order", [1, 2, 3], ids=["index", "longest_first", "xcd_groups"])
def test_batch_orders_match_oracle(dp, order):
    """Every batch order gives the oracle's swarms: a batch whose classes have
    8 or more members of equal work (24 instances of n = 50 and eight of
    n = 97), so XCD groups form and blocks past a group's end do nothing."""
    import torch
    gens = 4
    cases = [(50, 6, dict(ee_trigger=2))] * 24 + [(97, 4, dict(ee_trigger=2))] * 8
    members, refs = [], []
    for k, (n, S, kw) in enumerate(cases):
        sc = scenes.random_points(n, seed=700 + k, n_boxes=2)
        D = oracle.build_dist(sc)
        prm = scenes.swarm_params(S, gens, seed=k, instance=k, **kw)
        ref = oracle.new_state(D, prm)
        oracle.run(D, prm, ref, gens)
        members.append((D, prm))
        refs.append(ref)
    dp.tuning_reset()
    dp.batch_order_set(order)
    try:
        stream = torch.cuda.Stream()
        note(f"batch of {len(members)} instances, order {order}")
        b = dp.Batch([(_dev(D), p) for D, p in members], stream=stream).init()
        b.run(gens)
        for k, ((D, prm), st, ref) in enumerate(zip(members, b.states, refs)):
            bad = mismatches(dp.export_state(st, D.shape[0], prm["swarm_size"], stream), ref)
            assert not bad, f"order {order} instance {k} (n={D.shape[0]}): {bad}"
    finally:
        dp.batch_order_set(0)


@pytest.mark.parametrize("limit", [0, 1 << 40], ids=["classes_in_turn", "merged"])
def test_batch_merged_exchange_matches_oracle(dp, limit):
    """The 16-bit row classes of a batch (n = 9 ... 1001, n not a multiple of
    4 so that small n stage 16-bit rows too) launched one after another and
    merged into one launch, beside classes that never merge (int32 rows,
    node-swap, row-per-workgroup): every swarm equals the oracle's."""
    import torch
    gens = 4
    ee = dict(ee_trigger=2)
    cases = [(9, 8, ee), (50, 16, ee), (62, 8, ee), (70, 12, ee), (130, 8, ee), (255, 6, ee),
             (301, 6, ee), (509, 4, ee), (601, 4, ee), (1001, 3, ee), (40, 8, ee), (5, 8, ee),
             (33, 4, dict(ee_trigger=2, ee_neighbourhood=1)), (1030, 2, ee), (257, 4, {})]
    members, refs = [], []
    for k, (n, S, kw) in enumerate(cases):
        sc = scenes.random_points(n, seed=900 + k, n_boxes=2 if n > 3 else 0)
        D = oracle.build_dist(sc)
        prm = scenes.swarm_params(S, gens, seed=k, instance=k, **kw)
        ref = oracle.new_state(D, prm)
        oracle.run(D, prm, ref, gens)
        members.append((D, prm))
        refs.append(ref)
    dp.tuning_reset()
    dp.batch_merge_set(limit)
    try:
        stream = torch.cuda.Stream()
        note(f"batch of {len(members)} instances, merge limit {limit}")
        b = dp.Batch([(_dev(D), p) for D, p in members], stream=stream).init()
        b.run(gens)
        for k, ((D, prm), st, ref) in enumerate(zip(members, b.states, refs)):
            bad = mismatches(dp.export_state(st, D.shape[0], prm["swarm_size"], stream), ref)
            assert not bad, f"merge limit {limit} instance {k} (n={D.shape[0]}): {bad}"
    finally:
        dp.batch_merge_set(-1)

