"""Parity of the HIP library with the CPU oracle (bit-exact: all integer).

Each test feeds both sides the same seeded inputs and compares the whole
swarm state (tours, personal bests, velocities, costs, global best, trace,
counters of generations) element by element.
"""
import numpy as np
import pytest

import oracle
from paper_1706_04399_amd import scenes
from parity import as_host, mismatches, note, synthetic_state

pytestmark = pytest.mark.gpu


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


def _golden_detour_scene():
    from conftest import golden_lines
    rows = golden_lines("box_detour.txt")
    vp = [[int(v) for v in r[1:]] for r in rows if r[0] == "vp"]
    box = [[int(v) for v in r[1:]] for r in rows if r[0] == "box"]
    return scenes.Scene(np.array(vp), np.array(box), 500)


DIST_CASES = {
    "facade30": lambda: scenes.workload(1)[0],
    "bridge200": lambda: scenes.workload(2)[0],
    "facade1000": lambda: scenes.workload(3)[0],
    "random50_5boxes": lambda: scenes.random_points(50, seed=3, n_boxes=5),
    "random130_10boxes": lambda: scenes.random_points(130, seed=21, n_boxes=10),
    "serpentine1_long_finite": lambda: scenes.serpentine(1),
    "circle64": lambda: scenes.circle(64),
    "grid8x6": lambda: scenes.grid(8, 6),
    "detour": _golden_detour_scene,
    "single": lambda: scenes.line([7]),
    "batch_item_3": lambda: scenes.batch_instance(3),
}


@pytest.mark.parametrize("name", list(DIST_CASES))
def test_build_dist_matches_oracle(dp, name):
    sc = DIST_CASES[name]()
    note(f"build_dist {name} n={sc.n} boxes={len(sc.boxes_mm)}")
    got = dp.build_dist(sc).cpu().numpy()
    assert np.array_equal(got, oracle.build_dist(sc))


def test_build_dist_unreachable_pair(dp):
    slabs = [(-3000, -3000, -3000, -2000, 3000, 3000), (2000, -3000, -3000, 3000, 3000, 3000),
             (-3000, -3000, -3000, 3000, -2000, 3000), (-3000, 2000, -3000, 3000, 3000, 3000),
             (-3000, -3000, -3000, 3000, 3000, -2000), (-3000, -3000, 2000, 3000, 3000, 3000)]
    sc = scenes.Scene(np.array([(0, 0, 0), (10000, 0, 0), (10000, 5000, 0)]), np.array(slabs), 0)
    note("build_dist sealed viewpoint")
    got = dp.build_dist(sc).cpu().numpy()
    assert np.array_equal(got, oracle.build_dist(sc))
    assert got[0, 1] == dp.D_INF


@pytest.mark.parametrize("walls", [2, 20])
def test_build_dist_finite_path_beyond_sentinel_is_range_error(dp, walls):
    """Paths that weave through 2 or 20 walls are finite and longer than the
    blocked-pair cost (with 20 walls, longer than 2^32 mm): a range error on
    both sides, not a blocked pair."""
    sc = scenes.serpentine(walls)
    note(f"build_dist serpentine{walls}")
    with pytest.raises(ValueError, match="status -2"):
        oracle.build_dist(sc)
    with pytest.raises(dp.DpsoError) as ei:
        dp.build_dist(sc)
    assert ei.value.status == dp.E_RANGE


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 200, 1000, 4096])
def test_check_dist_matches_oracle(dp, n):
    """The device check reports the oracle's first broken entry, across tile
    edges and with breaks planted in several places."""
    note(f"check_dist n={n}")
    rng = np.random.default_rng(n)
    D = scenes.random_dist(n, seed=n)
    assert dp.check_dist(_dev(D)) == oracle.check_dist(D) == -1
    if n == 1:
        D1 = np.array([[3]], np.int32)
        assert dp.check_dist(_dev(D1)) == oracle.check_dist(D1) == 0
        return
    for trial in range(6):
        E = D.copy()
        for _ in range(int(rng.integers(1, 4))):
            i, j = (int(v) for v in rng.integers(0, n, size=2))
            kind = trial % 4
            if kind == 0:
                E[i, j] = -1 - int(rng.integers(0, 9))
            elif kind == 1:
                E[i, j] = (1 << 28) + int(rng.integers(0, 9))
            elif kind == 2:
                E[i, i] = 1 + int(rng.integers(0, 9))
            else:
                E[i, j] += 1 if i != j else 0
        assert dp.check_dist(_dev(E)) == oracle.check_dist(E), (n, trial)


def test_check_dist_on_built_matrices(dp):
    note("check_dist built matrices")
    for k in (1, 2, 3):
        D = dp.build_dist(scenes.workload(k)[0])
        assert dp.check_dist(D) == -1
    assert dp.check_dist(dp.build_dist_voxel(scenes.workload(2)[0], 500)) == -1


def lockstep(dp, D, prm, checkpoints, label):
    """Runs library and oracle from the same initial swarm, comparing the whole
    state at each checkpoint generation."""
    note(f"{label}: init n={D.shape[0]} S={prm['swarm_size']}")
    Dg = _dev(D)
    state = dp.init_nn(Dg, prm)
    ost = oracle.new_state(D, prm)
    bad = mismatches(dp.export_state(state, D.shape[0], prm["swarm_size"]), ost)
    assert not bad, f"after init: {bad}"
    done = 0
    for cp in checkpoints:
        note(f"{label}: run to generation {cp}")
        dp.run(Dg, prm, state, cp - done)
        oracle.run(D, prm, ost, cp - done)
        done = cp
        bad = mismatches(dp.export_state(state, D.shape[0], prm["swarm_size"]), ost)
        assert not bad, f"generation {cp}: {bad}"
    info = dp.get_info(state)
    assert (info["sweeps"], info["moves"], info["reshuffled"]) == \
        (ost.n_sweeps, ost.n_moves, ost.n_reshuffled)
    tour, cost, gen, trace = dp.get_best(state)
    assert np.array_equal(tour, ost.G) and cost == ost.FG and gen == ost.t
    return state, ost


def test_workload1_full_run(dp):
    sc, prm = scenes.workload(1)
    D = oracle.build_dist(sc)
    lockstep(dp, D, prm, [1, 2, 3, 4, 5, 6, 10, 50, 100, 200], "facade30")


def test_workload2_full_run(dp):
    sc, prm = scenes.workload(2)
    D = oracle.build_dist(sc)
    lockstep(dp, D, prm, [1, 2, 3, 30, 300, 1000], "bridge200")


def test_workload3_first_generations(dp):
    """The benchmark's workload and launch configuration, first generations."""
    sc, prm = scenes.workload(3)
    D = oracle.build_dist(sc)
    lockstep(dp, D, prm, [1, 3], "facade1000")


def test_workload3_late_generation_from_synthetic_state(dp):
    """One mutation generation (t = 1500) at full size from a seeded mid-run state."""
    sc, prm = scenes.workload(3)
    D = oracle.build_dist(sc)
    st = synthetic_state(D, prm, t=1499, seed=5)
    Dg = _dev(D)
    state = dp.new_state(D.shape[0], prm)
    dp.init_nn(Dg, prm, state)
    note("facade1000: import synthetic state at t=1499")
    dp.import_state(state, D.shape[0], prm["swarm_size"], as_host(st))
    dp.run(Dg, prm, state, 1)
    oracle.run(D, prm, st, 1)
    bad = mismatches(dp.export_state(state, D.shape[0], prm["swarm_size"]), st)
    assert not bad, bad


EDGE = [
    # (name, n, S, gens, overrides)
    ("n1", 1, 3, 6, {}),
    ("n2", 2, 5, 6, {}),
    ("n3", 3, 4, 6, {}),
    ("n4", 4, 7, 9, dict(ee_trigger=2)),
    ("n5_S1", 5, 1, 9, dict(ee_trigger=2)),
    ("n63", 63, 33, 12, {}),
    ("n64", 64, 64, 12, dict(ee_trigger=2, ee_max_moves=0)),
    ("n65", 65, 65, 12, dict(det_permille=1000)),
    ("n129_S257", 129, 257, 9, dict(det_permille=0, ee_trigger=2)),
    ("ee_off", 40, 50, 12, dict(ee_trigger=0)),
    ("no_mutation", 40, 50, 12, dict(mutation_period=0)),
    ("stall_limit", 20, 16, 60, dict(stall_limit=3)),
    ("w1_phi04", 50, 100, 12, dict(w=1.0, phi1=0.4, phi2=0.4)),
    ("coef_max", 50, 30, 9, dict(w=2.0, phi1=2.0, phi2=2.0)),
    # n a multiple of 4: rows staged straight into LDS, at every register-block
    # class and its edges
    ("n8_aligned", 8, 9, 9, dict(ee_trigger=2)),
    ("n68_aligned", 68, 20, 9, dict(ee_trigger=2)),
    ("n256_aligned", 256, 16, 6, dict(ee_trigger=2)),
    ("n260_aligned", 260, 16, 6, dict(ee_trigger=2)),
    ("n512_aligned", 512, 12, 5, dict(ee_trigger=2)),
    ("n516_aligned", 516, 12, 4, dict(ee_trigger=2)),
    ("n1024_aligned", 1024, 8, 3, dict(ee_trigger=2)),
]


@pytest.mark.parametrize("name,n,S,gens,kw", EDGE, ids=[e[0] for e in EDGE])
def test_edge_cases(dp, name, n, S, gens, kw):
    sc = scenes.random_points(n, seed=n + S, n_boxes=2 if n > 3 else 0)
    D = oracle.build_dist(sc)
    prm = scenes.swarm_params(S, gens, seed=17, instance=n, **kw)
    lockstep(dp, D, prm, sorted({1, 2, 3, gens // 2 or 1, gens}), name)


@pytest.mark.parametrize("n", [4096, 3001])
def test_largest_sizes(dp, n):
    """The largest supported n (and a ragged one near it): row-kernel edge
    exchange on every generation, a mutation generation, LDS at its largest."""
    D = scenes.random_dist(n, seed=n)
    prm = scenes.swarm_params(8, 3, seed=5, instance=n, ee_trigger=scenes.EE_ALWAYS,
                              det_permille=250)
    lockstep(dp, D, prm, [1, 3], f"n{n}")


def _packed_case_matrix(n, kind, seed):
    """Symmetric zero-diagonal matrices for the 16-bit row path: `kind` is the
    largest entry (the shift follows from it) or "ties" (entries 1 and 2) or
    "ties_wide" (entries 100000 or 200000 plus 0 or 1: shift 2 with ties) or
    "lowbit" / "lowbit2" (shift 1 / 2, near-ties decided by the dropped bits)."""
    if kind == "ties":
        return scenes.random_dist(n, seed=seed, max_mm=3)
    if kind == "ties_wide":
        rng = np.random.default_rng(seed)
        a = 100_000 * rng.integers(1, 3, size=(n, n)) + rng.integers(0, 2, size=(n, n))
        d = np.triu(a, 1)
        return np.ascontiguousarray(d + d.T, dtype=np.int32)
    if kind in ("lowbit", "lowbit2"):
        # shift 1 (or 2): sums of H tie often and the dropped low bits decide
        rng = np.random.default_rng(seed)
        if kind == "lowbit":
            a = 65_536 + 2 * rng.integers(0, 4, size=(n, n)) + rng.integers(0, 2, size=(n, n))
        else:
            a = 131_072 + 4 * rng.integers(0, 3, size=(n, n)) + rng.integers(0, 4, size=(n, n))
        d = np.triu(a, 1)
        return np.ascontiguousarray(d + d.T, dtype=np.int32)
    return scenes.random_dist(n, seed=seed, max_mm=kind)


PACKED = [
    # (name, n, S, gens, matrix, overrides): n above 256 or not a multiple of 4
    # stages 16-bit rows (padded to 8 entries); shifts 0, 1, 2, 4 and 12,
    # exchanges tied at the minimum in many rows (every row then evaluated
    # exactly), every register-block class, padded and unpadded rows
    ("n264_shift4", 264, 16, 4, 1 << 20, dict(ee_trigger=2)),
    ("n320_shift12_opt", 320, 8, 3, (1 << 28) - 1, dict(ee_trigger=2, ee_max_moves=0)),
    ("n264_ties_opt", 264, 8, 3, "ties", dict(ee_trigger=2, ee_max_moves=0)),
    ("n264_ties_shift2", 264, 16, 4, "ties_wide", dict(ee_trigger=2)),
    ("n512_shift1", 512, 12, 4, 100_000, dict(ee_trigger=2)),
    ("n520_shift4", 520, 12, 4, 1 << 20, dict(ee_trigger=2)),
    ("n1016_shift1", 1016, 8, 3, 100_000, dict(ee_trigger=2)),
    ("n1024_ties", 1024, 8, 2, "ties", dict(ee_trigger=2)),
    ("n400_shift0_opt", 400, 8, 3, 60_000, dict(ee_trigger=2, ee_max_moves=0)),
    ("n264_lowbit", 264, 16, 4, "lowbit", dict(ee_trigger=2)),
    ("n288_lowbit2_opt", 288, 8, 3, "lowbit2", dict(ee_trigger=2, ee_max_moves=0)),
    ("n1000_lowbit", 1000, 8, 2, "lowbit", dict(ee_trigger=2)),
    ("n9_pad_shift1", 9, 7, 6, 100_000, dict(ee_trigger=2, ee_max_moves=0)),
    ("n63_pad_ties_opt", 63, 16, 4, "ties", dict(ee_trigger=2, ee_max_moves=0)),
    ("n101_pad_lowbit", 101, 16, 4, "lowbit", dict(ee_trigger=2)),
    ("n250_pad_shift4", 250, 12, 4, 1 << 20, dict(ee_trigger=2)),
    ("n263_pad_lowbit2_opt", 263, 8, 3, "lowbit2", dict(ee_trigger=2, ee_max_moves=0)),
    ("n260_pad4_shift1", 260, 12, 4, 100_000, dict(ee_trigger=2)),
    ("n517_pad_ties", 517, 8, 3, "ties", dict(ee_trigger=2)),
    ("n1021_pad_shift12", 1021, 8, 2, (1 << 28) - 1, dict(ee_trigger=2)),
]


@pytest.mark.parametrize("name,n,S,gens,kind,kw", PACKED, ids=[c[0] for c in PACKED])
def test_packed_rows(dp, name, n, S, gens, kind, kw):
    D = _packed_case_matrix(n, kind, seed=n + 11)
    prm = scenes.swarm_params(S, gens, seed=29, instance=n, **kw)
    lockstep(dp, D, prm, sorted({1, 2, gens}), "packed_" + name)


NB = scenes.NB_NODE_SWAP
VARIANTS = [
    # (name, n, S, gens, overrides): node-swap exchange, disturbance mutation,
    # conventional DPSO
    ("swap_n2", 2, 5, 6, dict(ee_neighbourhood=NB, ee_trigger=2)),
    ("swap_n3", 3, 4, 6, dict(ee_neighbourhood=NB, ee_trigger=2)),
    ("swap_n4", 4, 7, 9, dict(ee_neighbourhood=NB, ee_trigger=2)),
    ("swap_n5_S1_opt", 5, 1, 9, dict(ee_neighbourhood=NB, ee_trigger=2, ee_max_moves=0)),
    ("swap_n40_stall", 40, 50, 12, dict(ee_neighbourhood=NB)),
    ("swap_n65_opt", 65, 33, 9, dict(ee_neighbourhood=NB, ee_trigger=2, ee_max_moves=0)),
    ("swap_n257", 257, 64, 6, dict(ee_neighbourhood=NB, ee_trigger=2)),
    ("swap_n1030", 1030, 16, 3, dict(ee_neighbourhood=NB, ee_trigger=2)),
    ("disturb_k1", 40, 50, 12, dict(mutation_swaps=1)),
    ("disturb_k7", 65, 64, 9, dict(mutation_swaps=7, ee_trigger=2)),
    ("disturb_k3000", 30, 20, 6, dict(mutation_swaps=3000)),      # several draw chunks
    ("conventional", 50, 64, 20, dict(det_permille=0, mutation_period=0, ee_trigger=0)),
    ("swap_and_disturb", 100, 64, 12, dict(ee_neighbourhood=NB, ee_trigger=2, mutation_swaps=4)),
    # velocity kept as the raw concatenation, with a cap
    ("raw_cap_n", 40, 50, 12, dict(velocity_cap=40)),
    ("raw_cap_10", 65, 33, 9, dict(velocity_cap=10, w=1.0, phi1=0.4, phi2=0.4)),
    ("raw_n1", 1, 3, 4, dict(velocity_cap=1)),
    ("raw_n1030", 1030, 16, 3, dict(velocity_cap=500, ee_trigger=2)),
    ("raw_all_variants", 100, 64, 12, dict(velocity_cap=60, ee_neighbourhood=NB, mutation_swaps=3,
                                           ee_trigger=2)),
]


@pytest.mark.parametrize("name,n,S,gens,kw", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_variants(dp, name, n, S, gens, kw):
    sc = scenes.random_points(n, seed=3 * n + S, n_boxes=2 if n > 3 else 0)
    D = oracle.build_dist(sc)
    prm = scenes.swarm_params(S, gens, seed=23, instance=n, **kw)
    lockstep(dp, D, prm, sorted({1, 2, 3, gens // 2 or 1, gens}), name)


def test_node_swap_on_a_random_matrix(dp):
    """Node-swap exchange to a local optimum on a non-metric matrix with many
    equal entries (ties between exchanges)."""
    D = scenes.random_dist(70, seed=8, max_mm=6)
    prm = scenes.swarm_params(24, 6, seed=4, ee_neighbourhood=NB, ee_trigger=2, ee_max_moves=0)
    lockstep(dp, D, prm, [1, 3, 6], "swap_ties")


@pytest.mark.parametrize("kw", [dict(ee_neighbourhood=NB, ee_trigger=2),
                                dict(velocity_cap=4096, mutation_swaps=9, ee_trigger=2)],
                         ids=["node_swap", "raw_velocity"])
def test_largest_size_variants(dp, kw):
    """The variants' kernels at n = 4096, where their LDS use is largest."""
    n = 4096
    D = scenes.random_dist(n, seed=n)
    prm = scenes.swarm_params(4, 3, seed=5, instance=n, det_permille=250, **kw)
    lockstep(dp, D, prm, [1, 3], f"n{n} {kw}")


def test_raw_velocity_import_and_mode_check(dp):
    """Arbitrary transposition lists imported into a raw-velocity state move
    the swarm exactly as in the oracle; a state is refused by a run in the
    other velocity mode."""
    n, S = 36, 20
    D = oracle.build_dist(scenes.random_points(n, seed=12, n_boxes=2))
    prm = scenes.swarm_params(S, 20, seed=6, velocity_cap=25, w=1.0)
    st = synthetic_state(D, prm, t=4, seed=31)
    rng = np.random.default_rng(5)
    st.VL[:] = rng.integers(0, 26, size=S)
    st.V[:] = rng.integers(0, n, size=st.V.shape)       # any labels, any order
    Dg = _dev(D)
    state = dp.init_nn(Dg, prm)
    dp.import_state(state, n, S, as_host(st))
    assert not mismatches(dp.export_state(state, n, S), st)
    note("raw velocity: generation 5 from an imported state")
    dp.run(Dg, prm, state, 2)
    oracle.run(D, prm, st, 2)
    bad = mismatches(dp.export_state(state, n, S), st)
    assert not bad, bad
    with pytest.raises(dp.DpsoError) as ei:
        dp.run(Dg, dict(prm, velocity_cap=0), state, 1)
        dp.get_info(state)
    assert ei.value.status == dp.E_STATE


def test_collapsed_swarm_mutation(dp):
    """All particles identical at a mutation generation: one is kept."""
    n, S = 48, 96
    D = oracle.build_dist(scenes.random_points(n, seed=2, n_boxes=3))
    prm = scenes.swarm_params(S, 10, seed=3)
    st = synthetic_state(D, prm, t=2, seed=9)
    st.X[:] = st.X[0]
    st.F[:] = st.F[0]
    st.P[:] = st.X[0]
    st.FP[:] = st.F[0]
    st.G[:] = st.X[0]
    st.FG = int(st.F[0])
    st.trace[:3] = st.FG
    st.VL[:] = 0
    Dg = _dev(D)
    state = dp.init_nn(Dg, prm)
    dp.import_state(state, n, S, as_host(st))
    note("collapsed swarm: generation 3")
    dp.run(Dg, prm, state, 1)
    oracle.run(D, prm, st, 1)
    bad = mismatches(dp.export_state(state, n, S), st)
    assert not bad, bad


def test_import_export_round_trip_and_rejection(dp):
    n, S = 40, 24
    D = oracle.build_dist(scenes.random_points(n, seed=8, n_boxes=2))
    prm = scenes.swarm_params(S, 20, seed=4)
    st = synthetic_state(D, prm, t=5, seed=21)
    Dg = _dev(D)
    state = dp.init_nn(Dg, prm)
    note("import / export round trip")
    dp.import_state(state, n, S, as_host(st))
    assert not mismatches(dp.export_state(state, n, S), st)
    bad = as_host(st)
    bad["V"][2, :2] = [[5, 7], [7, 9]]      # moves label 7 again after placing it: not canonical
    bad["vlen"][2] = 2
    with pytest.raises(dp.DpsoError) as ei:
        dp.import_state(state, n, S, bad)
    assert ei.value.status == dp.E_INVAL
    bad = as_host(st)
    bad["X"][3, [0, 1]] = bad["X"][3, 0]             # not a permutation
    with pytest.raises(dp.DpsoError):
        dp.import_state(state, n, S, bad)


def test_split_run_equals_single_run(dp):
    sc, prm = scenes.workload(1)
    D = oracle.build_dist(sc)
    Dg = _dev(D)
    a = dp.init_nn(Dg, prm)
    dp.run(Dg, prm, a, 37)
    b = dp.init_nn(Dg, prm)
    dp.run(Dg, prm, b, 20)
    dp.run(Dg, prm, b, 17)
    ea, eb = dp.export_state(a, sc.n, 64), dp.export_state(b, sc.n, 64)
    for k in ea:
        if k != "V":
            assert np.array_equal(np.asarray(ea[k]), np.asarray(eb[k])), k
    for p in range(64):      # slots past a velocity's length are unused
        L = ea["vlen"][p]
        assert np.array_equal(ea["V"][p, :L], eb["V"][p, :L]), p


@pytest.mark.parametrize("trigger", [0, 1, 2])
def test_timed_and_profiled_runs_equal_plain_runs(dp, trigger):
    """The two timing entry points leave the same state as dpso_run, and count
    one exchange launch a generation when the exchange is on."""
    sc, prm = scenes.workload(1)
    prm = dict(prm, ee_trigger=trigger)
    note(f"timed runs, trigger {trigger}")
    Dg = _dev(oracle.build_dist(sc))
    states = []
    for how in ("plain", "timed", "profiled"):
        st = dp.init_nn(Dg, prm)
        if how == "plain":
            dp.run(Dg, prm, st, 25)
        elif how == "timed":
            t = dp.run_timed(Dg, prm, st, 25)
            assert t["exchange_launches"] == (25 if trigger else 0) and t["generations"] == 25
            assert (t["ms_exchange"] > 0) == (trigger != 0) and t["ms_move"] == 0
        else:
            t = dp.run_profiled(Dg, prm, st, 25)
            assert t["ms_move"] > 0 and t["generations"] == 25
        states.append(dp.export_state(st, sc.n, prm["swarm_size"]))
    for other in states[1:]:
        for k in ("X", "P", "F", "FP", "G", "vlen", "trace"):
            assert np.array_equal(np.asarray(states[0][k]), np.asarray(other[k])), k


def test_state_mismatch_is_reported(dp):
    sc, prm = scenes.workload(1)
    D = oracle.build_dist(sc)
    Dg = _dev(D)
    state = dp.init_nn(Dg, prm)
    other = dict(prm, swarm_size=32)
    dp.run(Dg, other, state, 1)   # header says S = 64: the device rejects it
    with pytest.raises(dp.DpsoError) as ei:
        dp.get_info(state)
    assert ei.value.status == dp.E_STATE


BATCH = [
    # (n, swarm, overrides): every edge-exchange class, aligned and unaligned n
    (1, 2, {}), (3, 5, {}), (30, 16, {}), (64, 8, dict(ee_trigger=2)), (65, 12, {}),
    (127, 9, dict(mutation_period=0)), (128, 6, dict(ee_trigger=2, ee_max_moves=0)),
    (200, 20, {}), (257, 7, dict(ee_trigger=2)), (515, 6, dict(ee_trigger=2)),
    (1000, 5, dict(ee_trigger=2)), (1030, 3, dict(ee_trigger=2)),
    (260, 6, dict(ee_trigger=2)), (512, 5, dict(ee_trigger=2)), (1024, 3, dict(ee_trigger=2)),
    (50, 10, dict(stall_limit=2)), (40, 10, dict(ee_trigger=0)),
    # paper-literal variants in the same batch as the default instances
    (45, 10, dict(ee_neighbourhood=1, ee_trigger=2)), (2, 4, dict(ee_neighbourhood=1, ee_trigger=2)),
    (301, 6, dict(ee_neighbourhood=1, ee_trigger=2, mutation_swaps=3)), (88, 12, dict(mutation_swaps=5)),
    (77, 9, dict(velocity_cap=30, w=1.0, phi1=0.4, phi2=0.4)),
]


def _batch_case(gens):
    members = []
    for k, (n, S, kw) in enumerate(BATCH):
        sc = scenes.random_points(n, seed=100 + k, n_boxes=2 if n > 3 else 0)
        D = oracle.build_dist(sc)
        prm = scenes.swarm_params(S, gens if k != 0 else 5, seed=k, instance=k, **kw)
        members.append((D, prm))
    return members


@pytest.mark.parametrize("side", [False, True], ids=["null_stream", "side_stream"])
def test_batch_matches_oracle(dp, side):
    import torch
    gens = 9
    members = _batch_case(gens)
    stream = torch.cuda.Stream() if side else None
    note(f"batch of {len(members)} instances, side stream={side}")
    b = dp.Batch([(_dev(D), p) for D, p in members], stream=stream).init()
    b.run(4)
    b.run(gens - 4)
    for k, ((D, prm), st) in enumerate(zip(members, b.states)):
        ref = oracle.new_state(D, prm)
        oracle.run(D, prm, ref, gens)
        bad = mismatches(dp.export_state(st, D.shape[0], prm["swarm_size"], stream), ref)
        assert not bad, f"instance {k} (n={D.shape[0]}): {bad}"


@pytest.mark.parametrize("single,chunk", [(False, 0), (False, 4), (True, 0)],
                         ids=["batched", "continuous", "single_instance"])
def test_served_replans_match_oracle(dp, single, chunk):
    """A short re-planning stream through the server (5 sites, obstacle
    changes, swarm capacity of 3 runs, a budget that holds the two largest
    sites, so that sites are evicted): every served plan equals the oracle replaying the same sequence
    of actions per site (a fresh swarm for plan / rebuild / restart on the
    request's scene, the site's previous swarm run further for resume). The
    server runs requests as batches, or one at a time on the single-instance
    path, or by continuous batching (rounds of at most 4 generations, so
    swarms run in parts and requests join running ones)."""
    import collections
    from paper_1706_04399_amd import serve
    reqs = serve.replan_requests(40, rate=400.0, seed=9, sites=5, n_lo=20, n_hi=120, swarm=32,
                                 generations=15, change_permille=300, capacity_runs=3)
    sizes = sorted({r.key: dp.request_footprint(r.n, r.params, 1 << 40)[1] for r in reqs}.values())
    budget = sizes[-1] + sizes[-2]             # the two largest sites fit together, not all five
    ex = serve.GpuExecutor(budget_bytes=budget, single=single)
    sched = serve.Scheduler(budget, ex.footprint, max_batch=1 if single else 1024)
    note(f"served re-planning stream of 40 requests against the oracle, single={single}, chunk={chunk}")
    recs = serve.serve(reqs, ex, sched, chunk=chunk)
    assert sorted(r.rid for r in recs) == list(range(40)) and all(r.status == 0 for r in recs)
    acts = collections.Counter(r.action for r in recs)
    assert acts["resume"] and acts["rebuild"] and acts["restart"] and sched.n_evicted > 0, acts
    sites = {}
    for rec in sorted(recs, key=lambda r: r.rid):
        req = reqs[rec.rid]
        G, cap = req.generations, req.params["max_generations"]
        site = sites.get(req.key)
        if rec.action == "resume":
            assert site is not None and site["version"] == req.version and site["st"].t + G <= cap
        else:
            if rec.action == "rebuild":
                assert site is not None and site["version"] != req.version
            if rec.action == "restart":
                assert site is not None and site["version"] == req.version and site["st"].t + G > cap
            D = oracle.build_dist(req.scene)
            site = {"version": req.version, "D": D, "st": oracle.new_state(D, req.params)}
            sites[req.key] = site
        oracle.run(site["D"], req.params, site["st"], G)
        o = site["st"]
        assert (rec.cost, rec.generation) == (o.FG, o.t), (rec.rid, rec.action)
        assert np.array_equal(rec.tour, o.G), (rec.rid, rec.action)


def test_served_large_sites_match_oracle(dp):
    """Continuous batching over sites of n = 150 ... 700 (swarm 32, so a round
    of one to three requests takes the four- and two-wavefront rows, merged
    by group): every served plan equals the oracle replaying the site's
    actions in request order."""
    from paper_1706_04399_amd import serve
    reqs = serve.replan_requests(14, rate=300.0, seed=4, sites=3, n_lo=150, n_hi=700, swarm=32,
                                 generations=6, change_permille=300, capacity_runs=2)
    ns = sorted({r.n for r in reqs})
    forms = {dp.tuning_get(n, 96)["exchange_rows"] for n in ns} | {dp.tuning_get(n, 32)["exchange_rows"] for n in ns}
    assert dp.ROWS_U16_QUAD in forms, (ns, forms)
    ex = serve.GpuExecutor(budget_bytes=1 << 34)
    sched = serve.Scheduler(1 << 34, ex.footprint, max_batch=1024)
    note(f"served stream of 14 requests over sites n={ns} against the oracle, chunk=4")
    recs = serve.serve(reqs, ex, sched, chunk=4)
    assert sorted(r.rid for r in recs) == list(range(14)) and all(r.status == 0 for r in recs)
    sites = {}
    for rec in sorted(recs, key=lambda r: r.rid):
        req = reqs[rec.rid]
        site = sites.get(req.key)
        if rec.action != "resume":
            D = oracle.build_dist(req.scene)
            site = {"D": D, "st": oracle.new_state(D, req.params)}
            sites[req.key] = site
        oracle.run(site["D"], req.params, site["st"], req.generations)
        o = site["st"]
        assert (rec.cost, rec.generation) == (o.FG, o.t), (rec.rid, rec.action, req.n)
        assert np.array_equal(rec.tour, o.G), (rec.rid, rec.action, req.n)


def _costs(D, tours):
    """Tour costs recomputed with numpy (independent of both implementations)."""
    t = tours.astype(np.int64)
    return D.astype(np.int64)[t, np.roll(t, -1, axis=1)].sum(axis=1)


def test_workload3_full_length_properties(dp):
    """The benchmark run itself (2000 generations, n = 1000, swarm 4096): too
    long for the oracle, checked by properties that hold at any size."""
    sc, prm = scenes.workload(3)
    D = oracle.build_dist(sc)
    Dg = _dev(D)
    note("facade1000: full 2000-generation run")
    state = dp.init_nn(Dg, prm)
    dp.run(Dg, prm, state, prm["max_generations"])
    ex = dp.export_state(state, sc.n, prm["swarm_size"])
    info = dp.get_info(state)
    n, S, G = sc.n, prm["swarm_size"], prm["max_generations"]
    assert ex["generation"] == G and ex["done"] == 1
    for name in ("X", "P"):
        assert (np.sort(ex[name].astype(np.int64), axis=1) == np.arange(n)).all(), name
    assert (np.sort(ex["G"].astype(np.int64)) == np.arange(n)).all()
    assert np.array_equal(_costs(D, ex["X"]), ex["F"])
    assert np.array_equal(_costs(D, ex["P"]), ex["FP"])
    assert ex["best_cost"] == ex["FP"].min() == _costs(D, ex["G"][None, :])[0]
    assert (np.diff(ex["trace"]) <= 0).all() and ex["trace"][-1] == ex["best_cost"]
    assert (ex["FP"] <= ex["F"]).all()
    assert info["sweeps"] == S * G                  # one complete sweep per particle
    assert 0 < info["moves"] <= S * G
    assert (ex["vlen"] <= n - 1).all()
