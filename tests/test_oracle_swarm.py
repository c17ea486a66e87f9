"""Pins and invariants of the whole swarm iteration (Sect. 3.3 pseudo code)."""
import itertools
import os
import subprocess
import sys

import numpy as np
import pytest

from paper_1706_04399_amd import scenes
from test_oracle_tsp import brute_force_optimum, cost_py


def check_state(D, st):
    n, S = st.n, st.S
    for p in range(S):
        assert sorted(st.X[p].tolist()) == list(range(n))
        assert sorted(st.P[p].tolist()) == list(range(n))
        assert st.F[p] == cost_py(D, st.X[p])
        assert st.FP[p] == cost_py(D, st.P[p])
        assert 0 <= st.VL[p] <= max(n - 1, 0)
    assert sorted(st.G.tolist()) == list(range(n))
    assert st.FG == cost_py(D, st.G)
    assert st.FG == st.FP.min()


def test_init_layout(orc):
    sc, prm = scenes.workload(1)
    D = orc.build_dist(sc)
    st = orc.new_state(D, prm)
    S, n = prm["swarm_size"], sc.n
    m = -(-S * prm["det_permille"] // 1000)
    for p in range(S):
        if p < m:
            assert (st.X[p] == orc.nn_tour(D, p * n // m)).all()
        else:
            assert (st.X[p] == orc.fisher_yates(n, prm["seed"], prm["instance"], p, 0, 0)).all()
    assert (st.VL == 0).all() and (st.P == st.X).all() and (st.FP == st.F).all()
    g = int(np.argmin(st.FP))
    assert (st.G == st.P[g]).all() and st.trace[0] == st.FG and st.t == 0
    check_state(D, st)


def test_run_invariants_every_generation(orc):
    sc, prm = scenes.workload(1)
    D = orc.build_dist(sc)
    st = orc.new_state(D, prm)
    prev = st.copy()
    for t in range(1, 61):
        orc.generation(D, prm, st)
        assert st.t == t
        check_state(D, st)
        assert st.FG <= prev.FG
        assert (st.FP <= prev.FP).all()                      # personal bests never worsen
        improved = st.FG < prev.FG
        assert st.stall == (0 if improved else prev.stall + 1)
        prev = st.copy()
    assert (np.diff(st.trace[: st.t + 1]) <= 0).all()


def test_move_phase_matches_move_core(orc):
    """The swarm's move uses the first two draws of stream (VEL, p, t)."""
    sc, prm = scenes.workload(1)
    D = orc.build_dist(sc)
    st = orc.new_state(D, prm)
    orc.run(D, prm, st, 4)
    before = st.copy()
    t = st.t + 1
    for p in (0, 5, 63):
        u1, u2 = orc.draws(prm["seed"], prm["instance"], p, t, 1, 2)
        y, v = orc.move_core(before.X[p], before.P[p], before.G, before.velocity(p), prm["w_q16"],
                             prm["phi1_q16"], prm["phi2_q16"], int(u1), int(u2))
        orc.move_particle(D, prm, st, p, t)
        assert (st.X[p] == y).all() and (st.velocity(p) == v).all()
        assert st.F[p] == cost_py(D, y)
        assert st.FP[p] == min(before.FP[p], st.F[p])


def test_mutation_invariants(orc):
    sc, prm = scenes.workload(1)
    D = orc.build_dist(sc)
    st = orc.new_state(D, prm)
    orc.run(D, prm, st, 2)
    S, n = st.S, st.n
    # plant duplicates: particles 10..14 copy particle 3 (same tour, same cost)
    for p in range(10, 15):
        st.X[p] = st.X[3]
        st.F[p] = st.F[3]
        st.V[p] = st.V[3]
        st.VL[p] = st.VL[3]
    before = st.copy()
    t = 3
    count, kept = orc.mutation(D, prm, st, t)
    K = -(-S // 3)
    assert kept.sum() == K and count == S - K
    assert not kept[10:15].any()                      # duplicates of 3 are never kept
    order = sorted(range(S), key=lambda p: (before.F[p], p))
    dup = {p for p in range(S) if any(before.F[q] == before.F[p] and
                                      (before.X[q] == before.X[p]).all() for q in range(p))}
    assert set(range(10, 15)) <= dup
    expect_kept = [p for p in order if p not in dup][:K]
    assert sorted(np.flatnonzero(kept).tolist()) == sorted(expect_kept)
    for p in range(S):
        if kept[p]:
            assert (st.X[p] == before.X[p]).all() and st.VL[p] == before.VL[p]
        else:
            assert (st.X[p] == orc.fisher_yates(n, prm["seed"], prm["instance"], p, t, 2)).all()
            assert st.VL[p] == 0 and st.F[p] == cost_py(D, st.X[p])
            assert st.FP[p] == min(before.FP[p], st.F[p])


def test_mutation_with_all_particles_identical(orc):
    """A collapsed swarm keeps one particle and reshuffles every other."""
    sc, prm = scenes.workload(1)
    D = orc.build_dist(sc)
    st = orc.new_state(D, prm)
    st.X[:] = st.X[0]
    st.F[:] = st.F[0]
    count, kept = orc.mutation(D, prm, st, 3)
    assert kept.tolist() == [1] + [0] * (st.S - 1) and count == st.S - 1


def test_split_run_equals_single_run(orc):
    sc, prm = scenes.workload(1)
    D = orc.build_dist(sc)
    a = orc.new_state(D, prm)
    orc.run(D, prm, a, 37)
    b = orc.new_state(D, prm)
    orc.run(D, prm, b, 20)
    orc.run(D, prm, b, 17)
    for name in ("X", "P", "V", "VL", "F", "FP", "G", "trace"):
        assert (getattr(a, name) == getattr(b, name)).all(), name
    assert (a.t, a.stall, a.FG) == (b.t, b.stall, b.FG)


def test_results_do_not_depend_on_thread_count(tmp_path):
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import oracle, numpy as np\n"
        "from paper_1706_04399_amd import scenes\n"
        "sc, prm = scenes.workload(1)\n"
        "D = oracle.build_dist(sc)\n"
        "st = oracle.new_state(D, prm)\n"
        "oracle.run(D, prm, st, 30)\n"
        "print(int(st.FG), int(st.X.astype(np.int64).sum() * 7 + st.V.sum()), st.G.tolist())\n"
    ) % os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    outs = []
    for th in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=th)
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, capture_output=True,
                                   text=True, check=True).stdout)
    assert outs[0] == outs[1]


def test_stop_conditions(orc):
    sc, prm = scenes.workload(1)
    D = orc.build_dist(sc)
    p2 = dict(prm, max_generations=25)
    st = orc.new_state(D, p2)
    orc.run(D, p2, st, 1000)
    assert st.t == 25 and st.done
    p3 = dict(prm, stall_limit=4)
    st = orc.new_state(D, p3)
    orc.run(D, p3, st, 200)
    assert st.done and (st.stall >= 4 or st.t == 200)
    if st.t < 200:
        assert st.stall == 4
    p0 = dict(prm, max_generations=0)
    st = orc.new_state(D, p0)
    assert st.done


def test_small_instances_reach_brute_force_optimum(orc):
    """n <= 8: the swarm never beats the optimum and, on these seeds, finds it."""
    for n, seed in ((5, 1), (7, 2), (8, 3)):
        D = orc.build_dist(scenes.random_points(n, seed=seed, n_boxes=1))
        opt = brute_force_optimum(D)
        prm = scenes.swarm_params(16, 40, seed=seed)
        st = orc.new_state(D, prm)
        orc.run(D, prm, st, 40)
        assert st.FG >= opt
        assert st.FG == opt


@pytest.mark.parametrize("cols,rows", [(4, 4), (4, 6)])
def test_even_grid_reaches_closed_form_optimum(orc, cols, rows):
    """Every edge of a grid tour is at least one spacing, so N*s is a lower
    bound, and a back-and-forth tour attains it when N is even. With the
    nearest-neighbour seeding of Sect. 3.2.1 the swarm reaches it."""
    s = 1000
    D = orc.build_dist(scenes.grid(cols, rows, s))
    prm = scenes.swarm_params(32, 100, seed=11)
    st = orc.new_state(D, prm)
    orc.run(D, prm, st, 100)
    assert st.FG >= cols * rows * s
    assert st.FG == cols * rows * s


def test_edge_exchange_always_leaves_no_improving_move_when_run_to_optimum(orc):
    sc, prm = scenes.workload(1)
    D = orc.build_dist(sc)
    p = dict(prm, ee_trigger=scenes.EE_ALWAYS, ee_max_moves=0)
    st = orc.new_state(D, p)
    orc.run(D, p, st, 3)
    for q in range(0, st.S, 7):
        assert orc.best_2opt(D, st.X[q])[0] >= 0


def test_check_params_rejects_bad_values(orc):
    base = scenes.swarm_params(8, 10)
    assert orc.check_params(base, 10) == 0
    for k, v in (("swarm_size", 0), ("swarm_size", 65537), ("w_q16", 131073),
                 ("ee_trigger", 3), ("det_permille", 1001), ("mutation_period", -1)):
        assert orc.check_params(dict(base, **{k: v}), 10) == -1
    assert orc.check_params(base, 0) == -1 and orc.check_params(base, 65536) == -1
