"""Pins of the oracle's paper-literal variants: the node-swap exchange
neighbourhood (the edge-exchange kernel and pseudo code of Sect. 3.3 exchange
two nodes and keep the best), mutation as a disturbance by random position
exchanges (the mutation text of Sect. 3.2.2) and the velocity kept as the raw
concatenation of eq. velocity with a length cap."""
import itertools

import numpy as np
import pytest

from paper_1706_04399_amd import scenes
from test_oracle_rng import numpy_block
from test_oracle_swarm import check_state
from test_oracle_tsp import cost_py


def swapped(x, i, j):
    y = np.array(x, np.int64)
    y[i], y[j] = y[j], y[i]
    return y


def brute_best_swap(D, x):
    """Lexicographic minimum (delta, i, j) by recomputing every swapped tour."""
    c0 = cost_py(D, x)
    best = None
    for i, j in itertools.combinations(range(len(x)), 2):
        key = (cost_py(D, swapped(x, i, j)) - c0, i, j)
        best = key if best is None or key < best else best
    return best


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 9, 14])
def test_swap_delta_is_the_cost_difference(orc, n):
    rng = np.random.default_rng(n)
    for trial in range(4):
        D = scenes.random_dist(n, seed=100 * n + trial)         # not a metric
        x = rng.permutation(n)
        c0 = cost_py(D, x)
        for i, j in itertools.combinations(range(n), 2):
            assert orc.swap_delta(D, x, i, j) == cost_py(D, swapped(x, i, j)) - c0, (n, i, j)


@pytest.mark.parametrize("n", [2, 3, 4, 7, 12])
def test_best_swap_is_the_lexicographic_minimum(orc, n):
    rng = np.random.default_rng(7 + n)
    for trial in range(5):
        # few distinct values: many ties between candidate exchanges
        D = scenes.random_dist(n, seed=trial, max_mm=4)
        x = rng.permutation(n)
        assert orc.best_swap(D, x) == brute_best_swap(D, x)


def test_best_swap_needs_two_nodes(orc):
    D = np.zeros((1, 1), np.int32)
    assert orc.best_swap(D, np.array([0]))[1] == -1


def test_node_exchange_to_a_local_optimum(orc):
    rng = np.random.default_rng(3)
    for n in (5, 8, 13):
        D = scenes.random_dist(n, seed=n)
        x = rng.permutation(n)
        F0 = cost_py(D, x)
        y, F, moves, sweeps = orc.node_exchange(D, x, F0, 0)
        assert F == cost_py(D, y) and sorted(y.tolist()) == list(range(n))
        assert sweeps == moves + 1 and F <= F0
        assert brute_best_swap(D, y)[0] >= 0                     # no improving exchange left
        # one move: exactly the best exchange, when it improves
        d, i, j = brute_best_swap(D, x)
        y1, F1, m1, _ = orc.node_exchange(D, x, F0, 1)
        if d < 0:
            assert m1 == 1 and (y1 == swapped(x, i, j)).all() and F1 == F0 + d
        else:
            assert m1 == 0 and (y1 == x).all()


@pytest.mark.parametrize("a,b", [(1, 5), (0, 7), (2, 3), (0, 11)])
def test_collinear_points_one_exchange_from_optimal(orc, a, b):
    """Collinear points in order cost 2 x span, the least any closed tour can
    cost; a tour one exchange away from that order is fixed by one move."""
    n, s = 12, 1000
    sc = scenes.line([s * k for k in range(n)])
    D = orc.build_dist(sc)
    x = swapped(np.arange(n), a, b)
    y, F, moves, _ = orc.node_exchange(D, x, cost_py(D, x), 1)
    assert F == 2 * s * (n - 1) == cost_py(D, y)


def _numpy_disturb(x, k, seed, inst, p, t, purpose):
    """k exchanges of positions (uniform(n), uniform(n)) from numpy's Philox words."""
    n = len(x)
    words = np.concatenate([numpy_block(seed, inst, [b, p, t, purpose])
                            for b in range((2 * k + 7) // 8 + 1)])
    draws = []
    for w in words:
        draws += [int(w) & 0xFFFFFFFF, int(w) >> 32]
    y = list(x)
    for a in range(k):
        i = (draws[2 * a] * n) >> 32
        j = (draws[2 * a + 1] * n) >> 32
        y[i], y[j] = y[j], y[i]
    return np.array(y, np.int32)


@pytest.mark.parametrize("n,k", [(1, 3), (2, 1), (9, 4), (30, 5), (257, 40)])
def test_disturbance_matches_numpy_stream(orc, n, k):
    x = np.random.default_rng(n).permutation(n)
    got = orc.disturb(x, k, 5, 1, 3, 6, 2)
    assert (got == _numpy_disturb(x, k, 5, 1, 3, 6, 2)).all()
    assert sorted(got.tolist()) == list(range(n))


def test_mutation_by_disturbance(orc):
    sc, prm = scenes.workload(1)
    prm = dict(prm, mutation_swaps=3)
    D = orc.build_dist(sc)
    st = orc.new_state(D, prm)
    orc.run(D, prm, st, 2)
    before = st.copy()
    t = 3
    count, kept = orc.mutation(D, prm, st, t)
    S = st.S
    assert kept.sum() == -(-S // 3) and count == S - kept.sum()
    for p in range(S):
        if kept[p]:
            assert (st.X[p] == before.X[p]).all() and st.VL[p] == before.VL[p]
        else:
            expect = _numpy_disturb(before.X[p], 3, prm["seed"], prm["instance"], p, t, 2)
            assert (st.X[p] == expect).all()
            assert st.VL[p] == 0 and st.F[p] == cost_py(D, st.X[p])
            assert st.FP[p] == min(before.FP[p], st.F[p])


@pytest.mark.parametrize("variant", [
    dict(ee_neighbourhood=scenes.NB_NODE_SWAP),
    dict(ee_neighbourhood=scenes.NB_NODE_SWAP, ee_trigger=scenes.EE_ALWAYS, ee_max_moves=0),
    dict(mutation_swaps=2),
    dict(ee_neighbourhood=scenes.NB_NODE_SWAP, mutation_swaps=5, ee_trigger=scenes.EE_ALWAYS),
    dict(det_permille=0, mutation_period=0, ee_trigger=scenes.EE_OFF),   # conventional DPSO
])
def test_variant_runs_keep_the_invariants(orc, variant):
    sc = scenes.random_points(24, seed=4, n_boxes=2)
    D = orc.build_dist(sc)
    prm = scenes.swarm_params(40, 30, seed=2, **variant)
    st = orc.new_state(D, prm)
    prev = st.copy()
    for t in range(1, 31):
        orc.generation(D, prm, st)
        check_state(D, st)
        assert st.FG <= prev.FG and (st.FP <= prev.FP).all()
        prev = st.copy()
    if variant.get("ee_max_moves") == 0:
        for p in range(st.S):                      # every particle left node-swap optimal
            assert brute_best_swap(D, st.X[p])[0] >= 0


def test_variant_params_are_checked(orc):
    base = scenes.swarm_params(8, 5)
    assert orc.check_params(base, 10) == 0
    for bad in (dict(ee_neighbourhood=2), dict(ee_neighbourhood=-1), dict(mutation_swaps=-1),
                dict(mutation_swaps=65537)):
        assert orc.check_params(dict(base, **bad), 10) != 0


# ----------------------------------------------- raw concatenated velocity

def _golden_move(name):
    from conftest import golden_lines
    g = {row[0]: [int(v) for v in row[1:]] for row in golden_lines(name)}
    return g


def test_raw_velocity_worked_example(orc):
    g = _golden_move("move_step_raw.txt")
    w, p1, p2 = g["coef"]
    u1, u2 = g["draws"]
    for cap in (5, 4, 3, 1):
        y, v = orc.move_core_raw(g["x"], g["P"], g["G"], np.array(g["v"]).reshape(-1, 2), w, p1, p2,
                                 u1, u2, cap)
        assert y.tolist() == g["y"]
        assert v.reshape(-1).tolist() == g["vnew"][: 2 * cap]


def test_raw_velocity_properties(orc):
    """Same position as the renormalised move; the uncapped list applied to x
    gives y; a smaller cap keeps a prefix of the list."""
    rng = np.random.default_rng(11)
    for trial in range(200):
        n = int(rng.integers(2, 30))
        x, P, G = rng.permutation(n), rng.permutation(n), rng.permutation(n)
        v = orc.bss(rng.permutation(n), rng.permutation(n))
        w, p1, p2 = (int(c) for c in rng.integers(0, 131073, size=3))
        u1, u2 = (int(d) for d in rng.integers(0, 2**32, size=2))
        y0, _ = orc.move_core(x, P, G, v, w, p1, p2, u1, u2)
        y, full = orc.move_core_raw(x, P, G, v, w, p1, p2, u1, u2, n)
        assert (y == y0).all()
        if len(full) < n:                       # the cap did not cut the list
            assert (orc.apply_swaps(x, full) == y).all()
        cap = int(rng.integers(1, n + 1))
        _, short = orc.move_core_raw(x, P, G, v, w, p1, p2, u1, u2, cap)
        assert len(short) == min(cap, len(full)) and (short == full[: len(short)]).all()


def test_raw_velocity_runs_keep_the_invariants(orc):
    sc = scenes.random_points(24, seed=6, n_boxes=2)
    D = orc.build_dist(sc)
    prm = scenes.swarm_params(40, 30, seed=3, w=1.0, phi1=0.4, phi2=0.4, velocity_cap=20)
    st = orc.new_state(D, prm)
    prev = st.copy()
    grew = False
    for t in range(1, 31):
        orc.generation(D, prm, st)
        check_state(D, st)
        assert (st.VL <= 20).all()
        grew |= bool((st.VL > 0).any())
        assert st.FG <= prev.FG
        prev = st.copy()
    assert grew
    for bad in (-1, 25):
        assert orc.check_params(dict(prm, velocity_cap=bad), 24) != 0
