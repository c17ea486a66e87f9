"""Pins of the generation control of the pseudo code of Sect. 3.3.

One generation of the enhanced DPSO, as the pseudo code lists it: every
particle moves and updates its personal best; on every third generation (the
mutation period of Sect. 4) the swarm is ranked and all but the best third are
randomised; then the fittest personal best is found and installs the global
best if it is better; only when the global best did not improve does the edge
exchange run, after which the global best is updated again.

Each test below builds a swarm by hand whose outcome that order fixes, so a
phase moved, a trigger inverted, a mutation phase shifted or a global-best tie
sent to the wrong particle fails here, independently of the parity between the
oracle and the GPU (which share these readings). The last test composes the
oracle's unit-pinned phases in the pseudo code's order in Python and compares
whole generations with the oracle's own composition.
"""
import numpy as np
import pytest

from paper_1706_04399_amd import scenes

EE_OFF, EE_ON_STALL, EE_ALWAYS = 0, 1, 2
MUT = 2  # purpose of the mutation stream


def cost_py(D, x):
    return int(sum(int(D[x[k], x[(k + 1) % len(x)]]) for k in range(len(x))))


def frozen_params(S, gens, **kw):
    """Coefficients zero: a move leaves every tour where it is (k_w = k_1 =
    k_2 = 0), so only mutation and the edge exchange change the swarm."""
    p = scenes.swarm_params(S, gens, w=0.0, phi1=0.0, phi2=0.0, det_permille=0, seed=7)
    p.update(kw)
    return p


def set_swarm(orc, D, prm, tours):
    """A fresh oracle state whose particles hold the given tours (empty
    velocities, personal best = the tour) and whose global best is the
    cheapest of them, lowest index first, at generation 0."""
    st = orc.new_state(D, prm)
    for p, x in enumerate(tours):
        st.X[p] = x
        st.P[p] = x
        st.F[p] = st.FP[p] = cost_py(D, x)
    st.VL[:] = 0
    g = min(range(len(tours)), key=lambda p: (st.FP[p], p))
    st.G[:] = st.P[g]
    st.FG = int(st.FP[g])
    st.trace[0] = st.FG
    st.t, st.stall, st.done = 0, 0, 0
    return st


def cycle_matrix(order, cheap=1, dear=100):
    """Symmetric matrix whose cheapest closed tour is exactly `order` (and its
    rotations and reversal): its n edges cost `cheap`, every other pair `dear`."""
    n = len(order)
    D = np.full((n, n), dear, np.int32)
    np.fill_diagonal(D, 0)
    for k in range(n):
        a, b = order[k], order[(k + 1) % n]
        D[a, b] = D[b, a] = cheap
    return D


def test_mutation_precedes_the_global_best_update(orc):
    """A particle randomised on a mutation generation reaches the unique
    optimum: the global best must take it in that same generation (the
    pseudo code finds the fittest particle after the mutation), not one
    generation later."""
    n, S = 9, 6
    prm = frozen_params(S, 10, mutation_period=3, ee_trigger=EE_OFF)
    star = 5
    optimum = orc.fisher_yates(n, prm["seed"], prm["instance"], star, 3, MUT)
    D = cycle_matrix(optimum)
    # particles 0 and 1 are one exchange away from the optimum (cheapest, kept:
    # ceil(6/3) = 2); the others are farther, so particle 5 is randomised at t = 3
    rng = np.random.default_rng(3)
    tours = []
    for p in range(S):
        x = optimum.copy()
        if p < 2:
            i, j = (1 + p, 5 + p)
            x[i], x[j] = x[j], x[i]
        else:
            x = rng.permutation(n).astype(np.int32)
        tours.append(x)
    st = set_swarm(orc, D, prm, tours)
    start = st.FG
    assert start > n and min(cost_py(D, t) for t in tours[2:]) > max(cost_py(D, t) for t in tours[:2])
    orc.run(D, prm, st, 2)
    assert st.trace[1] == st.trace[2] == start and st.n_reshuffled == 0
    orc.run(D, prm, st, 1)                                 # t = 3: mutation generation
    assert st.n_reshuffled == S - 2
    assert (st.X[star] == optimum).all() and st.F[star] == n
    assert st.FG == n and st.trace[3] == n                 # taken in the same generation
    assert (st.G == optimum).all() and st.stall == 0


def test_mutation_only_on_multiples_of_the_period(orc):
    """Randomisation happens on generations t = 3, 6, 9 (t mod 3 = 0, t >= 1)
    and on no other."""
    sc, _ = scenes.workload(1)
    D = orc.build_dist(sc)
    S = 12
    prm = frozen_params(S, 12, mutation_period=3, ee_trigger=EE_OFF)
    st = orc.new_state(D, prm)
    grew = []
    for t in range(1, 13):
        before = st.n_reshuffled
        orc.generation(D, prm, st)
        grew.append(st.n_reshuffled - before)
    K = -(-S // 3)
    assert [t for t in range(1, 13) if grew[t - 1]] == [3, 6, 9, 12]
    assert all(g == S - K for g in grew if g)
    # period 0 switches it off
    st = orc.new_state(D, dict(prm, mutation_period=0))
    orc.run(D, dict(prm, mutation_period=0), st, 12)
    assert st.n_reshuffled == 0


def test_on_stall_exchange_runs_when_the_global_best_does_not_improve(orc):
    """Frozen moves and no mutation: the move phase can never lower a
    personal best, so the first global-best step never improves and the
    exchange runs every generation, one sweep per particle."""
    sc, _ = scenes.workload(1)
    D = orc.build_dist(sc)
    S = 16
    prm = frozen_params(S, 8, mutation_period=0, ee_trigger=EE_ON_STALL, ee_max_moves=1)
    st = orc.new_state(D, prm)
    for t in range(1, 9):
        orc.generation(D, prm, st)
        assert st.n_sweeps == S * t
    # the exchange improves some tour every generation here (random tours are
    # far from 2-opt optimal), and that improvement resets the stall counter
    assert st.n_moves > 0 and st.stall == 0


def test_on_stall_exchange_skipped_when_the_global_best_improves(orc):
    """The same swarm with a global best worse than every personal best:
    the first global-best step improves, so the exchange does not run."""
    sc, _ = scenes.workload(1)
    D = orc.build_dist(sc)
    S = 16
    prm = frozen_params(S, 8, mutation_period=0, ee_trigger=EE_ON_STALL, ee_max_moves=1)
    st = orc.new_state(D, prm)
    st.FG = int(st.FP.max()) + 1000
    orc.generation(D, prm, st)
    assert st.n_sweeps == 0 and st.stall == 0 and st.FG == int(st.FP.min())
    # the next generation cannot improve in the first step: exchange runs
    orc.generation(D, prm, st)
    assert st.n_sweeps == S


@pytest.mark.parametrize("trigger,expect", [(EE_OFF, 0), (EE_ALWAYS, 1)])
def test_off_and_always_triggers(orc, trigger, expect):
    sc, _ = scenes.workload(1)
    D = orc.build_dist(sc)
    S = 16
    prm = frozen_params(S, 4, mutation_period=0, ee_trigger=trigger, ee_max_moves=1)
    st = orc.new_state(D, prm)
    st.FG = int(st.FP.max()) + 1000       # the first step improves: ALWAYS still runs
    orc.run(D, prm, st, 4)
    assert st.n_sweeps == expect * S * 4


def test_global_best_ties_go_to_the_lowest_index(orc):
    """Two personal bests of equal, lowest cost and different tours: the
    global best is the lower-indexed particle's tour."""
    n, S = 8, 6
    order = np.arange(n, dtype=np.int32)
    D = cycle_matrix(order)
    prm = frozen_params(S, 4, mutation_period=0, ee_trigger=EE_OFF)
    rng = np.random.default_rng(11)
    tours = [rng.permutation(n).astype(np.int32) for _ in range(S)]
    a = order.copy()
    a[[1, 4]] = a[[4, 1]]
    b = order.copy()
    b[[2, 6]] = b[[6, 2]]
    assert cost_py(D, a) == cost_py(D, b) and not (a == b).all()
    tours[2], tours[4] = b, a            # particle 2 holds b, particle 4 holds a
    st = set_swarm(orc, D, prm, tours)
    assert (st.G == b).all()
    # the same through a generation's global-best step
    st.FG = 10 ** 9
    orc.generation(D, prm, st)
    assert (st.G == b).all() and st.FG == cost_py(D, b)
    # and through the function itself, with the tie planted higher up
    st.FP[5] = st.FP[2]
    st.P[5] = tours[0]
    st.FG = 10 ** 9
    assert orc.update_gbest(st) == 1 and (st.G == b).all()


def test_global_best_replaced_only_on_strict_improvement(orc):
    n, S = 8, 4
    D = cycle_matrix(np.arange(n, dtype=np.int32))
    prm = frozen_params(S, 4, mutation_period=0, ee_trigger=EE_OFF)
    rng = np.random.default_rng(5)
    st = set_swarm(orc, D, prm, [rng.permutation(n).astype(np.int32) for _ in range(S)])
    held = st.G.copy()
    g = int(np.argmin(st.FP))
    st.P[g] = np.roll(st.P[g], 1)        # same cost (a rotation), other tour
    assert orc.update_gbest(st) == 0 and (st.G == held).all()


def reference_generation(orc, D, prm, st):
    """One generation composed from the oracle's phases in the order of the
    pseudo code (written here, not taken from the oracle's composition)."""
    t = st.t + 1
    for p in range(st.S):
        orc.move_particle(D, prm, st, p, t)
    reshuffled = 0
    if prm["mutation_period"] > 0 and t % prm["mutation_period"] == 0:
        reshuffled, _ = orc.mutation(D, prm, st, t)
    improved = orc.update_gbest(st) == 1
    sweeps = moves = 0
    trig = prm["ee_trigger"]
    if trig == EE_ALWAYS or (trig == EE_ON_STALL and not improved):
        for p in range(st.S):
            y, f, m, sw = orc.edge_exchange(D, st.X[p], int(st.F[p]), prm["ee_max_moves"])
            st.X[p], st.F[p] = y, f
            sweeps += sw
            moves += m
            if st.F[p] < st.FP[p]:
                st.P[p], st.FP[p] = st.X[p], st.F[p]
        improved = (orc.update_gbest(st) == 1) or improved
    st.stall = 0 if improved else st.stall + 1
    st.t = t
    st.trace[t] = st.FG
    return reshuffled, sweeps, moves


@pytest.mark.parametrize("trigger", [EE_OFF, EE_ON_STALL, EE_ALWAYS])
def test_generation_equals_the_pseudo_code_composition(orc, trigger):
    sc, prm = scenes.workload(1)
    D = orc.build_dist(sc)
    prm = dict(prm, swarm_size=24, max_generations=12, ee_trigger=trigger)
    a = orc.new_state(D, prm)
    b = a.copy()
    res = sw = mv = 0
    for _ in range(12):
        orc.generation(D, prm, a)
        r, s, m = reference_generation(orc, D, prm, b)
        res, sw, mv = res + r, sw + s, mv + m
        for name in ("X", "P", "F", "FP", "G", "VL"):
            assert (getattr(a, name) == getattr(b, name)).all(), (name, a.t)
        assert (a.FG, a.stall, a.t) == (b.FG, b.stall, b.t)
    assert (a.n_reshuffled, a.n_sweeps, a.n_moves) == (res, sw, mv)
    assert (a.trace[:13] == b.trace[:13]).all()
