"""Pins of the tour cost, nearest-neighbour seeding and edge exchange."""
import itertools
import math

import numpy as np
import pytest

from paper_1706_04399_amd import scenes


def cost_py(D, x):
    n = len(x)
    return sum(int(D[x[k], x[(k + 1) % n]]) for k in range(n))


def test_cost_small_cases(orc):
    D = np.array([[0, 3, 4], [3, 0, 5], [4, 5, 0]], np.int32)
    assert orc.tour_cost(D[:1, :1], [0]) == 0
    assert orc.tour_cost(D[:2, :2], [1, 0]) == 6
    assert orc.tour_cost(D, [2, 0, 1]) == 12
    sq = orc.build_dist(scenes.grid(2, 2, 1000))
    assert orc.tour_cost(sq, [0, 1, 3, 2]) == 4000
    assert orc.tour_cost(sq, [0, 1, 2, 3]) == 2000 + 2 * 1414


def test_nn_collinear_sorted(orc):
    xs = [0, 130, 170, 1000, 1001, 4000, 4200, 9999]
    rng = np.random.default_rng(1)
    perm = rng.permutation(len(xs))
    sc = scenes.line([xs[i] for i in perm])
    D = orc.build_dist(sc)
    left = int(np.argmin(sc.vp_mm[:, 0]))
    tour = orc.nn_tour(D, left)
    assert sc.vp_mm[tour, 0].tolist() == sorted(xs)
    assert orc.tour_cost(D, tour) == 2 * (max(xs) - min(xs))


@pytest.mark.parametrize("cols,rows", [(3, 2), (5, 4), (8, 6), (4, 10)])
def test_nn_on_even_row_grid_is_back_and_forth(orc, cols, rows):
    """On a grid with an even number of rows and row-major labels, the
    nearest-neighbour tour from label 0 (smallest label on ties) is the
    back-and-forth tour of Sect. 3.2.1: cost (N - 1) s + (rows - 1) s."""
    s = 1000
    D = orc.build_dist(scenes.grid(cols, rows, s))
    tour = orc.nn_tour(D, 0)
    snake = []
    for r in range(rows):
        row = [r * cols + c for c in range(cols)]
        snake += row if r % 2 == 0 else row[::-1]
    assert tour.tolist() == snake
    assert orc.tour_cost(D, tour) == (cols * rows - 1) * s + (rows - 1) * s


def neighbours_by_recomputation(D, x):
    """Every 2-opt neighbour with its cost change, by reversing and re-costing."""
    n = len(x)
    base = cost_py(D, x)
    out = []
    for i in range(n):
        for j in range(i + 2, n):
            if i == 0 and j == n - 1:
                continue
            y = list(x[: i + 1]) + list(x[i + 1: j + 1])[::-1] + list(x[j + 1:])
            out.append((cost_py(D, y) - base, i, j))
    return out


@pytest.mark.parametrize("n", [4, 5, 6, 9, 23, 40])
def test_best_2opt_matches_recomputation(orc, n):
    rng = np.random.default_rng(100 + n)
    for trial in range(6):
        D = scenes.random_dist(n, seed=trial * 31 + n, max_mm=50 if trial % 2 else 100_000)
        x = rng.permutation(n)
        nb = neighbours_by_recomputation(D, x)
        assert len(nb) == n * (n - 3) // 2
        assert orc.best_2opt(D, x) == min(nb)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_no_exchange_below_four_nodes(orc, n):
    D = scenes.random_dist(n, seed=1)
    delta, i, j = orc.best_2opt(D, list(range(n)))
    assert (i, j) == (-1, -1)
    y, F, moves, sweeps = orc.edge_exchange(D, list(range(n)), cost_py(D, list(range(n))), 0)
    assert moves == 0 and sweeps == 1


def test_edge_exchange_one_move_and_local_optimum(orc):
    rng = np.random.default_rng(5)
    for n in (6, 15, 33):
        D = scenes.random_dist(n, seed=n)
        x = rng.permutation(n)
        F0 = cost_py(D, x)
        delta, i, j = min(neighbours_by_recomputation(D, x))
        y, F, moves, _ = orc.edge_exchange(D, x, F0, 1)
        assert F == cost_py(D, y)
        if delta < 0:
            assert moves == 1 and F == F0 + delta
            assert y.tolist() == list(x[: i + 1]) + list(x[i + 1: j + 1])[::-1] + list(x[j + 1:])
        y, F, moves, sweeps = orc.edge_exchange(D, x, F0, 0)
        assert F == cost_py(D, y) and sweeps == moves + 1
        assert min(d for d, _, _ in neighbours_by_recomputation(D, y)) >= 0
        assert sorted(y.tolist()) == list(range(n))


def _round_half_up(num_sq):
    r = math.isqrt(num_sq)
    return r + 1 if 4 * num_sq >= (2 * r + 1) ** 2 else r


@pytest.mark.parametrize("n", [8, 20, 64])
def test_circle_local_optimum_is_hull_order(orc, n):
    """For points on a circle every 2-opt local optimum is the angular order:
    any other tour has crossing edges, and uncrossing gains far more than the
    rounding slack (R * delta^3 / 2 > 2 mm for these n)."""
    sc = scenes.circle(n)
    D = orc.build_dist(sc)
    p = sc.vp_mm.astype(np.int64)
    hull = sum(_round_half_up(int(((p[k] - p[(k + 1) % n]) ** 2).sum())) for k in range(n))
    rng = np.random.default_rng(n)
    for _ in range(4):
        x = rng.permutation(n)
        y, F, _, _ = orc.edge_exchange(D, x, cost_py(D, x), 0)
        assert F == hull
        r = np.roll(y, -int(np.argmin(y)))
        assert r.tolist() in (list(range(n)), [0] + list(range(n - 1, 0, -1)))


def brute_force_optimum(D):
    n = len(D)
    best = None
    for perm in itertools.permutations(range(1, n)):
        if n > 2 and perm[0] > perm[-1]:
            continue                       # each cycle once per direction
        c = cost_py(D, (0,) + perm)
        best = c if best is None or c < best else best
    return best


def test_local_optimum_never_beats_brute_force(orc):
    for n in (5, 7, 8):
        D = orc.build_dist(scenes.random_points(n, seed=n, n_boxes=1))
        opt = brute_force_optimum(D)
        rng = np.random.default_rng(n)
        for _ in range(5):
            x = rng.permutation(n)
            _, F, _, _ = orc.edge_exchange(D, x, cost_py(D, x), 0)
            assert F >= opt
