"""Pins of the obstacle-aware distance builder (Sect. 2.2, 2.3)."""
import math

import numpy as np
import pytest
from conftest import golden_lines

from paper_1706_04399_amd import scenes


def _round_half_up(sq):
    r = math.isqrt(sq)
    return r + 1 if 4 * sq >= (2 * r + 1) ** 2 else r


def test_round_len_matches_exact_integer_rounding(orc):
    rng = np.random.default_rng(0)
    for _ in range(2000):
        d = [int(v) for v in rng.integers(-(1 << 26), 1 << 26, size=3)]
        assert orc.round_len(*d) == _round_half_up(sum(v * v for v in d))
    # s = r^2 + r lies just below (r + 1/2)^2 and rounds down; r^2 + r + 1 rounds up
    assert orc.round_len(3, 4, 0) == 5
    assert orc.round_len(1, 1, 0) == 1          # 1.414
    assert orc.round_len(1, 1, 1) == 2          # 1.732


@pytest.mark.parametrize("A,B,hit", [
    ((-10, 0, 0), (10, 0, 0), True),            # through the centre
    ((-10, 5, 0), (10, 5, 0), False),           # along the face y = 5
    ((-10, 6, 0), (10, 6, 0), False),           # beside the box
    ((-10, 5, 5), (10, 5, 5), False),           # along an edge
    ((-10, -10, 0), (10, 10, 0), True),         # diagonal through
    ((-10, 0, 0), (-5, 0, 0), False),           # ends on the face x = -5
    ((-10, 0, 0), (-4, 0, 0), True),            # ends just inside
    ((0, 0, 0), (0, 0, 0), True),               # a point inside
    ((-5, -5, -5), (5, 5, 5), True),            # corner to corner through
    ((-5, -5, 5), (5, 5, 5), False),            # diagonal of the top face
])
def test_segment_box_cases(orc, A, B, hit):
    assert orc.segment_hits_box(A, B, (-5, -5, -5), (5, 5, 5)) is hit
    assert orc.segment_hits_box(B, A, (-5, -5, -5), (5, 5, 5)) is hit


def test_hand_computed_detour(orc):
    rows = golden_lines("box_detour.txt")
    vp = [[int(v) for v in r[1:]] for r in rows if r[0] == "vp"]
    box = [[int(v) for v in r[1:]] for r in rows if r[0] == "box"]
    clr = int([r for r in rows if r[0] == "clearance"][0][1])
    cost = int([r for r in rows if r[0] == "cost"][0][1])
    D = orc.build_dist(scenes.Scene(np.array(vp), np.array(box), clr))
    assert D.tolist() == [[0, cost], [cost, 0]]


def _check_metric(D):
    n = len(D)
    assert (D == D.T).all()
    assert (np.diag(D) == 0).all()
    D64 = D.astype(np.int64)
    for k in range(n):
        assert (D64 <= D64[:, [k]] + D64[[k], :]).all()


@pytest.mark.parametrize("seed,nb", [(0, 0), (1, 2), (2, 5), (3, 9)])
def test_metric_properties(orc, seed, nb):
    sc = scenes.random_points(40, seed=seed, n_boxes=nb)
    D = orc.build_dist(sc)
    _check_metric(D)
    p = sc.vp_mm.astype(np.int64)
    straight = np.array([[_round_half_up(int(((p[i] - p[j]) ** 2).sum())) for j in range(len(p))]
                         for i in range(len(p))])
    if nb == 0:
        assert (D <= straight).all()
    # A path with L legs is at least the straight line minus L/2 of rounding;
    # no path here has more than 2 + 8 * nb legs.
    assert (D >= straight - (2 + 8 * nb) // 2 - 1).all()


def test_circle_distances_are_rounded_chords(orc):
    sc = scenes.circle(40)
    D = orc.build_dist(sc)
    p = sc.vp_mm.astype(np.int64)
    for i in range(40):
        for j in range(40):
            assert D[i, j] == _round_half_up(int(((p[i] - p[j]) ** 2).sum()))


def test_workload_scenes_build(orc):
    for k in (1, 2):
        sc, _ = scenes.workload(k)
        D = orc.build_dist(sc)
        _check_metric(D)
        assert D.max() < oracle_D_INF()


def oracle_D_INF():
    import oracle
    return oracle.D_INF


def test_unreachable_pair_gets_large_cost(orc):
    # a viewpoint sealed inside a hollow of boxes: six slabs around (0,0,0)
    slabs = [(-3000, -3000, -3000, -2000, 3000, 3000), (2000, -3000, -3000, 3000, 3000, 3000),
             (-3000, -3000, -3000, 3000, -2000, 3000), (-3000, 2000, -3000, 3000, 3000, 3000),
             (-3000, -3000, -3000, 3000, 3000, -2000), (-3000, -3000, 2000, 3000, 3000, 3000)]
    sc = scenes.Scene(np.array([(0, 0, 0), (10000, 0, 0)]), np.array(slabs), 0)
    D = orc.build_dist(sc)
    assert D[0, 1] == D[1, 0] == (1 << 28) - 1


# ------------------------------------------------------ the matrix contract

D_INF = (1 << 28) - 1


def plant(n, seed, kind, i, j):
    """A valid symmetric matrix with one planted break at (i, j)."""
    D = scenes.random_dist(n, seed=seed, max_mm=D_INF).astype(np.int64)
    if kind == "negative":
        D[i, j] = D[j, i] = -1
    elif kind == "above_inf":
        D[i, j] = D[j, i] = D_INF + 1
    elif kind == "diagonal":
        D[i, i] = 5
        j = i
    elif kind == "asymmetric":
        D[i, j] += 1
    return D.astype(np.int32), min(i, j) * n + max(i, j)


def test_check_dist_accepts_valid_matrices(orc):
    for sc in (scenes.workload(1)[0], scenes.random_points(40, seed=2, n_boxes=3)):
        assert orc.check_dist(orc.build_dist(sc)) == -1
    D = scenes.random_dist(17, seed=1)
    D[2, 9] = D[9, 2] = D_INF                     # a blocked pair is allowed
    assert orc.check_dist(D) == -1
    assert orc.check_dist(np.zeros((1, 1), np.int32)) == -1


@pytest.mark.parametrize("kind", ["negative", "above_inf", "diagonal", "asymmetric"])
def test_check_dist_finds_a_planted_break(orc, kind):
    rng = np.random.default_rng(len(kind))
    for n in (2, 7, 30):
        for _ in range(5):
            i, j = (int(v) for v in rng.choice(n, size=2, replace=False))
            D, first = plant(n, seed=n, kind=kind, i=i, j=j)
            assert orc.check_dist(D) == first, (kind, n, i, j)


def test_check_dist_reports_the_first_of_several(orc):
    D = scenes.random_dist(12, seed=4)
    D[7, 3] += 1                                   # asymmetric: first seen at row 3
    D[5, 5] = 1
    D[9, 1] = D[1, 9] = -4
    assert orc.check_dist(D) == 1 * 12 + 9         # row-major order: (1, 9) < (3, 7) < (5, 5)
