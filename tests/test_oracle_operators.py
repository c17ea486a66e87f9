"""Pins of the velocity operators (Sect. 3.1)."""
import itertools

import numpy as np
import pytest
from conftest import golden_lines


def test_paper_example_position_plus_velocity(orc):
    """The paper's worked example: transpositions exchange labels."""
    g = {row[0]: [int(v) for v in row[1:]] for row in golden_lines("position_plus_velocity.txt")}
    x = np.array(g["x"][:-1]) - 1            # drop the repeated first node, go 0-based
    v = np.array([g["swap1"], g["swap2"]]) - 1
    after1 = orc.apply_swaps(x, v, 1) + 1
    after2 = orc.apply_swaps(x, v, 2) + 1
    assert after1.tolist() + [after1[0]] == g["after1"]
    assert after2.tolist() + [after2[0]] == g["after2"]


def test_paper_example_rejects_position_swaps():
    """Exchanging positions instead of labels does not reproduce the example."""
    g = {row[0]: [int(v) for v in row[1:]] for row in golden_lines("position_plus_velocity.txt")}
    x = g["x"][:-1]
    i, j = g["swap1"]
    y = list(x)
    y[i - 1], y[j - 1] = y[j - 1], y[i - 1]
    assert y + [y[0]] != g["after1"]


def _cycles(x, T):
    pos = {v: i for i, v in enumerate(x)}
    rho = [pos[T[p]] for p in range(len(x))]
    seen, c = set(), 0
    for s in range(len(x)):
        if s not in seen:
            c += 1
            while s not in seen:
                seen.add(s)
                s = rho[s]
    return c


def test_subtraction_paper_pair(orc):
    """x1 + (x2 - x1) = x2 for the example's pair; the canonical velocity differs
    from the paper's but has the same (minimal) length."""
    x = np.array([1, 4, 2, 3, 5]) - 1
    T = np.array([3, 4, 1, 2, 5]) - 1
    v = orc.bss(x, T)
    assert (v + 1).tolist() == [[1, 3], [2, 1]]
    assert (orc.apply_swaps(x, v) == T).all()
    assert (orc.apply_swaps(x, np.array([[1, 2], [2, 3]]) - 1) == T).all()


@pytest.mark.parametrize("n", [1, 2, 3, 7, 50, 300])
def test_subtraction_property(orc, n):
    rng = np.random.default_rng(n)
    for _ in range(50):
        x, T = rng.permutation(n), rng.permutation(n)
        v = orc.bss(x, T)
        assert (orc.apply_swaps(x, v) == T).all()
        assert len(v) == n - _cycles(x.tolist(), T.tolist())


def _min_transpositions_bfs(x, T):
    """Fewest label exchanges carrying x to T, by breadth-first search."""
    start, goal = tuple(x), tuple(T)
    frontier, seen, d = [start], {start}, 0
    while goal not in seen:
        nxt = []
        for s in frontier:
            for a, b in itertools.combinations(range(len(s)), 2):
                t = list(s)
                t[a], t[b] = t[b], t[a]
                t = tuple(t)
                if t not in seen:
                    seen.add(t)
                    nxt.append(t)
        frontier, d = nxt, d + 1
    return d


def test_subtraction_is_minimal_brute_force(orc):
    for x in itertools.permutations(range(5)):
        T = (2, 0, 4, 1, 3)
        assert len(orc.bss(x, T)) == _min_transpositions_bfs(x, T)


def test_addition_of_velocities_is_concatenation(orc):
    """(x + v1) + v2 == x + (v1 (+) v2) for label transpositions."""
    rng = np.random.default_rng(4)
    x = rng.permutation(12)
    v1 = rng.integers(0, 12, size=(5, 2))
    v2 = rng.integers(0, 12, size=(4, 2))
    v1 = v1[v1[:, 0] != v1[:, 1]]
    v2 = v2[v2[:, 0] != v2[:, 1]]
    lhs = orc.apply_swaps(orc.apply_swaps(x, v1), v2)
    rhs = orc.apply_swaps(x, np.concatenate([v1, v2]))
    assert (lhs == rhs).all()


def test_truncation_counts_golden(orc):
    for row in golden_lines("truncation_counts.txt"):
        lv, lb, lc, w, p1, p2, u1, u2, kw, k1, k2 = (int(v) for v in row)
        assert orc.truncate_counts(lv, lb, lc, w, p1, p2, u1, u2) == (kw, k1, k2), row


def test_truncation_special_cases(orc):
    """c = 0 gives the empty velocity, c = 1 the whole velocity."""
    for L in range(0, 40):
        assert orc.truncate_counts(L, L, L, 0, 0, 0, 2**32 - 1, 2**32 - 1) == (0, 0, 0)
        assert orc.truncate_counts(L, L, L, 65536, 65536, 65536, 0, 0)[0] == L


def test_move_step_golden(orc):
    g = {row[0]: [int(v) for v in row[1:]] for row in golden_lines("move_step.txt")}
    w, p1, p2 = g["coef"]
    u1, u2 = g["draws"]
    y, v = orc.move_core(g["x"], g["P"], g["G"], np.array(g["v"]).reshape(-1, 2), w, p1, p2, u1, u2)
    assert y.tolist() == g["y"]
    assert v.reshape(-1).tolist() == g["vnew"]


def test_move_reaches_targets_with_full_coefficients(orc):
    """w = 0, phi1 = 0, phi2 r2 = 1 moves x onto G; phi1 r1 = 1 alone onto P."""
    rng = np.random.default_rng(7)
    for n in (5, 17, 64):
        x, P, G = rng.permutation(n), rng.permutation(n), rng.permutation(n)
        y, v = orc.move_core(x, P, G, np.zeros((0, 2)), 0, 0, 2 * 65536, 0, 2**32 - 1)
        assert (y == G).all()
        assert (orc.apply_swaps(x, v) == y).all()
        y, _ = orc.move_core(x, P, G, np.zeros((0, 2)), 0, 2 * 65536, 0, 2**32 - 1, 0)
        assert (y == P).all()
