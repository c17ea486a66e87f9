"""The prefix of the canonical subtraction, by cycle structure.

The HIP move kernel does not scan positions one by one. It relies on this
description of x + (first k transpositions of T - x), checked here against
the oracle's literal scan:

  rho(p) = position in x of the label T[p]. The scan exchanges labels at
  exactly the positions that are not the largest of their rho-cycle, in
  increasing order, so |T - x| = n - (number of cycles). After the first k
  exchanges, the first k such positions hold T[p]; every other position s
  holds x[rho(r)], where r is the nearest predecessor of s along rho (r, rho(r),
  ..., s) that is not among those k positions.
"""
import itertools

import numpy as np


def partial_by_cycles(frm, to, k):
    n = len(frm)
    pos = {v: i for i, v in enumerate(frm)}
    rho = [pos[to[p]] for p in range(n)]
    cmax = [None] * n
    for s in range(n):
        if cmax[s] is None:
            cyc, q = [s], rho[s]
            while q != s:
                cyc.append(q)
                q = rho[q]
            for q in cyc:
                cmax[q] = max(cyc)
    emit = [p for p in range(n) if cmax[p] != p]
    fixed = set(emit[:k])
    cur = [None] * n
    for p in fixed:
        cur[p] = to[p]
    for r in range(n):
        if r in fixed:
            continue
        s = rho[r]
        while s in fixed:
            s = rho[s]
        cur[s] = frm[rho[r]]
    return cur, len(emit)


def test_exhaustive_small(orc):
    rng = np.random.default_rng(0)
    for n in range(1, 6):
        for frm in itertools.permutations(range(n)):
            to = list(rng.permutation(n))
            v = orc.bss(frm, to)
            for k in range(len(v) + 1):
                got, L = partial_by_cycles(list(frm), to, k)
                assert L == len(v)
                assert got == orc.apply_swaps(frm, v, k).tolist(), (frm, to, k)


def test_random_larger(orc):
    rng = np.random.default_rng(1)
    for _ in range(200):
        n = int(rng.integers(6, 150))
        frm, to = list(rng.permutation(n)), list(rng.permutation(n))
        v = orc.bss(frm, to)
        for k in sorted({0, 1, len(v) // 3, len(v) // 2, max(len(v) - 1, 0), len(v)}):
            assert partial_by_cycles(frm, to, k)[0] == orc.apply_swaps(frm, v, k).tolist()
