"""Fisher-Yates without replaying the exchanges.

The HIP shuffle (initial tours, mutation) does not run the n - 1 exchanges
one after another. It relies on this description of the shuffle of the
identity with exchange targets j_i (i = n-1 down to 1, j_i <= i), checked
here against the oracle's serial shuffle on the same random stream:

  Step i fixes place i for good, with what place j_i holds just before it.
  With T(q) = {i > q : j_i = q} and W(i) = what place i holds just before
  step i (place 0: at the end),
    W(i)    = W(min T(i)), or i when T(i) is empty;
    tour[i] = W(i) when j_i = i or i = 0; otherwise W(u) with u the smallest
              member of T(j_i) above i, or j_i when there is none.
"""
import numpy as np
import pytest

import oracle


def shuffle_by_chains(j):
    n = len(j)
    members = {}
    for i in range(1, n):
        if j[i] < i:
            members.setdefault(j[i], []).append(i)
    W = [None] * n
    for i in range(n - 1, -1, -1):          # min T(i) > i is resolved first
        t = members.get(i)
        W[i] = W[min(t)] if t else i
    out = []
    for i in range(n):
        if i == 0 or j[i] == i:
            out.append(W[i])
            continue
        above = [u for u in members[j[i]] if u > i]
        out.append(W[min(above)] if above else j[i])
    return out


def targets(n, seed, inst, p, t, purpose):
    """j_i of the oracle's stream: step i uses draw n-1-i, scaled to [0, i]."""
    d = oracle.draws(seed, inst, p, t, purpose, max(n - 1, 0)).astype(np.uint64)
    j = [0] * n
    for i in range(1, n):
        j[i] = int((d[n - 1 - i] * np.uint64(i + 1)) >> np.uint64(32))
    return j


@pytest.mark.parametrize("n", [1, 2, 3, 5, 17, 64, 65, 200, 1000, 4096])
def test_chains_match_serial_shuffle(n):
    for p in range(6 if n <= 200 else 2):
        for purpose in (oracle.PURPOSE_INIT, oracle.PURPOSE_MUT):
            t = 0 if purpose == oracle.PURPOSE_INIT else 3 * (p + 1)
            ref = oracle.fisher_yates(n, 11, n, p, t, purpose)
            got = shuffle_by_chains(targets(n, 11, n, p, t, purpose))
            assert list(ref) == got, (n, p, purpose)


def test_chains_match_every_target_sequence_small():
    """Every sequence j_1..j_{n-1} with j_i <= i, n <= 6 (720 sequences)."""
    import itertools
    for n in range(1, 7):
        for tail in itertools.product(*[range(i + 1) for i in range(1, n)]):
            j = [0, *tail]
            a = list(range(n))
            for i in range(n - 1, 0, -1):
                a[i], a[j[i]] = a[j[i]], a[i]
            assert shuffle_by_chains(j) == a, j
