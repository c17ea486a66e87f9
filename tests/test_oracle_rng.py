"""Pins of the oracle's random streams against numpy's Philox4x64-10.

numpy.random.Philox is an independent implementation of the same published
generator; it advances its 256-bit counter before producing a block, so the
block for counter c is the first output of numpy's generator started at c - 1.
"""
import numpy as np
import pytest


def numpy_block(seed, inst, ctr):
    c = sum(int(v) << (64 * i) for i, v in enumerate(ctr))
    c = (c - 1) % (1 << 256)
    return np.random.Philox(key=[seed, inst], counter=c).random_raw(4).astype(np.uint64)


@pytest.mark.parametrize("seed,inst,ctr", [
    (0, 0, [0, 0, 0, 0]), (0, 0, [0, 1, 1, 1]), (12345, 7, [3, 17, 200, 2]),
    (2**64 - 1, 2**63, [2**64 - 1, 2**64 - 1, 5, 1]), (42, 0, [7, 4095, 1999, 0]),
])
def test_philox_block_matches_numpy(orc, seed, inst, ctr):
    assert (orc.philox_block(seed, inst, ctr) == numpy_block(seed, inst, ctr)).all()


def test_draw_stream_layout(orc):
    """Draw 8b + 2m is the low half of word m of block b, draw 8b+2m+1 the high half."""
    seed, inst, p, t, purpose = 99, 3, 11, 5, 1
    d = orc.draws(seed, inst, p, t, purpose, 40)
    words = np.concatenate([numpy_block(seed, inst, [b, p, t, purpose]) for b in range(5)])
    expect = np.empty(40, np.uint64)
    expect[0::2] = words & np.uint64(0xFFFFFFFF)
    expect[1::2] = words >> np.uint64(32)
    assert (d.astype(np.uint64) == expect).all()


def _numpy_fisher_yates(n, seed, inst, p, t, purpose):
    """Textbook Fisher-Yates driven by numpy's Philox words."""
    nblk = (n + 7) // 8 + 1
    words = np.concatenate([numpy_block(seed, inst, [b, p, t, purpose]) for b in range(nblk)])
    draws = []
    for w in words:
        draws += [int(w) & 0xFFFFFFFF, int(w) >> 32]
    x = list(range(n))
    k = 0
    for i in range(n - 1, 0, -1):
        j = (draws[k] * (i + 1)) >> 32
        k += 1
        x[i], x[j] = x[j], x[i]
    return np.array(x, np.int32)


@pytest.mark.parametrize("n", [1, 2, 3, 9, 30, 257])
@pytest.mark.parametrize("purpose", [0, 2])
def test_fisher_yates_matches_numpy_stream(orc, n, purpose):
    got = orc.fisher_yates(n, 5, 1, 3, 7, purpose)
    assert (got == _numpy_fisher_yates(n, 5, 1, 3, 7, purpose)).all()
    assert sorted(got.tolist()) == list(range(n))


def test_fisher_yates_uniform_on_small_n(orc):
    """All 3! orders occur with about equal frequency over many streams."""
    counts = {}
    for p in range(6000):
        key = tuple(orc.fisher_yates(3, 1, 0, p, 0, 0).tolist())
        counts[key] = counts.get(key, 0) + 1
    assert len(counts) == 6
    assert all(800 < c < 1200 for c in counts.values())
