"""Pins of the oracle's voxel-grid planner (Sect. 2.2): the grid's occupancy
in closed form, free-space costs in closed form (weighted Manhattan: a
diagonal step costs as much as the axis steps it replaces), brute-force
all-pairs shortest paths over every voxel on tiny grids, enclosure, and the
metric invariants."""
import itertools

import numpy as np
import pytest

from paper_1706_04399_amd import scenes

D_INF = (1 << 28) - 1


def scene(vp, boxes=(), clearance=0):
    return scenes.Scene(np.array(vp, np.int32).reshape(-1, 3),
                        np.array(boxes, np.int32).reshape(-1, 6), clearance, "voxel")


def grid_index(sc, s):
    """Voxel of each viewpoint, from the grid's definition (origin = smallest
    coordinate of viewpoints and box corners minus one voxel)."""
    pts = [sc.vp_mm] + ([sc.boxes_mm[:, :3], sc.boxes_mm[:, 3:]] if len(sc.boxes_mm) else [])
    origin = np.concatenate(pts).min(axis=0).astype(np.int64) - s
    return (sc.vp_mm.astype(np.int64) - origin) // s


def test_occupancy_of_box_interiors(orc):
    # centres at origin + (i + 1/2) s; a box covers the centres strictly inside it
    sc = scene([[0, 0, 0]], [[1000, 1000, 1000, 4000, 3000, 2000]])
    dims, origin, occ = orc.voxel_grid(sc, 500)
    assert list(origin) == [-500, -500, -500]
    cx = origin[0] + (np.arange(dims[0]) + 0.5) * 500
    cy = origin[1] + (np.arange(dims[1]) + 0.5) * 500
    cz = origin[2] + (np.arange(dims[2]) + 0.5) * 500
    inside = ((cx > 1000) & (cx < 4000)).sum() * ((cy > 1000) & (cy < 3000)).sum() * \
             ((cz > 1000) & (cz < 2000)).sum()
    assert occ.sum() == inside == 6 * 4 * 2


def test_inflation_is_a_sphere_of_voxels(orc):
    """One occupied voxel, inflated by 2 voxel edges: the 33 voxels whose
    centres are within 2 edges (offsets with squared length <= 4)."""
    s = 1000
    sc = scene([[0, 0, 0], [20000, 20000, 20000]], [[10100, 10100, 10100, 10900, 10900, 10900]], 2 * s)
    dims, origin, occ = orc.voxel_grid(sc, s)
    assert occ.sum() == 33
    k, j, i = np.argwhere(occ).T
    c = np.array([i, j, k]).T
    ctr = np.round(c.mean(axis=0)).astype(int)
    assert (((c - ctr) ** 2).sum(axis=1) <= 4).all()


@pytest.mark.parametrize("w", [(1, 1, 1), (3, 1, 2), (5, 7, 2)])
def test_free_space_is_weighted_manhattan(orc, w):
    rng = np.random.default_rng(sum(w))
    vp = rng.integers(0, 12_000, size=(9, 3))
    sc = scene(vp)
    s = 700
    D = orc.build_dist_voxel(sc, s, w)
    idx = grid_index(sc, s)
    expect = s * (np.abs(idx[:, None, :] - idx[None, :, :]) * np.array(w)).sum(axis=2)
    assert (D == expect).all()


def brute_force(dims, occ, src_vox, weights):
    """All-pairs over every voxel (Floyd-Warshall) with only free voxels as
    intermediates; the ends may be occupied."""
    nx, ny, nz = (int(d) for d in dims)
    G = nx * ny * nz
    INF = 1 << 50
    d = np.full((G, G), INF, np.int64)
    np.fill_diagonal(d, 0)
    coords = [(i, j, k) for k in range(nz) for j in range(ny) for i in range(nx)]
    for v, (i, j, k) in enumerate(coords):
        for di, dj, dk in itertools.product((-1, 0, 1), repeat=3):
            if (di, dj, dk) == (0, 0, 0):
                continue
            a, b, c = i + di, j + dj, k + dk
            if 0 <= a < nx and 0 <= b < ny and 0 <= c < nz:
                u = a + nx * (b + ny * c)
                d[v, u] = weights[0] * di * di + weights[1] * dj * dj + weights[2] * dk * dk
    free = occ.reshape(-1) == 0
    for k in np.flatnonzero(free):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    sub = d[np.ix_(src_vox, src_vox)]
    return sub, INF


@pytest.mark.parametrize("seed", range(6))
def test_tiny_grids_match_brute_force(orc, seed):
    rng = np.random.default_rng(seed)
    s = 1000
    vp = rng.integers(0, 5000, size=(6, 3))
    vp[:, 2] = rng.integers(0, 2500, size=6)
    boxes = []
    for _ in range(int(rng.integers(1, 4))):
        lo = rng.integers(0, 4000, size=3)
        hi = lo + rng.integers(800, 3000, size=3)
        boxes.append(np.concatenate([lo, hi]))
    w = tuple(int(x) for x in rng.integers(1, 4, size=3))
    sc = scene(vp, boxes, clearance=int(rng.choice([0, 600])))
    dims, origin, occ = orc.voxel_grid(sc, s)
    assert np.prod(dims) <= 1000
    idx = (sc.vp_mm.astype(np.int64) - origin) // s
    vox = idx[:, 0] + dims[0] * (idx[:, 1] + dims[1] * idx[:, 2])
    ref, INF = brute_force(dims, occ, vox, w)
    D = orc.build_dist_voxel(sc, s, w)
    expect = np.where(ref >= INF, D_INF, ref * s)
    assert (D == expect).all(), (seed, w)


def test_enclosed_viewpoint_is_unreachable(orc):
    # a viewpoint deep inside a box: every neighbour of its voxel is occupied
    sc = scene([[0, 0, 0], [10000, 10000, 10000]], [[8000, 8000, 8000, 12000, 12000, 12000]])
    D = orc.build_dist_voxel(sc, 1000)
    assert D[0, 1] == D[1, 0] == D_INF and D[0, 0] == D[1, 1] == 0


def test_metric_invariants_with_boxes(orc):
    sc = scenes.random_points(30, seed=7, extent_mm=15_000, n_boxes=4)
    s = 500
    D = orc.build_dist_voxel(sc, s, (2, 1, 3)).astype(np.int64)
    idx = grid_index(sc, s)
    assert (D == D.T).all() and (np.diag(D) == 0).all()
    fin = D < D_INF
    lower = s * (np.abs(idx[:, None, :] - idx[None, :, :]) * np.array([2, 1, 3])).sum(axis=2)
    assert (D[fin] >= lower[fin]).all()
    # through a viewpoint whose voxel is free (an occupied one is an end only)
    dims, origin, occ = orc.voxel_grid(sc, s)
    for k in range(len(D)):
        if occ[idx[k, 2], idx[k, 1], idx[k, 0]]:
            continue
        via = D[:, k:k + 1] + D[k:k + 1, :]
        ok = fin[:, k:k + 1] & fin[k:k + 1, :]
        assert (D[ok] <= via[ok]).all()


def test_bad_parameters_are_rejected(orc):
    sc = scene([[0, 0, 0], [1000, 0, 0]])
    for s, w in [(0, (1, 1, 1)), (100, (0, 1, 1)), (100, (1, -1, 1))]:
        with pytest.raises(ValueError):
            orc.build_dist_voxel(sc, s, w)
