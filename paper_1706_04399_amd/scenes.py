"""Seeded synthetic inspection scenes: viewpoints and box obstacles in integer mm.

This module only draws inputs. It holds none of the method's arithmetic (no
distances, tours or swarm steps), so both the CPU oracle and the HIP library
consume the same scene without sharing any computation.

The paper measures on two laser-scanned datasets (an office-building floor and
a bridge section, Sect. 4) that are not available. The generators below stand in
for them: viewpoints lie on working surfaces at a fixed standoff from the
inspected planes, as the viewpoint-selection step of Sect. 2.1 produces (a grid
of cells projected onto a parallel plane), and obstacles are axis-aligned boxes
that the UAV must clear by an inflation radius (Sect. 2.2).

Every generator uses ``numpy.random.default_rng(seed)`` and returns a
:class:`Scene` whose arrays are contiguous int32.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

CLEARANCE_MM = 500


@dataclasses.dataclass
class Scene:
    vp_mm: np.ndarray        # int32 [n, 3]  viewpoint positions x, y, z
    boxes_mm: np.ndarray     # int32 [b, 6]  lo x, lo y, lo z, hi x, hi y, hi z
    clearance_mm: int        # inflation radius applied to every box
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.vp_mm.shape[0])

    def __post_init__(self):
        self.vp_mm = np.ascontiguousarray(self.vp_mm, dtype=np.int32).reshape(-1, 3)
        self.boxes_mm = np.ascontiguousarray(self.boxes_mm, dtype=np.int32).reshape(-1, 6)
        self.clearance_mm = int(self.clearance_mm)


def _inside_inflated(p, boxes, c) -> bool:
    for b in boxes:
        if all(b[a] - c < p[a] < b[a + 3] + c for a in range(3)):
            return True
    return False


def _box_around(rng, centre, side_lo, side_hi):
    """Box with integer sides drawn per axis from [side_lo[a], side_hi[a]]."""
    lo, hi = [], []
    for a in range(3):
        s = int(rng.integers(side_lo[a], side_hi[a] + 1))
        l0 = int(centre[a]) - s // 2
        lo.append(l0)
        hi.append(l0 + s)
    return lo + hi


def _draw_points(rng, n, sampler, boxes, clearance, seen=None):
    """Draw n distinct points with ``sampler(rng)``, redrawing any point that
    falls inside an inflated box or repeats an earlier one."""
    seen = set() if seen is None else seen
    pts = []
    while len(pts) < n:
        p = tuple(int(v) for v in sampler(rng))
        if p in seen or _inside_inflated(p, boxes, clearance):
            continue
        seen.add(p)
        pts.append(p)
    return pts


def facade(n, width_mm, height_mm, n_boxes, seed, standoff_mm=2000,
           clearance_mm=CLEARANCE_MM, name="facade") -> Scene:
    """Wall in the plane y=0 spanning x in [0, width], z in [0, height].

    Viewpoints are uniform on the working plane y = standoff. Boxes are placed
    first, centred in the flight layer (y within 500 mm of the working plane)
    so that they block straight flights, with sides drawn from [500, 2000] mm
    in x and z and [500, 1500] mm in y.
    """
    rng = np.random.default_rng(seed)
    boxes = []
    for _ in range(n_boxes):
        centre = (rng.integers(0, width_mm + 1),
                  rng.integers(standoff_mm - 500, standoff_mm + 501),
                  rng.integers(0, height_mm + 1))
        boxes.append(_box_around(rng, centre, (500, 500, 500), (2000, 1500, 2000)))
    pts = _draw_points(
        rng, n,
        lambda r: (r.integers(0, width_mm + 1), standoff_mm, r.integers(0, height_mm + 1)),
        boxes, clearance_mm)
    return Scene(np.array(pts, np.int32), np.array(boxes, np.int32).reshape(-1, 6),
                 clearance_mm, name)


def bridge(n, length_mm, n_boxes, seed, depth_mm=8000, web_mm=8000,
           standoff_mm=2000, jitter_mm=200, clearance_mm=CLEARANCE_MM,
           name="bridge") -> Scene:
    """Bridge girder: two vertical webs (planes y=0 and y=depth, z in
    [0, web]) and a soffit (plane z=0, y in [0, depth]), all of length
    ``length_mm`` along x.

    Each plane gets a grid of cells (4 across its short side, ``ceil(n/12)+1``
    along the span); cell centres are projected to the working plane at
    ``standoff_mm`` along the outward normal and jittered by +-``jitter_mm``.
    Cells are taken in a seeded random order until n viewpoints are placed;
    a cell whose jittered centre keeps landing inside an obstacle is skipped. The girder body is
    box 0 (the UAV cannot fly through the structure); the remaining
    ``n_boxes`` boxes (sides 300..1000 mm, bearings and pipes) sit in the
    viewpoint layers.
    """
    rng = np.random.default_rng(seed)
    boxes = [[0, 0, 0, length_mm, depth_mm, web_mm]]
    layers = [  # (fixed axis, fixed value, axis u (span), axis v (across))
        (1, -standoff_mm, 0, 2, web_mm),
        (1, depth_mm + standoff_mm, 0, 2, web_mm),
        (2, -standoff_mm, 0, 1, depth_mm),
    ]
    for k in range(n_boxes):
        fa, fv, ua, va, vext = layers[k % 3]
        centre = [0, 0, 0]
        centre[fa] = fv
        centre[ua] = int(rng.integers(0, length_mm + 1))
        centre[va] = int(rng.integers(0, vext + 1))
        boxes.append(_box_around(rng, centre, (300, 300, 300), (1000, 1000, 1000)))
    per_plane = math.ceil(n / 3)
    cols = max(1, math.ceil(per_plane / 4)) + 1      # one spare column per plane
    cells = []
    for fa, fv, ua, va, vext in layers:
        for r in range(4):
            for c in range(cols):
                p = [0, 0, 0]
                p[fa] = fv
                p[ua] = (2 * c + 1) * length_mm // (2 * cols)
                p[va] = (2 * r + 1) * vext // 8
                cells.append((fa, p))
    pts, seen = [], set()
    for idx in rng.permutation(len(cells)):
        if len(pts) == n:
            break
        fa, base = cells[idx]
        for _ in range(50):          # a cell buried in an obstacle is skipped
            q = list(base)
            for a in range(3):
                if a != fa:
                    q[a] += int(rng.integers(-jitter_mm, jitter_mm + 1))
            q = tuple(q)
            if q not in seen and not _inside_inflated(q, boxes, clearance_mm):
                seen.add(q)
                pts.append(q)
                break
    if len(pts) < n:
        raise ValueError("bridge: obstacles leave fewer free cells than viewpoints")
    return Scene(np.array(pts, np.int32), np.array(boxes, np.int32), clearance_mm, name)


def circle(n, radius_mm=100_000) -> Scene:
    """n points on a circle in the plane z=0, rounded to integer mm; no boxes."""
    th = 2.0 * np.pi * np.arange(n) / n
    pts = np.stack([np.rint(radius_mm * np.cos(th)), np.rint(radius_mm * np.sin(th)),
                    np.zeros(n)], axis=1)
    return Scene(pts.astype(np.int32), np.zeros((0, 6), np.int32), 0, f"circle{n}")


def grid(cols, rows, spacing_mm=1000) -> Scene:
    """cols x rows grid in the plane z=0 with row-major labels; no boxes."""
    pts = [(c * spacing_mm, r * spacing_mm, 0) for r in range(rows) for c in range(cols)]
    return Scene(np.array(pts, np.int32), np.zeros((0, 6), np.int32), 0,
                 f"grid{cols}x{rows}")


def line(xs_mm) -> Scene:
    """Points on the x axis at the given integer positions; no boxes."""
    pts = [(int(x), 0, 0) for x in xs_mm]
    return Scene(np.array(pts, np.int32), np.zeros((0, 6), np.int32), 0, "line")


def serpentine(walls: int, gap_mm: int = 2_000_000, half_mm: int = 65_000_000) -> Scene:
    """Three viewpoints on the x axis near the ends of a cube of half-edge
    `half_mm`, separated by `walls` thin walls (planes of constant x) that span
    the whole cube in z and leave a gap of `gap_mm` at alternately the high and
    the low end of y, so a flight between the ends weaves through every gap
    (paths far longer than the cube, for the range limits of the costs)."""
    xs = np.linspace(-half_mm + 5_000_000, half_mm - 5_000_000, walls).astype(np.int64)
    far = half_mm + 1_000_000
    boxes = []
    for k, x in enumerate(xs):
        if k % 2 == 0:
            boxes.append((x - 1000, -far, -far, x + 1000, half_mm - gap_mm, far))
        else:
            boxes.append((x - 1000, -half_mm + gap_mm, -far, x + 1000, far, far))
    vp = [(-half_mm, 0, 0), (half_mm, 0, 0), (-half_mm, 1000, 0)]
    return Scene(np.array(vp, np.int32), np.array(boxes, np.int32).reshape(-1, 6), 0, f"serpentine{walls}")


def moved_box(scene: Scene, seed: int, shift_mm: int = 2000, tries: int = 32) -> Scene:
    """The scene with one obstacle moved (a changed site for re-planning): box
    k = seed mod b is shifted by a random offset of up to `shift_mm` per axis,
    redrawn while a viewpoint would fall inside its inflated volume; after
    `tries` failed draws the scene is returned unchanged. Scenes without
    boxes are returned unchanged."""
    b = len(scene.boxes_mm)
    if b == 0:
        return scene
    rng = np.random.default_rng(seed)
    k = seed % b
    boxes = [tuple(int(v) for v in row) for row in scene.boxes_mm]
    for _ in range(tries):
        d = rng.integers(-shift_mm, shift_mm + 1, size=3)
        moved = tuple(boxes[k][a] + int(d[a % 3]) for a in range(6))
        if not any(_inside_inflated(tuple(int(v) for v in p), [moved], scene.clearance_mm)
                   for p in scene.vp_mm):
            boxes[k] = moved
            return Scene(scene.vp_mm.copy(), np.array(boxes, np.int32), scene.clearance_mm,
                         scene.name)
    return scene


def random_points(n, seed, extent_mm=20_000, n_boxes=0, clearance_mm=CLEARANCE_MM) -> Scene:
    """Uniform points in a cube, optionally with random boxes (sides 500..3000)."""
    rng = np.random.default_rng(seed)
    boxes = []
    for _ in range(n_boxes):
        centre = rng.integers(0, extent_mm + 1, size=3)
        boxes.append(_box_around(rng, centre, (500, 500, 500), (3000, 3000, 3000)))
    pts = _draw_points(rng, n, lambda r: r.integers(0, extent_mm + 1, size=3), boxes,
                       clearance_mm)
    return Scene(np.array(pts, np.int32), np.array(boxes, np.int32).reshape(-1, 6),
                 clearance_mm, f"random{n}")


def random_dist(n, seed, max_mm=100_000) -> np.ndarray:
    """Symmetric random int32 matrix with zero diagonal (not a metric)."""
    rng = np.random.default_rng(seed)
    a = rng.integers(1, max_mm, size=(n, n), dtype=np.int64)
    d = np.triu(a, 1)
    d = d + d.T
    return np.ascontiguousarray(d, dtype=np.int32)


# --------------------------------------------------------------------------
# The workloads. Swarm parameters are carried as plain numbers; the Q16 fixed
# point encoding (value * 65536) is how both implementations receive them.
# --------------------------------------------------------------------------

Q16 = 65536
EE_OFF, EE_ON_STALL, EE_ALWAYS = 0, 1, 2
NB_TWO_OPT, NB_NODE_SWAP = 0, 1          # edge-exchange neighbourhoods


def swarm_params(swarm_size, max_generations, *, w=0.7, phi1=1.5, phi2=1.5,
                 mutation_period=3, ee_trigger=EE_ON_STALL, ee_max_moves=1,
                 stall_limit=0, det_permille=100, seed=0, instance=0,
                 ee_neighbourhood=NB_TWO_OPT, mutation_swaps=0, velocity_cap=0) -> dict:
    return dict(swarm_size=int(swarm_size), max_generations=int(max_generations),
                w_q16=int(round(w * Q16)), phi1_q16=int(round(phi1 * Q16)),
                phi2_q16=int(round(phi2 * Q16)), mutation_period=int(mutation_period),
                ee_trigger=int(ee_trigger), ee_max_moves=int(ee_max_moves),
                stall_limit=int(stall_limit), det_permille=int(det_permille),
                seed=int(seed), instance=int(instance),
                ee_neighbourhood=int(ee_neighbourhood), mutation_swaps=int(mutation_swaps),
                velocity_cap=int(velocity_cap))


def workload(k: int):
    """(scene, params) of the single-instance workloads.

    1: 30 viewpoints on a 10 x 6 m facade, 2 boxes; swarm 64, 200 generations.
    2: 200 viewpoints on a 40 m bridge girder (3 planes), 6 boxes; swarm 1024,
       1000 generations.
    3: 1000 viewpoints on a 100 x 30 m facade, 20 boxes; swarm 4096, 2000
       generations, edge exchange on every generation.
    """
    if k == 1:
        return (facade(30, 10_000, 6_000, 2, seed=0, name="facade30"),
                swarm_params(64, 200))
    if k == 2:
        return (bridge(200, 40_000, 6, seed=0, name="bridge200"),
                swarm_params(1024, 1000))
    if k == 3:
        return (facade(1000, 100_000, 30_000, 20, seed=0, name="facade1000"),
                swarm_params(4096, 2000, ee_trigger=EE_ALWAYS))
    raise ValueError(f"no single-instance workload {k}")


def batch_instance(i: int) -> Scene:
    """Instance i of the batched workload: n log-uniform in [20, 500] (seed
    1000+i); even i are facades of area 3 m^2 per viewpoint and aspect 10:3
    with round(n/50) boxes, odd i are bridges of length 40 m * n/200 with
    max(1, round(6n/200)) boxes."""
    rng = np.random.default_rng(1000 + i)
    n = int(round(math.exp(rng.uniform(math.log(20), math.log(500)))))
    if i % 2 == 0:
        h = int(round(math.sqrt(0.9e6 * n)))
        w = int(round(h * 10 / 3))
        return facade(n, w, h, int(round(n / 50)), seed=1000 + i, name=f"b{i}facade{n}")
    length = int(round(40_000 * n / 200))
    return bridge(n, length, max(1, int(round(6 * n / 200))), seed=1000 + i,
                  name=f"b{i}bridge{n}")
