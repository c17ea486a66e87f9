"""Viewpoint selection (Sect. 2.1): the oracle pinned by a hand-worked wall,
closed forms and a coverage property; the library's host implementation
matches the oracle exactly (no GPU needed)."""
import math

import numpy as np
import pytest

from conftest import golden_lines
from oracle import viewpoints as ov

CAM = dict(resolution_px=4000, feature_um=1000, overlap_permille=300, focal_um=35000, sensor_um=36000)


def _golden():
    g = {row[0]: [int(v) for v in row[1:]] for row in golden_lines("viewpoints_wall.txt")}
    cam = dict(zip(("resolution_px", "feature_um", "overlap_permille", "focal_um", "sensor_um"), g["camera"]))
    s = g["surface"]
    surf = dict(lo_mm=s[0:3], hi_mm=s[3:6], normal_axis=s[6], normal_sign=s[7])
    return g, cam, surf


def test_oracle_worked_wall():
    g, cam, surf = _golden()
    assert ov.camera_lengths(cam) == (2_000_000, 1_400_000, 1_944_444)
    v = ov.viewpoints([surf], cam)
    assert len(v) == g["count"][0]
    assert v[0] == g["first"] and v[1] == g["second"] and v[-1] == g["last"]


@pytest.mark.parametrize("w,h,overlap", [(10_000, 6_000, 300), (1_400, 2_800, 300), (1, 1, 0),
                                         (0, 5_000, 500), (33_333, 7_777, 123)])
def test_oracle_grid_closed_forms(w, h, overlap):
    cam = dict(CAM, overlap_permille=overlap)
    a, p, d = ov.camera_lengths(cam)
    surf = dict(lo_mm=[100, 200, 0], hi_mm=[100 + w, 200 + h, 0], normal_axis=2, normal_sign=1)
    v = np.array(ov.viewpoints([surf], cam))
    nx, ny = max(1, math.ceil(w * 1000 / p)), max(1, math.ceil(h * 1000 / p))
    assert len(v) == nx * ny
    assert (v[:, 2] == math.floor(d / 1000 + 0.5)).all()                  # viewed from +z, plane z = 0
    xs, ys = sorted(set(v[:, 0])), sorted(set(v[:, 1]))
    assert len(xs) == nx and len(ys) == ny
    # consecutive centres one cell apart (to the mm rounding)
    assert all(abs((b - a_) * 1000 - p) <= 1000 for a_, b in zip(xs, xs[1:]))
    # every point of the surface lies within half a cell of a viewpoint's foot
    rng = np.random.default_rng(w + h)
    for _ in range(200):
        q = np.array([100 + rng.integers(0, w + 1), 200 + rng.integers(0, h + 1)])
        cheb = np.abs(v[:, :2] - q).max(axis=1).min()
        assert cheb * 1000 <= p / 2 + 1000


def test_oracle_viewing_side_and_axes():
    surf = dict(lo_mm=[5_000, -300, 0], hi_mm=[5_000, 2_500, 4_000], normal_axis=0, normal_sign=-1)
    a, p, d = ov.camera_lengths(CAM)
    v = np.array(ov.viewpoints([surf], CAM))
    assert (v[:, 0] == math.floor(5_000 - d / 1000 + 0.5)).all()          # viewed from -x
    assert v[0, 1] == round(-300 + p / 2000) and v[1, 1] == v[0, 1]       # y outer, z inner
    assert v[1, 2] - v[0, 2] == p // 1000


def _random_case(rng):
    cam = dict(resolution_px=int(rng.integers(100, 9000)), feature_um=int(rng.integers(10, 3000)),
               overlap_permille=int(rng.integers(0, 1000)), focal_um=int(rng.integers(1000, 100000)),
               sensor_um=int(rng.integers(1000, 50000)))
    surfs = []
    for _ in range(int(rng.integers(1, 5))):
        ax = int(rng.integers(0, 3))
        lo = rng.integers(-50_000, 50_000, size=3)
        hi = lo + rng.integers(0, 20_000, size=3)
        hi[ax] = lo[ax]
        surfs.append(dict(lo_mm=[int(c) for c in lo], hi_mm=[int(c) for c in hi], normal_axis=ax,
                          normal_sign=int(rng.choice([-1, 1]))))
    return surfs, cam


def test_library_matches_oracle():
    from paper_1706_04399_amd import dpso
    rng = np.random.default_rng(2024)
    checked = 0
    for _ in range(300):
        surfs, cam = _random_case(rng)
        p = ov.camera_lengths(cam)[1]
        if p < 1:
            continue
        count = 0
        for f in surfs:
            cells = [max(1, math.ceil((f["hi_mm"][k] - f["lo_mm"][k]) * 1000 / p))
                     for k in range(3) if k != f["normal_axis"]]
            count += cells[0] * cells[1]
        if count > 3_000:
            continue
        ref = ov.viewpoints(surfs, cam)
        got = dpso.viewpoints(surfs, cam)
        assert got.tolist() == ref
        checked += 1
    assert checked > 100
    g, cam, surf = _golden()
    assert dpso.viewpoints([surf], cam).tolist() == ov.viewpoints([surf], cam)


def test_library_rejects_bad_input():
    from paper_1706_04399_amd import dpso
    good = dict(lo_mm=[0, 0, 0], hi_mm=[1000, 0, 1000], normal_axis=1, normal_sign=1)
    for bad_s, bad_c in [(dict(good, normal_axis=3), CAM), (dict(good, normal_sign=0), CAM),
                         (dict(good, hi_mm=[1000, 5, 1000]), CAM), (dict(good, hi_mm=[-1, 0, 1000]), CAM),
                         (good, dict(CAM, overlap_permille=1000)), (good, dict(CAM, sensor_um=0)),
                         (good, dict(CAM, resolution_px=1, feature_um=1))]:
        with pytest.raises(dpso.DpsoError) as ei:
            dpso.viewpoints([bad_s], bad_c)
        assert ei.value.status == dpso.E_INVAL
