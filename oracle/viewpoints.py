"""Viewpoint selection (Sect. 2.1), plain and exact.

TEST INFRASTRUCTURE: used only by the test suite. Written from the paper's
formulas with exact rational arithmetic, independently of the library:

  footprint           a = r_c s_f / 2                      (eq. fov)
  primitive (cell)    p = (1 - o_p) a                      (eq. premitive)
  working distance    d = a f / s_s                        (eq. cameraDistance)

Readings (the same the library documents): lengths in um are truncated to
whole um after each formula; a surface is an axis-aligned rectangle covered
by cells of size p from its low corner, max(1, ceil(L / p)) per in-plane axis;
a viewpoint is a cell centre moved d to the viewing side, rounded half up to
whole mm; output surface by surface, lower in-plane axis outer.
"""
from fractions import Fraction
import math


def camera_lengths(camera):
    """(a, p, d) in whole um."""
    a = math.floor(Fraction(camera["resolution_px"] * camera["feature_um"], 2))
    p = math.floor(Fraction(1000 - camera["overlap_permille"], 1000) * a)
    d = math.floor(Fraction(a * camera["focal_um"], camera["sensor_um"]))
    return a, p, d


def round_half_up(x: Fraction) -> int:
    return math.floor(x + Fraction(1, 2))


def viewpoints(surfaces, camera):
    a, p, d = camera_lengths(camera)
    out = []
    for f in surfaces:
        ax = f["normal_axis"]
        plane = [k for k in range(3) if k != ax]
        counts = []
        for k in plane:
            length_um = (f["hi_mm"][k] - f["lo_mm"][k]) * 1000
            counts.append(max(1, math.ceil(Fraction(length_um, p))))
        normal_mm = round_half_up(Fraction(f["lo_mm"][ax] * 1000 + f["normal_sign"] * d, 1000))
        for i in range(counts[0]):
            for j in range(counts[1]):
                v = [0, 0, 0]
                v[ax] = normal_mm
                for k, idx in zip(plane, (i, j)):
                    centre_um = f["lo_mm"][k] * 1000 + (idx + Fraction(1, 2)) * p
                    v[k] = round_half_up(centre_um / 1000)
                out.append(v)
    return out
