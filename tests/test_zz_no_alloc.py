"""The distance builder's entry point without a workspace argument (its
workspace is the library's static device buffer) gives, through the C ABI,
exactly the matrices of the entry point with a caller workspace: two calls
in a row, the second on a smaller scene, so the second reuses a buffer that
still holds the first call's contents."""
import numpy as np
import pytest

from paper_1706_04399_amd import scenes
from parity import note

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1706_04399_amd import dpso
    dpso.lib()
    return dpso


def test_noalloc_matches_workspace_entry_point(dp):
    cases = [("facade1000", scenes.workload(3)[0]), ("random130_10boxes",
             scenes.random_points(130, seed=21, n_boxes=10)), ("facade30", scenes.workload(1)[0])]
    for name, sc in cases:
        note(f"build_dist_noalloc {name} n={sc.n} boxes={len(sc.boxes_mm)}")
        ref = dp.build_dist(sc).cpu().numpy()
        got = dp.build_dist_noalloc(sc).cpu().numpy()
        assert got.shape == ref.shape == (sc.n, sc.n)
        assert np.array_equal(got, ref), name


def test_noalloc_unreachable_pair_after_larger_call(dp):
    note("build_dist_noalloc sealed viewpoint after facade1000")
    dp.build_dist_noalloc(scenes.workload(3)[0])
    slabs = [(-3000, -3000, -3000, -2000, 3000, 3000), (2000, -3000, -3000, 3000, 3000, 3000),
             (-3000, -3000, -3000, 3000, -2000, 3000), (-3000, 2000, -3000, 3000, 3000, 3000),
             (-3000, -3000, -3000, 3000, 3000, -2000), (-3000, -3000, 2000, 3000, 3000, 3000)]
    sc = scenes.Scene(np.array([(0, 0, 0), (10000, 0, 0), (10000, 5000, 0)]), np.array(slabs), 0)
    got = dp.build_dist_noalloc(sc).cpu().numpy()
    assert np.array_equal(got, dp.build_dist(sc).cpu().numpy())
    assert got[0, 1] == dp.D_INF


def test_noalloc_rejects_scene_beyond_static_buffer(dp):
    note("build_dist_noalloc oversized scene (rejected on the host)")
    sc = scenes.random_points(2000, seed=4, n_boxes=120)     # 2960 graph nodes
    with pytest.raises(dp.DpsoError) as ei:
        dp.build_dist_noalloc(sc)
    assert ei.value.status == dp.E_NOMEM
