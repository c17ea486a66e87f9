"""The HIP library loads, exports every declared entry point and validates
its arguments on the host (no device work, so these run without a GPU)."""
import ctypes as C
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "dpso.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dpso_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def dp():
    from paper_1706_04399_amd import dpso
    dpso.lib()
    return dpso


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("dpso_build_dist", "dpso_init_nn", "dpso_run", "dpso_get_best"):
        assert required in names


def test_every_declared_symbol_is_exported(dp):
    raw = C.CDLL(dp._LIB_PATH)
    for name in declared_functions():
        assert hasattr(raw, name), name
    assert set(declared_functions()) <= set(dp.EXPORTS)


def test_binding_covers_exports(dp):
    assert set(dp.EXPORTS) == set(declared_functions())


def test_status_codes_match_header(dp):
    src = open(HEADER).read()
    codes = dict(re.findall(r"#define DPSO_(OK|E_[A-Z]+)\s+\(?(-?\d+)\)?", src))
    assert set(codes) == {"OK", "E_INVAL", "E_RANGE", "E_NOMEM", "E_DEVICE", "E_STATE", "E_ADMIT"}
    for name, value in codes.items():
        assert getattr(dp, name) == int(value), name


def test_request_footprint(dp):
    """State plus distance matrix; E_ADMIT above the budget, on the host."""
    p = _params()
    need = dp.state_bytes(30, 64, 200) + 30 * 30 * 4
    assert dp.request_footprint(30, p, need) == (dp.OK, need)
    assert dp.request_footprint(30, p, need - 1) == (dp.E_ADMIT, need)
    assert "budget" in dp.lib().dpso_last_error().decode()
    with pytest.raises(dp.DpsoError) as ei:
        dp.request_footprint(0, p, 1 << 30)
    assert ei.value.status == dp.E_INVAL


def _params(**kw):
    from paper_1706_04399_amd import scenes
    return scenes.swarm_params(64, 200, **kw)


def test_validation_errors(dp):
    dp.validate_params(_params(), 30)
    dp.validate_params(_params(ee_neighbourhood=1, mutation_swaps=65536, velocity_cap=30), 30)
    bad = [(dict(swarm_size=0), 30, dp.E_INVAL), (dict(swarm_size=65537), 30, dp.E_INVAL),
           (dict(w_q16=131073), 30, dp.E_INVAL), (dict(ee_trigger=3), 30, dp.E_INVAL),
           (dict(det_permille=1001), 30, dp.E_INVAL), (dict(mutation_period=-1), 30, dp.E_INVAL),
           (dict(ee_max_moves=-1), 30, dp.E_INVAL), (dict(), 0, dp.E_INVAL),
           (dict(ee_neighbourhood=2), 30, dp.E_INVAL), (dict(ee_neighbourhood=-1), 30, dp.E_INVAL),
           (dict(mutation_swaps=-1), 30, dp.E_INVAL), (dict(mutation_swaps=65537), 30, dp.E_INVAL),
           (dict(velocity_cap=-1), 30, dp.E_INVAL), (dict(velocity_cap=31), 30, dp.E_INVAL),
           (dict(), dp.MAX_N + 1, dp.E_RANGE)]
    for kw, n, code in bad:
        p = _params()
        p.update(kw)
        with pytest.raises(dp.DpsoError) as ei:
            dp.validate_params(p, n)
        assert ei.value.status == code, (kw, n)
        assert dp.lib().dpso_last_error()


def test_state_bytes(dp):
    assert dp.state_bytes(0, 1, 1) == 0
    assert dp.state_bytes(10, 0, 1) == 0
    assert dp.state_bytes(dp.MAX_N + 1, 1, 1) == 0
    a = dp.state_bytes(1000, 4096, 2000)
    # tours, personal bests and velocities dominate: 2 + 2 + 4 bytes per label;
    # n = 1000 adds the 16-bit copy of D the exchange stages (rows padded to 8)
    assert 4096 * 1024 * 8 + 2 * 1000 * 1000 <= a < 4096 * 1024 * 8 + 2 * 1000 * 1000 + (1 << 20)
    b = dp.state_bytes(1001, 4096, 2000)
    assert 4096 * 1024 * 8 + 2 * 1001 * 1008 <= b < 4096 * 1024 * 8 + 2 * 1001 * 1008 + (1 << 20)
    # every 8 <= n <= 1024 holds the 16-bit copy (the tuning table may pick
    # 16-bit rows for any of them); n below 8 and above 1024 hold none
    c = dp.state_bytes(256, 64, 10)
    assert 64 * 256 * 8 + 256 * 256 * 2 <= c < 64 * 256 * 8 + 256 * 256 * 2 + (1 << 16)
    d = dp.state_bytes(255, 64, 10)
    assert d >= 255 * 256 * 2
    assert dp.state_bytes(7, 64, 10) < 64 * 64 * 8 + (1 << 16)
    assert dp.state_bytes(1025, 8, 10) < 8 * 1088 * 8 + (1 << 16)


def test_tuning_table(dp):
    """Buckets, defaults, validation and reset of the per-device table (host only)."""
    dp.tuning_reset()
    # defaults: one wavefront per particle in the move for a lone swarm of at
    # most 128 and for n <= 512 among more than 8192 particles, else 256
    # threads; int32 rows for multiples of 4 up to 256 among at most 1024
    # particles and below n = 8, where no 16-bit copy exists, 16-bit rows for
    # other n up to 1024, one workgroup per particle above
    assert dp.tuning_get(1000, 4096) == {"move_threads": 256, "exchange_rows": dp.ROWS_U16}
    assert dp.tuning_get(30, 64) == {"move_threads": 64, "exchange_rows": dp.ROWS_U16}
    assert dp.tuning_get(200, 1024) == {"move_threads": 256, "exchange_rows": dp.ROWS_I32}
    assert dp.tuning_get(200, 1025) == {"move_threads": 256, "exchange_rows": dp.ROWS_U16}
    assert dp.tuning_get(200, 65536) == {"move_threads": 64, "exchange_rows": dp.ROWS_U16}
    assert dp.tuning_get(384, 65536) == {"move_threads": 64, "exchange_rows": dp.ROWS_U16}
    assert dp.tuning_get(384, 512) == {"move_threads": 256, "exchange_rows": dp.ROWS_U16_QUAD}
    assert dp.tuning_get(384, 513)["exchange_rows"] == dp.ROWS_U16_PAIR
    assert dp.tuning_get(256, 512)["exchange_rows"] == dp.ROWS_I32
    assert dp.tuning_get(255, 512)["exchange_rows"] == dp.ROWS_U16_PAIR
    assert dp.tuning_get(129, 1024)["exchange_rows"] == dp.ROWS_U16_PAIR
    assert dp.tuning_get(128, 1024)["exchange_rows"] == dp.ROWS_I32
    assert dp.tuning_get(127, 1024)["exchange_rows"] == dp.ROWS_U16
    assert dp.tuning_get(384, 1025)["exchange_rows"] == dp.ROWS_U16
    assert dp.tuning_get(516, 65536) == {"move_threads": 256, "exchange_rows": dp.ROWS_U16}
    assert dp.tuning_get(2000, 8) == {"move_threads": 256, "exchange_rows": dp.ROWS_BLOCK}
    assert dp.tuning_get(2000, 64)["move_threads"] == 256     # 64 threads serve n <= 1024 only
    assert dp.tuning_get(5, 8)["exchange_rows"] == dp.ROWS_I32
    assert dp.tuning_get(5, 65536)["exchange_rows"] == dp.ROWS_I32
    try:
        dp.tuning_set(200, 1024, {"move_threads": 128, "exchange_rows": dp.ROWS_U16})
        # the whole bucket: n in (128, 256], 513 .. 1024 particles launched together
        assert dp.tuning_get(129, 513) == {"move_threads": 128, "exchange_rows": dp.ROWS_U16}
        assert dp.tuning_get(256, 1024) == {"move_threads": 128, "exchange_rows": dp.ROWS_U16}
        assert dp.tuning_get(128, 1024)["move_threads"] == 256
        assert dp.tuning_get(200, 1025)["move_threads"] == 256
        assert dp.tuning_get(200, 8193)["move_threads"] == 64
        assert dp.tuning_get(200, 512)["move_threads"] == 256
        # int32 rows for an n off 16 bytes resolve to 16-bit rows
        dp.tuning_set(200, 1024, {"exchange_rows": dp.ROWS_I32})
        assert dp.tuning_get(200, 1024)["exchange_rows"] == dp.ROWS_I32
        assert dp.tuning_get(201, 1024)["exchange_rows"] == dp.ROWS_U16
        # a partial entry: the other field keeps its default
        dp.tuning_set(30, 64, {"move_threads": 128})
        assert dp.tuning_get(30, 64) == {"move_threads": 128, "exchange_rows": dp.ROWS_U16}
        dp.tuning_set(200, 1024, None)
        assert dp.tuning_get(200, 1024) == {"move_threads": 256, "exchange_rows": dp.ROWS_I32}
        # 64 threads serve n up to 1024, 128 up to 2048; the wavefront exchange n up to 1024
        dp.tuning_set(1024, 64, {"move_threads": 64})
        for n, cfg in ((1025, {"move_threads": 64}), (2049, {"move_threads": 128}),
                       (1500, {"exchange_rows": dp.ROWS_U16}), (1500, {"exchange_rows": dp.ROWS_I32}),
                       (1500, {"exchange_rows": dp.ROWS_U16_PAIR}), (1500, {"exchange_rows": dp.ROWS_U16_QUAD})):
            with pytest.raises(dp.DpsoError) as e:
                dp.tuning_set(n, 64, cfg)
            assert e.value.status == dp.E_RANGE, (n, cfg)
        for cfg in ({"move_threads": 32}, {"move_threads": 1024}, {"exchange_rows": 6}, {"exchange_rows": -1}):
            with pytest.raises(dp.DpsoError) as e:
                dp.tuning_set(100, 64, cfg)
            assert e.value.status == dp.E_INVAL, cfg
        for bad in ((0, 64), (dp.MAX_N + 1, 64)):
            with pytest.raises(dp.DpsoError):
                dp.tuning_get(*bad)
        with pytest.raises(dp.DpsoError):
            dp.tuning_get(100, 0)
        # a 16-bit entry over a bucket whose smallest n has no 16-bit copy
        dp.tuning_set(6, 64, {"exchange_rows": dp.ROWS_U16})
        assert dp.tuning_get(8, 64)["exchange_rows"] == dp.ROWS_U16
        assert dp.tuning_get(7, 64)["exchange_rows"] == dp.ROWS_I32
        # two wavefronts per particle split n > 128; smaller n of a bucket take one
        dp.tuning_set(200, 64, {"exchange_rows": dp.ROWS_U16_PAIR})
        assert dp.tuning_get(129, 64)["exchange_rows"] == dp.ROWS_U16_PAIR
        dp.tuning_set(100, 64, {"exchange_rows": dp.ROWS_U16_PAIR})
        assert dp.tuning_get(100, 64)["exchange_rows"] == dp.ROWS_U16
        # four wavefronts split n > 256; the bucket's smaller n take two
        dp.tuning_set(400, 64, {"exchange_rows": dp.ROWS_U16_QUAD})
        assert dp.tuning_get(257, 64)["exchange_rows"] == dp.ROWS_U16_QUAD
        dp.tuning_set(200, 64, {"exchange_rows": dp.ROWS_U16_QUAD})
        assert dp.tuning_get(200, 64)["exchange_rows"] == dp.ROWS_U16_PAIR
        # the batch order
        assert dp.batch_order_get() == dp.ORDER_LPT
        for o in (dp.ORDER_INDEX, dp.ORDER_XCD, dp.ORDER_LPT):
            dp.batch_order_set(o)
            assert dp.batch_order_get() == o
        dp.batch_order_set(dp.ORDER_XCD)
        for bad in (-1, 4):
            with pytest.raises(dp.DpsoError) as e:
                dp.batch_order_set(bad)
            assert e.value.status == dp.E_INVAL
        # the merge limit of the batched exchange classes
        assert dp.batch_merge_get() == dp.MERGE_DEFAULT_PARTICLES
        for m in (0, 1, 1 << 40):
            dp.batch_merge_set(m)
            assert dp.batch_merge_get() == m
        dp.batch_merge_set(-5)
        assert dp.batch_merge_get() == dp.MERGE_DEFAULT_PARTICLES
        dp.batch_merge_set(3)
    finally:
        dp.tuning_reset()
    assert dp.tuning_get(1024, 64)["move_threads"] == 64
    assert dp.batch_order_get() == dp.ORDER_LPT
    assert dp.batch_merge_get() == dp.MERGE_DEFAULT_PARTICLES


def test_autotune_validation(dp):
    """Argument checks that fail before any device work."""
    import ctypes as C
    p = dp._params(_params())
    lib = dp.lib()
    res = (dp.TuneResult * 4)()
    cnt, ch = C.c_int32(), dp.Tuning()
    fake = C.c_void_p(0x1000)
    need = dp.state_bytes(30, p.swarm_size, p.max_generations)
    cases = [
        ((None, 30, C.byref(p), fake, need, 3, fake, need, res, 4, C.byref(cnt), C.byref(ch), None), dp.E_INVAL),
        ((fake, 30, C.byref(p), fake, need, 0, fake, need, res, 4, C.byref(cnt), C.byref(ch), None), dp.E_INVAL),
        ((fake, 30, C.byref(p), fake, need, 3, fake, need - 1, res, 4, C.byref(cnt), C.byref(ch), None), dp.E_NOMEM),
        ((fake, 30, C.byref(p), fake, need - 1, 3, fake, need, res, 4, C.byref(cnt), C.byref(ch), None), dp.E_NOMEM),
        ((fake, 30, C.byref(p), fake, need, 3, None, need, res, 4, C.byref(cnt), C.byref(ch), None), dp.E_INVAL),
        ((fake, 30, C.byref(p), fake, need, 3, fake, need, None, 4, C.byref(cnt), C.byref(ch), None), dp.E_INVAL),
        ((fake, 0, C.byref(p), fake, need, 3, fake, need, res, 4, C.byref(cnt), C.byref(ch), None), dp.E_INVAL),
    ]
    for args, code in cases:
        assert lib.dpso_autotune(*args) == code, args


def test_calls_reject_null_pointers_before_device_work(dp):
    L = dp.lib()
    p = dp._params(_params())
    assert L.dpso_init_nn(None, 30, C.byref(p), None, 0, None) == dp.E_INVAL
    assert L.dpso_run(None, 30, C.byref(p), None, 0, 1, None) == dp.E_INVAL
    assert L.dpso_build_dist(None, None, None, 0, None) == dp.E_INVAL
    assert L.dpso_get_info(None, None, None) == dp.E_INVAL
    # state buffer too small is caught on the host
    fake = C.c_void_p(0x1000)
    need = dp.state_bytes(30, 64, 200)
    assert L.dpso_init_nn(fake, 30, C.byref(p), fake, need - 1, None) == dp.E_NOMEM
    assert L.dpso_run(fake, 30, C.byref(p), fake, need - 1, 1, None) == dp.E_NOMEM
    assert L.dpso_run(fake, 30, C.byref(p), fake, need, -1, None) == dp.E_INVAL


def test_build_dist_validation(dp):
    import numpy as np
    L = dp.lib()
    vp = np.array([[0, 0, 0], [1 << 26, 0, 0]], np.int32)
    sc = dp.Scene(vp.ctypes.data, 2, None, 0, 0)
    fake = C.c_void_p(0x1000)
    assert L.dpso_build_dist(C.byref(sc), fake, fake, 1 << 20, None) == dp.E_RANGE
    vp = np.array([[0, 0, 0], [5, 0, 0]], np.int32)
    box = np.array([[5, 5, 5, 0, 0, 0]], np.int32)   # lo > hi
    sc = dp.Scene(vp.ctypes.data, 2, box.ctypes.data, 1, 0)
    assert L.dpso_build_dist(C.byref(sc), fake, fake, 1 << 20, None) == dp.E_INVAL
    sc = dp.Scene(vp.ctypes.data, 2, None, 0, 0)
    assert L.dpso_build_dist(C.byref(sc), fake, fake, 16, None) == dp.E_NOMEM


def test_build_dist_noalloc_validation(dp):
    """The entry point without a workspace checks the scene as dpso_build_dist
    does, and refuses a scene whose workspace exceeds its static buffer, all
    before any device work."""
    import numpy as np
    L = dp.lib()
    fake = C.c_void_p(0x1000)
    assert L.dpso_build_dist_noalloc(None, fake, None) == dp.E_INVAL
    vp = np.array([[0, 0, 0], [1 << 26, 0, 0]], np.int32)
    sc = dp.Scene(vp.ctypes.data, 2, None, 0, 0)
    assert L.dpso_build_dist_noalloc(C.byref(sc), fake, None) == dp.E_RANGE
    # 2000 viewpoints and 120 boxes: 2960 graph nodes, a 2960^2 x 4 byte matrix
    vp = np.zeros((2000, 3), np.int32)
    vp[:, 0] = np.arange(2000) * 10
    box = np.tile(np.array([[0, 5000, 0, 10, 5010, 10]], np.int32), (120, 1))
    sc = dp.Scene(vp.ctypes.data, 2000, box.ctypes.data, 120, 0)
    assert L.dpso_dist_work_bytes(2000, 120) > dp.NOALLOC_WORK_BYTES
    assert L.dpso_build_dist_noalloc(C.byref(sc), fake, None) == dp.E_NOMEM
    assert "static buffer" in L.dpso_last_error().decode()
    assert L.dpso_dist_work_bytes(1000, 20) <= dp.NOALLOC_WORK_BYTES


def test_voxel_planner_validation(dp):
    """Host checks of the voxel planner: bad arguments give a zero workspace
    size and an error before any device work."""
    import numpy as np
    L = dp.lib()
    fake = C.c_void_p(0x1000)
    vp = np.array([[0, 0, 0], [5000, 0, 0]], np.int32)
    box = np.array([[1000, -500, -500, 2000, 500, 500]], np.int32)
    sc = dp.Scene(vp.ctypes.data, 2, box.ctypes.data, 1, 300)
    good = dp.VoxelParams(250, (C.c_int32 * 3)(1, 2, 3))
    need = L.dpso_voxel_work_bytes(C.byref(sc), C.byref(good))
    assert need > 0
    assert L.dpso_build_dist_voxel(C.byref(sc), C.byref(good), fake, fake, need - 1, None) == dp.E_NOMEM
    assert L.dpso_build_dist_voxel(C.byref(sc), C.byref(good), None, fake, need, None) == dp.E_INVAL
    for s, w in [(0, (1, 1, 1)), (-3, (1, 1, 1)), (100, (0, 1, 1)), (100, (1, 1, -2)),
                 (100, (1, 1 << 21, 1))]:
        bad = dp.VoxelParams(s, (C.c_int32 * 3)(*w))
        assert L.dpso_voxel_work_bytes(C.byref(sc), C.byref(bad)) == 0
        assert L.dpso_build_dist_voxel(C.byref(sc), C.byref(bad), fake, fake, 1 << 30, None) == dp.E_INVAL
    # 1 mm voxels: 5003 x 1003 x 1003 here, 10003^3 over a 10 m cube: above 2^26
    assert L.dpso_voxel_work_bytes(C.byref(sc), C.byref(dp.VoxelParams(1, (C.c_int32 * 3)(1, 1, 1)))) == 0
    cube = np.array([[0, 0, 0], [10000, 10000, 10000]], np.int32)
    sc2 = dp.Scene(cube.ctypes.data, 2, None, 0, 0)
    one = dp.VoxelParams(1, (C.c_int32 * 3)(1, 1, 1))
    assert L.dpso_voxel_work_bytes(C.byref(sc2), C.byref(one)) == 0
    assert L.dpso_build_dist_voxel(C.byref(sc2), C.byref(one), fake, fake, 1 << 30, None) == dp.E_RANGE
    assert L.dpso_voxel_work_bytes(None, C.byref(good)) == 0
    neg = dp.Scene(vp.ctypes.data, 2, box.ctypes.data, 1, -1)
    assert L.dpso_voxel_work_bytes(C.byref(neg), C.byref(good)) == 0


def test_check_dist_validation(dp):
    L = dp.lib()
    fake = C.c_void_p(0x1000)
    bad = C.c_int64(7)
    assert L.dpso_check_dist(None, 10, fake, 8, C.byref(bad), None) == dp.E_INVAL
    assert L.dpso_check_dist(fake, 10, None, 8, C.byref(bad), None) == dp.E_INVAL
    assert L.dpso_check_dist(fake, 10, fake, 8, None, None) == dp.E_INVAL
    assert L.dpso_check_dist(fake, 0, fake, 8, C.byref(bad), None) == dp.E_RANGE
    assert L.dpso_check_dist(fake, 4097, fake, 8, C.byref(bad), None) == dp.E_RANGE
    assert L.dpso_check_dist(fake, 10, fake, 7, C.byref(bad), None) == dp.E_NOMEM
    assert bad.value == 7                                   # untouched on a host-side error


def test_library_does_not_link_the_oracle(dp):
    data = open(dp._LIB_PATH, "rb").read()
    assert b"liboracle" not in data and b"or_build_dist" not in data


def test_batch_validation(dp):
    L = dp.lib()
    assert dp.batch_work_bytes(0) == 0 and dp.batch_work_bytes(4) > 0
    items = (dp.BatchItem * 2)()
    fake = C.c_void_p(0x1000)
    assert L.dpso_run_batch(items, 0, 1, fake, 1 << 20, None) == dp.E_INVAL
    assert L.dpso_run_batch(items, 2, 1, fake, 16, None) == dp.E_NOMEM
    need = dp.batch_work_bytes(2)
    # items with zero swarm size are rejected before any device work
    assert L.dpso_run_batch(items, 2, 1, fake, need, None) == dp.E_INVAL
    assert L.dpso_run_batch(items, 2, -1, fake, need, None) == dp.E_INVAL


def test_ceiling_benchmarks_load_and_check_arguments():
    """The memory-path micro-benchmarks the benchmark uses for its ceilings:
    exported, and invalid arguments are rejected before any launch."""
    raw = C.CDLL(os.path.join(ROOT, "paper_1706_04399_amd", "libceilings.so"))
    for name in ("ceil_l2_stream", "ceil_l2_gather", "ceil_lds_gather", "ceil_lds_write", "ceil_lds_dma",
                 "ceil_lds_gather16", "ceil_lds_dma16"):
        assert hasattr(raw, name), name
    vp, i32 = C.c_void_p, C.c_int32
    raw.ceil_l2_stream.argtypes = [vp, C.c_size_t, i32, i32, vp, vp]
    raw.ceil_l2_gather.argtypes = [vp, C.c_uint32, i32, i32, vp, vp]
    raw.ceil_lds_gather.argtypes = [i32, i32, vp, vp]
    raw.ceil_lds_write.argtypes = [i32, i32, vp, vp]
    raw.ceil_lds_dma.argtypes = [vp, i32, i32, i32, i32, vp, vp]
    raw.ceil_lds_gather16.argtypes = [i32, i32, vp, vp]
    raw.ceil_lds_dma16.argtypes = [vp, i32, i32, i32, i32, vp, vp]
    fake = vp(256)                     # never dereferenced: rejected first
    assert raw.ceil_l2_stream(None, 1 << 24, 1024, 1, fake, None) != 0
    assert raw.ceil_l2_stream(fake, 1 << 24, 1020, 1, fake, None) != 0   # not a multiple of 8
    assert raw.ceil_l2_stream(fake, 1 << 10, 1024, 1, fake, None) != 0   # slice below 16 KB
    assert raw.ceil_l2_gather(fake, 1000, 8, 1, fake, None) != 0         # not a power of two
    assert raw.ceil_lds_gather(0, 1, fake, None) != 0
    assert raw.ceil_lds_dma(fake, 1000, 1002, 8, 1, fake, None) != 0     # not a multiple of 4
    assert raw.ceil_lds_dma(fake, 1000, 2048, 8, 1, fake, None) != 0     # longer than a buffer
    assert raw.ceil_lds_dma(None, 1000, 1000, 8, 1, fake, None) != 0
    assert raw.ceil_lds_gather16(0, 1, fake, None) != 0
    assert raw.ceil_lds_gather16(8, 1, None, None) != 0
    assert raw.ceil_lds_dma16(fake, 1000, 1004, 8, 1, fake, None) != 0   # not a multiple of 8
    assert raw.ceil_lds_dma16(fake, 1000, 2048, 8, 1, fake, None) != 0   # longer than a buffer
    assert raw.ceil_lds_dma16(None, 1000, 1000, 8, 1, fake, None) != 0
    assert raw.ceil_lds_write(8, 0, fake, None) != 0
