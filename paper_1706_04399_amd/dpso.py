"""Python binding of the C ABI in ``include/dpso.h`` (argument marshalling only).

Device memory comes from torch tensors on the current HIP device and work is
enqueued on torch's current stream unless a stream is given. Every step of
the swarm runs in ``libdpso.so``; if the library is missing this module
raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # loaded first so libdpso binds to the HIP runtime torch already uses

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdpso.so")

OK, E_INVAL, E_RANGE, E_NOMEM, E_DEVICE, E_STATE, E_ADMIT = 0, -1, -2, -3, -4, -5, -6
D_INF = (1 << 28) - 1
NOALLOC_WORK_BYTES = 32 << 20   # static workspace of dpso_build_dist_noalloc
MAX_N = 4096
MAX_SWARM = 65536
EE_OFF, EE_ON_STALL, EE_ALWAYS = 0, 1, 2
NB_TWO_OPT, NB_NODE_SWAP = 0, 1
ROWS_AUTO, ROWS_U16, ROWS_I32, ROWS_BLOCK, ROWS_U16_PAIR, ROWS_U16_QUAD = 0, 1, 2, 3, 4, 5
ORDER_DEFAULT, ORDER_INDEX, ORDER_LPT, ORDER_XCD = 0, 1, 2, 3
MERGE_DEFAULT_PARTICLES = 8192


class DpsoError(RuntimeError):
    def __init__(self, status: int, text: str):
        super().__init__(f"dpso status {status}: {text}")
        self.status = status


class Scene(C.Structure):
    _fields_ = [("vp_mm", C.c_void_p), ("n", C.c_int32), ("boxes_mm", C.c_void_p),
                ("n_boxes", C.c_int32), ("clearance_mm", C.c_int32)]


class Surface(C.Structure):
    _fields_ = [("lo_mm", C.c_int32 * 3), ("hi_mm", C.c_int32 * 3), ("normal_axis", C.c_int32),
                ("normal_sign", C.c_int32)]


class Camera(C.Structure):
    _fields_ = [("resolution_px", C.c_int32), ("feature_um", C.c_int32),
                ("overlap_permille", C.c_int32), ("focal_um", C.c_int32), ("sensor_um", C.c_int32)]


class VoxelParams(C.Structure):
    _fields_ = [("voxel_mm", C.c_int32), ("weight", C.c_int32 * 3)]


class Params(C.Structure):
    _fields_ = [("swarm_size", C.c_int32), ("max_generations", C.c_int32),
                ("w_q16", C.c_uint32), ("phi1_q16", C.c_uint32), ("phi2_q16", C.c_uint32),
                ("mutation_period", C.c_int32), ("ee_trigger", C.c_int32),
                ("ee_max_moves", C.c_int32), ("stall_limit", C.c_int32),
                ("det_permille", C.c_int32), ("seed", C.c_uint64), ("instance", C.c_uint64),
                ("ee_neighbourhood", C.c_int32), ("mutation_swaps", C.c_int32),
                ("velocity_cap", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int32), ("swarm_size", C.c_int32), ("trace_capacity", C.c_int32),
                ("generation", C.c_int32), ("stall", C.c_int32), ("done", C.c_int32),
                ("best_cost", C.c_int64), ("sweeps", C.c_int64), ("moves", C.c_int64),
                ("reshuffled", C.c_int64)]


class PhaseTimes(C.Structure):
    _fields_ = [("ms_total", C.c_float), ("ms_move", C.c_float), ("ms_mutation", C.c_float),
                ("ms_gbest", C.c_float), ("ms_exchange", C.c_float), ("ms_control", C.c_float),
                ("generations", C.c_int32), ("exchange_launches", C.c_int32)]


class BatchItem(C.Structure):
    _fields_ = [("d_dist", C.c_void_p), ("n", C.c_int32), ("params", Params),
                ("d_state", C.c_void_p), ("state_bytes", C.c_size_t)]


class Tuning(C.Structure):
    _fields_ = [("move_threads", C.c_int32), ("exchange_rows", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("config", Tuning), ("ms", C.c_float), ("digest", C.c_uint64)]


class HostState(C.Structure):
    _fields_ = [("X", C.c_void_p), ("P", C.c_void_p), ("V", C.c_void_p), ("vlen", C.c_void_p),
                ("F", C.c_void_p), ("FP", C.c_void_p), ("G", C.c_void_p), ("trace", C.c_void_p),
                ("generation", C.c_int32), ("stall", C.c_int32), ("done", C.c_int32),
                ("best_cost", C.c_int64)]


EXPORTS = {
    "dpso_version": (C.c_char_p, []),
    "dpso_last_error": (C.c_char_p, []),
    "dpso_validate_params": (C.c_int32, [C.c_void_p, C.c_int32]),
    "dpso_state_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32]),
    "dpso_dist_work_bytes": (C.c_size_t, [C.c_int32, C.c_int32]),
    "dpso_build_dist_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "dpso_request_footprint": (C.c_int32, [C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p]),
    "dpso_build_dist": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "dpso_init_nn": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t,
                                 C.c_void_p]),
    "dpso_run": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t,
                             C.c_int32, C.c_void_p]),
    "dpso_run_profiled": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t,
                                      C.c_int32, C.c_void_p, C.c_void_p]),
    "dpso_run_timed": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t,
                                      C.c_int32, C.c_void_p, C.c_void_p]),
    "dpso_batch_work_bytes": (C.c_size_t, [C.c_int32]),
    "dpso_init_batch": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p]),
    "dpso_run_batch": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_size_t,
                                   C.c_void_p]),
    "dpso_get_info": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "dpso_get_best": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
    "dpso_export_state": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "dpso_import_state": (C.c_int32, [C.c_void_p, C.c_size_t, C.c_int32, C.c_int32, C.c_void_p,
                                      C.c_void_p]),
    "dpso_viewpoints": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                    C.c_void_p]),
    "dpso_check_dist": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "dpso_voxel_work_bytes": (C.c_size_t, [C.c_void_p, C.c_void_p]),
    "dpso_build_dist_voxel": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                          C.c_void_p]),
    "dpso_tuning_get": (C.c_int32, [C.c_int32, C.c_int32, C.c_void_p]),
    "dpso_tuning_set": (C.c_int32, [C.c_int32, C.c_int32, C.c_void_p]),
    "dpso_tuning_reset": (C.c_int32, []),
    "dpso_batch_order_set": (C.c_int32, [C.c_int32]),
    "dpso_batch_order_get": (C.c_int32, []),
    "dpso_batch_merge_set": (C.c_int32, [C.c_int64]),
    "dpso_batch_merge_get": (C.c_int64, []),
    "dpso_autotune": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_size_t, C.c_int32,
                                  C.c_void_p, C.c_size_t, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                  C.c_void_p]),
}

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                               "`python -m paper_1706_04399_amd.build` (no fallback exists)")
        L = C.CDLL(_LIB_PATH, mode=C.RTLD_GLOBAL)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status: int):
    if status != OK:
        raise DpsoError(status, lib().dpso_last_error().decode())


def _stream(stream):
    """The HIP stream a call enqueues on. A torch stream other than the
    current one first waits for the work already queued on the current stream
    (torch's pool streams do not synchronise with it), so tensors the caller
    just wrote there, such as an uploaded distance matrix, are complete
    before the library reads them. A raw handle is used as given."""
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        cur = torch.cuda.current_stream(stream.device)
        if cur.cuda_stream != stream.cuda_stream:
            stream.wait_stream(cur)
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _params(p) -> Params:
    if isinstance(p, Params):
        return p
    # fields added later (the exchange neighbourhood, the disturbance size)
    # default to 0, their original behaviour
    return Params(**{k: int(p.get(k, 0)) for k, _ in Params._fields_})


def _dev(t: torch.Tensor, dtype) -> C.c_void_p:
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"expected a contiguous {dtype} tensor on the GPU")
    return C.c_void_p(t.data_ptr())


def version() -> str:
    return lib().dpso_version().decode()


def validate_params(params, n: int):
    _check(lib().dpso_validate_params(C.byref(_params(params)), n))


def state_bytes(n: int, swarm_size: int, max_generations: int) -> int:
    return int(lib().dpso_state_bytes(n, swarm_size, max_generations))


def dist_work_bytes(n: int, n_boxes: int) -> int:
    return int(lib().dpso_dist_work_bytes(n, n_boxes))


def build_dist(scene, out: torch.Tensor | None = None, stream=None, device=None) -> torch.Tensor:
    """Travelling-cost matrix of a scene as an int32 [n, n] GPU tensor."""
    vp = np.ascontiguousarray(scene.vp_mm, dtype=np.int32)
    bx = np.ascontiguousarray(scene.boxes_mm, dtype=np.int32)
    n, nb = vp.shape[0], bx.shape[0]
    dev = device if device is not None else (out.device if out is not None else "cuda")
    if out is None:
        out = torch.empty((n, n), dtype=torch.int32, device=dev)
    work = torch.empty(max(dist_work_bytes(n, nb), 1), dtype=torch.uint8, device=dev)
    sc = Scene(vp.ctypes.data, n, bx.ctypes.data if nb else None, nb, int(scene.clearance_mm))
    _check(lib().dpso_build_dist(C.byref(sc), _dev(out, torch.int32), C.c_void_p(work.data_ptr()),
                                 work.numel(), _stream(stream)))
    return out


def build_dist_noalloc(scene, out: torch.Tensor | None = None, stream=None, device=None) -> torch.Tensor:
    """As build_dist, through the entry point whose workspace is the library's
    static device buffer (no workspace tensor is allocated)."""
    vp = np.ascontiguousarray(scene.vp_mm, dtype=np.int32)
    bx = np.ascontiguousarray(scene.boxes_mm, dtype=np.int32)
    n, nb = vp.shape[0], bx.shape[0]
    if out is None:
        out = torch.empty((n, n), dtype=torch.int32, device=device if device is not None else "cuda")
    sc = Scene(vp.ctypes.data, n, bx.ctypes.data if nb else None, nb, int(scene.clearance_mm))
    _check(lib().dpso_build_dist_noalloc(C.byref(sc), _dev(out, torch.int32), _stream(stream)))
    return out


def check_dist(D: torch.Tensor, stream=None) -> int:
    """Row-major index of the first entry of a device matrix that breaks the
    matrix contract (zero diagonal, symmetric, 0..D_INF), or -1."""
    if D.dim() != 2 or D.shape[0] != D.shape[1]:
        raise ValueError("expected a square matrix")
    work = torch.empty(8, dtype=torch.uint8, device=D.device)
    bad = C.c_int64(-1)
    st = lib().dpso_check_dist(_dev(D, torch.int32), D.shape[0], C.c_void_p(work.data_ptr()), 8,
                               C.byref(bad), _stream(stream))
    if st not in (OK, E_RANGE):
        _check(st)
    return int(bad.value)


def request_footprint(n: int, params, budget: int):
    """(status, bytes): the device bytes a served request holds while resident
    (swarm state and distance matrix) and OK, or E_ADMIT if they exceed the
    budget; other statuses raise."""
    nbytes = C.c_size_t(0)
    st = lib().dpso_request_footprint(int(n), C.byref(_params(params)), int(budget), C.byref(nbytes))
    if st not in (OK, E_ADMIT):
        _check(st)
    return st, int(nbytes.value)


def new_state(n: int, params, device="cuda") -> torch.Tensor:
    p = _params(params)
    nbytes = state_bytes(n, p.swarm_size, p.max_generations)
    if nbytes == 0:
        raise DpsoError(E_RANGE, f"no state layout for n={n}, swarm={p.swarm_size}")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def init_nn(D: torch.Tensor, params, state: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    n = D.shape[0]
    if state is None:
        state = new_state(n, params, D.device)
    _check(lib().dpso_init_nn(_dev(D, torch.int32), n, C.byref(_params(params)),
                              _dev(state, torch.uint8), state.numel(), _stream(stream)))
    return state


def run(D: torch.Tensor, params, state: torch.Tensor, generations: int, stream=None):
    n = D.shape[0]
    _check(lib().dpso_run(_dev(D, torch.int32), n, C.byref(_params(params)),
                          _dev(state, torch.uint8), state.numel(), int(generations),
                          _stream(stream)))


def run_profiled(D: torch.Tensor, params, state: torch.Tensor, generations: int,
                 stream=None) -> dict:
    """run() with HIP events between phases; returns device ms per phase."""
    n = D.shape[0]
    t = PhaseTimes()
    _check(lib().dpso_run_profiled(_dev(D, torch.int32), n, C.byref(_params(params)),
                                   _dev(state, torch.uint8), state.numel(), int(generations),
                                   C.byref(t), _stream(stream)))
    return {k: getattr(t, k) for k, _ in PhaseTimes._fields_}


def run_timed(D: torch.Tensor, params, state: torch.Tensor, generations: int, stream=None) -> dict:
    """run() with HIP events around the edge-exchange launches only; returns
    their summed device ms (the other phase fields are 0)."""
    n = D.shape[0]
    t = PhaseTimes()
    _check(lib().dpso_run_timed(_dev(D, torch.int32), n, C.byref(_params(params)),
                                _dev(state, torch.uint8), state.numel(), int(generations),
                                C.byref(t), _stream(stream)))
    return {k: getattr(t, k) for k, _ in PhaseTimes._fields_}


def get_info(state: torch.Tensor, stream=None) -> dict:
    info = Info()
    _check(lib().dpso_get_info(_dev(state, torch.uint8), C.byref(info), _stream(stream)))
    return {k: getattr(info, k) for k, _ in Info._fields_}


def get_best(state: torch.Tensor, stream=None):
    """(tour int32[n], cost, generation, trace int64[generation + 1])."""
    info = get_info(state, stream)
    tour = np.zeros(info["n"], np.int32)
    trace = np.zeros(info["generation"] + 1, np.int64)
    cost, gen = C.c_int64(), C.c_int32()
    _check(lib().dpso_get_best(_dev(state, torch.uint8), tour.ctypes.data, C.byref(cost),
                               C.byref(gen), trace.ctypes.data, _stream(stream)))
    return tour, cost.value, gen.value, trace[: gen.value + 1]


def _voxel_args(scene, voxel_mm, weights):
    vp = np.ascontiguousarray(scene.vp_mm, dtype=np.int32)
    bx = np.ascontiguousarray(scene.boxes_mm, dtype=np.int32)
    sc = Scene(vp.ctypes.data, vp.shape[0], bx.ctypes.data if bx.size else None, bx.shape[0],
               int(scene.clearance_mm))
    vpp = VoxelParams(int(voxel_mm), (C.c_int32 * 3)(*[int(w) for w in weights]))
    return vp, bx, sc, vpp


def voxel_work_bytes(scene, voxel_mm: int, weights=(1, 1, 1)) -> int:
    vp, bx, sc, vpp = _voxel_args(scene, voxel_mm, weights)
    return int(lib().dpso_voxel_work_bytes(C.byref(sc), C.byref(vpp)))


def build_dist_voxel(scene, voxel_mm: int, weights=(1, 1, 1), device="cuda", stream=None) -> torch.Tensor:
    """Travelling costs from the voxel-grid planner (device int32 [n][n])."""
    vp, bx, sc, vpp = _voxel_args(scene, voxel_mm, weights)
    wb = int(lib().dpso_voxel_work_bytes(C.byref(sc), C.byref(vpp)))
    if wb == 0:
        _check(lib().dpso_build_dist_voxel(C.byref(sc), C.byref(vpp), None, None, 0, _stream(stream)))
    n = vp.shape[0]
    D = torch.empty((n, n), dtype=torch.int32, device=device)
    work = torch.empty(wb, dtype=torch.uint8, device=device)
    _check(lib().dpso_build_dist_voxel(C.byref(sc), C.byref(vpp), _dev(D, torch.int32),
                                       _dev(work, torch.uint8), wb, _stream(stream)))
    return D


def viewpoints(surfaces, camera: dict) -> np.ndarray:
    """Viewpoints (int32 [n][3] mm) covering the surfaces: each surface is a
    dict with lo_mm, hi_mm (3 ints), normal_axis and normal_sign; camera has
    the fields of dpso_camera. Host computation."""
    arr = (Surface * max(len(surfaces), 1))()
    for k, f in enumerate(surfaces):
        arr[k] = Surface((C.c_int32 * 3)(*f["lo_mm"]), (C.c_int32 * 3)(*f["hi_mm"]),
                         int(f["normal_axis"]), int(f["normal_sign"]))
    cam = Camera(**{k: int(camera[k]) for k, _ in Camera._fields_})
    count = C.c_int32()
    _check(lib().dpso_viewpoints(arr, len(surfaces), C.byref(cam), None, 0, C.byref(count)))
    out = np.zeros((max(count.value, 1), 3), np.int32)
    _check(lib().dpso_viewpoints(arr, len(surfaces), C.byref(cam), out.ctypes.data, count.value,
                                 C.byref(count)))
    return out[: count.value]


def export_state(state: torch.Tensor, n: int, swarm_size: int, stream=None) -> dict:
    info = get_info(state, stream)
    a = dict(X=np.zeros((swarm_size, n), np.uint16), P=np.zeros((swarm_size, n), np.uint16),
             V=np.zeros((swarm_size, n, 2), np.uint16), vlen=np.zeros(swarm_size, np.int32),
             F=np.zeros(swarm_size, np.int64), FP=np.zeros(swarm_size, np.int64),
             G=np.zeros(n, np.uint16), trace=np.zeros(info["trace_capacity"], np.int64))
    hs = HostState(*[a[k].ctypes.data for k in ("X", "P", "V", "vlen", "F", "FP", "G", "trace")])
    _check(lib().dpso_export_state(_dev(state, torch.uint8), n, swarm_size, C.byref(hs),
                                   _stream(stream)))
    a.update(generation=hs.generation, stall=hs.stall, done=hs.done, best_cost=hs.best_cost)
    a["trace"] = a["trace"][: hs.generation + 1]
    return a


def import_state(state: torch.Tensor, n: int, swarm_size: int, host: dict, stream=None):
    arr = {k: np.ascontiguousarray(host[k], dtype=dt) for k, dt in
           (("X", np.uint16), ("P", np.uint16), ("V", np.uint16), ("vlen", np.int32),
            ("F", np.int64), ("FP", np.int64), ("G", np.uint16), ("trace", np.int64))}
    hs = HostState(*[arr[k].ctypes.data for k in ("X", "P", "V", "vlen", "F", "FP", "G", "trace")],
                   int(host["generation"]), int(host["stall"]), int(host["done"]),
                   int(host["best_cost"]))
    _check(lib().dpso_import_state(_dev(state, torch.uint8), state.numel(), n, swarm_size,
                                   C.byref(hs), _stream(stream)))


def tuning_get(n: int, particles: int) -> dict:
    """The configuration the library uses for n among `particles` particles
    launched together on the current device."""
    t = Tuning()
    _check(lib().dpso_tuning_get(int(n), int(particles), C.byref(t)))
    return {"move_threads": t.move_threads, "exchange_rows": t.exchange_rows}


def tuning_set(n: int, particles: int, config: dict | None):
    """Sets (or, with None, clears) the table entry of the bucket of
    (n, particles) on the current device."""
    if config is None:
        _check(lib().dpso_tuning_set(int(n), int(particles), None))
        return
    t = Tuning(int(config.get("move_threads", 0)), int(config.get("exchange_rows", ROWS_AUTO)))
    _check(lib().dpso_tuning_set(int(n), int(particles), C.byref(t)))


def tuning_reset():
    _check(lib().dpso_tuning_reset())


def batch_order_set(order: int):
    """Order of the particles in batched launches on the current device
    (ORDER_INDEX, ORDER_LPT, ORDER_XCD or ORDER_DEFAULT)."""
    _check(lib().dpso_batch_order_set(int(order)))


def batch_order_get() -> int:
    return int(lib().dpso_batch_order_get())


def batch_merge_set(max_particles: int):
    """Batches of at most this many particles run their 16-bit row exchange
    classes in one launch (0: never, negative: the library default)."""
    _check(lib().dpso_batch_merge_set(int(max_particles)))


def batch_merge_get() -> int:
    return int(lib().dpso_batch_merge_get())


def autotune(D: torch.Tensor, params, state: torch.Tensor, generations: int, stream=None) -> dict:
    """Times every candidate configuration on `generations` generations of the
    swarm in `state` (left unchanged), records the fastest for the bucket of
    (n, swarm_size) and returns {"chosen": config, "results": [...]}."""
    n = D.shape[0]
    scratch = torch.empty_like(state)
    res = (TuneResult * 16)()
    count = C.c_int32(0)
    chosen = Tuning()
    _check(lib().dpso_autotune(_dev(D, torch.int32), n, C.byref(_params(params)), _dev(state, torch.uint8),
                               state.numel(), int(generations), _dev(scratch, torch.uint8), scratch.numel(),
                               res, 16, C.byref(count), C.byref(chosen), _stream(stream)))
    out = [{"move_threads": r.config.move_threads, "exchange_rows": r.config.exchange_rows,
            "ms": float(r.ms), "digest": int(r.digest)} for r in res[: count.value]]
    return {"chosen": {"move_threads": chosen.move_threads, "exchange_rows": chosen.exchange_rows},
            "results": out}


def batch_work_bytes(count: int) -> int:
    return int(lib().dpso_batch_work_bytes(count))


class Batch:
    """Many independent swarms driven by batched launches.

    members: list of (D tensor, params dict). `states` (optional) are existing
    state buffers, one per member (resident swarms resume from them); `work`
    (optional) a device buffer of at least batch_work_bytes(len(members))
    bytes for the batch tables. Whatever is not given is allocated here."""

    def __init__(self, members, stream=None, states=None, work: torch.Tensor | None = None):
        self.stream = stream
        self.members = [(D, dict(p)) for D, p in members]
        dev = self.members[0][0].device
        self.states = list(states) if states is not None else \
            [new_state(D.shape[0], p, dev) for D, p in self.members]
        n = len(self.members)
        if work is None or work.numel() < batch_work_bytes(n):
            work = torch.empty(max(batch_work_bytes(n), 1), dtype=torch.uint8, device=dev)
        self.work = work
        self.items = (BatchItem * n)()
        for i, ((D, p), st) in enumerate(zip(self.members, self.states)):
            self.items[i] = BatchItem(_dev(D, torch.int32).value, D.shape[0], _params(p),
                                      _dev(st, torch.uint8).value, st.numel())

    def init(self):
        _check(lib().dpso_init_batch(self.items, len(self.members), C.c_void_p(self.work.data_ptr()),
                                     self.work.numel(), _stream(self.stream)))
        return self

    def run(self, generations: int):
        _check(lib().dpso_run_batch(self.items, len(self.members), int(generations),
                                    C.c_void_p(self.work.data_ptr()), self.work.numel(),
                                    _stream(self.stream)))
        return self

    def best(self, i: int):
        return get_best(self.states[i], self.stream)


class Solver:
    """One swarm on one GPU: distance matrix and state stay in device memory."""

    def __init__(self, scene=None, params=None, D: torch.Tensor | None = None, device="cuda",
                 stream=None):
        self.params = dict(params)
        self.stream = stream
        self.D = D if D is not None else build_dist(scene, stream=stream, device=device)
        self.n = self.D.shape[0]
        self.state = init_nn(self.D, self.params, stream=stream)

    def run(self, generations: int):
        run(self.D, self.params, self.state, generations, self.stream)
        return self

    def best(self):
        return get_best(self.state, self.stream)

    def info(self):
        return get_info(self.state, self.stream)
