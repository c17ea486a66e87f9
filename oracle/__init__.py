"""ctypes access to the CPU oracle (``dpso_oracle.c``).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use this package. The HIP library never imports, links or
calls it, and it never imports the library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dpso_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

PURPOSE_INIT, PURPOSE_VEL, PURPOSE_MUT = 0, 1, 2
D_INF = (1 << 28) - 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O3, OpenMP over particles).

    The library is built on one machine and may run on another host CPU, so
    it targets x86-64-v3 (AVX2, FMA, BMI2) rather than -march=native. Every
    result is integer arithmetic, so the flags change speed only."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-std=c11", "-O3", "-march=x86-64-v3", "-fopenmp", "-fPIC",
                               "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("swarm_size", C.c_int32), ("max_generations", C.c_int32),
                ("w_q16", C.c_uint32), ("phi1_q16", C.c_uint32), ("phi2_q16", C.c_uint32),
                ("mutation_period", C.c_int32), ("ee_trigger", C.c_int32),
                ("ee_max_moves", C.c_int32), ("stall_limit", C.c_int32),
                ("det_permille", C.c_int32), ("seed", C.c_uint64), ("instance", C.c_uint64),
                ("ee_neighbourhood", C.c_int32), ("mutation_swaps", C.c_int32),
                ("velocity_cap", C.c_int32)]


class _State(C.Structure):
    _fields_ = [("n", C.c_int32), ("S", C.c_int32),
                ("X", C.c_void_p), ("P", C.c_void_p), ("V", C.c_void_p), ("VL", C.c_void_p),
                ("F", C.c_void_p), ("FP", C.c_void_p), ("G", C.c_void_p), ("trace", C.c_void_p),
                ("trace_cap", C.c_int32), ("t", C.c_int32), ("stall", C.c_int32),
                ("done", C.c_int32), ("FG", C.c_int64),
                ("n_sweeps", C.c_int64), ("n_moves", C.c_int64), ("n_reshuffled", C.c_int64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # DPSO_ORACLE_LIB names another build of this source (the tests load
        # copies with planted mistakes through it to show the pins fail)
        _lib = C.CDLL(os.environ.get("DPSO_ORACLE_LIB") or build())
        P = C.c_void_p
        i32, i64, u32, u64 = C.c_int32, C.c_int64, C.c_uint32, C.c_uint64
        sig = {
            "or_philox4x64_10": (None, [P, P, P]),
            "or_draws": (None, [u64, u64, u64, u64, u64, i32, P]),
            "or_tour_cost": (i64, [P, i32, P]),
            "or_check_dist": (i64, [P, i32]),
            "or_apply_swaps": (None, [P, i32, P, i32]),
            "or_bss": (i32, [P, P, i32, P]),
            "or_truncate_counts": (None, [i32, i32, i32, u32, u32, u32, u32, u32, P]),
            "or_nn_tour": (None, [P, i32, i32, P]),
            "or_fisher_yates": (None, [i32, u64, u64, u64, u64, u64, P]),
            "or_best_2opt": (i64, [P, i32, P, P, P]),
            "or_edge_exchange": (i32, [P, i32, P, P, i32, P]),
            "or_swap_delta": (i64, [P, i32, P, i32, i32]),
            "or_best_swap": (i64, [P, i32, P, P, P]),
            "or_node_exchange": (i32, [P, i32, P, P, i32, P]),
            "or_disturb": (None, [i32, i32, u64, u64, u64, u64, u64, P]),
            "or_update_gbest": (i32, [P]),
            "or_check_params": (i32, [P, i32]),
            "or_init": (i32, [P, P, P]),
            "or_move_core": (i32, [P, P, P, P, i32, i32, u32, u32, u32, u32, u32, P]),
            "or_move_core_raw": (i32, [P, P, P, P, i32, i32, u32, u32, u32, u32, u32, i32, P]),
            "or_move_particle": (None, [P, P, P, i32, i32]),
            "or_mutation": (i32, [P, P, P, i32, P]),
            "or_generation": (i32, [P, P, P]),
            "or_run": (i32, [P, P, P, i32]),
            "or_round_len": (i64, [i64, i64, i64]),
            "or_segment_hits_box": (i32, [P, P, P, P]),
            "or_build_dist": (i32, [P, i32, P, i32, i32, P]),
            "or_voxel_grid": (i32, [P, i32, P, i32, i32, i32, P, P, P]),
            "or_build_dist_voxel": (i32, [P, i32, P, i32, i32, i32, i32, i32, i32, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.c_void_p)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


def params(d: dict) -> Params:
    return Params(**{k: d.get(k, 0) for k, _ in Params._fields_})


# ----------------------------------------------------------------- primitives

def philox_block(seed, instance, ctr):
    out = np.zeros(4, np.uint64)
    c = np.array(ctr, np.uint64)
    k = np.array([seed, instance], np.uint64)
    lib().or_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def draws(seed, instance, p, t, purpose, count):
    out = np.zeros(count, np.uint32)
    lib().or_draws(seed, instance, p, t, purpose, count, _p(out))
    return out


def tour_cost(D, x) -> int:
    D = _i32(D)
    return int(lib().or_tour_cost(_p(D), D.shape[0], _p(_i32(x))))


def apply_swaps(x, pairs, k=None):
    y = _i32(x).copy()
    pr = _i32(pairs).reshape(-1)
    k = len(pr) // 2 if k is None else k
    lib().or_apply_swaps(_p(y), len(y), _p(pr if pr.size else np.zeros(2, np.int32)), k)
    return y


def bss(x, T):
    x, T = _i32(x), _i32(T)
    pairs = np.zeros(2 * max(len(x), 1), np.int32)
    ln = lib().or_bss(_p(x), _p(T), len(x), _p(pairs))
    return pairs[: 2 * ln].reshape(-1, 2)


def truncate_counts(lv, lb, lc, w_q16, phi1_q16, phi2_q16, u1, u2):
    out = np.zeros(3, np.int32)
    lib().or_truncate_counts(lv, lb, lc, w_q16, phi1_q16, phi2_q16, u1, u2, _p(out))
    return tuple(int(v) for v in out)


def nn_tour(D, start):
    D = _i32(D)
    out = np.zeros(D.shape[0], np.int32)
    lib().or_nn_tour(_p(D), D.shape[0], start, _p(out))
    return out


def fisher_yates(n, seed, instance, p, t, purpose):
    out = np.zeros(n, np.int32)
    lib().or_fisher_yates(n, seed, instance, p, t, purpose, _p(out))
    return out


def best_2opt(D, x):
    D = _i32(D)
    bi, bj = C.c_int32(), C.c_int32()
    d = lib().or_best_2opt(_p(D), D.shape[0], _p(_i32(x)), C.byref(bi), C.byref(bj))
    return int(d), bi.value, bj.value


def edge_exchange(D, x, F, max_moves):
    D = _i32(D)
    y = _i32(x).copy()
    f = C.c_int64(F)
    sw = C.c_int64(0)
    m = lib().or_edge_exchange(_p(D), D.shape[0], _p(y), C.byref(f), max_moves, C.byref(sw))
    return y, f.value, m, sw.value


def swap_delta(D, x, i, j) -> int:
    D = _i32(D)
    return int(lib().or_swap_delta(_p(D), D.shape[0], _p(_i32(x)), i, j))


def best_swap(D, x):
    D = _i32(D)
    bi, bj = C.c_int32(), C.c_int32()
    d = lib().or_best_swap(_p(D), D.shape[0], _p(_i32(x)), C.byref(bi), C.byref(bj))
    return int(d), bi.value, bj.value


def node_exchange(D, x, F, max_moves):
    D = _i32(D)
    y = _i32(x).copy()
    f = C.c_int64(F)
    sw = C.c_int64(0)
    m = lib().or_node_exchange(_p(D), D.shape[0], _p(y), C.byref(f), max_moves, C.byref(sw))
    return y, f.value, m, sw.value


def disturb(x, k, seed, instance, p, t, purpose):
    y = _i32(x).copy()
    lib().or_disturb(len(y), k, seed, instance, p, t, purpose, _p(y))
    return y


def round_len(dx, dy, dz) -> int:
    return int(lib().or_round_len(dx, dy, dz))


def segment_hits_box(A, B, L, H) -> bool:
    a = [np.ascontiguousarray(v, dtype=np.int64) for v in (A, B, L, H)]
    return bool(lib().or_segment_hits_box(*[_p(v) for v in a]))


def check_dist(D):
    """Row-major index of the first entry of D breaking the matrix contract, or -1."""
    D = _i32(D)
    return int(lib().or_check_dist(_p(D), D.shape[0]))


def build_dist(scene):
    vp = _i32(scene.vp_mm)
    bx = _i32(scene.boxes_mm)
    n = vp.shape[0]
    D = np.zeros((n, n), np.int32)
    st = lib().or_build_dist(_p(vp), n, _p(bx) if bx.size else None, bx.shape[0],
                             scene.clearance_mm, _p(D))
    if st != 0:
        raise ValueError(f"oracle build_dist failed with status {st}")
    return D


def voxel_grid(scene, voxel_mm):
    """(dims (3,), origin (3,), occupancy uint8 [dims z][y][x]) of the planner's grid."""
    vp = _i32(scene.vp_mm)
    bx = _i32(scene.boxes_mm)
    dims = np.zeros(3, np.int32)
    origin = np.zeros(3, np.int64)
    st = lib().or_voxel_grid(_p(vp), vp.shape[0], _p(bx) if bx.size else None, bx.shape[0],
                             scene.clearance_mm, voxel_mm, _p(dims), _p(origin), None)
    if st != 0:
        raise ValueError(f"oracle voxel_grid failed with status {st}")
    occ = np.zeros(int(np.prod(dims.astype(np.int64))), np.uint8)
    lib().or_voxel_grid(_p(vp), vp.shape[0], _p(bx) if bx.size else None, bx.shape[0],
                        scene.clearance_mm, voxel_mm, _p(dims), _p(origin), _p(occ))
    return dims, origin, occ.reshape(dims[2], dims[1], dims[0])


def build_dist_voxel(scene, voxel_mm, weights=(1, 1, 1)):
    vp = _i32(scene.vp_mm)
    bx = _i32(scene.boxes_mm)
    n = vp.shape[0]
    D = np.zeros((n, n), np.int32)
    st = lib().or_build_dist_voxel(_p(vp), n, _p(bx) if bx.size else None, bx.shape[0],
                                   scene.clearance_mm, voxel_mm, *[int(w) for w in weights], _p(D))
    if st != 0:
        raise ValueError(f"oracle build_dist_voxel failed with status {st}")
    return D


# ---------------------------------------------------------------- swarm state

class State:
    """Swarm state held in numpy arrays (int32 labels) plus scalars."""

    def __init__(self, n: int, S: int, trace_cap: int):
        self.n, self.S = n, S
        self.X = np.zeros((S, n), np.int32)
        self.P = np.zeros((S, n), np.int32)
        self.V = np.zeros((S, n, 2), np.int32)
        self.VL = np.zeros(S, np.int32)
        self.F = np.zeros(S, np.int64)
        self.FP = np.zeros(S, np.int64)
        self.G = np.zeros(n, np.int32)
        self.trace = np.zeros(max(trace_cap, 1), np.int64)
        self._c = _State(n=n, S=S, X=self.X.ctypes.data, P=self.P.ctypes.data,
                         V=self.V.ctypes.data, VL=self.VL.ctypes.data, F=self.F.ctypes.data,
                         FP=self.FP.ctypes.data, G=self.G.ctypes.data,
                         trace=self.trace.ctypes.data, trace_cap=len(self.trace))

    # scalar views
    t = property(lambda s: s._c.t, lambda s, v: setattr(s._c, "t", v))
    stall = property(lambda s: s._c.stall, lambda s, v: setattr(s._c, "stall", v))
    done = property(lambda s: s._c.done, lambda s, v: setattr(s._c, "done", v))
    FG = property(lambda s: s._c.FG, lambda s, v: setattr(s._c, "FG", v))
    n_sweeps = property(lambda s: s._c.n_sweeps)
    n_moves = property(lambda s: s._c.n_moves)
    n_reshuffled = property(lambda s: s._c.n_reshuffled)

    @property
    def ref(self):
        return C.byref(self._c)

    def velocity(self, p):
        return self.V[p, : self.VL[p]].copy()

    def copy(self) -> "State":
        o = State(self.n, self.S, len(self.trace))
        for name in ("X", "P", "V", "VL", "F", "FP", "G", "trace"):
            getattr(o, name)[...] = getattr(self, name)
        for name in ("t", "stall", "done", "FG"):
            setattr(o, name, getattr(self, name))
        return o


def new_state(D, prm: dict) -> State:
    D = _i32(D)
    st = State(D.shape[0], prm["swarm_size"], prm["max_generations"] + 1)
    pp = params(prm)
    r = lib().or_init(_p(D), C.byref(pp), st.ref)
    if r != 0:
        raise ValueError(f"oracle init failed with status {r}")
    return st


def generation(D, prm: dict, st: State) -> int:
    D = _i32(D)
    pp = params(prm)
    r = lib().or_generation(_p(D), C.byref(pp), st.ref)
    if r < 0:
        raise ValueError(f"oracle generation failed with status {r}")
    return r


def run(D, prm: dict, st: State, generations: int) -> State:
    D = _i32(D)
    pp = params(prm)
    r = lib().or_run(_p(D), C.byref(pp), st.ref, generations)
    if r != 0:
        raise ValueError(f"oracle run failed with status {r}")
    return st


def move_core(x, Pp, G, v, w_q16, phi1_q16, phi2_q16, u1, u2):
    """One particle's move with given draws; returns (y, new velocity)."""
    x = _i32(x)
    n = len(x)
    vv = np.zeros((max(n, 1), 2), np.int32)
    v = _i32(v).reshape(-1, 2)
    vv[: len(v)] = v
    y = np.zeros(n, np.int32)
    ln = lib().or_move_core(_p(x), _p(_i32(Pp)), _p(_i32(G)), _p(vv), len(v), n, w_q16,
                            phi1_q16, phi2_q16, u1, u2, _p(y))
    return y, vv[:ln].copy()


def move_core_raw(x, Pp, G, v, w_q16, phi1_q16, phi2_q16, u1, u2, cap):
    """The move with the raw concatenated velocity truncated to `cap`."""
    x = _i32(x)
    n = len(x)
    vv = np.zeros((max(n, 1), 2), np.int32)
    v = _i32(v).reshape(-1, 2)
    vv[: len(v)] = v
    y = np.zeros(n, np.int32)
    ln = lib().or_move_core_raw(_p(x), _p(_i32(Pp)), _p(_i32(G)), _p(vv), len(v), n, w_q16,
                                phi1_q16, phi2_q16, u1, u2, cap, _p(y))
    return y, vv[:ln].copy()


def move_particle(D, prm, st: State, p: int, t: int):
    D = _i32(D)
    pp = params(prm)
    lib().or_move_particle(_p(D), C.byref(pp), st.ref, p, t)


def mutation(D, prm, st: State, t: int):
    D = _i32(D)
    pp = params(prm)
    kept = np.zeros(st.S, np.int32)
    r = lib().or_mutation(_p(D), C.byref(pp), st.ref, t, _p(kept))
    return r, kept


def update_gbest(st: State) -> int:
    return int(lib().or_update_gbest(st.ref))


def check_params(prm: dict, n: int) -> int:
    pp = params(prm)
    return int(lib().or_check_params(C.byref(pp), n))
