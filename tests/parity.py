"""Helpers for comparing the HIP library with the oracle.

Inputs flow one way only: scenes come from the seeded generators, distance
matrices and synthetic swarm states are produced on the oracle side and fed
to both implementations. Nothing computed by the library is ever fed to the
oracle.
"""
import hashlib
import sys

import numpy as np

import oracle


def note(msg):
    """Names the case about to run on the GPU (visible even if the run dies)."""
    sys.stdout.write(f"[gpu] {msg}\n")
    sys.stdout.flush()


def as_host(st: "oracle.State") -> dict:
    """Oracle state in the library's host layout (for dpso.import_state)."""
    return dict(X=st.X.astype(np.uint16), P=st.P.astype(np.uint16),
                V=st.V.astype(np.uint16), vlen=st.VL.copy(), F=st.F.copy(), FP=st.FP.copy(),
                G=st.G.astype(np.uint16), trace=st.trace[: st.t + 1].copy(), generation=st.t,
                stall=st.stall, done=st.done, best_cost=st.FG)


def mismatches(gpu: dict, st: "oracle.State") -> list:
    """Fields where an exported library state differs from the oracle state."""
    bad = []
    for name, ref in (("X", st.X), ("P", st.P), ("F", st.F), ("FP", st.FP), ("G", st.G),
                      ("vlen", st.VL)):
        got = gpu[name]
        if not np.array_equal(got.astype(np.int64), ref.astype(np.int64)):
            rows = np.flatnonzero((got.astype(np.int64) != ref.astype(np.int64)).reshape(
                got.shape[0], -1).any(axis=1)) if got.ndim > 0 else []
            bad.append(f"{name} differs (rows {list(rows[:8])})")
    if np.array_equal(gpu["vlen"], st.VL):
        for p in range(st.S):
            L = st.VL[p]
            if not np.array_equal(gpu["V"][p, :L].astype(np.int64), st.V[p, :L].astype(np.int64)):
                bad.append(f"V[{p}] differs")
                break
    for name, ref in (("generation", st.t), ("stall", st.stall), ("done", st.done),
                      ("best_cost", st.FG)):
        if int(gpu[name]) != int(ref):
            bad.append(f"{name}: gpu {gpu[name]} oracle {ref}")
    if not np.array_equal(gpu["trace"], st.trace[: st.t + 1]):
        bad.append("trace differs")
    return bad


def synthetic_state(D: np.ndarray, prm: dict, t: int, seed: int, max_vlen=None) -> "oracle.State":
    """A mid-run swarm state at generation t: random tours, personal bests and
    velocities, costs from the oracle, G the cheapest personal best. A
    velocity is the canonical difference of two tours, as every velocity the
    method produces is; some are short (a few exchanges apart), some long.
    The trace is flat at F_G."""
    n, S = D.shape[0], prm["swarm_size"]
    rng = np.random.default_rng(seed)
    st = oracle.State(n, S, prm["max_generations"] + 1)
    for p in range(S):
        st.X[p] = rng.permutation(n)
        st.P[p] = rng.permutation(n) if p % 4 else st.X[p]
        ref = rng.permutation(n)
        if p % 3 == 0:
            tgt = rng.permutation(n)
        else:
            tgt = ref.copy()
            for _ in range(int(rng.integers(0, 6))):
                i, j = rng.integers(0, n, size=2)
                tgt[i], tgt[j] = tgt[j], tgt[i]
        v = oracle.bss(ref, tgt)
        if max_vlen is not None:
            v = v[:max_vlen] if len(v) <= max_vlen else oracle.bss(ref, ref)
        st.V[p, : len(v)] = v
        st.VL[p] = len(v)
        st.F[p] = oracle.tour_cost(D, st.X[p])
        st.FP[p] = oracle.tour_cost(D, st.P[p])
        if st.FP[p] > st.F[p]:
            st.P[p], st.FP[p] = st.X[p], st.F[p]
    g = int(np.argmin(st.FP))
    st.G[:] = st.P[g]
    st.FG = int(st.FP[g])
    st.t = t
    st.stall = 0
    st.done = 0
    st.trace[: t + 1] = st.FG
    return st


# ---------------------------------------------------------------- digests
# A whole swarm state reduced to a few hashes, so that the oracle's state at
# the end of a full-length run can be stored as a small fixture and compared
# field by field with the library's exported state. Labels hash as int32,
# costs as int64, a velocity as the concatenation of every particle's
# transposition list (its first vlen pairs).

def _h(a, dtype) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype=dtype).tobytes()).hexdigest()[:16]


def _velocity_words(V, vlen) -> np.ndarray:
    parts = [np.asarray(V[p, : int(vlen[p])], dtype=np.int64).reshape(-1) for p in range(len(vlen))]
    return np.concatenate(parts) if parts else np.zeros(0, np.int64)


def digest(*, X, P, F, FP, vlen, V, G, trace, best_cost, generation, stall, done, sweeps, moves,
           reshuffled, full=False) -> dict:
    d = {"best_cost": int(best_cost), "generation": int(generation), "stall": int(stall),
         "done": int(done), "sweeps": int(sweeps), "moves": int(moves), "reshuffled": int(reshuffled),
         "h_G": _h(G, np.int32), "h_trace": _h(trace, np.int64), "h_X": _h(X, np.int32),
         "h_P": _h(P, np.int32), "h_F": _h(F, np.int64), "h_FP": _h(FP, np.int64),
         "h_vlen": _h(vlen, np.int32), "h_V": _h(_velocity_words(V, vlen), np.int32)}
    if full:
        d["G"] = [int(v) for v in G]
        d["trace"] = [int(v) for v in trace]
    return d


def oracle_digest(st: "oracle.State", full=False) -> dict:
    return digest(X=st.X, P=st.P, F=st.F, FP=st.FP, vlen=st.VL, V=st.V, G=st.G,
                  trace=st.trace[: st.t + 1], best_cost=st.FG, generation=st.t, stall=st.stall,
                  done=st.done, sweeps=st.n_sweeps, moves=st.n_moves, reshuffled=st.n_reshuffled,
                  full=full)


def library_digest(dp, state, n: int, S: int, stream=None, full=False) -> dict:
    """The same digest of a library state (exported through the C ABI)."""
    ex = dp.export_state(state, n, S, stream)
    info = dp.get_info(state, stream)
    return digest(X=ex["X"], P=ex["P"], F=ex["F"], FP=ex["FP"], vlen=ex["vlen"], V=ex["V"],
                  G=ex["G"], trace=ex["trace"], best_cost=ex["best_cost"],
                  generation=ex["generation"], stall=ex["stall"], done=ex["done"],
                  sweeps=info["sweeps"], moves=info["moves"], reshuffled=info["reshuffled"],
                  full=full)


def digest_mismatches(got: dict, want: dict) -> list:
    return [f"{k}: library {got.get(k)!r:.60} oracle {want[k]!r:.60}"
            for k in want if k in got and got[k] != want[k]]
