"""Helpers for comparing the HIP library with the oracle.

Inputs flow one way only: scenes come from the seeded generators, distance
matrices and synthetic swarm states are produced on the oracle side and fed
to both implementations. Nothing computed by the library is ever fed to the
oracle.
"""
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
