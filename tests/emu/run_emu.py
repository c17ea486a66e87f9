"""Drives the host build of the library (tests/emu/libdpso_emu.so, see
build_emu.py) through its C ABI and compares every result with the oracle.
Run it under the sanitizers the library was built with; AddressSanitizer
then reports any access outside a buffer of the emulated device (distance
matrices, states, tables and the exact-size dynamic LDS of each workgroup):

    LD_PRELOAD=$(gcc -print-file-name=libasan.so):$(gcc -print-file-name=libubsan.so) \\
        ASAN_OPTIONS=detect_leaks=0 python tests/emu/run_emu.py quick|batch|serve [count]

Exit status 0 when every compared state equals the oracle's.
"""
import ctypes as C
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path[:0] = [ROOT, os.path.dirname(HERE)]

import oracle  # noqa: E402
from paper_1706_04399_amd import scenes  # noqa: E402
from parity import mismatches  # noqa: E402

LIB = os.path.join(HERE, "libdpso_emu.so")


class Params(C.Structure):
    _fields_ = [("swarm_size", C.c_int32), ("max_generations", C.c_int32),
                ("w_q16", C.c_uint32), ("phi1_q16", C.c_uint32), ("phi2_q16", C.c_uint32),
                ("mutation_period", C.c_int32), ("ee_trigger", C.c_int32),
                ("ee_max_moves", C.c_int32), ("stall_limit", C.c_int32),
                ("det_permille", C.c_int32), ("seed", C.c_uint64), ("instance", C.c_uint64),
                ("ee_neighbourhood", C.c_int32), ("mutation_swaps", C.c_int32),
                ("velocity_cap", C.c_int32)]


class Scene(C.Structure):
    _fields_ = [("vp_mm", C.c_void_p), ("n", C.c_int32), ("boxes_mm", C.c_void_p),
                ("n_boxes", C.c_int32), ("clearance_mm", C.c_int32)]


class BatchItem(C.Structure):
    _fields_ = [("d_dist", C.c_void_p), ("n", C.c_int32), ("params", Params),
                ("d_state", C.c_void_p), ("state_bytes", C.c_size_t)]


class HostState(C.Structure):
    _fields_ = [("X", C.c_void_p), ("P", C.c_void_p), ("V", C.c_void_p), ("vlen", C.c_void_p),
                ("F", C.c_void_p), ("FP", C.c_void_p), ("G", C.c_void_p), ("trace", C.c_void_p),
                ("generation", C.c_int32), ("stall", C.c_int32), ("done", C.c_int32),
                ("best_cost", C.c_int64)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int32), ("swarm_size", C.c_int32), ("trace_capacity", C.c_int32),
                ("generation", C.c_int32), ("stall", C.c_int32), ("done", C.c_int32),
                ("best_cost", C.c_int64), ("sweeps", C.c_int64), ("moves", C.c_int64),
                ("reshuffled", C.c_int64)]


def params(p: dict) -> Params:
    return Params(**{k: int(p.get(k, 0)) for k, _ in Params._fields_})


class Emu:
    def __init__(self):
        L = C.CDLL(LIB)
        L.emu_alloc.restype = C.c_void_p
        L.emu_alloc.argtypes = [C.c_size_t]
        L.emu_free.argtypes = [C.c_void_p]
        L.dpso_last_error.restype = C.c_char_p
        L.dpso_state_bytes.restype = C.c_size_t
        L.dpso_state_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32]
        L.dpso_batch_work_bytes.restype = C.c_size_t
        L.dpso_batch_work_bytes.argtypes = [C.c_int32]
        self.L = L

    def check(self, st):
        if st != 0:
            raise RuntimeError(f"status {st}: {self.L.dpso_last_error().decode()}")

    def alloc(self, nbytes: int) -> int:
        return self.L.emu_alloc(nbytes)

    def free(self, ptr: int):
        self.L.emu_free(C.c_void_p(ptr))

    def build_dist(self, sc):
        vp = np.ascontiguousarray(sc.vp_mm, np.int32)
        bx = np.ascontiguousarray(sc.boxes_mm, np.int32)
        n = vp.shape[0]
        D = self.alloc(4 * n * n)
        s = Scene(vp.ctypes.data, n, bx.ctypes.data if bx.size else None, bx.shape[0], sc.clearance_mm)
        self.check(self.L.dpso_build_dist_noalloc(C.byref(s), C.c_void_p(D), None))
        return D

    def read_dist(self, D: int, n: int) -> np.ndarray:
        out = np.zeros((n, n), np.int32)
        C.memmove(out.ctypes.data, D, out.nbytes)
        return out

    def new_state(self, n: int, p: dict):
        nbytes = self.L.dpso_state_bytes(n, p["swarm_size"], p["max_generations"])
        return self.alloc(nbytes), nbytes

    def init_nn(self, D, n, p, st):
        self.check(self.L.dpso_init_nn(C.c_void_p(D), n, C.byref(params(p)), C.c_void_p(st[0]),
                                       C.c_size_t(st[1]), None))

    def run(self, D, n, p, st, g):
        self.check(self.L.dpso_run(C.c_void_p(D), n, C.byref(params(p)), C.c_void_p(st[0]),
                                   C.c_size_t(st[1]), g, None))

    def _items(self, members):
        arr = (BatchItem * len(members))()
        for i, (D, n, p, st) in enumerate(members):
            arr[i] = BatchItem(D, n, params(p), st[0], st[1])
        return arr

    def init_batch(self, members):
        items = self._items(members)
        wb = self.L.dpso_batch_work_bytes(len(members))
        work = self.alloc(wb)
        self.check(self.L.dpso_init_batch(items, len(members), C.c_void_p(work), C.c_size_t(wb), None))
        self.free(work)

    def run_batch(self, members, g):
        items = self._items(members)
        wb = self.L.dpso_batch_work_bytes(len(members))
        work = self.alloc(wb)
        self.check(self.L.dpso_run_batch(items, len(members), g, C.c_void_p(work), C.c_size_t(wb), None))
        self.free(work)

    def export(self, st, n, S):
        info = Info()
        self.check(self.L.dpso_get_info(C.c_void_p(st[0]), C.byref(info), None))
        a = dict(X=np.zeros((S, n), np.uint16), P=np.zeros((S, n), np.uint16),
                 V=np.zeros((S, n, 2), np.uint16), vlen=np.zeros(S, np.int32),
                 F=np.zeros(S, np.int64), FP=np.zeros(S, np.int64),
                 G=np.zeros(n, np.uint16), trace=np.zeros(info.trace_capacity, np.int64))
        hs = HostState(*[a[k].ctypes.data for k in ("X", "P", "V", "vlen", "F", "FP", "G", "trace")])
        self.check(self.L.dpso_export_state(C.c_void_p(st[0]), n, S, C.byref(hs), None))
        a.update(generation=hs.generation, stall=hs.stall, done=hs.done, best_cost=hs.best_cost)
        a["trace"] = a["trace"][: hs.generation + 1]
        a["counters"] = (info.sweeps, info.moves, info.reshuffled)
        return a


def compare(label, got, ref) -> bool:
    bad = mismatches(got, ref)
    if got["counters"] != (ref.n_sweeps, ref.n_moves, ref.n_reshuffled):
        bad.append(f"counters {got['counters']} oracle {(ref.n_sweeps, ref.n_moves, ref.n_reshuffled)}")
    print(f"{label}: {'ok' if not bad else bad}", flush=True)
    return not bad


def case_quick(emu: Emu) -> bool:
    ok = True
    sc, prm = scenes.workload(1)
    prm = dict(prm, swarm_size=16, max_generations=6)
    D = emu.build_dist(sc)
    Dref = oracle.build_dist(sc)
    same = np.array_equal(emu.read_dist(D, sc.n), Dref)
    print(f"facade30 distance matrix: {'ok' if same else 'differs'}", flush=True)
    ok &= same
    st = emu.new_state(sc.n, prm)
    emu.init_nn(D, sc.n, prm, st)
    ref = oracle.new_state(Dref, prm)
    for g in (1, 1, 1, 3):
        emu.run(D, sc.n, prm, st, g)
        oracle.run(Dref, prm, ref, g)
        ok &= compare(f"facade30 S=16 generation {ref.t}", emu.export(st, sc.n, 16), ref)
    return ok


def _batch_members(emu, cases, gens):
    members, refs = [], []
    for k, (n, S, kw) in enumerate(cases):
        sc = scenes.random_points(n, seed=100 + k, n_boxes=2 if n > 3 else 0)
        Dref = oracle.build_dist(sc)
        D = emu.alloc(4 * n * n)
        C.memmove(D, np.ascontiguousarray(Dref).ctypes.data, 4 * n * n)
        prm = scenes.swarm_params(S, gens, seed=k, instance=k, **kw)
        members.append((D, n, prm, emu.new_state(n, prm)))
        refs.append((Dref, prm))
    return members, refs


BATCH = [
    # every edge-exchange class (int32 rows through registers or straight into
    # LDS, 16-bit rows, the row-per-workgroup kernel above 1024), aligned and
    # unaligned n, and the variants: node-swap exchange, disturbance
    # mutation, raw velocity
    (1, 2, {}), (3, 5, {}), (5, 4, {}), (7, 3, dict(ee_trigger=2)), (30, 6, {}),
    (64, 3, dict(ee_trigger=2)), (65, 4, {}), (100, 3, dict(ee_trigger=2)),
    (127, 3, dict(mutation_period=0)), (128, 3, dict(ee_trigger=2, ee_max_moves=0)),
    (200, 4, {}), (257, 3, dict(ee_trigger=2)), (260, 2, dict(ee_trigger=2)), (301, 2, dict(ee_trigger=2)),
    (512, 2, dict(ee_trigger=2)), (515, 2, dict(ee_trigger=2)), (1000, 2, dict(ee_trigger=2)),
    (1030, 2, dict(ee_trigger=2)), (50, 5, dict(stall_limit=2)), (40, 5, dict(ee_trigger=0)),
    (45, 5, dict(ee_neighbourhood=1, ee_trigger=2)), (2, 4, dict(ee_neighbourhood=1, ee_trigger=2)),
    (131, 3, dict(ee_neighbourhood=1, ee_trigger=2, mutation_swaps=3)), (88, 6, dict(mutation_swaps=5)),
    (77, 5, dict(velocity_cap=30, w=1.0, phi1=0.4, phi2=0.4)),
]


def case_batch(emu: Emu) -> bool:
    gens = 4
    members, refs = _batch_members(emu, BATCH, gens)
    emu.init_batch(members)
    emu.run_batch(members, 2)
    emu.run_batch(members, gens - 2)
    ok = True
    for (D, n, prm, st), (Dref, _) in zip(members, refs):
        ref = oracle.new_state(Dref, prm)
        oracle.run(Dref, prm, ref, gens)
        ok &= compare(f"batch n={n} S={prm['swarm_size']}", emu.export(st, n, prm["swarm_size"]), ref)
    return ok


class Tuning(C.Structure):
    _fields_ = [("move_threads", C.c_int32), ("exchange_rows", C.c_int32)]


class TuneResult(C.Structure):
    _fields_ = [("config", Tuning), ("ms", C.c_float), ("digest", C.c_uint64)]


# forced configurations: (threads per particle in the move, exchange rows:
# 1 16-bit, 2 int32, 3 one workgroup per particle); a field a bucket cannot
# take is left to the default there
TUNINGS = [(64, 1), (128, 2), (256, 3), (64, 3), (128, 1), (64, 2)]


def force_tuning(emu: Emu, tpb: int, rows: int):
    """Sets every bucket of the table to (tpb, rows) where it can serve it."""
    L = emu.L
    L.dpso_tuning_reset()
    for b in range(1, 13):
        n = min(1 << b, 4096)
        for particles in (100, 500, 1000, 2000, 5000, 10000):
            for t in ((tpb, rows), (tpb, 0), (0, rows)):
                if L.dpso_tuning_set(n, particles, C.byref(Tuning(*t))) == 0:
                    break


def case_tuned(emu: Emu, full: bool) -> bool:
    """The batch of every class and single swarms under each forced
    configuration: results equal to the oracle's whatever the table. Without
    `full`, the first three tables, the batch's instances up to n = 131 and
    two single swarms."""
    ok = True
    gens = 3
    refs_cache = {}
    batch = BATCH if full else [c for c in BATCH if c[0] <= 131]
    for tpb, rows in (TUNINGS if full else TUNINGS[:3]):
        force_tuning(emu, tpb, rows)
        members, refs = _batch_members(emu, batch, gens)
        emu.init_batch(members)
        emu.run_batch(members, gens)
        for k, ((D, n, prm, st), (Dref, _)) in enumerate(zip(members, refs)):
            if k not in refs_cache:
                ref = oracle.new_state(Dref, prm)
                oracle.run(Dref, prm, ref, gens)
                refs_cache[k] = ref
            ok &= compare(f"tuning {tpb}/{rows} batch n={n} S={prm['swarm_size']}",
                          emu.export(st, n, prm["swarm_size"]), refs_cache[k])
            emu.free(D)
            emu.free(st[0])
        # a single swarm whose n is in no other bucket of the batch
        for n in ((12, 200, 700) if full else (12, 100)):
            sc = scenes.random_points(n, seed=7, n_boxes=2)
            Dref = oracle.build_dist(sc)
            D = emu.alloc(4 * n * n)
            C.memmove(D, np.ascontiguousarray(Dref).ctypes.data, 4 * n * n)
            prm = scenes.swarm_params(3, gens, seed=1, instance=2, ee_trigger=2)
            st = emu.new_state(n, prm)
            emu.init_nn(D, n, prm, st)
            emu.run(D, n, prm, st, gens)
            ref = oracle.new_state(Dref, prm)
            oracle.run(Dref, prm, ref, gens)
            ok &= compare(f"tuning {tpb}/{rows} single n={n}", emu.export(st, n, 3), ref)
            emu.free(D)
            emu.free(st[0])
    emu.L.dpso_tuning_reset()
    return ok


def case_autotune(emu: Emu) -> bool:
    """dpso_autotune on a small swarm: every candidate's digest agrees, the
    state is left as it was, the pick lands in the table and a run after it
    still equals the oracle."""
    ok = True
    n, gens = 90, 2
    sc = scenes.random_points(n, seed=3, n_boxes=2)
    Dref = oracle.build_dist(sc)
    D = emu.alloc(4 * n * n)
    C.memmove(D, np.ascontiguousarray(Dref).ctypes.data, 4 * n * n)
    prm = scenes.swarm_params(4, 6, seed=2, instance=1, ee_trigger=2)
    st = emu.new_state(n, prm)
    emu.init_nn(D, n, prm, st)
    emu.run(D, n, prm, st, 1)
    before = emu.export(st, n, 4)
    scratch = emu.alloc(st[1])
    res = (TuneResult * 16)()
    count, chosen = C.c_int32(0), Tuning()
    p = params(prm)
    status = emu.L.dpso_autotune(C.c_void_p(D), n, C.byref(p), C.c_void_p(st[0]), C.c_size_t(st[1]), gens,
                                 C.c_void_p(scratch), C.c_size_t(st[1]), res, 16, C.byref(count),
                                 C.byref(chosen), None)
    if status != 0:
        print("autotune failed:", emu.L.dpso_last_error().decode(), flush=True)
        return False
    digests = {res[k].digest for k in range(count.value)}
    cfgs = [(res[k].config.move_threads, res[k].config.exchange_rows) for k in range(count.value)]
    print(f"autotune: {count.value} candidates {cfgs}, {len(digests)} digest(s), chosen "
          f"{(chosen.move_threads, chosen.exchange_rows)}", flush=True)
    ok &= len(digests) == 1 and count.value >= 4
    after = emu.export(st, n, 4)
    same = all(np.array_equal(np.asarray(before[k]), np.asarray(after[k])) for k in before)
    print(f"autotune leaves the state unchanged: {same}", flush=True)
    ok &= same
    got = Tuning()
    emu.L.dpso_tuning_get(n, 4, C.byref(got))
    ok &= (got.move_threads, got.exchange_rows) == (chosen.move_threads, chosen.exchange_rows)
    emu.run(D, n, prm, st, 2)
    ref = oracle.new_state(Dref, prm)
    oracle.run(Dref, prm, ref, 3)
    ok &= compare(f"run after autotune n={n}", emu.export(st, n, 4), ref)
    emu.L.dpso_tuning_reset()
    return ok


def case_orders(emu: Emu) -> bool:
    """A batch whose classes have 8 or more members (16 instances of n = 50,
    eight of n = 97, one move class and two exchange classes) in
    each batch order: index, longest first, and XCD groups (balanced here, so
    every launch is grouped and blocks past a group's end do nothing)."""
    ok = True
    gens = 3
    cases = [(50, 6, dict(ee_trigger=2))] * 16 + [(97, 4, dict(ee_trigger=2))] * 8
    refs = None
    for order in (1, 2, 3):
        emu.L.dpso_batch_order_set(order)
        members, rr = _batch_members(emu, cases, gens)
        if refs is None:
            refs = []
            for (D, n, prm, st), (Dref, _) in zip(members, rr):
                ref = oracle.new_state(Dref, prm)
                oracle.run(Dref, prm, ref, gens)
                refs.append(ref)
        emu.init_batch(members)
        emu.run_batch(members, gens)
        for k, ((D, n, prm, st), ref) in enumerate(zip(members, refs)):
            ok &= compare(f"order {order} instance {k} n={n}", emu.export(st, n, prm["swarm_size"]), ref)
            emu.free(D)
            emu.free(st[0])
    emu.L.dpso_batch_order_set(0)
    return ok


def case_merge(emu: Emu) -> bool:
    """One batch with instances of every 16-bit row class (n = 9 ... 601, n not
    a multiple of 4 so small n take 16-bit rows too) beside int32, node-swap
    and row-per-workgroup ones, with the 16-bit row classes merged into one
    launch and launched one after another; then the same with two wavefronts
    per particle above n = 128, and with four above n = 256 (each width's
    classes merged apart from the others), the last with the move at 512
    threads per particle."""
    ok = True
    for tpb, rows in ((0, 0), (256, 4), (256, 5), (512, 5)):
        L = emu.L
        L.dpso_tuning_reset()
        if rows:
            force_tuning(emu, tpb, rows)
        ok &= _case_merge_once(emu)
    emu.L.dpso_tuning_reset()
    return ok


def _case_merge_once(emu: Emu) -> bool:
    ok = True
    gens = 3
    L = emu.L
    L.dpso_batch_merge_set.argtypes = [C.c_int64]
    L.dpso_batch_merge_get.restype = C.c_int64
    cases = [(9, 3, dict(ee_trigger=2)), (50, 4, dict(ee_trigger=2)), (70, 3, dict(ee_trigger=2)),
             (130, 2, dict(ee_trigger=2)), (301, 2, dict(ee_trigger=2)), (601, 2, dict(ee_trigger=2)),
             (62, 3, dict(ee_trigger=2)), (5, 3, dict(ee_trigger=2)), (40, 2, dict(ee_trigger=2)),
             (33, 2, dict(ee_trigger=2, ee_neighbourhood=1)), (1030, 1, dict(ee_trigger=2))]
    refs = None
    for limit in (1 << 40, 0):
        L.dpso_batch_merge_set(limit)
        ok &= L.dpso_batch_merge_get() == limit
        members, rr = _batch_members(emu, cases, gens)
        if refs is None:
            refs = []
            for (D, n, prm, st), (Dref, _) in zip(members, rr):
                ref = oracle.new_state(Dref, prm)
                oracle.run(Dref, prm, ref, gens)
                refs.append(ref)
        emu.init_batch(members)
        emu.run_batch(members, gens)
        for k, ((D, n, prm, st), ref) in enumerate(zip(members, refs)):
            ok &= compare(f"merge limit {limit} instance {k} n={n}", emu.export(st, n, prm["swarm_size"]), ref)
            emu.free(D)
            emu.free(st[0])
    L.dpso_batch_merge_set(-1)
    ok &= L.dpso_batch_merge_get() == 8192
    return ok


def case_plain(emu: Emu, count: int) -> bool:
    """The batched workload's instances (n log-uniform in [20, 500]) solved
    one after another on the single-instance path, swarm 8, 6 generations."""
    ok = True
    for i in range(count):
        sc = scenes.batch_instance(i)
        prm = scenes.swarm_params(8, 6, seed=0, instance=i)
        Dref = oracle.build_dist(sc)
        D = emu.build_dist(sc)
        st = emu.new_state(sc.n, prm)
        emu.init_nn(D, sc.n, prm, st)
        emu.run(D, sc.n, prm, st, 6)
        ref = oracle.new_state(Dref, prm)
        oracle.run(Dref, prm, ref, 6)
        ok &= compare(f"instance {i} n={sc.n}", emu.export(st, sc.n, 8), ref)
        emu.free(D)
        emu.free(st[0])
    return ok


def case_serve(emu: Emu, count: int) -> bool:
    """The re-planning server's sequence of library calls (as serve.GpuExecutor
    makes them) on a scaled-down stream: sites with n log-uniform in [50, 800],
    swarm 8, 6 generations per request, capacity of 3 runs, 30 % of re-plans
    after a moved obstacle, batches of up to 6 requests (one per site)."""
    from paper_1706_04399_amd import serve
    reqs = serve.replan_requests(count, rate=50.0, seed=int(os.environ.get("EMU_SEED", "5")), sites=12,
                                 n_lo=50, n_hi=800, swarm=8,
                                 generations=6, change_permille=300, capacity_runs=3)
    sites, oracle_sites, ok = {}, {}, True
    pending = list(reqs)
    batch_no = 0
    while pending:
        batch, keys = [], set()
        while pending and len(batch) < 6 and pending[0].key not in keys:
            keys.add(pending[0].key)
            batch.append(pending.pop(0))
        cold, run = [], []
        t0 = time.time()
        for req in batch:
            G = req.run_generations
            site = sites.get(req.key)
            if site is None:
                D = emu.build_dist(req.scene)
                site = dict(version=req.version, D=D, st=emu.new_state(req.n, req.params), t=0,
                            params=dict(req.params), n=req.n)
                sites[req.key] = site
                act = "plan"
            elif site["version"] != req.version:
                emu.free(site["D"])
                site["D"] = emu.build_dist(req.scene)
                site["version"] = req.version
                act = "rebuild"
            elif site["t"] + G > site["params"]["max_generations"]:
                act = "restart"
            else:
                act = "resume"
            if act != "resume":
                cold.append(site)
                site["t"] = 0
            site["t"] += G
            run.append((site, act, req))
        if cold:
            emu.init_batch([(s["D"], s["n"], s["params"], s["st"]) for s in cold])
        emu.run_batch([(s["D"], s["n"], s["params"], s["st"]) for s, _, _ in run], batch[0].run_generations)
        dt = time.time() - t0
        for site, act, req in run:
            o = oracle_sites.get(req.key)
            if act != "resume":
                Dref = oracle.build_dist(req.scene)
                o = dict(D=Dref, st=oracle.new_state(Dref, req.params))
                oracle_sites[req.key] = o
            oracle.run(o["D"], req.params, o["st"], req.run_generations)
            ok &= compare(f"batch {batch_no} request {req.rid} {req.key} n={req.n} {act}",
                          emu.export(site["st"], req.n, req.params["swarm_size"]), o["st"])
        print(f"batch {batch_no}: {len(batch)} requests, {dt:.1f} s emulated", flush=True)
        batch_no += 1
    return ok


def main(argv):
    emu = Emu()
    case = argv[0] if argv else "quick"
    if case == "quick":
        ok = case_quick(emu)
    elif case == "batch":
        ok = case_batch(emu)
    elif case == "tuned":
        ok = case_tuned(emu, len(argv) > 1 and argv[1] == "full")
    elif case == "orders":
        ok = case_orders(emu)
    elif case == "merge":
        ok = case_merge(emu)
    elif case == "autotune":
        ok = case_autotune(emu)
    elif case == "plain":
        ok = case_plain(emu, int(argv[1]) if len(argv) > 1 else 24)
    elif case == "serve":
        ok = case_serve(emu, int(argv[1]) if len(argv) > 1 else 24)
    else:
        raise SystemExit(f"unknown case {case}")
    print("EMU RESULT", "ok" if ok else "MISMATCH", flush=True)
    return 0 if ok else 1


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
