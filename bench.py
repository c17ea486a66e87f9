"""Throughput of the enhanced DPSO swarm update on one MI355X.

Workload: 1000 viewpoints on a 100 x 30 m facade with 20 box obstacles
(obstacle-aware int32 mm distances, 4 MB), swarm 4096, edge exchange on
every generation (w = 0.7, phi1 = phi2 = 1.5, mutation every 3 generations).
One step is one generation of the whole swarm: move, mutation, global-best
update, complete 2-opt sweep per particle. The metric is particle-iterations
per second (swarm size x generations / seconds) with the distance matrix and
swarm state resident in HBM; the timed run (fresh swarm, W warm-up
generations, K timed) is repeated and the median reported.

The same line carries the edge-exchange kernel's LDS roofline and HBM
traffic, the whole step against the L2 roofline of the distance reads, the
measured memory-path ceilings, the n = 30 and n = 200 workloads, the batched
workload against the plain single-instance path, a served re-planning run
and the oracle timed on the host.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--reps R] [--no-extras]
    python bench.py --batch 256 | --serve 3000 [--plain] | --ablation 15 | --voxel 3
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

VALU_LANE_OPS_PER_S = 256 * 4 * 16 * 2.4e9
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_facade1000.md")
# continuous batching of the served runs: rounds of at most this many generations
SERVE_CHUNK = 32
KERNEL_SRC = os.path.join(ROOT, "paper_1706_04399_amd", "csrc", "twoopt.hip")


def exchange_kernel_name(n: int, rows: int) -> str:
    """The edge-exchange kernel an instance of n runs with the row form
    `rows` (1: 16-bit, 2: int32, 3: one workgroup per particle, 4: 16-bit,
    two wavefronts per particle above n = 128, 5: four above n = 256):
    <columns per lane / 64, rows go straight into LDS, 16-bit rows>; 16-bit
    rows are padded to 16 bytes, so they always go straight into LDS."""
    if rows == 3 or n > 1024:
        return "k_2opt_rows"
    mb = next(m for m in (1, 2, 4, 8, 16) if n <= 64 * m)
    if rows == 5 and n > 256:
        return f"k_2opt_quad<{mb}>"
    if rows in (4, 5) and n > 128:
        return f"k_2opt_pair<{mb}>"
    packed = rows == 1
    direct = packed or n % 4 == 0
    return f"k_2opt_wave<{mb}, {'true' if direct else 'false'}, {'true' if packed else 'false'}>"


def setup_tuning(run_tuner: bool) -> dict:
    """Fills the library's tuning table: the saved picks for this device if
    there are any, else the autotuner's run over the default buckets (saved
    for later runs). Outside every timed region."""
    from paper_1706_04399_amd import tune
    if not run_tuner:
        return {"source": "built-in defaults"}
    t0 = time.time()
    loaded = tune.load()
    if loaded:
        return {"source": "saved picks", "entries": loaded, "path": tune.cache_path(),
                "seconds": round(time.time() - t0, 2)}
    table = tune.tune()
    try:
        path = tune.save(table)
    except OSError:
        path = None
    return {"source": "autotuner", "entries": len(table["entries"]), "seconds": table["seconds"],
            "path": path, "picks": [{"n": e["n"], "particles": e["particles"], **e["chosen"],
                                     "candidates_ms": {f"{r['move_threads']}/{r['exchange_rows']}": round(r["ms"], 3)
                                                       for r in e["results"]}}
                                    for e in table["entries"]]}


def hbm_traffic_per_launch():
    """HBM bytes per edge-exchange launch from the committed rocprofv3 counter
    summary, or None if the kernel source changed since it was taken."""
    import hashlib
    import re
    try:
        text = open(TRAFFIC_FILE).read()
        src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    h = re.search(r"source_sha256_16:\s*([0-9a-f]{16})", text)
    b = re.search(r"traffic_bytes_per_launch:\s*(\d+)", text)
    if not h or not b or h.group(1) != src:
        return None
    return int(b.group(1))


def measure_ceilings():
    """Measured rates of the memory paths (micro-benchmarks of
    ``libceilings.so``), each timed with events on the stream it runs on:
    16-byte reads streamed from L2 (a 16 MB buffer of which each XCD reads its
    own 2 MB), random 4-byte reads over a 4 MB buffer (a distance matrix at
    n = 1000), random 4-byte LDS reads within a 4 KB row per wave and random
    2-byte reads within a 2 KB row, 16-byte LDS writes of 4 KB rows, and rows
    loaded straight into LDS (4 KB int32 rows, 2 KB 16-bit rows). Occupancy of
    the LDS tests matches the edge-exchange kernel (16 waves per CU)."""
    import ctypes as C
    import torch
    lib = C.CDLL(os.path.join(ROOT, "paper_1706_04399_amd", "libceilings.so"))
    u64, i32 = C.c_uint64, C.c_int32
    lib.ceil_l2_stream.argtypes = [C.c_void_p, C.c_size_t, i32, i32, C.c_void_p, C.c_void_p]
    lib.ceil_l2_gather.argtypes = [C.c_void_p, C.c_uint32, i32, i32, C.c_void_p, C.c_void_p]
    lib.ceil_lds_gather.argtypes = [i32, i32, C.c_void_p, C.c_void_p]
    lib.ceil_lds_write.argtypes = [i32, i32, C.c_void_p, C.c_void_p]
    lib.ceil_lds_dma.argtypes = [C.c_void_p, i32, i32, i32, i32, C.c_void_p, C.c_void_p]
    lib.ceil_lds_gather16.argtypes = [i32, i32, C.c_void_p, C.c_void_p]
    lib.ceil_lds_dma16.argtypes = [C.c_void_p, i32, i32, i32, i32, C.c_void_p, C.c_void_p]
    stream = torch.cuda.current_stream()
    sh = C.c_void_p(stream.cuda_stream)
    big = torch.randint(0, 1 << 20, (4 << 20,), dtype=torch.int32, device="cuda")   # 16 MB
    mat = torch.randint(0, 1 << 20, (1 << 20,), dtype=torch.int32, device="cuda")   # 4 MB
    sink = torch.zeros(1024 * 256, dtype=torch.int32, device="cuda")
    blocks = 1024

    def timed(call):
        call()                                   # warm-up (and caches)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(3):
            st = call()
            if st != 0:
                raise RuntimeError(f"ceiling kernel launch failed: {st}")
        b.record(stream)
        b.synchronize()
        return a.elapsed_time(b) / 3 / 1e3      # seconds per launch

    reps = 400
    t = timed(lambda: lib.ceil_l2_stream(C.c_void_p(big.data_ptr()), big.numel() * 4, blocks, reps,
                                         C.c_void_p(sink.data_ptr()), sh))
    slice_bytes = big.numel() * 4 // blocks // 16384 * 16384
    l2_stream = slice_bytes * blocks * reps / t / 1e9
    reps = 64
    t = timed(lambda: lib.ceil_l2_gather(C.c_void_p(mat.data_ptr()), mat.numel(), 2048, reps,
                                         C.c_void_p(sink.data_ptr()), sh))
    l2_gather = 2048 * 256 * reps * 16 * 4 / t / 1e9
    reps = 2000
    t = timed(lambda: lib.ceil_lds_gather(blocks, reps, C.c_void_p(sink.data_ptr()), sh))
    lds_gather = blocks * 256 * reps * 16 / t / 1e9               # G reads/s
    t = timed(lambda: lib.ceil_lds_write(blocks, reps, C.c_void_p(sink.data_ptr()), sh))
    lds_write = blocks * 4 * reps * 4096 / t / 1e9               # GB/s
    reps, waves = 200, 4096
    t = timed(lambda: lib.ceil_lds_dma(C.c_void_p(mat.data_ptr()), 1000, 1000, waves, reps,
                                       C.c_void_p(sink.data_ptr()), sh))
    lds_dma = waves * (reps + 1) * 4096 / t / 1e9                 # GB/s of 4 KB rows staged
    t = timed(lambda: lib.ceil_lds_dma16(C.c_void_p(mat.data_ptr()), 1000, 1000, waves, reps,
                                         C.c_void_p(sink.data_ptr()), sh))
    lds_dma16 = waves * (reps + 1) * 2048 / t / 1e9               # GB/s of 2 KB rows staged
    reps = 2000
    t = timed(lambda: lib.ceil_lds_gather16(blocks, reps, C.c_void_p(sink.data_ptr()), sh))
    lds_gather16 = blocks * 256 * reps * 16 / t / 1e9             # G reads/s
    torch.cuda.synchronize()
    return {"l2_stream_GBs": round(l2_stream, 1), "l2_random_gather_GBs": round(l2_gather, 1),
            "lds_random_read_G_per_s": round(lds_gather, 1), "lds_row_write_GBs": round(lds_write, 1),
            "lds_dma_row_GBs": round(lds_dma, 1), "lds_random_read16_G_per_s": round(lds_gather16, 1),
            "lds_dma_row16_GBs": round(lds_dma16, 1)}


def cpu_baseline(seconds: float):
    """The oracle on the same workload, timed on the host cores for a bounded
    number of generations, then one more generation on a single thread."""
    import ctypes as C
    import oracle
    from paper_1706_04399_amd import scenes
    sc, prm = scenes.workload(3)
    D = oracle.build_dist(sc)
    st = oracle.new_state(D, prm)
    gomp = C.CDLL("libgomp.so.1")               # the OpenMP runtime the oracle runs on
    threads = int(gomp.omp_get_max_threads())
    gens, t0 = 0, time.perf_counter()
    while gens < 40:
        oracle.generation(D, prm, st)
        gens += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    gomp.omp_set_num_threads(1)
    t1 = time.perf_counter()
    oracle.generation(D, prm, st)
    dt1 = time.perf_counter() - t1
    gomp.omp_set_num_threads(threads)
    return {"value": round(prm["swarm_size"] * gens / dt, 1), "unit": "particle-iters/s",
            "cores": threads, "kind": "oracle",
            "value_1_core": round(prm["swarm_size"] / dt1, 1),
            "sample": f"generations 1-{gens} of the same workload (n=1000, swarm 4096, "
                      f"edge exchange every generation) on {threads} threads, {dt:.1f} s; "
                      f"generation {gens + 1} on 1 thread, {dt1:.1f} s"}


def batch_cpu_baseline(sc, prm, generations: int, seconds: float, gpu_best):
    """The oracle solving the batch's instances one after another (the first
    ones, until about `seconds` of solving), distance builds excluded as on
    the GPU side; also whether each best cost equals the batched result."""
    import ctypes as C
    import oracle
    gomp = C.CDLL("libgomp.so.1")               # the OpenMP runtime the oracle runs on
    threads = int(gomp.omp_get_max_threads())
    done, same, t_solve = 0, True, 0.0
    for i, (s, p) in enumerate(zip(sc, prm)):
        D = oracle.build_dist(s)
        t0 = time.perf_counter()
        st = oracle.new_state(D, p)
        oracle.run(D, p, st, generations)
        t_solve += time.perf_counter() - t0
        done += 1
        same = same and int(st.FG) == int(gpu_best[i])
        if t_solve >= seconds:
            break
    return {"value": round(done / t_solve, 3), "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": f"instances 0-{done - 1} of the same batch, one after another on {threads} "
                      f"threads, {t_solve:.1f} s of solving (distance builds excluded)",
            "identical_best_costs": same}


def bench_batch(count: int, generations: int, cpu_seconds: float = 0.0, plain_leg: bool = True,
                one_at_a_time: bool = False):
    """Batched workload: `count` independent instances (n log-uniform in
    [20, 500], facades and bridges by seed), swarm 256 each, edge exchange on
    stall. Solves/s of the batched path (one captured graph per run) against
    the plain single-instance path solving the same instances one after
    another (`plain_leg`: dpso_init_nn and dpso_run per instance, on the same
    stream), optionally the batched path with one instance per call
    (`one_at_a_time`), and the oracle on the host for about cpu_seconds (0:
    skipped)."""
    import torch
    from paper_1706_04399_amd import dpso, scenes

    sc = [scenes.batch_instance(i) for i in range(count)]
    prm = [scenes.swarm_params(256, generations, seed=0, instance=i) for i in range(count)]
    Ds = [dpso.build_dist(s) for s in sc]
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    b = dpso.Batch(list(zip(Ds, prm)), stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.init().run(generations)
    stream.synchronize()
    t_batch = time.perf_counter() - t0
    batch_best = [dpso.get_best(st, stream)[1] for st in b.states]
    out = {}
    if plain_leg:
        states = [dpso.new_state(D.shape[0], p) for D, p in zip(Ds, prm)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for D, p, st in zip(Ds, prm, states):
            dpso.init_nn(D, p, st, stream=stream)
            dpso.run(D, p, st, generations, stream=stream)
        stream.synchronize()
        t_plain = time.perf_counter() - t0
        plain_best = [dpso.get_best(st, stream)[1] for st in states]
        del states
        out.update({"plain_value": round(count / t_plain, 3),
                    "plain_path": "dpso_init_nn + dpso_run per instance, one after another on one stream",
                    "speedup_vs_plain": round(t_plain / t_batch, 3), "seconds_plain": round(t_plain, 3),
                    "identical_results_plain": plain_best == batch_best})
    if one_at_a_time:
        t0 = time.perf_counter()
        ones = [dpso.Batch([(D, p)], stream=stream).init().run(generations) for D, p in zip(Ds, prm)]
        stream.synchronize()
        t_one = time.perf_counter() - t0
        one_best = [o.best(0)[1] for o in ones]
        del ones
        out.update({"one_per_call_value": round(count / t_one, 3),
                    "one_per_call_path": "dpso_run_batch with one instance per call, in sequence",
                    "speedup_vs_one_per_call": round(t_one / t_batch, 3),
                    "identical_results_one_per_call": one_best == batch_best})
    ns = [s.n for s in sc]
    cpu = batch_cpu_baseline(sc, prm, generations, cpu_seconds, batch_best) if cpu_seconds > 0 else None
    return {
        "metric": "batched solves/s", "value": round(count / t_batch, 3), "unit": "solves/s",
        "seconds_batched": round(t_batch, 3), **out,
        "particle_iters_per_s": round(256 * generations * count / t_batch, 1),
        "n_gpus": 1, "higher_is_better": True, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"{count} instances, n log-uniform in [20, 500] (min {min(ns)}, "
                               f"max {max(ns)}), facade/bridge by seed, swarm 256, "
                               f"{generations} generations, edge exchange on stall",
                   "instances": count, "generations": generations},
        "cpu_baseline": cpu,
    }


def bench_serve(count: int, rate: float, warmup: int, budget_mb: int, one_at_a_time: bool = False,
                sites: int = 100, plain: bool = False, chunk: int = 0):
    """Served re-planning: Poisson arrivals at `rate`/s over `sites` sites (n
    log-uniform in [50, 800], facades and bridges), swarm 512, 300 generations
    per request, one in five re-plans after a moved obstacle; sites keep their
    distance matrix and swarm resident on the device under the memory budget
    (least recently used evicted), requests admitted first come, first served
    and run as batches. With `one_at_a_time`, every admitted batch holds one
    request; with `plain` as well, each request runs on the plain
    single-instance path (dpso_init_nn, dpso_run) instead of a batch of one
    (the baseline). With `chunk` > 0 the batched server batches continuously:
    running swarms advance in rounds of at most `chunk` generations and
    waiting requests join between rounds."""
    import torch
    from paper_1706_04399_amd import serve

    reqs = serve.replan_requests(count, rate, sites=sites)
    budget = budget_mb << 20
    warm = serve.GpuExecutor(budget)         # untimed: load kernels, warm the allocator
    warm.solve([serve.Request(0, 0.0, reqs[0].scene, dict(reqs[0].params, max_generations=5))])
    del warm
    torch.cuda.synchronize()
    ex = serve.GpuExecutor(budget, single=plain)
    sched = serve.Scheduler(budget, ex.footprint, max_batch=1 if one_at_a_time or plain else 1024)
    chunk = 0 if one_at_a_time or plain else chunk
    t0 = time.perf_counter()
    recs = serve.serve(reqs, ex, sched, chunk=chunk)
    wall = time.perf_counter() - t0
    s = serve.summary(recs, warmup=warmup, scheduler=sched)
    return {
        "metric": "served re-planning p99 latency" + (" (one request at a time, single-instance path)"
                                                      if plain else " (one request per batch)"
                                                      if one_at_a_time else ""),
        "value": round(s["p99_ms"], 2), "unit": "ms", "p50_ms": round(s["p50_ms"], 2),
        "mean_ms": round(s["mean_ms"], 2), "max_ms": round(s["max_ms"], 2),
        "solves_per_s": round(s["solves_per_s"], 2), "batches": s["batches"],
        "mean_batch": round(s["mean_batch"], 2), "actions": s["actions"],
        "state_hit_rate": round(s["state_hit_rate"], 4), "dist_hit_rate": round(s["dist_hit_rate"], 4),
        "evictions": s["evictions"], "rejected": s["rejected"], "wall_s": round(wall, 2),
        "higher_is_better": False, "n_gpus": 1, "dtype": "int32", "data": "synthetic",
        "config": {"workload": f"Poisson arrivals at {rate}/s over {sites} sites, n log-uniform in "
                               f"[50, 800], swarm 512, 300 generations per request, 20 % of re-plans "
                               f"after a moved obstacle, {count} requests (first {warmup} not "
                               f"counted), budget {budget_mb} MiB",
                   "server": "one request at a time on the single-instance path" if plain else
                             "one request per batch" if one_at_a_time else
                             f"continuous batching (rounds of at most {chunk} generations), FCFS "
                             "admission, resident sites" if chunk else "batched, FCFS admission, resident sites"},
    }


ABLATION = [
    # (name, overrides of the enhanced configuration)
    ("DPSO (random init, no mutation, no exchange)", dict(det_permille=0, mutation_period=0, ee_trigger=0)),
    ("+ initialization", dict(mutation_period=0, ee_trigger=0)),
    ("+ random mutation", dict(ee_trigger=0)),
    ("enhanced DPSO (+ 2-opt edge exchange)", dict()),
    ("enhanced, node-swap exchange", dict(ee_neighbourhood=1)),
    ("enhanced, mutation by disturbance", dict(mutation_swaps=-1)),   # -1: n / 10 exchanges
    ("enhanced, raw concatenated velocity", dict(velocity_cap=-1)),   # -1: capped at n
]


# The same augmentations from random starts: the nearest-neighbour seeds of
# the synthetic scenes are so strong that the swarm moves at phi = 0.4 never
# improve on them, and every seeded variant then ends on the exchange's local
# optimum of the seed; from random tours the mutation, the exchange and the
# velocity and mutation variants act on the swarm itself.
ABLATION_RANDOM = [
    ("DPSO (random init, no mutation, no exchange)", dict(det_permille=0, mutation_period=0, ee_trigger=0)),
    ("+ random mutation", dict(det_permille=0, ee_trigger=0)),
    ("+ 2-opt edge exchange, no mutation", dict(det_permille=0, mutation_period=0)),
    ("+ random mutation + 2-opt edge exchange", dict(det_permille=0)),
    ("+ random mutation + node-swap exchange", dict(det_permille=0, ee_neighbourhood=1)),
    ("mutation by disturbance + 2-opt exchange", dict(det_permille=0, mutation_swaps=-1)),
    ("raw concatenated velocity + mutation + 2-opt", dict(det_permille=0, velocity_cap=-1)),
]


def _ablation_rows(dpso, scenes, np, torch, stream, sc, D, k, variants, trials, generations):
    """One table of the ablation: every variant's trials as one batch."""
    rows = []
    for name, kw in variants:
        kw = dict(kw)
        if kw.get("mutation_swaps") == -1:
            kw["mutation_swaps"] = max(2, sc.n // 10)
        if kw.get("velocity_cap") == -1:
            kw["velocity_cap"] = sc.n
        prm = [scenes.swarm_params(100, generations, w=1.0, phi1=0.4, phi2=0.4, seed=s,
                                   instance=k, **kw) for s in range(trials)]
        b = dpso.Batch([(D, p) for p in prm], stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.init().run(generations)
        stream.synchronize()
        dt = time.perf_counter() - t0
        costs, reach = [], []
        for i in range(trials):
            _, cost, _, trace = b.best(i)
            costs.append(cost)
            reach.append(int(np.argmax(trace == cost)))
        rows.append({"variant": name, "cost_mean": round(float(np.mean(costs)), 1),
                     "cost_std": round(float(np.std(costs)), 1),
                     "reached_at_generation_mean": round(float(np.mean(reach)), 1),
                     "seconds_for_all_trials": round(dt, 3), "params": kw})
    base = rows[0]["cost_mean"]
    for r in rows:
        r["cost_improvement_vs_dpso_pct"] = round(100.0 * (base - r["cost_mean"]) / base, 2)
    return rows


def bench_ablation(trials: int, generations: int):
    """Effect of each augmentation, and enhanced vs conventional DPSO, on the
    two synthetic stand-ins for the paper's datasets (facade n=30, bridge
    girder n=200) with the paper's experiment settings (w = 1, phi1 = phi2 =
    0.4, 100 particles, mutation every 3 generations, edge exchange when the
    global best did not improve). Each variant runs `trials` seeds as one
    batch; reported: final cost mean and std, the generation at which the
    best cost was first reached, and the batch's wall time. A second table
    starts every variant from random tours (ABLATION_RANDOM). Also times the
    n=1000 benchmark workload with the node-swap neighbourhood against 2-opt."""
    import numpy as np
    import torch
    from paper_1706_04399_amd import dpso, scenes

    out = {"metric": "ablation", "unit": "mm", "trials": trials, "generations": generations,
           "higher_is_better": False, "n_gpus": 1, "dtype": "int32", "data": "synthetic",
           "settings": "w=1, phi1=phi2=0.4, swarm 100, mutation every 3 generations, exchange on stall",
           "scenes": []}
    stream = torch.cuda.Stream()
    sc, _ = scenes.workload(1)                 # untimed: loads kernels, warms the allocator
    warm = dpso.Batch([(dpso.build_dist(sc), scenes.swarm_params(100, 5))], stream=stream)
    warm.init().run(5)
    stream.synchronize()
    for k, label in ((1, "building stand-in: facade n=30"), (2, "bridge stand-in: girder n=200")):
        sc, _ = scenes.workload(k)
        D = dpso.build_dist(sc)
        entry = {"scene": label, "n": sc.n}
        for key, variants in (("rows", ABLATION), ("rows_random_start", ABLATION_RANDOM)):
            entry[key] = _ablation_rows(dpso, scenes, np, torch, stream, sc, D, k, variants, trials, generations)
        out["scenes"].append(entry)
    # throughput of the two neighbourhoods on the benchmark workload
    sc, prm3 = scenes.workload(3)
    D = dpso.build_dist(sc)
    thr = {}
    for nb, name in ((0, "2-opt"), (1, "node swap")):
        prm = dict(prm3, max_generations=25, ee_neighbourhood=nb)
        st = dpso.init_nn(D, prm)
        dpso.run(D, prm, st, 5)
        torch.cuda.synchronize()
        ph = dpso.run_profiled(D, prm, st, 20)
        torch.cuda.synchronize()
        thr[name] = {"particle_iters_per_s": round(prm["swarm_size"] * 20 / (ph["ms_total"] / 1e3), 1),
                     "exchange_us_per_launch": round(ph["ms_exchange"] / ph["exchange_launches"] * 1e3, 1)}
    out["throughput_n1000_swarm4096"] = thr
    return out


VOXEL_CASES = [("facade n=30", 1, 250), ("bridge girder n=200", 2, 250),
               ("facade n=1000", 3, 500), ("facade n=1000", 3, 250), ("facade n=1000", 3, 125)]


def bench_voxel(reps: int, oracle_seconds: float):
    """The voxel-grid planner (unit step weights) on the three synthetic
    scenes at several voxel edges: milliseconds per all-pairs build on the GPU
    (the whole call: host set-up, uploads, kernels, synchronisation), the
    visibility-graph builder on the same scene for comparison, and the oracle
    on the host cores while a case stays under `oracle_seconds`."""
    import ctypes as C
    import numpy as np
    import torch
    import oracle
    from paper_1706_04399_amd import dpso, scenes

    gomp = C.CDLL("libgomp.so.1")
    out = {"metric": "voxel_planner_ms", "unit": "ms", "higher_is_better": False, "n_gpus": 1,
           "dtype": "int32", "data": "synthetic", "weights": [1, 1, 1], "reps": reps,
           "oracle_threads": int(gomp.omp_get_max_threads()), "cases": []}
    dpso.build_dist_voxel(scenes.workload(1)[0], 500)      # untimed: loads the kernels
    rate = None
    for label, k, s in VOXEL_CASES:
        sc = scenes.workload(k)[0]
        row = {"scene": label, "voxel_mm": s, "n": sc.n}
        vp = sc.vp_mm.astype(np.int64)
        pts = [vp] + ([sc.boxes_mm[:, :3], sc.boxes_mm[:, 3:]] if len(sc.boxes_mm) else [])
        lo = np.concatenate(pts).min(axis=0) - s
        hi = np.concatenate(pts).max(axis=0)
        dims = (hi - lo) // s + 2
        row["grid"] = [int(d) for d in dims]
        row["voxels"] = int(np.prod(dims))
        D = dpso.build_dist_voxel(sc, s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            D = dpso.build_dist_voxel(sc, s)
        torch.cuda.synchronize()
        row["gpu_ms"] = round((time.perf_counter() - t0) / reps * 1e3, 3)
        row["unreachable_pairs"] = int((D == dpso.D_INF).sum().item())
        dpso.build_dist(sc)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            dpso.build_dist(sc)
        torch.cuda.synchronize()
        row["visibility_builder_ms"] = round((time.perf_counter() - t0) / reps * 1e3, 3)
        size = row["voxels"] * sc.n
        if rate is None or size / rate < oracle_seconds:
            t0 = time.perf_counter()
            ref = oracle.build_dist_voxel(sc, s)
            dt = time.perf_counter() - t0
            row["oracle_ms"] = round(dt * 1e3, 1)
            row["equal_to_oracle"] = bool(np.array_equal(ref, D.cpu().numpy()))
            rate = size / dt                  # voxel-sources per second, to skip slow cases
        out["cases"].append(row)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the memory-path micro-benchmarks")
    ap.add_argument("--reps", type=int, default=5,
                    help="repetitions of the timed run (fresh swarm each); the median is reported")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (n=30, n=200, batched, served) in the default line")
    ap.add_argument("--extra-serve", type=int, default=3000,
                    help="requests of the served run in the default line")
    ap.add_argument("--batch", type=int, default=0,
                    help="run the batched workload with this many instances instead")
    ap.add_argument("--batch-generations", type=int, default=500)
    ap.add_argument("--no-plain-leg", action="store_true",
                    help="with --batch: skip solving the instances one at a time on the "
                         "single-instance path")
    ap.add_argument("--serve", type=int, default=0,
                    help="serve this many re-planning requests instead")
    ap.add_argument("--rate", type=float, default=50.0)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--serve-chunk", type=int, default=SERVE_CHUNK,
                    help="continuous batching: rounds of at most this many generations "
                         "(0: whole batches)")
    ap.add_argument("--budget-mb", type=int, default=2048)
    ap.add_argument("--plain", action="store_true",
                    help="with --serve: one request at a time on the single-instance path")
    ap.add_argument("--one-per-batch", action="store_true",
                    help="with --serve: admit one request per batch (the baseline)")
    ap.add_argument("--one-per-call", action="store_true",
                    help="with --batch: also solve the instances one per call of the batched path")
    ap.add_argument("--ablation", type=int, default=0,
                    help="run the augmentation ablation with this many trials per variant instead")
    ap.add_argument("--ablation-generations", type=int, default=200)
    ap.add_argument("--voxel", type=int, default=0,
                    help="time the voxel-grid planner (this many builds per case) instead")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the library's built-in launch configuration instead of the autotuner's picks")
    ap.add_argument("--batch-merge", type=int, default=-1,
                    help="batches of at most this many particles launch their 16-bit row exchange "
                         "classes as one (0: never; default: the library's)")
    ap.add_argument("--batch-order", type=int, default=0,
                    help="order of the batched launches: 0 default, 1 index, 2 longest first, 3 XCD groups")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (each swarm runs "
              "on one GPU; see the multi-GPU design notes)", file=sys.stderr)
        sys.exit(2)

    tuning = None
    if not (args.ablation or args.voxel):
        from paper_1706_04399_amd import dpso
        tuning = setup_tuning(not args.no_tune)
        dpso.batch_order_set(args.batch_order)
        tuning["batch_order"] = dpso.batch_order_get()
        dpso.batch_merge_set(args.batch_merge)
        tuning["batch_merge_particles"] = dpso.batch_merge_get()
    if args.batch:
        print(json.dumps(bench_batch(args.batch, args.batch_generations,
                                     0.0 if args.no_cpu else args.cpu_seconds,
                                     not args.no_plain_leg, args.one_per_call)), flush=True)
        return
    if args.ablation:
        print(json.dumps(bench_ablation(args.ablation, args.ablation_generations)), flush=True)
        return
    if args.voxel:
        print(json.dumps(bench_voxel(args.voxel, args.cpu_seconds)), flush=True)
        return
    if args.serve:
        print(json.dumps(bench_serve(args.serve, args.rate, min(args.serve_warmup, args.serve // 4),
                                     args.budget_mb, args.one_per_batch, plain=args.plain,
                                     chunk=args.serve_chunk)), flush=True)
        return

    import torch
    from paper_1706_04399_amd import dpso, scenes

    sc, prm = scenes.workload(3)
    phase_gens = min(args.steps, 100)          # the untimed phase breakdown afterwards
    prm = dict(prm, max_generations=args.warmup + args.steps + phase_gens)
    n, S = sc.n, prm["swarm_size"]
    D = dpso.build_dist(sc)
    config = dpso.tuning_get(n, S)
    # the same run (fresh swarm, W warm-up generations, then K timed) repeated;
    # the median repetition is reported
    runs = []
    for _ in range(max(1, args.reps)):
        state = dpso.init_nn(D, prm)
        dpso.run(D, prm, state, args.warmup)
        torch.cuda.synchronize()
        info0 = dpso.get_info(state)
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        timed = dpso.run_timed(D, prm, state, args.steps)   # events around the exchange launches only
        end.record()
        torch.cuda.synchronize()
        info1 = dpso.get_info(state)
        assert info1["generation"] - info0["generation"] == args.steps
        runs.append((start.elapsed_time(end), timed, info1["sweeps"] - info0["sweeps"], info1, state))
    order = sorted(range(len(runs)), key=lambda r: runs[r][0])
    ms, timed, sweeps, info1, state = runs[order[len(runs) // 2]]
    gens = args.steps

    bytes_per_sweep = 4 * n * (n - 3) + 4 * n     # two gathers per exchange + edge costs
    launches = timed["exchange_launches"]
    avg_launch_s = timed["ms_exchange"] / launches / 1e3
    per_launch = sweeps / launches                 # sweeps in one exchange launch
    algorithmic_GBs = per_launch * bytes_per_sweep / avg_launch_s / 1e9
    exchanges_G = per_launch * n * (n - 3) / 2 / avg_launch_s / 1e9
    tb = hbm_traffic_per_launch()
    traffic = round(tb / avg_launch_s / 1e9, 2) if tb is not None else None
    value = S * gens / (ms / 1e3)

    line = {
        "metric": "particle-iters/s at n=1000",
        "value": round(value, 1),
        "unit": "particle-iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 4),
        "ms_per_step_repetitions": [round(r[0] / args.steps, 4) for r in runs],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": "facade n=1000, 20 boxes, swarm 4096, edge exchange every "
                               "generation", "n": n, "swarm": S, "generations": args.steps,
                   "repetitions": len(runs), "parallelism": "none (1 GPU)"},
        "exchange_ms_per_launch": round(avg_launch_s * 1e3, 4),
        "best_cost_mm": info1["best_cost"],
        "launch_config": config,
        "tuning": tuning,
    }
    # device time per generation of each phase, from a profiled run after the
    # timed region (its events between phases add a little time of their own)
    phases = dpso.run_profiled(D, prm, state, phase_gens)
    line["phases_ms_per_generation"] = {k[3:]: round(v / phase_gens, 4) for k, v in phases.items()
                                        if k.startswith("ms_")}
    del runs
    # the distance builder, timed on its own after the timed region: median of 5
    build_ms = []
    for _ in range(6):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dpso.build_dist(sc, out=D)
        b.record()
        b.synchronize()
        build_ms.append(a.elapsed_time(b))
    line["build_dist_ms_median5"] = round(sorted(build_ms[1:])[2], 3)
    c = measure_ceilings() if not args.no_ceilings else None
    packed = config["exchange_rows"] == dpso.ROWS_U16
    # The dominant kernel (the edge exchange) is bound by its LDS: every
    # exchange evaluation is one random LDS read of a staged row (the matrix
    # itself is served from L2 and its HBM traffic is small, see `traffic`).
    # achieved: exchange evaluations per second of its launches = random LDS
    # reads per second; peak: the measured random LDS read rate at the same
    # occupancy and width (2-byte reads for 16-bit rows).
    peak = None
    if c is not None:
        peak = c["lds_random_read16_G_per_s"] if packed else c["lds_random_read_G_per_s"]
    line["roofline"] = {
        "bound": "lds", "kernel": exchange_kernel_name(n, config["exchange_rows"]),
        "achieved": round(exchanges_G, 1), "peak": peak, "unit": "G LDS reads/s",
        "frac": round(exchanges_G / peak, 4) if peak else None, "traffic": traffic,
        "traffic_unit": "GB/s of HBM (counters)",
        "algorithmic_GBs": round(algorithmic_GBs, 1), "hbm_peak_GBs": HBM_PEAK_GBS,
    }
    counters = exchange_counters()
    if counters is not None:
        line["roofline"]["counters"] = counters
    if c is not None:
        bpi = 4 * n * (n - 1)                       # algorithmic bytes per particle-iteration
        # time the exchange kernel cannot go below at the measured rates: one
        # random LDS read per exchange, and one staged row per row of the sweep
        # (n - 1 rows). Rows that go straight from memory into LDS (16-bit rows
        # for n above 256 or not a multiple of 4, int32 rows otherwise) stream
        # while the gathers run: the bound is the larger of the two (the LDS
        # serves both, so their sum is given too). Rows staged through
        # registers take LDS store time as well: the sum.
        mb = next(m for m in (1, 2, 4, 8, 16) if n <= 64 * m)
        if packed:
            gather_s = per_launch * n * (n - 3) / 2 / (c["lds_random_read16_G_per_s"] * 1e9)
            row_bytes = 1024 * ((mb + 7) // 8)      # staged per row (whole 1 KB chunks)
            stage_s = per_launch * (n - 1) * row_bytes / (c["lds_dma_row16_GBs"] * 1e9)
            bound_s = max(gather_s, stage_s)
        elif n % 4 == 0:
            gather_s = per_launch * n * (n - 3) / 2 / (c["lds_random_read_G_per_s"] * 1e9)
            row_bytes = 1024 * ((mb + 3) // 4)
            stage_s = per_launch * (n - 1) * row_bytes / (c["lds_dma_row_GBs"] * 1e9)
            bound_s = max(gather_s, stage_s)
        else:
            gather_s = per_launch * n * (n - 3) / 2 / (c["lds_random_read_G_per_s"] * 1e9)
            stage_s = per_launch * (n - 2) * 4 * n / (c["lds_row_write_GBs"] * 1e9)
            bound_s = gather_s + stage_s
        l2_bound = c["l2_stream_GBs"] * 1e9 / bpi
        c.update({
            "l2_stream_bound_piters_per_s": round(l2_bound, 1),
            "l2_gather_bound_piters_per_s": round(c["l2_random_gather_GBs"] * 1e9 / bpi, 1),
            "exchange_gather_us": round(gather_s * 1e6, 1),
            "exchange_staging_us": round(stage_s * 1e6, 1),
            "exchange_bound_us": round(bound_s * 1e6, 1),
            "exchange_rows": "16-bit" if packed else "int32",
            "exchange_lds_sum_us": round((gather_s + stage_s) * 1e6, 1),
            "exchange_measured_us": round(avg_launch_s * 1e6, 1),
            "exchange_frac_of_bound": round(bound_s / avg_launch_s, 4),
            # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, at ~8 integer operations per exchange
            "valu_bound_piters_per_s": round(VALU_LANE_OPS_PER_S / (8 * n * (n - 3) / 2), 1),
        })
        line["ceilings"] = c
        # the whole step against the L2 roofline of the distance reads (the
        # stream rate over 4 n (n - 1) int32 bytes per particle-iteration)
        line["l2_roofline"] = {"bound_piters_per_s": round(l2_bound, 1), "frac": round(value / l2_bound, 4)}
    if not args.no_extras:
        line["workloads"] = {"facade30": small_workload(1, 5), "bridge200": small_workload(2, 5)}
        line["batched"] = compact_batch(bench_batch(256, 500))
        line["served"] = compact_serve(bench_serve(args.extra_serve, 50.0, min(200, args.extra_serve // 4), 2048,
                                                   chunk=args.serve_chunk))
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


def small_workload(k: int, reps: int):
    """Particle-iterations/s of a whole single-instance run of workload k
    (1: facade n=30, swarm 64, 200 generations; 2: bridge girder n=200, swarm
    1024, 1000 generations; exchange on stall), init excluded, median of
    `reps` fresh runs, with the oracle-equal best cost."""
    import torch
    from paper_1706_04399_amd import dpso, scenes
    sc, prm = scenes.workload(k)
    D = dpso.build_dist(sc)
    G, S = prm["max_generations"], prm["swarm_size"]
    ms, best = [], None
    for _ in range(reps + 1):
        st = dpso.init_nn(D, prm)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        dpso.run(D, prm, st, G)
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
        best = dpso.get_best(st)[1]
    m = sorted(ms[1:])[len(ms[1:]) // 2]
    return {"particle_iters_per_s": round(S * G / (m / 1e3), 1), "ms_per_run": round(m, 3),
            "n": sc.n, "swarm": S, "generations": G, "best_cost_mm": best,
            "note": "median of %d runs after one warm-up, init excluded" % reps}


def compact_batch(r: dict) -> dict:
    keys = ("value", "unit", "seconds_batched", "plain_value", "speedup_vs_plain", "identical_results_plain",
            "particle_iters_per_s")
    return {k: r[k] for k in keys if k in r} | {"workload": r["config"]["workload"]}


def compact_serve(r: dict) -> dict:
    keys = ("p50_ms", "value", "solves_per_s", "mean_batch", "state_hit_rate", "dist_hit_rate", "evictions",
            "rejected")
    out = {k: r[k] for k in keys}
    out["p99_ms"] = out.pop("value")
    out["workload"] = r["config"]["workload"]
    out["server"] = r["config"]["server"]
    return out


def exchange_counters():
    """VALU busy, LDS and L2 figures of the edge-exchange kernel from the
    committed rocprofv3 counter summary, or None if the kernel source changed
    since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "counters_facade1000.md")
    try:
        text = open(path).read()
        src = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    h = re.search(r"source_sha256_16:\s*([0-9a-f]{16})", text)
    if not h or h.group(1) != src:
        return None
    out = {}
    for key in ("valu_busy_pct", "lds_active_pct", "lds_bank_conflict_pct", "l2_read_GBs", "l2_hit_pct"):
        m = re.search(key + r":\s*([0-9.]+)", text)
        if m:
            out[key] = float(m.group(1))
    out["source"] = "profiles/counters_facade1000.md"
    return out


if __name__ == "__main__":
    main()
