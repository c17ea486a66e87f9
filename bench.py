"""Throughput of the enhanced DPSO swarm update on one MI355X.

Workload: 1000 viewpoints on a 100 x 30 m facade with 20 box obstacles
(obstacle-aware int32 mm distances, 4 MB), swarm 4096, edge exchange on
every generation (w = 0.7, phi1 = phi2 = 1.5, mutation every 3 generations).
One step is one generation of the whole swarm: move, mutation, global-best
update, complete 2-opt sweep per particle. The metric is particle-iterations
per second (swarm size x generations / seconds) with the distance matrix and
swarm state resident in HBM.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_facade1000.md")
KERNEL_SRC = os.path.join(ROOT, "paper_1706_04399_amd", "csrc", "twoopt.hip")


def exchange_kernel_name(n: int) -> str:
    for mb in (1, 2, 4, 8, 16):
        if n <= 64 * mb:
            return f"k_2opt_wave<{mb}, {'true' if n % 4 == 0 else 'false'}>"
    return "k_2opt_rows"


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


def cpu_baseline(seconds: float):
    """The oracle on the same workload, timed on the host cores for a bounded
    number of generations."""
    import oracle
    from paper_1706_04399_amd import scenes
    sc, prm = scenes.workload(3)
    D = oracle.build_dist(sc)
    st = oracle.new_state(D, prm)
    gens, t0 = 0, time.perf_counter()
    while gens < 40:
        oracle.generation(D, prm, st)
        gens += 1
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(prm["swarm_size"] * gens / dt, 1), "unit": "particle-iters/s",
            "cores": cores, "kind": "oracle",
            "sample": f"generations 1-{gens} of the same workload (n=1000, swarm 4096, "
                      f"edge exchange every generation), {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (each swarm runs "
              "on one GPU; see the multi-GPU design notes)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1706_04399_amd import dpso, scenes

    sc, prm = scenes.workload(3)
    prm = dict(prm, max_generations=args.warmup + args.steps)
    n, S = sc.n, prm["swarm_size"]
    D = dpso.build_dist(sc)
    state = dpso.init_nn(D, prm)
    dpso.run(D, prm, state, args.warmup)
    torch.cuda.synchronize()
    info0 = dpso.get_info(state)

    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    phases = dpso.run_profiled(D, prm, state, args.steps)
    end.record()
    torch.cuda.synchronize()
    ms = start.elapsed_time(end)
    info1 = dpso.get_info(state)
    gens = info1["generation"] - info0["generation"]
    assert gens == args.steps, (gens, args.steps)

    sweeps = info1["sweeps"] - info0["sweeps"]
    bytes_per_sweep = 4 * n * (n - 3) + 4 * n     # two gathers per exchange + edge costs
    launches = phases["exchange_launches"]
    avg_launch_s = phases["ms_exchange"] / launches / 1e3
    achieved = sweeps / launches * bytes_per_sweep / avg_launch_s / 1e9
    tb = hbm_traffic_per_launch()
    traffic = round(tb / avg_launch_s / 1e9, 2) if tb is not None else None

    line = {
        "metric": "particle-iters/s at n=1000",
        "value": round(S * gens / (ms / 1e3), 1),
        "unit": "particle-iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32", "data": "synthetic",
        "config": {"workload": "facade n=1000, 20 boxes, swarm 4096, edge exchange every "
                               "generation", "n": n, "swarm": S, "generations": args.steps,
                   "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "hbm", "kernel": exchange_kernel_name(n),
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
        "phases_ms": {k: round(v, 2) for k, v in phases.items() if k.startswith("ms_")},
        "best_cost_mm": info1["best_cost"],
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
