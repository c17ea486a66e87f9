"""Autotuning of the generation loop's launch configuration, per device.

For each (n, particles) bucket the library's autotuner (dpso_autotune) times
every candidate configuration on a synthetic facade of that size and records
the fastest in the device's table; the candidates' swarms must agree bit for
bit. The picks are saved to a JSON file per device and library version and
loaded back into the table on a later run (`load`), so the search runs once
per device.

    python -m paper_1706_04399_amd.tune            # tune the default buckets, save
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

from . import dpso, scenes

# (n, particles launched together), one per table bucket: the single-instance
# workloads (facade n = 30 / swarm 64, bridge n = 200 / swarm 1024, facade
# n = 1000 / swarm 4096). Batches keep the built-in defaults: a single
# instance's fastest configuration can split a batch into more classes,
# whose launches run one after another.
DEFAULT_BUCKETS = [(30, 64), (200, 1024), (1000, 4096)]


def cache_path(device=None) -> str:
    import torch
    props = torch.cuda.get_device_properties(device if device is not None else torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "gpu").split(":")[0]
    name = "".join(c if c.isalnum() else "_" for c in props.name)
    ver = "".join(c if c.isalnum() or c == "." else "_" for c in dpso.version())
    root = os.environ.get("DPSO_TUNING_DIR", os.path.join(os.path.expanduser("~"), ".cache", "dpso_mi355x"))
    return os.path.join(root, f"tuning_{arch}_{name}_{ver}.json")


def _scene(n: int, seed: int):
    """A facade of n viewpoints (3 m^2 each, aspect 10:3) with round(n/50) boxes."""
    h = int(round(math.sqrt(0.9e6 * n)))
    w = int(round(h * 10 / 3))
    return scenes.facade(n, w, h, max(1, round(n / 50)), seed=seed, name=f"tune{n}")


def _generations(n: int, particles: int) -> int:
    """Generations per timed trial: a few ms of work or more per trial."""
    work = n * n * particles
    return max(4, min(64, int(4e9 / max(work, 1))))


def tune_bucket(n: int, particles: int, seed: int = 0, stream=None) -> dict:
    """Runs the autotuner on one synthetic instance of the bucket; the pick
    goes into the device's table. Returns the pick and every candidate."""
    D = dpso.build_dist(_scene(n, seed), stream=stream)
    gens = _generations(n, particles)
    prm = scenes.swarm_params(particles, gens + 4, seed=seed, ee_trigger=scenes.EE_ALWAYS)
    state = dpso.init_nn(D, prm, stream=stream)
    dpso.run(D, prm, state, 2, stream)  # past the nearest-neighbour start
    out = dpso.autotune(D, prm, state, gens, stream)
    out.update(n=n, particles=particles, generations=gens)
    return out


def tune(buckets=DEFAULT_BUCKETS, verbose=False, stream=None) -> dict:
    """Tunes every bucket; returns the table as saved by `save`."""
    entries = []
    t0 = time.time()
    for n, particles in buckets:
        e = tune_bucket(n, particles, stream=stream)
        entries.append(e)
        if verbose:
            cands = ", ".join(f"{r['move_threads']}/{r['exchange_rows']}: {r['ms']:.2f}" for r in e["results"])
            print(f"n={n:5d} particles={particles:5d} gens={e['generations']:3d} -> "
                  f"{e['chosen']}  [{cands}]", flush=True)
    return {"library": dpso.version(), "seconds": round(time.time() - t0, 2), "entries": entries}


def save(table: dict, path: str | None = None) -> str:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1)
    os.replace(tmp, path)
    return path


def load(path: str | None = None) -> int:
    """Loads saved picks into the device's table; returns how many (0 when no
    file exists for this device and library version)."""
    path = path or cache_path()
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        table = json.load(f)
    if table.get("library") != dpso.version():
        return 0
    for e in table["entries"]:
        dpso.tuning_set(e["n"], e["particles"], e["chosen"])
    return len(table["entries"])


def main(argv) -> int:
    table = tune(verbose=True)
    print("saved", save(table), f"({table['seconds']} s)")
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
