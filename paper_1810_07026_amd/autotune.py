"""Launch-shape autotuner for the AIREBO kernels.

Tunables (airebo_options): threads per block of the bonded kernel (one
wavefront: its LDS stage is sized for 64 threads), the size of its
persistent grid, threads per block of the deferred-pair kernel and of the
short-list kernel, and the force-kernel schedule (0 automatic, 1 far LJ
pairs beside the near pairs, 2 far pairs after them).  Tuning is a
coordinate search: starting from the defaults, each tunable in turn is swept over its candidates with the others
fixed, timing a short NVE run of the actual workload, and the best value is
kept.  Results are cached in a JSON file keyed by GPU architecture, workload
class (atom count and number of systems, rounded to powers of two) and
precision.
"""
import json
import math
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tune_cache.json")

CANDIDATES = {
    "bond_block": [64],
    "bond_grid": [0, 256, 512, 1024, 2048, 4096],
    "defer_block": [64],
    "short_block": [256, 512, 1024],
    "schedule": [0, 1, 2],
}


def workload_key(arch, n_atoms, nsys, precision):
    nb = 2 ** int(round(math.log2(max(n_atoms, 1))))
    sb = 2 ** int(round(math.log2(max(nsys, 1))))
    return f"{arch}|n{nb}|sys{sb}|{precision}"


def load_cache(path=CACHE):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def lookup(key, path=CACHE):
    return load_cache(path).get(key, {}).get("best")


def tune(run, key, steps=30, repeats=2, path=CACHE, log=print):
    """run(tune_dict, steps) -> seconds for `steps` NVE steps of the workload.

    Returns the best launch shapes and stores them with the timings."""
    best = {k: 0 if k == "bond_grid" else v[0] for k, v in CANDIDATES.items()}
    best_t = min(run(best, steps) for _ in range(repeats))
    trials = [{"tune": dict(best), "s": best_t}]
    for name, values in CANDIDATES.items():
        for val in values:
            if val == best[name]:
                continue
            cand = dict(best, **{name: val})
            t = min(run(cand, steps) for _ in range(repeats))
            trials.append({"tune": dict(cand), "s": t})
            log(f"autotune {key}: {cand} -> {1e3 * t / steps:.4f} ms/step")
            if t < best_t:
                best, best_t = cand, t
    cache = load_cache(path)
    cache[key] = {"best": best, "ms_per_step": 1e3 * best_t / steps, "trials": trials,
                  "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    with open(path, "w") as f:
        json.dump(cache, f, indent=1)
    return best
