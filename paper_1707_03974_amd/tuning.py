"""Persistent cache of autotuned H.v plans (JSON).

Key: device architecture, lattice (sites and a hash of the bond list),
fillings and precision.  U does not change the sparsity pattern, so it is not
part of the key.  Location: $PDZ_TUNE_CACHE, else ~/.cache/pdz/hv_plans.json.
"""
import hashlib
import json
import os


def cache_path():
    return os.environ.get("PDZ_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "pdz",
                                                             "hv_plans.json")


def plan_key(problem, dtype_name, arch):
    h = hashlib.sha1()
    for b in problem.bonds:
        i, j, t = (b.i, b.j, b.t) if hasattr(b, "i") else b
        h.update(f"{int(i)},{int(j)},{float(t)!r};".encode())
    return f"{arch}|N{problem.n_sites}|{problem.n_up}+{problem.n_dn}|{h.hexdigest()[:16]}|{dtype_name}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def tuned_plan(problem, dtype_name, reps=5, path=None, retune=False):
    """Plan from the cache, or tune now (libpdz autotuner) and store it."""
    import torch
    path = path or cache_path()
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    key = plan_key(problem, dtype_name, arch)
    cache = _load(path)
    if not retune and key in cache:
        entry = cache[key]
        problem.set_plan(dtype_name, entry["down"], entry["up_cw"], entry.get("up", 0), entry.get("map", 0))
        return entry, None
    best, trials = problem.tune(dtype_name, reps=reps)
    entry = dict(best, ms=min(t["ms"] for t in trials))
    cache[key] = entry
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return entry, trials
