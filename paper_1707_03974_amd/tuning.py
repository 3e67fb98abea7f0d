"""Persistent cache of autotuned launch plans (JSON): single-problem H.v plans and batch plans.

Key of a problem: device architecture, lattice (sites and a hash of the bond list), fillings and
precision.  U does not change the sparsity pattern, so it is not part of the key.  Key of a batch:
architecture, the ordered list of its problems' keys (hashed) and precision.  Location:
$PDZ_TUNE_CACHE, else ~/.cache/pdz/hv_plans.json.
"""
import hashlib
import json
import os


def cache_path():
    return os.environ.get("PDZ_TUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "pdz",
                                                             "hv_plans.json")


def _problem_sig(problem):
    h = hashlib.sha1()
    for b in problem.bonds:
        i, j, t = (b.i, b.j, b.t) if hasattr(b, "i") else b
        h.update(f"{int(i)},{int(j)},{float(t)!r};".encode())
    return f"N{problem.n_sites}|{problem.n_up}+{problem.n_dn}|{h.hexdigest()[:16]}"


def plan_key(problem, dtype_name, arch):
    return f"{arch}|{_problem_sig(problem)}|{dtype_name}"


def batch_key(problems, dtype_name, arch):
    h = hashlib.sha1()
    for q in problems:
        h.update((_problem_sig(q) + ";").encode())
    return f"{arch}|batch{len(problems)}|{h.hexdigest()[:16]}|{dtype_name}"


def _arch():
    import torch
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, key, entry):
    cache = _load(path)
    cache[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned_plan(problem, dtype_name, reps=5, path=None, retune=False, arch=None):
    """H.v plan from the cache, or tune now (libpdz autotuner) and store it; returns (entry, trials)."""
    path = path or cache_path()
    key = plan_key(problem, dtype_name, arch or _arch())
    cache = _load(path)
    if not retune and key in cache:
        entry = cache[key]
        problem.set_plan(dtype_name, entry["down"], entry["up_cw"], entry.get("up", 0), entry.get("map", 0))
        return entry, None
    best, trials = problem.tune(dtype_name, reps=reps)
    entry = dict(best, ms=min(t["ms"] for t in trials))
    _store(path, key, entry)
    return entry, trials


def tuned_batch_plan(batch, dtype_name, reps=5, path=None, retune=False, arch=None):
    """Batched H.v plan from the cache, or tune now (libpdz batch autotuner) and store it."""
    path = path or cache_path()
    key = batch_key(batch.problems, dtype_name, arch or _arch())
    cache = _load(path)
    if not retune and key in cache:
        entry = cache[key]
        batch.set_plan(entry["tile_elems"], entry["block"], entry["wgs_per_cu"], entry["order"])
        return entry, None
    best, trials = batch.tune(dtype_name, reps=reps)
    entry = dict(best, ms=min(t["ms"] for t in trials))
    _store(path, key, entry)
    return entry, trials
