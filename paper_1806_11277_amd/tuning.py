"""Cache of the launch-shape autotuner's tables (ehh_autotune), as JSON.

A table depends on the device, the grid and hierarchy, the cycle precision,
the domain decomposition and the number of sources; tune() looks it up by that
key and runs the library's autotuner only on a miss, storing the result.  The
cache file is EHH_TUNE_CACHE, else ~/.cache/ehh/tuning.json; it is rewritten
atomically (a temporary file renamed over it).
"""
from __future__ import annotations

import json
import os
import tempfile


def cache_path() -> str:
    p = os.environ.get("EHH_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "ehh", "tuning.json")


def key(solver, nrhs: int, device: str) -> str:
    p, o = solver.problem, solver.options
    return json.dumps({"device": device, "dim": p.dim, "n": list(p.n)[:p.dim], "levels": o.levels,
                       "precond_bits": o.precond_bits, "coarse_bits": o.coarse_bits,
                       "dd_parts": list(o.dd_parts)[:p.dim], "dd_overlap": o.dd_overlap, "dd_pad": o.dd_pad,
                       "coarse_dd_parts": list(o.coarse_dd_parts)[:p.dim], "vanka": o.vanka, "nrhs": int(nrhs)},
                      sort_keys=True)


def load(path: str) -> dict:
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def store(path: str, k: str, table) -> None:
    d = load(path)
    d[k] = [int(v) for v in table]
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=os.path.dirname(os.path.abspath(path)), suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(solver, nrhs: int, path: str = None, device: str = None):
    """Install the tuned launch shapes for nrhs sources on solver: from the cache
    when present, else by running the autotuner and caching its table.
    Returns (table, "cache" or "tuned")."""
    if device is None:
        import torch
        device = torch.cuda.get_device_name()
    path = path or cache_path()
    k = key(solver, nrhs, device)
    cached = load(path).get(k)
    if cached is not None and len(cached) == 2 * solver.levels:
        solver.set_tuning(cached)
        return list(cached), "cache"
    table = solver.autotune(nrhs)
    store(path, k, table)
    return table, "tuned"
