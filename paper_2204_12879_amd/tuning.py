"""Autotuner cache: launch shapes chosen per (device, batch of cube shapes,
precision), measured by the library (lrstv_autotune) the first time and
reused afterwards from a JSON file."""
from __future__ import annotations

import json
import os
import tempfile
from typing import Optional


def default_cache_path() -> str:
    return os.environ.get("LRSTV_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "lrstv", "tuning.json"))


def batch_key(solver) -> str:
    import torch
    dev = torch.cuda.get_device_name(torch.cuda.current_device())
    shapes = ";".join(f"{b}x{h}x{w}" for b, h, w in sorted(solver.shapes))
    return f"{dev}|precision={solver.params.precision}|{shapes}"


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path: str, data: dict) -> None:
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d or ".", prefix=".tuning.")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(solver, cache_path: Optional[str] = None, reps: int = 3, refresh: bool = False) -> dict:
    """Apply the cached choice for this batch, or measure and cache it.
    Returns the choice with "cached": True/False."""
    path = cache_path or default_cache_path()
    key = batch_key(solver)
    cache = _load(path)
    hit = cache.get(key) if not refresh else None
    if isinstance(hit, dict) and hit.get("tridiag_shape") in solver.get_tuning()["shapes"]:
        solver.set_tuning(hit["tridiag_shape"])
        return dict(hit, cached=True)
    res = solver.autotune(reps)
    entry = {"tridiag_shape": res["tridiag_shape"],
             "tridiag_ms": {str(k): v for k, v in res["tridiag_ms"].items()}}
    cache = _load(path)
    cache[key] = entry
    try:
        _store(path, cache)
    except OSError:
        pass  # a read-only cache location only loses the reuse
    return dict(entry, cached=False)
