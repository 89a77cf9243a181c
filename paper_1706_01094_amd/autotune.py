"""Schedule autotuner for the fused stream+collide kernel.

A schedule is (chunks per lane per tile, threads per block, LDS image
bytes).  Every schedule gives identical bits (the image only caches table
rows; misses read the exact rows), so the tuner is free to pick the fastest.
It times candidates on a scratch lattice with the same replica sizes and
densities as the target -- the target's own state is never stepped -- and
caches the winner in a JSON file keyed by a signature of the workload shape.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Iterable, Optional, Sequence, Tuple

import numpy as np

from . import mclg as M

Schedule = Tuple[int, int, int]

DEFAULT_CANDIDATES: Sequence[Schedule] = (
    (1, 1024, 146176), (1, 1024, 128 * 1024), (1, 1024, 112 * 1024), (1, 1024, 96 * 1024),
    (1, 1024, 64 * 1024), (1, 768, 112 * 1024), (1, 512, 64 * 1024), (1, 256, 32 * 1024),
)

CACHE_PATH = os.environ.get(
    "MCLG_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "mclg_autotune.json"))


def signature(L, rho, u0, C: int, lam, n_max: int, device_name: str) -> str:
    """Workload shape: sizes bucketed to powers of two, densities to integers."""
    Ls = np.atleast_1d(np.asarray(L, dtype=np.float64))
    r = np.broadcast_to(np.asarray(rho, dtype=np.float64), Ls.shape)
    u = np.broadcast_to(np.asarray(0.0 if u0 is None else u0, dtype=np.float64), Ls.shape)
    key = {
        "n": int(len(Ls)), "sites_log2": int(np.round(np.log2(Ls.sum()))),
        "L_hist": np.bincount(np.round(np.log2(Ls)).astype(int), minlength=32).tolist(),
        "rho": int(np.round(np.average(r, weights=Ls))), "u": round(float(np.average(np.abs(u), weights=Ls)), 2),
        "C": C, "lam": list(lam), "n_max": n_max, "device": device_name,
    }
    return hashlib.sha256(json.dumps(key, sort_keys=True).encode()).hexdigest()[:24]


def _load_cache() -> dict:
    try:
        with open(CACHE_PATH) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(cache: dict) -> None:
    try:
        os.makedirs(os.path.dirname(CACHE_PATH), exist_ok=True)
        tmp = CACHE_PATH + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE_PATH)
    except OSError:
        pass


def time_schedule(lat: "M.Lattice", sch: Schedule, steps: int, warmup: int = 2) -> float:
    """Seconds per step of `lat` under schedule `sch` (HIP events)."""
    torch = lat.torch
    lat.set_schedule(*sch)
    lat.step(warmup)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(lat.stream)
    lat.step(steps)
    e1.record(lat.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def tune(L, rho, u0=None, C: int = 10, lam=(1, 1), n_max: int = 255, seed: int = 0x5EED,
         candidates: Optional[Iterable[Schedule]] = None, steps: int = 20,
         use_cache: bool = True, replica_id=None) -> dict:
    """Pick the fastest schedule for this workload shape; returns
    {"schedule": (g, t, b), "seconds_per_step": s, "trials": [...], "cached": bool}."""
    import torch
    name = torch.cuda.get_device_name(0)
    sig = signature(L, rho, u0, C, lam, n_max, name)
    cache = _load_cache() if use_cache else {}
    if use_cache and sig in cache:
        hit = dict(cache[sig])
        hit["schedule"] = tuple(hit["schedule"])
        hit["cached"] = True
        return hit
    scratch = M.Lattice(L, seed, C=C, lam=lam, n_max=n_max, rho=rho, u0=u0,
                        replica_id=replica_id)
    trials = []
    for sch in (candidates or DEFAULT_CANDIDATES):
        try:
            sec = time_schedule(scratch, tuple(sch), steps)
        except M.MclgError as e:  # e.g. the image does not fit this device's LDS
            trials.append({"schedule": list(sch), "error": str(e)})
            continue
        trials.append({"schedule": list(sch), "seconds_per_step": sec})
    scratch.close()
    ok = [t for t in trials if "seconds_per_step" in t]
    if not ok:
        raise RuntimeError("no schedule could be timed")
    best = min(ok, key=lambda t: t["seconds_per_step"])
    res = {"schedule": tuple(best["schedule"]), "seconds_per_step": best["seconds_per_step"],
           "trials": trials, "cached": False}
    if use_cache:
        cache[sig] = {"schedule": list(res["schedule"]), "seconds_per_step": res["seconds_per_step"],
                      "trials": trials, "when": time.time()}
        _store_cache(cache)
    return res


def apply(lat: "M.Lattice", rho, u0=None, **kw) -> dict:
    """Tune for `lat`'s shape and set the winning schedule on it."""
    res = tune(lat.L, rho, u0, **kw)
    lat.set_schedule(*res["schedule"])
    return res
