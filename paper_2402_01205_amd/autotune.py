"""Autotuner of the launch shapes of the tracking library.

Tunes, by coordinate descent on a sample of the workload, the grid cell density
(cells per cluster), the workgroup sizes of the neighbour and tracklet kernels
the number of resident waves of the persistent tracklet kernel (0 = plain grid
launch) and how it hands out work (lane refill or 64 tracklets per wave).  Every candidate's tracks are compared with the reference
configuration's: tuning may change speed only, never the result.  Choices are
cached per (device name, size class) in a JSON file.
"""
from __future__ import annotations

import hashlib
import json
import math
import os

import numpy as np

from .tpc import DeviceClusters, Tracker, default_tuning

SPACE = [
    ("tracklet_order", [0, 1]),
    ("cells_per_cluster", [0.25, 0.5, 1.0, 2.0]),
    ("block_links", [64, 128, 256]),
    ("persistent_waves", [0, 16, 32]),
    ("persistent_refill", [0, 1]),
    ("block_tracklets", [64, 128, 256]),
]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "tpc_mi355x_autotune.json")


def size_class(n_clusters: int, n_jobs: int) -> str:
    return f"n2^{int(math.log2(max(n_clusters, 1)))}_j2^{int(math.log2(max(n_jobs, 1)))}"


def _digest(tr: Tracker) -> str:
    t = tr.tracks()
    h = hashlib.sha256()
    for k in ("off", "hits", "param", "ndf"):
        h.update(np.ascontiguousarray(t[k]).tobytes())
    return h.hexdigest()


def _measure(ev: DeviceClusters, tuning, reps: int, device: int):
    mode = "persistent" if tuning.persistent_waves > 0 else "batched"
    tr = Tracker(device, mode=mode, tuning=tuning)
    tr.run(ev)                      # warm-up (workspace, code objects)
    tr.sync()
    tr.profile(True)
    tr.profile_read(reset=True)
    for _ in range(reps):
        tr.run(ev)
    prof = tr.profile_read(reset=True)
    ms = sum(v[0] for v in prof.values()) / reps
    return ms, _digest(tr), prof


def tune(ev: DeviceClusters, device: int = 0, reps: int = 2, verbose: bool = False):
    """Returns (best tpc_tuning, report dict).  Raises if any candidate changes the result."""
    best = default_tuning(use_graph=0)
    best_ms, ref, _ = _measure(ev, best, reps, device)
    trials = [(dict(_as_dict(best)), best_ms)]
    for name, values in SPACE:
        for v in values:
            if getattr(best, name) == v:
                continue
            cand = default_tuning(**{**_as_dict(best), name: v})
            ms, dig, _ = _measure(ev, cand, reps, device)
            if dig != ref:
                raise RuntimeError(f"tuning {name}={v} changed the tracking result")
            trials.append((dict(_as_dict(cand)), ms))
            if verbose:
                print(f"autotune {name}={v}: {ms:.3f} ms (best {best_ms:.3f})", flush=True)
            if ms < best_ms:
                best, best_ms = cand, ms
    best.use_graph = 1
    return best, dict(best=_as_dict(best), best_ms=best_ms, trials=trials, verified=True)


def _as_dict(t) -> dict:
    return {k: getattr(t, k) for k, _ in t._fields_}


def load_or_tune(ev: DeviceClusters, device: int = 0, cache: str | None = DEFAULT_CACHE, reps: int = 2,
                 verbose: bool = False):
    import torch
    key_dev = torch.cuda.get_device_name(device)
    key_sz = size_class(ev.n, ev.n_jobs)
    db = {}
    if cache and os.path.exists(cache):
        try:
            with open(cache) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
    hit = db.get(key_dev, {}).get(key_sz)
    if hit:
        return default_tuning(**hit), dict(best=hit, cached=True)
    t, rep = tune(ev, device, reps, verbose)
    if cache:
        db.setdefault(key_dev, {})[key_sz] = _as_dict(t)
        try:
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(db, f, indent=1)
        except OSError:
            pass
    return t, rep
