"""Tracking quality against the generator's Monte-Carlo truth.

A track's label is its majority particle; purity = majority hits / hits; a
track with purity < 0.9 is a fake.  A particle is findable if it left at least
30 clusters in one sector.  Efficiency = findable particles with at least one
non-fake track / findable particles; clones are extra non-fake tracks of an
already-found particle (merged tracks count once).
"""
from __future__ import annotations

import numpy as np

MIN_FINDABLE = 30
PURITY = 0.9


PT_BINS = (0.1, 0.2, 0.5, 1.0, 10.0001)


def quality(label, job_off, sector, trk_off, trk_hits, part_off=None, part_pt=None, by_job=False):
    """Efficiency, fake and clone rates (and efficiency per pT bin); with by_job, the counts
    behind them per job as well (findable particles, found ones, tracks, fakes)."""
    label = np.asarray(label)
    job_off = np.asarray(job_off, np.int64)
    n_jobs = len(job_off) - 1
    job_of = np.repeat(np.arange(n_jobs), np.diff(job_off))
    if part_off is None:  # particles per job = max label + 1
        mx = np.full(n_jobs, -1, np.int64)
        if label.size:
            np.maximum.at(mx, job_of, label.astype(np.int64))
        part_off = np.concatenate([[0], np.cumsum(mx + 1)])
    part_off = np.asarray(part_off, np.int64)
    gl = np.where(label >= 0, part_off[job_of] + label, -1)
    n_part = int(part_off[-1])
    sig = gl >= 0
    key = gl[sig] * 36 + np.asarray(sector)[sig]
    uk, cnt = np.unique(key, return_counts=True)
    findable = np.zeros(n_part, bool)
    findable[uk[cnt >= MIN_FINDABLE] // 36] = True
    trk_off = np.asarray(trk_off, np.int64)
    K = len(trk_off) - 1
    if K == 0:
        return dict(n_tracks=0, n_findable=int(findable.sum()), efficiency=0.0, fake_rate=0.0,
                    clone_rate=0.0, hits_in_tracks=0)
    nh = np.diff(trk_off)
    tid = np.repeat(np.arange(K), nh)
    lab = gl[np.asarray(trk_hits)]
    m = lab >= 0
    # majority label per track: count (track, label) pairs
    pair = tid[m].astype(np.int64) * (n_part + 1) + lab[m]
    up, pc = np.unique(pair, return_counts=True)
    pt = up // (n_part + 1)
    pl = up % (n_part + 1)
    order = np.lexsort((-pc, pt))          # per track, largest count first
    first = np.ones(len(order), bool)
    first[1:] = pt[order][1:] != pt[order][:-1]
    best_t = pt[order][first]
    best_l = pl[order][first]
    best_c = pc[order][first]
    good = best_c >= PURITY * nh[best_t]
    found = np.zeros(n_part, np.int64)
    np.add.at(found, best_l[good], 1)
    n_good = int(good.sum())
    nf = int(findable.sum())
    eff = float((found[findable] > 0).sum()) / nf if nf else float("nan")
    clones = int(np.maximum(found - 1, 0).sum())
    out = dict(n_tracks=K, n_findable=nf, efficiency=eff, fake_rate=(K - n_good) / K,
               clone_rate=clones / K, hits_in_tracks=int(trk_off[-1]))
    if by_job:
        part_job = np.searchsorted(part_off, np.arange(n_part), side="right") - 1
        trk_job = job_of[np.asarray(trk_hits)[trk_off[:-1]]]
        out["per_job"] = dict(findable=np.bincount(part_job[findable], minlength=n_jobs),
                              found=np.bincount(part_job[findable & (found > 0)], minlength=n_jobs),
                              tracks=np.bincount(trk_job, minlength=n_jobs),
                              fakes=np.bincount(trk_job, minlength=n_jobs)
                              - np.bincount(trk_job[best_t[good]], minlength=n_jobs))
    if part_pt is not None:
        pt = np.asarray(part_pt)
        eff_pt = {}
        for lo, hi in zip(PT_BINS[:-1], PT_BINS[1:]):
            m = findable & (pt >= lo) & (pt < hi)
            eff_pt[f"{lo:g}-{min(hi, 10):g}"] = float((found[m] > 0).mean()) if m.any() else None
        out["efficiency_vs_pt"] = eff_pt
    return out
