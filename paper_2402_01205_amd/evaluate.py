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


def quality(label, job_off, sector, trk_off, trk_hits, trk_job=None, part_off=None):
    label = np.asarray(label)
    n_jobs = len(job_off) - 1
    job_of = np.repeat(np.arange(n_jobs), np.diff(job_off))
    # global particle id = part_off[job] + label
    if part_off is None:
        part_off = np.zeros(n_jobs + 1, np.int64)
        for j in range(n_jobs):
            lab = label[job_off[j]:job_off[j + 1]]
            part_off[j + 1] = part_off[j] + (int(lab.max()) + 1 if lab.size and lab.max() >= 0 else 0)
    gl = np.where(label >= 0, part_off[job_of] + label, -1)
    n_part = int(part_off[-1])
    # findable: >= MIN_FINDABLE clusters of the particle in one sector
    sig = gl >= 0
    key = gl[sig].astype(np.int64) * 36 + np.asarray(sector)[sig]
    uk, cnt = np.unique(key, return_counts=True)
    findable = np.zeros(n_part, bool)
    findable[(uk[cnt >= MIN_FINDABLE] // 36)] = True
    K = len(trk_off) - 1
    nh = np.diff(trk_off)
    found = np.zeros(n_part, np.int64)
    fakes = 0
    for t in range(K):
        hl = gl[trk_hits[trk_off[t]:trk_off[t + 1]]]
        good = hl[hl >= 0]
        if good.size == 0:
            fakes += 1
            continue
        vals, c = np.unique(good, return_counts=True)
        m = c.argmax()
        if c[m] < PURITY * nh[t]:
            fakes += 1
            continue
        found[vals[m]] += 1
    nf = int(findable.sum())
    eff = float((found[findable] > 0).sum()) / nf if nf else float("nan")
    clones = int(np.maximum(found - 1, 0).sum())
    return dict(n_tracks=K, n_findable=nf, efficiency=eff, fake_rate=fakes / K if K else 0.0,
                clone_rate=clones / K if K else 0.0, hits_in_tracks=int(trk_off[-1]),
                found_any=int((found > 0).sum()))
