"""The oracle's index tie-breaks on inputs with exact ties (readings R10, R16, R20).

Clusters on a 1/32-cm (or coarser) lattice with a fraction duplicated exactly: a
duplicate has the same coordinates as its original, so every score, chi2 and merge
chi2 computed with it equals the original's.  The method then defines the winner by
the smaller input index (links: of u, then of d; following: of the cluster; merge:
of the track id).  These tests check that definition directly on the oracle's
outputs: whenever a picked cluster or track has an identical twin, the pick is the
smallest index of its group.  A tie-break that takes the first candidate found, the
larger index, or compares the wrong index would fail them.
"""
import numpy as np
import pytest

import oracle.oracle as O
import tpcsynth as g


def _group_min(groups):
    """Per cluster: the smallest input index with the same group."""
    order = np.argsort(groups, kind="stable")
    gs = groups[order]
    first = np.r_[True, gs[1:] != gs[:-1]]
    mins = order[first]
    return mins[np.cumsum(first) - 1][np.argsort(order)]


def _dup_info(cs):
    grp = cs.meta["dup_group"]
    size = np.bincount(grp)[grp]
    return grp, size, _group_min(grp)


@pytest.mark.parametrize("cfg,seed,scale,q", [("c1", 11, 1.0, 1 / 32), ("c1", 12, 1.0, 1 / 4),
                                              ("c2", 21, 0.1, 1 / 32)])
def test_links_and_tracklets_take_the_smallest_index_of_a_tie(cfg, seed, scale, q):
    cs = g.with_exact_ties(g.make_config(cfg, seed, scale=scale), q, 0.15, seed + 100)
    grp, size, gmin = _dup_info(cs)
    r = O.Run.from_set(cs)
    L = r.links()
    n_tie = 0
    for key in ("up_raw", "down_raw"):
        v = L[key]
        has = v >= 0
        tied = has & (size[np.maximum(v, 0)] > 1)
        n_tie += int(tied.sum())
        assert np.all(v[tied] == gmin[v[tied]]), key
    assert n_tie > 200
    # a duplicate sees the same candidates as its twin, so identical clusters pick
    # identical raw links
    for key in ("up_raw", "down_raw"):
        v = L[key]
        assert np.array_equal(v, v[gmin]), key
    # only the smallest index of a group can hold a clean link (the others lose mutuality)
    for key in ("up", "down"):
        v = L[key]
        assert np.all(v[v >= 0] == gmin[v[v >= 0]])
        assert np.all(v[gmin != np.arange(cs.n)] == -1)
    T = r.tracklets()
    h = T["hits"]
    tied = size[h] > 1
    assert tied.sum() > 200
    assert np.all(h[tied] == gmin[h[tied]])


def test_merge_takes_the_smaller_track_id_of_a_tie():
    """A full event split into per-sector jobs of one event, every sector job present
    twice: each boundary crosser has two identical candidates on either side, whose
    merge chi2 are equal; the mutual best pair is the one of the smaller ids."""
    cs = g.make_config("c2", 23, scale=0.2)
    order = np.argsort(cs.sector, kind="stable")
    cuts = np.searchsorted(cs.sector[order], np.arange(37)).astype(np.int32)
    split = g.ClusterSet(cs.sector[order], cs.row[order], cs.y[order], cs.z[order], cs.time[order],
                         cs.label[order], cuts, cs.part_pt, cs.part_eta, cs.part_phi, cs.part_q,
                         np.array([0] + [0] * 35 + [len(cs.part_pt)]), {})
    twice = g.concat([split, split])
    ev = np.zeros(twice.n_jobs, np.int32)
    r = O.Run.from_set(twice, job_event=ev)
    all_t = O.Run.from_set(twice, last_stage=O.STAGE_FIT, job_event=ev).tracks(merged=False)
    K = len(all_t["tracklet"])
    half = K // 2
    assert K == 2 * half
    # the two copies find identical pieces (hits relative to their job's first cluster)
    jo = twice.job_off
    rel = all_t["hits"] - np.repeat(jo[all_t["job"]], np.diff(all_t["off"]))
    H = all_t["off"][half]
    assert np.array_equal(rel[:H], rel[H:]) and np.array_equal(all_t["job"][:half] + 36, all_t["job"][half:])
    assert np.array_equal(all_t["P"][:half].view(np.uint32), all_t["P"][half:].view(np.uint32))
    m = r.tracks(merged=True)
    merged = m["sector2"] >= 0
    assert merged.sum() > 50
    # every merged chain is made of first-copy tracks only: the second copies' candidates
    # tie with the first copies' and lose on the id
    for i in np.nonzero(merged)[0]:
        assert np.all(m["hits"][m["off"][i]:m["off"][i + 1]] < twice.job_off[36])
    # the second copy's pieces stay unmerged
    second = m["job"] >= 36
    assert second.sum() > 0 and not np.any(merged & second)
