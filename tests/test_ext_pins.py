"""Pins of the oracle's downward extension of the selected tracks (reading A13).

What the geometry fixes: a link spans at most two rows, so rows that hold clusters only
every third row (all particles alike) form no chain, and every tracklet starts above
them.  The extension visits every row below a track's innermost hit and tolerates
max_miss consecutive empty rows, so it must recover every lower cluster of the track when
the gaps are shorter than max_miss and none when they are longer.  With exact clusters
the extended track's FP64 fit is the exact helix state at its new innermost hit (from the
generator's closed form).  Two tracks that both find the same clusters: the one with more
owned hits takes them and the other keeps nothing after the first cluster it lost.
Invariants on a realistic event: the extension takes only clusters that no selected track
owns, below the track's selected hits and in its sector, and no cluster ends on two
tracks.  Which cluster the window search picks among several is pinned only by these
special cases and invariants (the same holds for the following above the chains).
"""
import math

import numpy as np
import pytest

import oracle.oracle as O
import tpcsynth as g
from tests.truth import true_state

R_CUT = 60          # rows below this keep clusters only every k-th row


def _particle_clusters(pt, eta, phi, q, rows):
    """Exact (FP32) crossings of one primary with the given rows of sector 0."""
    out = []
    for r in rows:
        x = float(O.row_x(r))
        ok, y, z, s, t, k = true_state(pt, eta, phi, q, 0, x)
        if ok and abs(y) <= x * math.tan(math.radians(10.0)) and abs(z) <= 250.0:
            out.append((r, np.float32(y), np.float32(z)))
    return out


def _cluster_set(parts):
    """A one-job, sector-0 cluster list from [(label, [(row, y, z), ...]), ...]."""
    rows, ys, zs, lab = [], [], [], []
    for p, cl in parts:
        for r, y, z in cl:
            rows.append(r); ys.append(y); zs.append(z); lab.append(p)
    n = len(rows)
    return dict(sector=np.zeros(n, np.uint8), row=np.array(rows, np.int16),
                y=np.array(ys, np.float32), z=np.array(zs, np.float32),
                job_off=np.array([0, n], np.int32), label=np.array(lab, np.int32))


def _thinned_event(seed, n, step, r_cut=R_CUT):
    """n primaries in sector 0 (pT 0.5-5 GeV), all rows from r_cut up, below it every
    `step`-th row counted down from r_cut."""
    rng = np.random.default_rng(seed)
    a = float(g.sector_alpha(0))
    lower = [r for r in range(r_cut - step, -1, -step)]
    parts, truth = [], []
    for p in range(n):
        pt = float(np.exp(rng.uniform(np.log(0.5), np.log(5.0))))
        eta = float(rng.uniform(0.05, 0.85))
        phi = float(a + rng.uniform(-0.12, 0.12))
        q = float(rng.choice([-1.0, 1.0]))
        parts.append((p, _particle_clusters(pt, eta, phi, q, list(range(r_cut, 152)) + lower)))
        truth.append((pt, eta, phi, q))
    return _cluster_set(parts), truth


def _run(ev, stage=O.STAGE_FIT, **over):
    return O.Run(ev["sector"], ev["row"], ev["y"], ev["z"], ev["job_off"], O.params(**over), stage)


def test_extension_recovers_every_lower_cluster():
    ev, truth = _thinned_event(3, 25, 3)
    t0 = _run(ev, ext_down=0).tracks()
    t1 = _run(ev, ext_down=1).tracks()
    lab, row = ev["label"], ev["row"]
    assert len(t0["ndf"]) == len(t1["ndf"]) >= 15
    assert np.array_equal(t0["tracklet"], t1["tracklet"])
    checked = 0
    for i in range(len(t1["ndf"])):
        h0 = t0["hits"][t0["off"][i]:t0["off"][i + 1]]
        h1 = t1["hits"][t1["off"][i]:t1["off"][i + 1]]
        p = lab[h0[0]]
        assert np.all(lab[h0] == p)
        # without the extension the track starts at R_CUT or above: nothing below forms a chain
        assert row[h0].min() >= R_CUT and t0["n_ext"][i] == 0
        # with it the track holds every cluster of its particle, rows ascending
        mine = np.flatnonzero(lab == p)
        assert sorted(h1.tolist()) == sorted(mine.tolist())
        assert np.all(np.diff(row[h1]) > 0)
        assert t1["n_ext"][i] == int((row[mine] < R_CUT).sum())
        assert np.array_equal(h1[t1["n_ext"][i]:], h0)
        if t1["n_ext"][i] == 0:
            continue
        # the FP64 fit of the extended track: the exact state at its new innermost hit
        pt, eta, phi, q = truth[p]
        xi = float(O.row_x(int(row[h1[0]])))
        assert t1["xd"][i] == pytest.approx(xi, abs=1e-5)
        _, yi, zi, si, ti, ki = true_state(pt, eta, phi, q, 0, xi)
        P = t1["Pd"][i]
        assert abs(P[0] - yi) < 1e-4 and abs(P[1] - zi) < 1e-4, (P, yi, zi)
        assert abs(P[2] - si) < 1e-5 and abs(P[3] - ti) < 1e-5
        assert abs(P[4] - ki) < 1e-3 * abs(ki)
        assert t1["ndf"][i] == 2 * len(h1) - 5 and t1["ndfd"][i] == 2 * len(h1) - 5
        checked += 1
    assert checked >= 12


@pytest.mark.parametrize("max_miss,found", [(4, False), (6, True)])
def test_extension_stops_after_max_miss_empty_rows(max_miss, found):
    """Lower clusters every 6th row: five empty rows between them end the extension at
    max_miss = 4 and not at max_miss = 6."""
    ev, _ = _thinned_event(4, 12, 6)
    t0 = _run(ev, ext_down=0, max_miss=max_miss).tracks()
    t1 = _run(ev, ext_down=1, max_miss=max_miss).tracks()
    assert len(t1["ndf"]) >= 10
    if not found:
        assert t1["n_ext"].sum() == 0
        for k in ("off", "hits", "P", "C", "x", "chi2", "ndf"):
            assert np.array_equal(t0[k], t1[k], equal_nan=True), k
    else:
        lab, row = ev["label"], ev["row"]
        for i in range(len(t1["ndf"])):
            h1 = t1["hits"][t1["off"][i]:t1["off"][i + 1]]
            mine = np.flatnonzero(lab == lab[h1[-1]])
            assert t1["n_ext"][i] == int((row[mine] < R_CUT).sum()) > 0


@pytest.mark.parametrize("longer", ["A", "B"])
def test_contested_clusters_go_to_the_track_with_more_hits(longer):
    """Particle B runs 0.08-0.2 cm beside A (same vertex, phi 1.5 mrad apart, 2 GeV) and has
    no clusters below R_CUT; A has them every third row.  Both tracks find A's lower
    clusters.  The longer track takes them all; the shorter one loses the first and keeps
    nothing."""
    a = float(g.sector_alpha(0))
    top_a = 151 if longer == "A" else 130
    top_b = 130 if longer == "A" else 151
    lower = list(range(R_CUT - 3, -1, -3))
    ca = _particle_clusters(2.0, 0.3, a, 1.0, list(range(R_CUT, top_a + 1)) + lower)
    cb = _particle_clusters(2.0, 0.3, a + 0.0015, 1.0, list(range(R_CUT, top_b + 1)))
    ev = _cluster_set([(0, ca), (1, cb)])
    t = _run(ev, ext_down=1).tracks()
    lab, row = ev["label"], ev["row"]
    assert len(t["ndf"]) == 2
    owner = [int(lab[t["hits"][t["off"][i + 1] - 1]]) for i in range(2)]
    assert sorted(owner) == [0, 1]
    ia, ib = owner.index(0), owner.index(1)
    low_a = np.flatnonzero((lab == 0) & (row < R_CUT))
    ha = t["hits"][t["off"][ia]:t["off"][ia + 1]]
    hb = t["hits"][t["off"][ib]:t["off"][ib + 1]]
    if longer == "A":
        assert t["n_ext"][ia] == len(low_a) and t["n_ext"][ib] == 0
        assert sorted(ha[:len(low_a)].tolist()) == sorted(low_a.tolist())
        assert np.all(lab[hb] == 1)
    else:
        assert t["n_ext"][ia] == 0 and t["n_ext"][ib] == len(low_a)
        assert sorted(hb[:len(low_a)].tolist()) == sorted(low_a.tolist())
        assert np.all(lab[ha] == 0)


@pytest.fixture(scope="module")
def dense():
    cs = g.make_config("c4", 41, jobs=[0, 8, 120])
    sel = O.Run.from_set(cs, last_stage=O.STAGE_SELECT).tracks(merged=False)
    ext = O.Run.from_set(cs, O.params(ext_down=1), last_stage=O.STAGE_FIT).tracks(merged=False)
    return cs, sel, ext


def test_extension_invariants_on_dense_jobs(dense):
    cs, sel, ext = dense
    assert np.array_equal(sel["tracklet"], ext["tracklet"])
    owned = np.zeros(cs.n, bool)
    owned[sel["hits"]] = True
    seen = np.zeros(cs.n, np.int32)
    np.add.at(seen, ext["hits"], 1)
    assert seen.max() == 1, "a cluster on two tracks"
    n_ext_total = 0
    for i in range(len(ext["ndf"])):
        hs = sel["hits"][sel["off"][i]:sel["off"][i + 1]]
        he = ext["hits"][ext["off"][i]:ext["off"][i + 1]]
        m = int(ext["n_ext"][i])
        assert np.array_equal(he[m:], hs)
        if m == 0:
            continue
        n_ext_total += m
        xh = he[:m]
        assert not owned[xh].any()
        assert np.all(np.diff(cs.row[xh]) > 0) and cs.row[xh].max() < cs.row[hs].min()
        assert np.all(cs.sector[xh] == cs.sector[hs[0]])
        assert np.all((xh >= cs.job_off[ext["job"][i]]) & (xh < cs.job_off[ext["job"][i] + 1]))
    assert n_ext_total > 1000


def test_extension_refits_the_extended_list(dense):
    """The reported state of an extended track is the fit of its whole hit list."""
    cs, sel, ext = dense
    r = O.Run.from_set(cs, O.params(ext_down=1), last_stage=O.STAGE_TRACKLETS)
    trk = r.tracklets()
    idx = np.flatnonzero(ext["n_ext"] > 0)[::50]
    assert len(idx) >= 10
    for i in idx:
        he = ext["hits"][ext["off"][i]:ext["off"][i + 1]]
        stk = trk["P"][ext["tracklet"][i], 2:5]
        ok, P, Cv, x, c2 = r.fit_hits(he, stk, fp64=False)
        if ext["ndf"][i] < 0:
            assert not ok
            continue
        assert ok
        assert np.array_equal(P[:5].astype(np.float32), ext["P"][i]) and np.float32(x) == ext["x"][i]
        assert np.array_equal(Cv.astype(np.float32), ext["C"][i])
