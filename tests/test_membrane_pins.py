"""Pins of the oracle's merge across the central membrane (reading A21).

What the geometry fixes: a primary from a vertex at z0 != 0 whose z = z0 + tan(lambda) arc
changes sign inside the chamber leaves a piece on each side of the membrane, in the same
sector frame.  With exact clusters the two pieces must become one track holding every
cluster, whose FP64 fit is the exact helix state (generator's closed form) at the innermost
hit.  In a time frame the two sides' measured z are off by v t0 in opposite directions, so
the merged track's collision time must come back from the z offset between the pieces: to
FP32 rounding of z for exact clusters, and with its error set by the cluster resolution in a
smeared time frame (where the vertex-based time of T1 is off by z0 / v).  Pieces that do not
belong together (a track leaving the membrane on the other side, a parameter mismatch) are
not merged, and nothing is merged with the membrane merge off.
"""
import math

import numpy as np
import pytest

import oracle.oracle as O
import tpcsynth as g
from tests.truth import true_state

V_D = float(np.float32(2.58))


def _crosser(pt, eta, phi, q, z0):
    """Exact crossings of one primary from (0, 0, z0), sector-0 phi, both sides."""
    ti, sec, row, y, z, _ = g.crossings(np.array([pt]), np.array([eta]), np.array([phi]),
                                        np.array([q]), None, np.array([z0]))
    return sec.astype(np.uint8), row.astype(np.int16), y, z


def _set(parts, t0=0.0):
    """One job from [(sec, row, y, z), ...]; z shifted as a time frame shifts it for a
    collision at t0 (side A: z - v t0, side C: z + v t0)."""
    sec = np.concatenate([p[0] for p in parts])
    row = np.concatenate([p[1] for p in parts])
    y = np.concatenate([p[2] for p in parts]).astype(np.float32)
    z = np.concatenate([p[3] for p in parts])
    z = np.where(sec < 18, z - V_D * t0, z + V_D * t0).astype(np.float32)
    lab = np.concatenate([np.full(len(p[0]), i) for i, p in enumerate(parts)]).astype(np.int32)
    return dict(sector=sec, row=row, y=y, z=z, job_off=np.array([0, len(y)], np.int32), label=lab)


def _run(ev, **over):
    return O.Run(ev["sector"], ev["row"], ev["y"], ev["z"], ev["job_off"], O.params(**over))


PHI0 = float(g.sector_alpha(0))
# (pT, eta, z0, phi - sector centre): crossing the membrane at radii from ~110 to ~200 cm,
# both directions, positive charges turning clockwise from phi inside sector 0 to its end
CROSSERS = [(1.5, -0.045, 6.0, 0.06), (0.8, -0.03, 5.0, 0.12), (3.0, 0.05, -8.0, 0.03),
            (0.6, 0.06, -12.0, 0.15)]


@pytest.mark.parametrize("t0", [0.0, 123.4])
@pytest.mark.parametrize("pt,eta,z0,dphi", CROSSERS)
def test_crossing_track_is_one_track_with_its_collision_time(pt, eta, z0, dphi, t0):
    sec, row, y, z = _crosser(pt, eta, PHI0 + dphi, 1.0, z0)
    assert (sec < 18).sum() >= 15 and (sec >= 18).sum() >= 15 and set(sec % 18) == {0}
    ev = _set([(sec, row, y, z)], t0)
    off = _run(ev, merge_membrane=0).tracks()
    assert len(off["ndf"]) == 2 and np.all(off["sector2"] < 0)
    t = _run(ev, merge_membrane=1).tracks()
    assert len(t["ndf"]) == 1
    h = t["hits"]
    assert sorted(h.tolist()) == list(range(len(sec)))
    inner = int(t["sector"][0])
    assert inner == int(sec[np.argmin(row)]) and int(t["sector2"][0]) == (inner + 18) % 36
    # the time from the pieces' z offset: FP32 rounding of z (|z| up to ~320 cm)
    assert abs(t["t0"][0] - t0) < 2e-4, (t["t0"][0], t0)
    assert abs(t["t0d"][0] - t0) < 2e-4
    # the FP64 fit of the whole list: the exact state at the innermost hit, in the inner
    # side's measured z
    xi = float(O.row_x(int(row[h[0]])))
    ok, yi, zi, si, ti, ki = true_state(pt, eta, PHI0 + dphi, 1.0, inner, xi, z0)
    zi_meas = zi - V_D * t0 if inner < 18 else zi + V_D * t0
    P = t["Pd"][0]
    assert abs(P[0] - yi) < 1e-4 and abs(P[1] - zi_meas) < 2e-3, (P, yi, zi_meas)
    assert abs(P[2] - si) < 1e-5 and abs(P[3] - ti) < 1e-5
    assert abs(P[4] - ki) < 1e-3 * abs(ki)
    assert t["ndf"][0] == 2 * len(h) - 5


def test_pieces_that_leave_the_membrane_are_not_merged():
    """The C-side piece of a crosser together with an A-side track from the vertex that
    runs away from the membrane (tan lambda > 0) at the same y: no membrane link."""
    sec, row, y, z = _crosser(1.5, -0.045, PHI0 + 0.06, 1.0, 6.0)
    c_side = sec >= 18
    sa, ra, ya, za = _crosser(1.5, 0.02, PHI0 + 0.06, 1.0, 0.5)
    a_side = sa < 18
    ev = _set([(sec[c_side], row[c_side], y[c_side], z[c_side]),
               (sa[a_side], ra[a_side], ya[a_side], za[a_side])])
    t = _run(ev, merge_membrane=1).tracks()
    assert len(t["ndf"]) == 2 and np.all(t["sector2"] < 0)


def test_mismatched_pieces_are_not_merged():
    """The two sides of two different crossers (curvatures of opposite sign): no link."""
    s1, r1, y1, z1 = _crosser(1.5, -0.045, PHI0 + 0.06, 1.0, 6.0)
    s2, r2, y2, z2 = _crosser(1.5, -0.045, PHI0 - 0.06, -1.0, 6.0)
    ev = _set([(s1[s1 < 18], r1[s1 < 18], y1[s1 < 18], z1[s1 < 18]),
               (s2[s2 >= 18], r2[s2 >= 18], y2[s2 >= 18], z2[s2 >= 18])])
    t = _run(ev, merge_membrane=1).tracks()
    assert len(t["ndf"]) == 2 and np.all(t["sector2"] < 0)


def _truth_time_and_vertex(cs):
    off = np.asarray(cs.meta["coll_part_off"], np.int64)
    coll = np.repeat(np.arange(len(off) - 1), np.diff(off))
    return np.asarray(cs.meta["t_collisions"])[coll], np.asarray(cs.meta["vertex_z"])[coll]


@pytest.fixture(scope="module")
def tf():
    pool = g.gen_collision_pool(77, 6, vz_sigma=8.0)
    cs = g.assemble_timeframe(78, pool, np.arange(6), 500.0)
    return cs, O.Run.from_set(cs, O.params(merge_membrane=1)).tracks()


def test_time_frame_membrane_merges(tf):
    """Smeared time frame, vertices at z ~ N(0, 8 cm): every membrane-merged track joins the
    two sides of one particle; their collision times scatter around the truth by the z
    resolution, while the vertex-based time of the same particles is off by z0 / v."""
    cs, t = tf
    truth_t, truth_vz = _truth_time_and_vertex(cs)
    memb = (t["sector2"] >= 0) & ((t["sector"] < 18) != (t["sector2"] < 18))
    assert memb.sum() > 100
    labs, pure = [], 0
    for i in np.flatnonzero(memb):
        h = t["hits"][t["off"][i]:t["off"][i + 1]]
        l = cs.label[h]
        v, c = np.unique(l[l >= 0], return_counts=True)
        p = v[np.argmax(c)]
        labs.append(p)
        mine = cs.sector[h[l == p]]
        pure += int(c.max() >= 0.9 * len(h) and (mine < 18).any() and (mine >= 18).any())
    assert pure >= 0.98 * memb.sum()
    labs = np.array(labs)
    d = t["t0"][memb] - truth_t[labs]
    assert np.median(np.abs(d)) < 0.02 and np.percentile(np.abs(d), 95) < 0.06
    # the same tracks' vertex-based time (T1) carries the vertex offset
    x = t["x"][memb]
    tv = np.array([O.collision_time(t["P"][i], float(t["x"][i]), int(t["sector"][i]))
                   for i in np.flatnonzero(memb)])
    bias = tv - truth_t[labs]
    vz = truth_vz[labs]
    sgn = np.where(t["sector"][memb] < 18, 1.0, -1.0)
    assert np.median(np.abs(bias + sgn * vz / V_D)) < 0.05


def test_membrane_merge_off_and_sync_change_nothing(tf):
    cs, t = tf
    base = O.Run.from_set(cs).tracks()
    assert not ((base["sector2"] >= 0) & ((base["sector"] < 18) != (base["sector2"] < 18))).any()
    sync = O.Run.from_set(cs, O.params(**dict(O.SYNC, merge_membrane=1))).tracks()
    assert np.all(sync["sector2"] < 0)
