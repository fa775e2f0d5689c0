"""Pins of the tracking of loopers' return legs (reading A25 with the return legs generated).

A primary whose circle turns back inside the chamber (2R < 245 cm / cos 10 deg) crosses the
rows a second time on its way in.  The tracker runs along increasing x, so it describes such
a return leg against the momentum: the same circle with sin(phi), tan(lambda) and q/pT of
the opposite sign.  What the geometry fixes, with exact clusters in one sector: the return
leg's clusters there form one track of their own (separate from the outgoing leg's), and its
FP64 fit is the reversed exact state at the innermost hit (the generator's closed form on
the second half turn).  On a full event with return legs: both legs of most loopers are
found, every pure return-leg track of 20 hits or more has a q/pT of the opposite sign of its
particle's charge, and few tracks mix the legs (near the turning point).  The pairing of the
two legs (same circle centre, opposite curvature and tan(lambda), the same z at the turning
point): the legs of exact loopers pair with each other and with nothing across events or
with a flipped curvature; on a full event every pair joins the two legs of one particle.
"""
import math

import numpy as np
import pytest

import oracle.oracle as O
import tpcsynth as g
from tests.truth import true_state, true_state_return


def _looper(pt, eta, phi, q):
    """Both legs of one looper from the origin, every sector, exact clusters."""
    out = []
    for leg in (0, 1):
        ti, sec, row, y, z, _ = g.crossings(np.array([pt]), np.array([eta]), np.array([phi]),
                                            np.array([q]), None, None, leg)
        out.append((sec.astype(np.uint8), row.astype(np.int16), y.astype(np.float32),
                    z.astype(np.float32), np.full(len(sec), leg)))
    sec, row, y, z, leg = (np.concatenate([o[i] for o in out]) for i in range(5))
    return dict(sector=sec, row=row, y=y, z=z, leg=leg, job_off=np.array([0, len(y)], np.int32))


# (pT, eta, phi, q): loopers turning at 2R = 145..200 cm, both charges, both sides
LOOPERS = [(0.12, 0.3, 0.3, 1.0), (0.15, -0.2, 2.0, -1.0), (0.13, 0.5, 4.0, 1.0), (0.11, 0.1, 5.5, -1.0)]


@pytest.mark.parametrize("pt,eta,phi,q", LOOPERS)
def test_return_leg_tracks_carry_the_reversed_state(pt, eta, phi, q):
    """Every track made of return-leg clusters has, at its innermost hit in its sector, the
    FP64 state of the second half turn reversed; the outgoing leg's tracks the forward one;
    no track mixes the legs; most clusters of both legs are on tracks (the rows near the
    turn, where |sin phi| reaches 0.95, cannot be followed)."""
    ev = _looper(pt, eta, phi, q)
    legs = ev["leg"]
    assert (legs == 1).sum() >= 30
    r = O.Run(ev["sector"], ev["row"], ev["y"], ev["z"], ev["job_off"], O.params(merge_edge=-1.0),
              O.STAGE_FIT)
    t = r.tracks(merged=False)
    n_leg = [0, 0]
    checked = [0, 0]
    for i in range(len(t["ndf"])):
        h = t["hits"][t["off"][i]:t["off"][i + 1]]
        lg = legs[h]
        assert (lg == lg[0]).all(), "a track mixes the legs"
        assert t["ndfd"][i] >= 0
        n_leg[lg[0]] += len(h)
        if len(h) < 20:   # a short piece's curvature still leans on the fit's prior
            continue
        sec = int(t["sector"][i])
        xi = float(O.row_x(int(ev["row"][h[0]])))
        fn = true_state_return if lg[0] == 1 else true_state
        ok, yi, zi, si, ti, ki = fn(pt, eta, phi, q, sec, xi)
        assert ok
        P = t["Pd"][i]
        # exact clusters (FP32), the fit's priors pulling a little on these strongly curved
        # tracks: 10^-3 cm, 10^-4 in sin(phi) and tan(lambda), 10^-3 relative in q/pT
        assert abs(P[0] - yi) < 1e-3 and abs(P[1] - zi) < 1e-3, (lg[0], P, yi, zi)
        assert abs(P[2] - si) < 1e-4 and abs(P[3] - ti) < 1e-4, (lg[0], P, si, ti)
        assert abs(P[4] - ki) < 1e-3 * abs(ki), (lg[0], P[4], ki)
        checked[lg[0]] += 1
    assert n_leg[0] >= 0.7 * (legs == 0).sum() and n_leg[1] >= 0.7 * (legs == 1).sum(), n_leg
    assert checked[0] >= 1 and checked[1] >= 1


def test_full_event_with_return_legs():
    cs = g.gen_event(21, 3000, loopers=True)
    leg = cs.meta["leg"]
    t = O.Run.from_set(cs).tracks()
    has_ret = np.unique(cs.label[leg == 1])
    found_ret, mixed, sign_ok, n_ret = set(), 0, 0, 0
    for i in range(len(t["ndf"])):
        h = t["hits"][t["off"][i]:t["off"][i + 1]]
        lg = leg[h]
        if (lg == 1).all():
            p = int(cs.label[h][0])
            found_ret.add(p)
            if (cs.label[h] == p).all() and len(h) >= 20 and t["ndf"][i] >= 0:
                n_ret += 1
                sign_ok += int(np.sign(t["P"][i][4]) == -cs.part_q[p])
        elif not (lg == 0).all():
            mixed += 1
    assert len(has_ret) > 500
    assert len(found_ret) >= 0.75 * len(has_ret)
    assert n_ret > 300 and sign_ok == n_ret
    assert mixed <= 0.03 * len(t["ndf"])


@pytest.mark.parametrize("pt,eta,phi,q", LOOPERS)
def test_the_two_legs_of_an_exact_looper_pair(pt, eta, phi, q):
    """Exact looper, sector merge on: one track per leg, and the pairing joins them."""
    ev = _looper(pt, eta, phi, q)
    t = O.Run(ev["sector"], ev["row"], ev["y"], ev["z"], ev["job_off"], O.params()).tracks()
    kinds = [int(ev["leg"][t["hits"][t["off"][i]]]) for i in range(len(t["ndf"]))]
    assert sorted(kinds) == [0, 1]
    leg = O.pair_legs(t, np.zeros(len(kinds), np.int32))
    assert leg.tolist() == [1, 0]
    # no pair across events, nor with the curvature of one leg flipped
    assert O.pair_legs(t, np.array([0, 1], np.int32)).tolist() == [-1, -1]
    t2 = dict(t)
    t2["P"] = t["P"].copy()
    t2["P"][1, 4] = -t2["P"][1, 4]
    assert O.pair_legs(t2, np.zeros(2, np.int32)).tolist() == [-1, -1]


def test_legs_pair_within_their_particle_on_a_full_event():
    """Full event with return legs: nearly every return-leg track is paired, every pair joins
    the two legs of one particle, and only looper curvatures pair."""
    cs = g.gen_event(21, 3000, loopers=True)
    leg = cs.meta["leg"]
    t = O.Run.from_set(cs).tracks()
    pairs = O.pair_legs(t, np.zeros(len(t["ndf"]), np.int32))
    assert np.all(pairs[pairs[pairs >= 0]] == np.flatnonzero(pairs >= 0))   # mutual
    # the centre cells only prune: every pair of tracks compared gives the same pairs
    assert np.array_equal(pairs, O.pair_legs(t, np.zeros(len(t["ndf"]), np.int32), brute=True))
    n_ret, good, n_pairs = 0, 0, 0
    cmin = 2.0 / (245.0 / math.cos(math.radians(10.0)))
    for i in range(len(t["ndf"])):
        h = t["hits"][t["off"][i]:t["off"][i + 1]]
        lab = cs.label[h]
        maj = np.bincount(lab[lab >= 0]).argmax()
        lg = np.bincount(leg[h][leg[h] >= 0]).argmax()
        n_ret += int(lg == 1 and (lab == maj).mean() >= 0.9)
        j = pairs[i]
        if j < 0 or j < i:
            continue
        n_pairs += 1
        assert abs(0.299792458e-2 * 0.5 * t["P"][i][4]) > cmin
        hj = t["hits"][t["off"][j]:t["off"][j + 1]]
        mj = np.bincount(cs.label[hj][cs.label[hj] >= 0]).argmax()
        lj = np.bincount(leg[hj][leg[hj] >= 0]).argmax()
        good += int(maj == mj and lg != lj)
    assert n_pairs >= 0.9 * n_ret and good == n_pairs, (n_pairs, n_ret, good)
