"""Pins of the oracle's collision time (continuous read-out) against what the geometry fixes.

A collision at time t0 after the frame start shifts every measured z by v_d t0 towards the
far side of the central membrane (z - v_d t0 on side A, z + v_d t0 on side C), so a primary
from the nominal vertex crosses the beam line at measured z = -v_d t0 (A) or +v_d t0 (C).
Checked against: exact helix states from the generator's closed form shifted by known
times (one state at a time), zero-smear time frames whose tracks must return their
collision's time, and the generator's collision times on a smeared time frame.
"""
import numpy as np
import pytest

import oracle.oracle as O
import tpcsynth as g
from tests.truth import true_state

V_D = float(np.float32(2.58))     # the parameter is FP32


def _particles(n, seed):
    rng = np.random.default_rng(seed)
    pt = np.exp(rng.uniform(np.log(0.15), np.log(10.0), n))
    eta = rng.uniform(-0.9, 0.9, n)
    phi = rng.uniform(0.02, 0.33, n)          # sector 0 (A) or 18 (C) by the sign of eta
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    t0 = rng.uniform(0.0, 1000.0, n)
    return pt, eta, phi, q, t0


@pytest.mark.parametrize("fp64", [True, False])
def test_collision_time_of_exact_shifted_states(fp64):
    """A true helix state at a pad-row plane, its z shifted by the drift of a known time:
    the collision time comes back (FP64 to 1e-8 us, FP32 to its rounding)."""
    pt, eta, phi, q, t0 = _particles(400, 5)
    n_ok = 0
    for i in range(len(pt)):
        sec = 0 if eta[i] >= 0 else 18
        for x in (O.row_x(0), O.row_x(60), O.row_x(140)):
            ok, y, z, s, t, k = true_state(pt[i], eta[i], phi[i], q[i], sec, x)
            if not ok or abs(s) >= 0.9:
                continue
            zm = z - V_D * t0[i] if sec < 18 else z + V_D * t0[i]
            P = np.array([y, zm, s, t, k])
            got = O.collision_time(P, x, sec, fp64=fp64)
            if fp64:
                assert abs(got - t0[i]) < 1e-8 * max(1.0, t0[i]), (i, x, got, t0[i])
            else:
                # FP32: z up to ~2600 cm carries ~1.5e-4 cm of rounding (6e-5 us)
                assert abs(got - t0[i]) < 2e-4 + 2e-6 * t0[i], (i, x, got, t0[i])
            n_ok += 1
    assert n_ok > 600


def test_collision_time_sign_per_side():
    """The same state in a sector of side A and of side C: opposite times."""
    P = np.array([1.0, -30.0, 0.1, 0.2, 0.5])
    ta = O.collision_time(P, O.row_x(10), 3, fp64=True)
    tc = O.collision_time(P, O.row_x(10), 21, fp64=True)
    assert ta > 0 and abs(ta + tc) < 1e-12


def _truth_times(cs):
    """Collision time of every particle of a time frame."""
    off = np.asarray(cs.meta["coll_part_off"], np.int64)
    tk = np.asarray(cs.meta["t_collisions"])
    coll = np.repeat(np.arange(len(tk)), np.diff(off))
    return tk[coll]


def _majority(cs, t):
    lab = np.full(len(t["tracklet"]), -1, np.int64)
    pur = np.zeros(len(t["tracklet"]))
    nh = np.diff(t["off"])
    for i in range(len(lab)):
        ls = cs.label[t["hits"][t["off"][i]:t["off"][i + 1]]]
        ls = ls[ls >= 0]
        if len(ls):
            v, c = np.unique(ls, return_counts=True)
            lab[i] = v[np.argmax(c)]
            pur[i] = c.max() / nh[i]
    return lab, pur, nh


def test_zero_smear_time_frame_returns_each_collision_time():
    """Four collisions without smear, noise or inefficiency, inside a wide window: every
    pure track's FP64 collision time equals its collision's time."""
    pool = g.gen_collision_pool(71, 4, mult_range=(150, 150), ineff=0.0, smear=0.0)
    cs = g.assemble_timeframe(72, pool, np.arange(4), 1000.0, noise=0.0)
    t = O.Run.from_set(cs).tracks()
    lab, pur, nh = _majority(cs, t)
    truth = _truth_times(cs)
    sel = (pur == 1.0) & (nh >= 20) & (t["ndfd"] >= 0) & (lab >= 0)
    assert sel.sum() > 300
    # the clusters are FP32 (z up to ~1000 cm: ~3e-5 cm of rounding each), which the
    # extrapolation to the beam line can amplify a few times: well under 1e-3 us
    d = np.abs(t["t0d"][sel] - truth[lab[sel]])
    assert np.median(d) < 1e-5 and d.max() < 1e-3, (np.median(d), d.max())
    # the FP32 fit of the same hits: within its precision (z of ~1000 cm in FP32)
    d32 = np.abs(t["t0"][sel] - truth[lab[sel]])
    assert d32.max() < 5e-3, d32.max()
    sides = t["sector"][sel] < 18
    assert sides.any() and (~sides).any()
    assert len(np.unique(truth[lab[sel]])) == 4


def test_smeared_time_frame_collision_times():
    """Five collisions of the time-frame workload's law (smear 0.1 cm, noise, inefficiency):
    the collision times of good tracks scatter around the truth by the z resolution."""
    cs = g.make_config("c3", 31, scale=0.1)
    t = O.Run.from_set(cs).tracks()
    lab, pur, nh = _majority(cs, t)
    truth = _truth_times(cs)
    sel = (pur >= 0.9) & (nh >= 30) & (t["ndf"] >= 0) & (lab >= 0)
    assert sel.sum() > 1000
    d = t["t0"][sel] - truth[lab[sel]]
    assert abs(np.median(d)) < 0.01
    assert np.median(np.abs(d)) < 0.05
    # pulls against the error of the fitted z transported to the beam line (FP64 covariance)
    sig = np.zeros(int(sel.sum()))
    for j, i in enumerate(np.flatnonzero(sel)):
        ok, _, Cv = O.propagate(t["Pd"][i], t["Cd"][i], float(t["xd"][i]), 0.0, fp64=True)
        assert ok
        sig[j] = np.sqrt(Cv[2]) / V_D          # C_zz: lower-triangle index 2
    pull = d / sig
    assert 0.8 < np.std(pull[np.abs(pull) < 6]) < 1.3, np.std(pull)
    assert np.mean(np.abs(pull) < 5) > 0.995
    # FP32 and FP64 agree within their rounding
    assert np.nanmax(np.abs(t["t0"][sel] - t["t0d"][sel])) < 2e-3
