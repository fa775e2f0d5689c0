"""Pins of the oracle's track-model compression (section 5: clusters stored as residuals to
the fitted tracks).

The prediction is checked against the generator's closed-form helix (circle/plane
intersection in FP64, rotated sector frames included); clusters placed exactly on the
generated helices must give residual codes of at most one step; codes of clusters in no
track are numpy's round-half-even of v/q; and decoding restores every cluster within half a
quantisation step.
"""
import math

import numpy as np
import pytest

import oracle.oracle as O
import tpcsynth as g
from tests.truth import true_state

ROWX32 = np.array([np.float32(85.0 + r * 160.0 / 151.0) for r in range(152)], np.float32)
Q = 1.0 / 32.0


def _tracks(cs, seed_params=None):
    r = O.Run.from_set(cs, seed_params)
    return r.tracks(merged=True)


def _permutation(n, t):
    """Stream order of the clusters: track hits in track order, then the rest in input order."""
    rest = np.setdiff1d(np.arange(n), t["hits"])
    return np.concatenate([t["hits"], rest]).astype(np.int64)


@pytest.mark.parametrize("steps", [0, 1, -1, 2, -2])
def test_prediction_against_the_closed_form_helix(steps):
    """C1: rotate sector by sector, then transport: the FP32 prediction equals the exact
    circle/plane crossing in the target sector's frame within FP32 rounding."""
    rng = np.random.default_rng(100 + steps)
    checked = 0
    for _ in range(400):
        pt = float(np.exp(rng.uniform(np.log(0.4), np.log(5.0))))
        eta = float(rng.uniform(-0.8, 0.8))
        q = float(rng.choice([-1.0, 1.0]))
        s0 = int(rng.integers(0, 18)) + (18 if eta < 0 else 0)
        phi = float(g.sector_alpha(s0)) + float(rng.uniform(-0.15, 0.15))
        r0 = int(rng.integers(0, 40))
        s1 = (s0 // 18) * 18 + (s0 % 18 + steps) % 18
        r1 = int(rng.integers(0, 152))
        ok0, y0, z0, sn0, t0, k0 = true_state(pt, eta, phi, q, s0, float(ROWX32[r0]))
        ok1, y1, z1, _, _, _ = true_state(pt, eta, phi, q, s1, float(ROWX32[r1]))
        if not (ok0 and ok1) or abs(sn0) > 0.8:
            continue
        P = np.array([y0, z0, sn0, t0, k0], np.float32)
        ok, py, pz = O.predict(P, float(ROWX32[r0]), s0, s1, r1)
        if not ok:
            continue
        assert abs(py - y1) < 2e-3 and abs(pz - z1) < 2e-3, (pt, eta, phi, q, s0, s1, r0, r1, py, y1, pz, z1)
        checked += 1
    assert checked >= 50


def test_prediction_refuses_other_side_and_failed_fits():
    P = np.array([1.0, 2.0, 0.1, 0.2, 0.5], np.float32)
    assert not O.predict(P, 100.0, 3, 21, 50)[0]          # across the membrane
    assert not O.predict(P, 100.0, 3, 40, 50)[0]          # no such sector
    ok, py, pz = O.predict(P, 100.0, 3, 3, 50)
    assert ok
    # a straight track (q/pT = 0) in its own sector: y and z move linearly in x
    Ps = np.array([1.0, 2.0, 0.1, 0.2, 0.0], np.float32)
    ok, py, pz = O.predict(Ps, 100.0, 3, 3, 50)
    dx = float(ROWX32[50]) - 100.0
    c = math.sqrt(1 - 0.1 ** 2)
    assert ok and abs(py - (1.0 + dx * 0.1 / c)) < 1e-5
    assert abs(pz - (2.0 + 0.2 * dx / c)) < 1e-5
    # |sin phi| reaching smax on the way fails
    assert not O.predict(np.array([0.0, 0.0, 0.9, 0.0, 10.0], np.float32), 100.0, 0, 0, 151)[0]


def test_clusters_on_the_helix_give_zero_residuals():
    """Zero-smear event over all sectors: the fitted tracks pass through their clusters, so
    every cluster of a successfully fitted track gets residual codes of at most one step
    (FP32 fit), most of them zero, merged tracks (rotations) included."""
    cs = g.gen_event(31, 300, smear=0.0)
    t = _tracks(cs)
    c = O.compress(cs.sector, cs.row, cs.y, cs.z, t, Q, Q)
    assert c["status"] == 0
    H = c["n_attached"]
    good = np.repeat(t["ndf"] >= 0, np.diff(t["off"]))
    assert good.sum() > 0.95 * H
    rs, ey, ez = c["rs"][:H][good], c["ey"][:H][good], c["ez"][:H][good]
    assert np.all(rs >> 15 == 0)
    assert np.abs(ey).max() <= 1 and np.abs(ez).max() <= 1
    assert np.mean((ey == 0) & (ez == 0)) > 0.9
    merged = np.nonzero((t["sector2"] >= 0) & (t["ndf"] >= 0))[0]
    assert len(merged) >= 3
    outer = np.concatenate([np.arange(t["off"][i], t["off"][i + 1])[cs.sector[t["hits"][t["off"][i]:t["off"][i + 1]]]
                                                                  != t["sector"][i]] for i in merged])
    assert len(outer) > 0
    assert np.all(c["rs"][outer] >> 15 == 0) and np.abs(c["ey"][outer]).max() <= 1


def test_codes_of_clusters_in_no_track_are_rounded_absolute_values():
    cs = g.gen_event(32, 50, noise=0.3)
    t = _tracks(cs)
    c = O.compress(cs.sector, cs.row, cs.y, cs.z, t, Q, 1.0 / 16.0)
    H = c["n_attached"]
    rest = np.setdiff1d(np.arange(cs.n), t["hits"])
    assert len(c["rs"]) == H + len(rest)
    iq_y, iq_z = np.float32(1.0) / np.float32(Q), np.float32(1.0) / np.float32(1.0 / 16.0)
    assert np.array_equal(c["ey"][H:], np.rint(cs.y[rest] * iq_y).astype(np.int16))
    assert np.array_equal(c["ez"][H:], np.rint(cs.z[rest] * iq_z).astype(np.int16))
    assert np.array_equal(c["rs"][H:], (cs.row[rest].astype(np.uint16) | (cs.sector[rest].astype(np.uint16) << 8)
                                        | np.uint16(1 << 15)))


def test_round_trip_within_half_a_step():
    """C5: decoding restores sector and row exactly and y, z within q/2 plus FP32 rounding."""
    cs = g.make_config("c1", 11)
    t = _tracks(cs)
    for qy, qz in ((Q, Q), (0.1, 0.5), (0.5, 1.0 / 64.0)):
        c = O.compress(cs.sector, cs.row, cs.y, cs.z, t, qy, qz)
        assert c["status"] == 0
        d = O.decompress(t, c, qy, qz)
        perm = _permutation(cs.n, t)
        assert len(d["y"]) == cs.n
        assert np.array_equal(d["sector"], cs.sector[perm]) and np.array_equal(d["row"], cs.row[perm])
        assert np.abs(d["y"] - cs.y[perm]).max() <= qy / 2 + 1e-4
        assert np.abs(d["z"] - cs.z[perm]).max() <= qz / 2 + 1e-4
        # residual codes are much smaller than absolute ones (the point of the method)
        H = c["n_attached"]
        res = (c["rs"][:H] >> 15) == 0
        assert res.mean() > 0.99
        assert np.std(c["ey"][:H][res]) < 0.2 * np.std(c["ey"][H:]) + 4 * 0.1 / qy


def test_failed_fits_invalid_clusters_and_saturation():
    cs = g.gen_event(33, 40)
    t = _tracks(cs)
    K = len(t["ndf"])
    assert K >= 5
    t = dict(t)
    t["ndf"] = t["ndf"].copy()
    t["ndf"][0] = -1                                           # failed fit: absolute codes
    z = cs.z.copy()
    y = cs.y.copy()
    rest = np.setdiff1d(np.arange(cs.n), t["hits"])
    z[rest[0]] = 5000.0                                        # beyond the code range: saturates
    y[rest[1]] = np.nan                                        # invalid cluster
    c = O.compress(cs.sector, cs.row, y, z, t, Q, Q)
    assert c["status"] == 1
    a, b = t["off"][0], t["off"][1]
    assert np.all(c["rs"][a:b] >> 15 == 1)
    assert np.array_equal(c["ey"][a:b], np.rint(cs.y[t["hits"][a:b]] * np.float32(32.0)).astype(np.int16))
    H = c["n_attached"]
    assert c["ez"][H] == 32767 and c["rs"][H] >> 15 == 1
    assert c["rs"][H + 1] == 0x7FFF and c["ey"][H + 1] == 0 and c["ez"][H + 1] == 0
    d = O.decompress(t, c, Q, Q)
    assert d["sector"][H + 1] == 255 and d["row"][H + 1] == -1 and np.isnan(d["y"][H + 1])
    assert abs(d["z"][H] - 32767 * Q) < 1e-3
    # a hit index outside the cluster list is an invalid record
    t2 = dict(t)
    t2["hits"] = t["hits"].copy()
    t2["hits"][0] = cs.n + 5
    c2 = O.compress(cs.sector, cs.row, cs.y, cs.z, t2, Q, Q)
    assert c2["status"] == 1 and c2["rs"][0] == 0x7FFF


# ------------------------------------------------------------------ C7: time frames
def test_wide_absolute_z_codes_split_and_saturate():
    """C7: a 24-bit absolute z code is numpy's round-half-even of z/q, split into its low 16
    bits and signed high byte; it saturates at +-(2^23 - 1) with the range status."""
    rng = np.random.default_rng(7)
    n = 20000
    z = np.concatenate([rng.uniform(-2600.0, 2600.0, n - 6),
                        [0.0, -0.5 * Q, 1.5 * Q, 262143.9, -262143.5, 1e6]]).astype(np.float32)
    sector = (np.arange(len(z)) % 36).astype(np.uint8)
    row = (np.arange(len(z)) % 152).astype(np.int16)
    y = rng.uniform(-15.0, 15.0, len(z)).astype(np.float32)
    none = dict(off=np.zeros(1, np.int32), hits=np.zeros(0, np.int32), P=np.zeros((0, 5), np.float32),
                x=np.zeros(0, np.float32), sector=np.zeros(0, np.int32), ndf=np.zeros(0, np.int32))
    c = O.compress(sector, row, y, z, none, Q, Q, wide_z=True)
    iq = np.float32(1.0) / np.float32(Q)
    e = np.clip(np.rint(z * iq).astype(np.float64), -(2 ** 23 - 1), 2 ** 23 - 1).astype(np.int64)
    got = c["ez_hi"].astype(np.int64) * 65536 + c["ez"].view(np.uint16).astype(np.int64)
    assert np.array_equal(got, e)
    assert c["status"] == 1                     # the last value saturates
    c2 = O.compress(sector[:-1], row[:-1], y[:-1], z[:-1], none, Q, Q, wide_z=True)
    assert c2["status"] == 0
    # 16-bit codes: everything beyond +-1024 cm saturates
    c16 = O.compress(sector[:-1], row[:-1], y[:-1], z[:-1], none, Q, Q)
    assert c16["status"] == 1
    d = O.decompress(none, c2, Q, Q)
    assert np.abs(d["z"] - z[:-1]).max() <= Q / 2
    assert np.array_equal(d["y"], (np.rint(y[:-1] * iq).astype(np.float32) * np.float32(Q)))


def test_time_frame_compresses_with_wide_codes():
    """C7 on a time frame of the workload's law spread over a whole 1 ms window (six
    collisions 150 us apart on average, drift-shifted z beyond 1024 cm): 16-bit absolute
    codes saturate, 24-bit ones do not; residual records carry a zero high byte; every
    cluster decodes within half a step."""
    pool = g.gen_collision_pool(73, 6, mult_range=(500, 1500))
    cs = g.assemble_timeframe(74, pool, np.arange(6), 1000.0, mean_spacing_us=150.0)
    assert np.abs(cs.z).max() > 1100.0
    t = _tracks(cs)
    c16 = O.compress(cs.sector, cs.row, cs.y, cs.z, t, Q, Q)
    assert c16["status"] == 1
    c = O.compress(cs.sector, cs.row, cs.y, cs.z, t, Q, Q, wide_z=True)
    assert c["status"] == 0
    H = c["n_attached"]
    res = (c["rs"] >> 15) == 0
    assert res[:H].mean() > 0.99 and not res[H:].any()
    assert np.all(c["ez_hi"][res] == 0)
    assert np.array_equal(c["ey"], c16["ey"]) and np.array_equal(c["rs"], c16["rs"])
    assert np.array_equal(c["ez"][res], c16["ez"][res])
    d = O.decompress(t, c, Q, Q)
    perm = _permutation(cs.n, t)
    assert np.array_equal(d["sector"], cs.sector[perm]) and np.array_equal(d["row"], cs.row[perm])
    assert np.abs(d["y"] - cs.y[perm]).max() <= Q / 2 + 1e-5
    assert np.abs(d["z"] - cs.z[perm]).max() <= Q / 2 + 2e-4
