"""Pins of the oracle's TPC cluster finder (section 5: cluster finding on the GPUs, the step
before the tracking) against hand-computed charge patterns and the generator's truth.

Exact centroids and widths of symmetric and asymmetric 3 x 3 patterns (values worked out by
hand below), the tie rule between equal neighbouring maxima, the threshold, the pad-plane
edges, translation invariance, invalid digits, and the recovery of the generator's clusters
from its digits (efficiency and resolution against the positions the digits were made from).
"""
import math

import numpy as np

import oracle.oracle as O
import tpcsynth as g
from tpcsynth import digits as D

PITCH, BIN = 0.5, 0.5


def _pattern(sec, row, p0, t0, grid):
    """Digits of a 3 x 3 charge grid[dp + 1][dt + 1] around (p0, t0); zeros are not digits."""
    s, r, p, t, a = [], [], [], [], []
    for i, dp in enumerate((-1, 0, 1)):
        for j, dt in enumerate((-1, 0, 1)):
            if grid[i][j]:
                s.append(sec); r.append(row); p.append(p0 + dp); t.append(t0 + dt); a.append(grid[i][j])
    return [np.array(x) for x in (s, r, p, t, a)]


def _cat(*ds):
    return [np.concatenate([d[k] for d in ds]) for k in range(5)]


def _y(row, pad):
    return (pad + 0.5) * PITCH - O.cf_pads(row) * PITCH / 2


def test_pad_plane():
    assert [O.cf_pads(r) for r in (0, 75, 151)] == [60, 118, 174]
    assert np.array_equal([O.cf_pads(r) for r in range(152)], D.PADS)


def test_symmetric_pattern_is_centred_exactly():
    c = O.find_clusters(*_pattern(3, 40, 20, 100, [[10, 20, 10], [20, 40, 20], [10, 20, 10]]))
    assert len(c["y"]) == 1 and c["digit"][0] == 4
    assert c["y"][0] == np.float32(_y(40, 20)) and c["z"][0] == np.float32(100.5 * BIN)
    # sum q dp^2 / Q = (40 + 40) / 160 = 0.5 in both directions
    assert c["sigma_pad"][0] == np.float32(math.sqrt(0.5)) and c["sigma_time"][0] == np.float32(math.sqrt(0.5))
    assert c["q_tot"][0] == 160 and c["q_max"][0] == 40


def test_hand_computed_asymmetric_pattern():
    # time mean 100 + 5/15, pad mean 20; time variance 5/15 - (5/15)^2 = 2/9
    c = O.find_clusters(*_pattern(20, 7, 20, 100, [[0, 0, 0], [0, 10, 5], [0, 0, 0]]))
    assert len(c["y"]) == 1
    assert abs(c["z"][0] - (-(100 + 1 / 3 + 0.5) * BIN)) < 2e-5          # side C: negative z
    assert c["y"][0] == np.float32(_y(7, 20)) and c["sigma_pad"][0] == 0
    assert abs(c["sigma_time"][0] - math.sqrt(2 / 9)) < 1e-6 and c["q_tot"][0] == 15
    # the same along the pads, towards the smaller pad: pad mean 20 - 1/3, variance 2/9
    c = O.find_clusters(*_pattern(2, 7, 20, 100, [[0, 5, 0], [0, 10, 0], [0, 0, 0]]))
    assert abs(c["y"][0] - (_y(7, 20) - PITCH / 3)) < 2e-5 and c["sigma_time"][0] == 0
    assert abs(c["sigma_pad"][0] - math.sqrt(2 / 9)) < 1e-6


def test_equal_neighbouring_maxima_give_one_peak_at_the_earlier_cell():
    d = _pattern(0, 10, 30, 50, [[0, 0, 0], [0, 19, 0], [0, 19, 0]])   # (30, 50) and (31, 50)
    c = O.find_clusters(*d)
    assert len(c["y"]) == 1 and d[2][c["digit"][0]] == 30
    d = _pattern(0, 10, 30, 50, [[0, 0, 0], [0, 19, 19], [0, 0, 0]])   # (30, 50) and (30, 51)
    c = O.find_clusters(*d)
    assert len(c["y"]) == 1 and d[3][c["digit"][0]] == 50


def test_threshold_edges_and_separation():
    low = _pattern(0, 0, 10, 10, [[0, 0, 0], [0, 9, 0], [0, 0, 0]])
    assert len(O.find_clusters(*low)["y"]) == 0
    assert len(O.find_clusters(*low, q_min=9)["y"]) == 1
    # a peak at pad 0 and time 0: cells outside the plane count as 0
    edge = _pattern(0, 0, 0, 0, [[0, 0, 0], [0, 20, 6], [0, 6, 3]])
    c = O.find_clusters(*edge)
    assert len(c["y"]) == 1 and c["q_tot"][0] == 35
    # two peaks three cells apart are two clusters; adjacent unequal ones are one
    two = _cat(_pattern(1, 5, 10, 10, [[1, 2, 1], [2, 30, 2], [1, 2, 1]]),
               _pattern(1, 5, 13, 10, [[1, 2, 1], [2, 25, 2], [1, 2, 1]]))
    assert len(O.find_clusters(*two)["y"]) == 2
    one = _cat(_pattern(1, 5, 10, 10, [[0, 0, 0], [0, 30, 0], [0, 0, 0]]),
               _pattern(1, 5, 11, 10, [[0, 0, 0], [0, 25, 0], [0, 0, 0]]))
    assert len(O.find_clusters(*one)["y"]) == 1


def test_translation_moves_clusters_by_whole_cells():
    cs, d, _ = D.digit_config("d1", 11)
    a = O.find_clusters(d.sector, d.row, d.pad, d.time, d.adc)
    b = O.find_clusters(d.sector, d.row, d.pad, d.time + 7, d.adc)
    # near the time edge the shifted copy keeps clusters the original cut
    keep = (d.time[a["digit"]] >= 1) & (d.time[a["digit"]] + 7 < 499)
    bm = {int(i): k for k, i in enumerate(b["digit"])}
    idx = [bm[int(i)] for i in a["digit"][keep]]
    assert np.allclose(b["z"][idx] - a["z"][keep], 7 * BIN, atol=2e-5)
    assert np.array_equal(b["y"][idx], a["y"][keep]) and np.array_equal(b["q_tot"][idx], a["q_tot"][keep])


def test_invalid_digits_are_dropped_and_reported():
    d = _pattern(0, 10, 30, 50, [[1, 2, 1], [2, 40, 2], [1, 2, 1]])
    bad = [np.array([40]), np.array([10]), np.array([30]), np.array([50]), np.array([99])]
    c = O.find_clusters(*_cat(d, bad))
    assert c["status"] == 1 and len(c["y"]) == 1
    for col, v in ((1, 152), (2, O.cf_pads(10)), (3, 500), (2, -1), (3, -1)):
        b = [x.copy() for x in bad]
        b[0][0] = 0
        b[col][0] = v
        assert O.find_clusters(*_cat(d, b))["status"] == 1


def test_generator_clusters_are_recovered():
    """Single-sector event: every isolated generated cluster (no other within 3 pads and
    3 bins) is found within 0.35 pad / bin of where its charge was deposited, with an RMS
    residual well below the 0.6-cell charge spread."""
    cs, d, _ = D.digit_config("d1", 11)
    c = O.find_clusters(d.sector, d.row, d.pad, d.time, d.adc)
    u_f = (c["y"] + D.PADS[c["row"]] * PITCH / 2) / PITCH - 0.5
    v_f = np.abs(c["z"]) / BIN - 0.5
    found = {}
    for k in range(len(u_f)):
        found.setdefault(int(c["row"][k]), []).append((u_f[k], v_f[k]))
    iso, res = 0, []
    for r in range(152):
        m = np.nonzero(cs.row == r)[0]
        if len(m) == 0:
            continue
        u, v = d.true_pad[m], d.true_time[m]
        du = np.abs(u[:, None] - u[None, :])
        dv = np.abs(v[:, None] - v[None, :])
        crowd = ((du < 3) & (dv < 3)).sum(1) > 1
        fr = np.array(found.get(r, np.zeros((0, 2))))
        for i in np.nonzero(~crowd)[0]:
            if not (1 <= u[i] <= D.PADS[r] - 2 and 1 <= v[i] <= 498):
                continue
            iso += 1
            dist = np.hypot(fr[:, 0] - u[i], fr[:, 1] - v[i]) if len(fr) else np.array([np.inf])
            res.append(dist.min())
    res = np.array(res)
    assert iso > 3000
    assert np.mean(res < 0.35) > 0.99
    assert np.sqrt(np.mean(np.minimum(res, 1.0) ** 2)) < 0.15
