"""Synthetic input generator: reproducibility, laws and exact geometry."""
import math

import numpy as np
import pytest

import tpcsynth as g
from tests.truth import rk4_crossing, true_state


def test_seed_reproducible():
    a = g.make_config("c1", 11)
    b = g.make_config("c1", 11)
    for f in ("sector", "row", "y", "z", "time", "label"):
        assert np.array_equal(getattr(a, f), getattr(b, f))
    c = g.make_config("c1", 12)
    assert a.n != c.n or not np.array_equal(a.y, c.y)


def test_c1_layout():
    cs = g.make_config("c1", 11)
    assert cs.n_jobs == 1
    assert np.all(cs.sector == 0)
    assert cs.row.dtype == np.int16 and cs.row.min() >= 0 and cs.row.max() < 152
    assert cs.y.dtype == np.float32 and cs.z.dtype == np.float32
    # acceptance |y| <= x tan10 (plus smear), z on side A
    x = g.ROW_X[cs.row]
    assert np.all(np.abs(cs.y) <= x * g.TAN_HALF + 1.0)
    assert np.all(cs.z > -1.0)
    assert np.all(cs.label >= 0) and cs.label.max() < 200
    assert 5000 < cs.n < 20000


def test_c2_noise_and_inefficiency():
    cs = g.make_config("c2", 21, scale=0.25)
    sig = (cs.label >= 0).sum()
    noise = (cs.label < 0).sum()
    assert abs(noise - round(0.05 * sig)) <= 1
    assert set(np.unique(cs.sector)) == set(range(36))
    # inefficiency: same seed without it has ~1/0.9 as many signal clusters
    ev = g.gen_event(21, 2000, noise=0.0, ineff=0.0)
    ev_i = g.gen_event(21, 2000, noise=0.0, ineff=0.1)
    frac = ev_i.n / ev.n
    assert abs(frac - 0.9) < 4 * math.sqrt(0.09 / ev.n) + 1e-3


def test_pt_law_clamped():
    rng = np.random.default_rng(5)
    pt, eta, phi, q = g.draw_primaries(rng, 200000)
    assert pt.min() == 0.1 and pt.max() <= 10.0
    # fraction clamped at 0.1: P(Exp(0.6) < 0.1) = 1 - exp(-1/6)
    assert abs((pt == 0.1).mean() - (1 - math.exp(-1 / 6))) < 0.005
    assert abs(eta).max() <= 0.9 and set(np.unique(q)) == {-1, 1}


def test_crossings_exact_on_circle():
    rng = np.random.default_rng(3)
    pt, eta, phi, q = g.draw_primaries(rng, 300)
    ti, sec, row, y, z, arc = g.crossings(pt, eta, phi, q)
    R, h, xc, yc = g.helix_geometry(pt[ti], phi[ti], q[ti])
    a = g.sector_alpha(sec)
    X = g.ROW_X[row] * np.cos(a) - y * np.sin(a)
    Y = g.ROW_X[row] * np.sin(a) + y * np.cos(a)
    # on the circle, and z = tan(lambda) * arc with the arc at most half a turn
    assert np.max(np.abs(np.hypot(X - xc, Y - yc) - R)) < 1e-9
    assert np.max(np.abs(z - np.sinh(eta[ti]) * arc)) < 1e-9
    assert np.all(arc <= math.pi * R + 1e-9)
    # inside the sector acceptance, correct side
    assert np.all(np.abs(y) <= g.ROW_X[row] * g.TAN_HALF)
    assert np.all((sec < 18) == (eta[ti] >= 0))


@pytest.mark.parametrize("pt,q,phi", [(0.3, 1, 0.1), (0.3, -1, 0.2), (2.0, 1, 0.15), (0.12, -1, 0.05)])
def test_crossing_matches_lorentz_force_rk4(pt, q, phi):
    """The generator's circle (and its sense of rotation) against a direct RK4 integration of
    the equations of motion dp/dl = kappa q (p/|p| x B)."""
    eta = 0.4
    sec = int(np.floor(phi / math.radians(20.0))) % 18
    for r in (0, 30, 60):
        x = g.ROW_X[r]
        ok, y, z, s, t, k = true_state(pt, eta, phi, q, sec, x)
        if not ok:
            continue
        yr, zr = rk4_crossing(pt, eta, phi, q, sec, x)
        assert abs(float(y) - yr) < 1e-6 and abs(float(z) - zr) < 1e-6


def test_timeframe_shift():
    pool = g.gen_collision_pool(7, 3, (50, 60))
    tf = g.assemble_timeframe(8, pool, [0, 1, 2], window_us=100.0, noise=0.0, shuffle=False)
    tk = np.array(tf.meta["t_collisions"])
    assert np.all(tf.time < 100.0)
    # measured z is the arrival time mapped to a drift distance on the cluster's side
    sgn = np.where(tf.sector < 18, 1.0, -1.0)
    assert np.allclose(tf.z, sgn * (g.DRIFT_LENGTH - g.V_DRIFT * tf.time.astype(np.float64)),
                       atol=2e-3)
    assert tk[0] > 0 and np.all(np.diff(tk) > 0)


def test_c4_job_sizes_law():
    s = g.c4_job_sizes(41)
    assert s.shape == (512,) and s.min() >= 100 and s.max() <= 20000
    # log-uniform: the median is near sqrt(100 * 20000)
    assert 700 < np.median(s) < 2300
    one = g.make_config("c4", 41, jobs=[3], scale=0.05)
    assert np.all(one.sector == 3)


# ------------------------------------------------------------------ digit simulator
def test_digits_layout_and_charge():
    """Digits are unique cells in read-out order inside the pad plane, 10-bit, above the
    zero-suppression threshold; an isolated deposit keeps its charge up to the suppressed
    tails and the rounding."""
    from tpcsynth import digits as D
    cs, d, nt = D.digit_config("d1", 11)
    assert nt == D.N_TIME
    key = ((d.sector.astype(np.int64) * 152 + d.row) * 256 + d.pad) * 1024 + d.time
    assert np.all(np.diff(key) > 0)
    assert np.all(d.pad >= 0) and np.all(d.pad < D.PADS[d.row])
    assert np.all(d.time >= 0) and np.all(d.time < nt)
    assert d.adc.min() >= D.ZS_THRESHOLD and d.adc.max() <= D.ADC_MAX
    # one cluster alone: its 5 x 5 deposit sums to Q within the suppressed and rounded part
    one = g.ClusterSet(np.zeros(1, np.uint8), np.array([70], np.int16), np.array([1.3], np.float32),
                       np.array([100.2], np.float32), np.zeros(1, np.float32), np.zeros(1, np.int32),
                       np.array([0, 1], np.int32), np.zeros(0), np.zeros(0), np.zeros(0),
                       np.zeros(0, np.int8), np.array([0, 0]), {})
    d1 = D.make_digits(one, 5)
    q = float(d1.true_q[0])
    assert abs(float(d1.adc.sum()) - q) < 25 * (D.ZS_THRESHOLD + 0.5)
    # the charge-weighted centre of its digits is the deposit's centre
    u, v = D.cluster_coordinates(one.sector, one.row, one.y, one.z)
    w = d1.adc.astype(np.float64)
    assert abs((w * d1.pad).sum() / w.sum() - u[0]) < 0.1
    assert abs((w * d1.time).sum() / w.sum() - v[0]) < 0.1


def test_digits_time_shift():
    """A collision placed later in the read-out window moves its digits by whole bins."""
    from tpcsynth import digits as D
    cs = g.make_config("c1", 11)
    a = D.make_digits(cs, 3)
    b = D.make_digits(cs, 3, n_time=2 * D.N_TIME, shift=np.full(cs.n, 200.0))
    m = (b.time >= 200) & (b.time < 200 + D.N_TIME)   # the cells the shorter window also has
    assert np.array_equal(a.adc, b.adc[m]) and np.array_equal(a.pad, b.pad[m])
    assert np.array_equal(a.time.astype(np.int32) + 200, b.time[m].astype(np.int32))
