"""Synthetic TPC digits (input data only): the pad-plane charge that a cluster list leaves.

Each cluster of a ``ClusterSet`` deposits a charge Q (30 ADC plus a Gamma(2, 30) tail, a
stand-in for the Landau-like ionisation) spread as a two-dimensional Gaussian over the pads of
its row and the time bins of its drift coordinate (sigma 0.6 pad and 0.6 bin, integrated over
each cell of the 5 x 5 cells around it); overlapping deposits add; every cell is rounded to an
integer ADC count (10-bit, saturating at 1023) and zero-suppressed below 3.  The digits come
out sorted by (sector, row, pad, time), the order of a read-out stream.  This is detector
simulation only: no peak finding and no centroid arithmetic.

Pad plane (the geometry the paper does not give): pads of pitch 0.5 cm, row r holding
2 ceil(x_r tan 10 deg / 0.5) pads centred on y = 0; time bins of 0.5 cm of drift (|z|),
500 bins over the 250 cm drift length.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
from scipy.special import erf

from . import N_ROWS, N_SECTORS, ROW_X, TAN_HALF

PAD_PITCH = 0.5
TIME_BIN = 0.5
N_TIME = 500
SIGMA_PAD = 0.6
SIGMA_TIME = 0.6
ZS_THRESHOLD = 3
ADC_MAX = 1023
PADS = (2 * np.ceil(ROW_X * TAN_HALF / PAD_PITCH)).astype(np.int64)


@dataclass
class Digits:
    sector: np.ndarray   # uint8
    row: np.ndarray      # int16
    pad: np.ndarray      # int16
    time: np.ndarray     # int16
    adc: np.ndarray      # uint16
    # truth per cluster (pad and time coordinates of the deposit's centre, charge)
    true_pad: np.ndarray
    true_time: np.ndarray
    true_q: np.ndarray

    @property
    def n(self) -> int:
        return int(self.adc.shape[0])


def cluster_coordinates(sector, row, y, z):
    """(pad, time) coordinates of a position, pad p and bin t centred on integers."""
    u = (np.asarray(y, np.float64) + PADS[row] * PAD_PITCH / 2) / PAD_PITCH - 0.5
    v = np.abs(np.asarray(z, np.float64)) / TIME_BIN - 0.5
    return u, v


def _cdf(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0)))




def make_digits(cs, seed: int, n_time: int = N_TIME, shift=None) -> Digits:
    """``shift`` (time bins per cluster) places collisions later in the read-out window."""
    rng = np.random.default_rng(seed)
    n = cs.n
    q = 30.0 + rng.gamma(2.0, 30.0, n)
    u, v = cluster_coordinates(cs.sector, cs.row, cs.y, cs.z)
    if shift is not None:
        v = v + shift
    row_off = np.concatenate([[0], np.cumsum(PADS * n_time)])   # first cell of each row in a sector
    row_all = cs.row.astype(np.int64)
    by_sector = np.argsort(cs.sector, kind="stable")
    bounds = np.searchsorted(cs.sector[by_sector], np.arange(N_SECTORS + 1))
    charge = np.zeros(int(row_off[-1]))          # one sector's cells, reused
    out = {k: [] for k in ("sector", "row", "pad", "time", "adc")}
    for s in range(N_SECTORS):
        idx = by_sector[bounds[s]:bounds[s + 1]]
        if len(idx) == 0:
            continue
        us, vs, qs, row = u[idx], v[idx], q[idx], row_all[idx]
        uc, vc = np.rint(us).astype(np.int64), np.rint(vs).astype(np.int64)
        cells, vals = [], []
        wps = []
        for dp in range(-2, 3):
            pp = uc + dp
            wps.append((pp, _cdf((pp + 0.5 - us) / SIGMA_PAD) - _cdf((pp - 0.5 - us) / SIGMA_PAD)))
        for dt in range(-2, 3):
            tt = vc + dt
            wt = _cdf((tt + 0.5 - vs) / SIGMA_TIME) - _cdf((tt - 0.5 - vs) / SIGMA_TIME)
            okt = (tt >= 0) & (tt < n_time)
            for pp, wp in wps:
                ok = okt & (pp >= 0) & (pp < PADS[row])
                cells.append((row_off[row] + pp * n_time + tt)[ok])
                vals.append((qs * wp * wt)[ok])
        cell = np.concatenate(cells)
        np.add.at(charge, cell, np.concatenate(vals))
        c = np.unique(cell)
        adc = np.minimum(np.floor(charge[c] + 0.5), ADC_MAX)
        charge[c] = 0.0
        keep = adc >= ZS_THRESHOLD
        c, adc = c[keep], adc[keep]
        r = np.searchsorted(row_off, c, side="right") - 1
        w = c - row_off[r]
        out["sector"].append(np.full(len(c), s, np.uint8))
        out["row"].append(r.astype(np.int16))
        out["pad"].append((w // n_time).astype(np.int16))
        out["time"].append((w % n_time).astype(np.int16))
        out["adc"].append(adc.astype(np.uint16))
    cat = {k: (np.concatenate(v) if v else np.zeros(0, dt)) for (k, v), dt in
           zip(out.items(), (np.uint8, np.int16, np.int16, np.int16, np.uint16))}
    return Digits(cat["sector"], cat["row"], cat["pad"], cat["time"], cat["adc"], u, v, q)


def digit_config(cfg: str, seed: int):
    """(clusters, digits, n_time) of a workload: 'd1' one sector of one event, 'd2' the full
    TPC event, 'd3' eight such events at uniform times over two drift lengths (1000 bins)."""
    from . import concat, make_config
    if cfg in ("d1", "d2"):
        cs = make_config({"d1": "c1", "d2": "c2"}[cfg], seed)
        return cs, make_digits(cs, seed + 1000), N_TIME
    assert cfg == "d3"
    rng = np.random.default_rng(seed)
    evs = [make_config("c2", seed * 100 + k) for k in range(8)]
    cs = concat(evs, {})
    offs = rng.uniform(0.0, N_TIME, len(evs))
    shift = np.repeat(offs, [e.n for e in evs])
    return cs, make_digits(cs, seed + 1000, n_time=2 * N_TIME, shift=shift), 2 * N_TIME
