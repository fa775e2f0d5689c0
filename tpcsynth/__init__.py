"""Seeded synthetic TPC cluster generator (input data only).

This module produces the inputs that both the CPU oracle and the HIP library
consume.  It simulates charged primaries moving on helices in a uniform
solenoidal field and records one smeared cluster per crossed pad-row plane.
It contains none of the tracking method's arithmetic: no neighbour search,
no Kalman filter and no track model beyond the physical motion used to place
the clusters.  Geometry constants are defined here independently of the
oracle and of the HIP path.

Workloads (sizes and laws of the paper's Pb-Pb running conditions, section 2
and section 7, stated concretely because the paper prints no event sample):

* ``c1``  single sector, 200 primaries, no noise, no inefficiency
* ``c2``  full TPC (36 sectors), 8000 primaries, 5% noise, 10% inefficiency
* ``c3``  1 ms time-frame slice: 50 collisions at 50 kHz Poisson spacing,
          multiplicity U{500..8000}, z shifted by the drift of the collision time
* ``c4``  512 single-sector jobs, 100..20000 primaries each (log-uniform)
* ``c5``  serving: chunks of U{10..200} collisions drawn from a pre-generated pool

All randomness comes from ``numpy.random.default_rng`` seeded per job or per
collision via ``SeedSequence.spawn`` so that every item is reproducible alone.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np

GENERATOR_VERSION = 1

N_ROWS = 152
N_SECTORS = 36
X_FIRST = 85.0
X_LAST = 245.0
ROW_X = X_FIRST + np.arange(N_ROWS, dtype=np.float64) * (X_LAST - X_FIRST) / (N_ROWS - 1)
TAN_HALF = math.tan(math.radians(10.0))
B_TESLA = 0.5
KAPPA = 0.299792458e-2          # GeV / (T cm)
DRIFT_LENGTH = 250.0            # cm
V_DRIFT = 2.58                  # cm / us
SIGMA_YZ = 0.1                  # cm, cluster smear
R_MAX = X_LAST / math.cos(math.radians(10.0))


def sector_alpha(sector):
    """Azimuth of the centre of a sector, radians (sectors 0..17 side A, 18..35 side C)."""
    return np.deg2rad(10.0 + 20.0 * (np.asarray(sector) % 18))


@dataclass
class ClusterSet:
    """Cluster list in caller order, grouped into independent jobs.

    Arrays are ``N`` long; job ``j`` owns clusters ``job_off[j]:job_off[j+1]``.
    ``label`` is the particle index within its job (or -1 for noise);
    particle arrays are concatenated over jobs with ``part_off``.
    """
    sector: np.ndarray       # uint8
    row: np.ndarray          # int16
    y: np.ndarray            # float32, sector-local
    z: np.ndarray            # float32
    time: np.ndarray         # float32, us
    label: np.ndarray        # int32
    job_off: np.ndarray      # int32 [J+1]
    part_pt: np.ndarray      # float64
    part_eta: np.ndarray
    part_phi: np.ndarray
    part_q: np.ndarray       # int8
    part_off: np.ndarray     # int64 [J+1]
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.y.shape[0])

    @property
    def n_jobs(self) -> int:
        return int(self.job_off.shape[0] - 1)

    def job(self, j: int) -> "ClusterSet":
        a, b = int(self.job_off[j]), int(self.job_off[j + 1])
        pa, pb = int(self.part_off[j]), int(self.part_off[j + 1])
        return ClusterSet(self.sector[a:b], self.row[a:b], self.y[a:b], self.z[a:b],
                          self.time[a:b], self.label[a:b], np.array([0, b - a], np.int32),
                          self.part_pt[pa:pb], self.part_eta[pa:pb], self.part_phi[pa:pb],
                          self.part_q[pa:pb], np.array([0, pb - pa], np.int64),
                          dict(self.meta, job=j))

    def subset_jobs(self, jobs) -> "ClusterSet":
        return concat([self.job(int(j)) for j in jobs], dict(self.meta, jobs=list(map(int, jobs))))


def concat(sets, meta=None) -> ClusterSet:
    """Concatenate cluster sets; each input job stays a job."""
    job_off = [0]
    part_off = [0]
    for s in sets:
        job_off.extend((s.job_off[1:] + job_off[-1]).tolist())
        part_off.extend((s.part_off[1:] + part_off[-1]).tolist())
    cat = lambda name, dt: (np.concatenate([getattr(s, name) for s in sets]).astype(dt, copy=False)
                            if sets else np.zeros(0, dt))
    return ClusterSet(cat("sector", np.uint8), cat("row", np.int16), cat("y", np.float32),
                      cat("z", np.float32), cat("time", np.float32), cat("label", np.int32),
                      np.asarray(job_off, np.int32), cat("part_pt", np.float64),
                      cat("part_eta", np.float64), cat("part_phi", np.float64),
                      cat("part_q", np.int8), np.asarray(part_off, np.int64), meta or {})


# --------------------------------------------------------------------------------------
# Particle kinematics and exact helix / pad-row-plane crossings
# --------------------------------------------------------------------------------------

def draw_primaries(rng, n, eta_range=(-0.9, 0.9), phi_range=(0.0, 2 * math.pi)):
    """pT ~ Exp(mean 0.6 GeV) clamped to [0.1, 10]; eta, phi uniform; charge +-1."""
    pt = np.clip(rng.exponential(0.6, n), 0.1, 10.0)
    eta = rng.uniform(eta_range[0], eta_range[1], n)
    phi = rng.uniform(phi_range[0], phi_range[1], n)
    q = np.where(rng.random(n) < 0.5, -1, 1).astype(np.int8)
    return pt, eta, phi, q


def helix_geometry(pt, phi, q):
    """Radius (cm), rotation sense h (+1 = counter-clockwise seen from +z) and centre of the
    transverse circle of a particle leaving the origin.  A positive charge in a field
    along +z turns clockwise (Lorentz force q v x B)."""
    R = pt / (KAPPA * B_TESLA)
    h = -np.asarray(q, np.float64)
    xc = -h * R * np.sin(phi)
    yc = h * R * np.cos(phi)
    return R, h, xc, yc


def crossings(pt, eta, phi, q, only_sector=None, z0=None, leg=0):
    """Exact crossings of each primary with every pad-row plane on its outgoing half turn.

    Returns (track_index, sector, row, y_local, z, arc) for crossings inside the sector
    acceptance |y| <= x tan10 and |z| <= drift length.  Without ``z0`` every primary starts
    at the origin and its z side follows the sign of eta; with ``z0`` (vertex z per primary)
    z = z0 + tan(lambda) * arc and each crossing's side follows the sign of its own z, so a
    primary whose z changes sign inside the chamber crosses the central membrane and leaves
    clusters on both sides.  ``only_sector`` restricts to one sector (single-sector
    workloads).

    ``leg`` = 1 gives instead the crossings of the return leg of a looper: a primary whose
    circle turns back inside the chamber (2R < R_MAX) crosses the rows again on the second
    half turn (turned angle in (pi, 2 pi)), moving inwards, while z keeps growing with the
    arc; primaries that leave the chamber first have no return leg.
    """
    n = pt.shape[0]
    R, h, xc, yc = helix_geometry(pt, phi, q)
    tanl = np.sinh(eta)
    side_c = eta < 0
    if leg == 0:
        # polar angle of the position at radius rho on the first half turn: phi + h asin(rho / 2R)
        th_a = phi + h * np.arcsin(np.minimum(1.0, X_FIRST / (2 * R)))
        th_b = phi + h * np.arcsin(np.minimum(1.0, R_MAX / (2 * R)))
        reach = 2 * R >= X_FIRST
    else:
        # on the second half turn: phi + h (pi - asin(rho / 2R)), from the turn (rho = 2R) inwards
        th_a = phi + h * (math.pi / 2)
        th_b = phi + h * (math.pi - np.arcsin(np.minimum(1.0, X_FIRST / (2 * R))))
        reach = (2 * R >= X_FIRST) & (2 * R < R_MAX)
    lo = np.floor(np.minimum(th_a, th_b) / math.radians(20.0)).astype(np.int64)
    hi = np.floor(np.maximum(th_a, th_b) / math.radians(20.0)).astype(np.int64)
    out = []
    for k in range(0, 7):
        m = reach & (lo + k <= hi)
        if only_sector is not None:
            if z0 is None:
                sec_k = np.mod(lo + k, 18) + np.where(side_c, 18, 0)
                m &= sec_k == only_sector
            else:
                m &= np.mod(lo + k, 18) == only_sector % 18
        idx = np.nonzero(m)[0]
        if idx.size == 0:
            continue
        sec = np.mod(lo[idx] + k, 18) + np.where(side_c[idx], 18, 0)
        a = sector_alpha(sec)
        ca, sa = np.cos(a), np.sin(a)
        xcl = xc[idx] * ca + yc[idx] * sa
        ycl = -xc[idx] * sa + yc[idx] * ca
        Ri = R[idx][:, None]
        hi_ = h[idx][:, None]
        dxr = ROW_X[None, :] - xcl[:, None]
        D = Ri * Ri - dxr * dxr
        ok = D >= 0
        root = -hi_ if leg == 0 else hi_
        yy = ycl[:, None] + root * np.sqrt(np.where(ok, D, 0.0))
        # turned angle from the origin's phase (-xcl, -ycl) to the crossing's phase
        py = yy - ycl[:, None]
        ox, oy = -xcl[:, None], -ycl[:, None]
        dphi = np.mod(hi_ * np.arctan2(ox * py - oy * dxr, ox * dxr + oy * py), 2 * math.pi)
        if leg == 0:
            ok &= (dphi > 0) & (dphi <= math.pi)
        else:
            ok &= (dphi > math.pi) & (dphi < 2 * math.pi)
        arc = Ri * dphi
        zz = tanl[idx][:, None] * arc
        if z0 is not None:
            zz = zz + np.asarray(z0, np.float64)[idx][:, None]
        ok &= np.abs(yy) <= ROW_X[None, :] * TAN_HALF
        ok &= np.abs(zz) <= DRIFT_LENGTH
        ti, ri = np.nonzero(ok)
        sec_c = sec[ti]
        if z0 is not None:  # the side of each crossing from the sign of its z
            sec_c = np.mod(sec_c, 18) + np.where(zz[ti, ri] < 0, 18, 0)
            if only_sector is not None:
                keep = sec_c == only_sector
                ti, ri, sec_c = ti[keep], ri[keep], sec_c[keep]
        out.append((idx[ti], sec_c, ri, yy[ti, ri], zz[ti, ri], arc[ti, ri]))
    if not out:
        e = np.zeros(0)
        return (e.astype(np.int64), e.astype(np.int64), e.astype(np.int64), e, e, e)
    return tuple(np.concatenate([o[i] for o in out]) for i in range(6))


# --------------------------------------------------------------------------------------
# Events, collisions and time frames
# --------------------------------------------------------------------------------------

def _signal_clusters(rng, n, *, eta_range, phi_range, only_sector=None, smear=SIGMA_YZ,
                     ineff=0.0, block=20000, vertex_z=None, loopers=False, legs_out=None):
    pt, eta, phi, q = draw_primaries(rng, n, eta_range, phi_range)
    parts = []
    for b0 in range(0, n, block):
        sl = slice(b0, min(n, b0 + block))
        z0 = None if vertex_z is None else np.full(sl.stop - sl.start, float(vertex_z))
        for leg in ((0, 1) if loopers else (0,)):
            ti, sec, row, y, z, _ = crossings(pt[sl], eta[sl], phi[sl], q[sl], only_sector, z0, leg)
            parts.append((ti + b0, sec, row, y, z, np.full(len(ti), leg, np.int8)))
    ti, sec, row, y, z, lg = (np.concatenate([p[i] for p in parts]) for i in range(6))
    m = len(ti)
    if smear > 0:
        y = y + rng.normal(0.0, smear, m)
        z = z + rng.normal(0.0, smear, m)
    if ineff > 0:
        keep = rng.random(m) >= ineff
        ti, sec, row, y, z, lg = ti[keep], sec[keep], row[keep], y[keep], z[keep], lg[keep]
    if legs_out is not None:
        legs_out.append(lg)
    return (pt, eta, phi, q), (ti, sec, row, y, z)


def _noise_clusters(rng, n_noise, *, window_us=None):
    sec = rng.integers(0, N_SECTORS, n_noise)
    row = rng.integers(0, N_ROWS, n_noise)
    x = ROW_X[row]
    y = rng.uniform(-1.0, 1.0, n_noise) * x * TAN_HALF
    sgn = np.where(sec < 18, 1.0, -1.0)
    if window_us is None:
        az = rng.uniform(0.0, DRIFT_LENGTH, n_noise)
        t = (DRIFT_LENGTH - az) / V_DRIFT
    else:
        t = rng.uniform(0.0, window_us, n_noise)
        az = DRIFT_LENGTH - V_DRIFT * t
    return sec, row, y, sgn * az, t


def _finish_job(rng, sig, noise, parts, shuffle=True, meta=None):
    ti, sec, row, y, z, t = sig
    nsec, nrow, ny, nz, nt = noise
    sector = np.concatenate([sec, nsec]).astype(np.uint8)
    rowa = np.concatenate([row, nrow]).astype(np.int16)
    ya = np.concatenate([y, ny]).astype(np.float32)
    za = np.concatenate([z, nz]).astype(np.float32)
    ta = np.concatenate([t, nt]).astype(np.float32)
    lab = np.concatenate([ti, np.full(len(nsec), -1)]).astype(np.int32)
    if shuffle:
        p = rng.permutation(len(ya))
        sector, rowa, ya, za, ta, lab = sector[p], rowa[p], ya[p], za[p], ta[p], lab[p]
        if meta and "leg" in meta:
            meta["leg"] = meta["leg"][p]
    pt, eta, phi, q = parts
    return ClusterSet(sector, rowa, ya, za, ta, lab, np.array([0, len(ya)], np.int32),
                      pt, eta, phi, q.astype(np.int8), np.array([0, len(pt)], np.int64),
                      meta or {})


def gen_event(seed, n_primaries, *, sector=None, noise=0.0, ineff=0.0, smear=SIGMA_YZ,
              shuffle=True, vertex_z=None, loopers=False):
    """One collision at t=0 from the origin, or from (0, 0, vertex_z) when given (then the
    clusters' sides follow their own z: primaries near eta 0 cross the central membrane).
    ``sector`` given: a single-sector event with phi inside that sector and eta on its side
    (clusters elsewhere dropped).  ``loopers``: the return legs of primaries that turn back
    inside the chamber are generated too; ``meta["leg"]`` then gives each cluster's leg (0
    outgoing, 1 return, -1 noise)."""
    rng = np.random.default_rng(seed)
    if sector is None:
        eta_r, phi_r = (-0.9, 0.9), (0.0, 2 * math.pi)
    else:
        a = float(sector_alpha(sector))
        eta_r = (0.0, 0.9) if sector < 18 else (-0.9, 0.0)
        phi_r = (a - math.radians(10.0), a + math.radians(10.0))
    legs = [] if loopers else None
    parts, (ti, sec, row, y, z) = _signal_clusters(rng, n_primaries, eta_range=eta_r,
                                                   phi_range=phi_r, only_sector=sector,
                                                   smear=smear, ineff=ineff, vertex_z=vertex_z,
                                                   loopers=loopers, legs_out=legs)
    t = (DRIFT_LENGTH - np.abs(z)) / V_DRIFT
    n_noise = int(round(noise * len(ti)))
    nz = _noise_clusters(rng, n_noise)
    meta = dict(kind="event", seed=seed, n_primaries=n_primaries, sector=sector, vertex_z=vertex_z)
    if loopers:
        meta["leg"] = np.concatenate([legs[0], np.full(n_noise, -1, np.int8)])
    return _finish_job(rng, (ti, sec, row, y, z, t), nz, parts, shuffle, meta)


def gen_collision_pool(seed, n_collisions, mult_range=(500, 8000), ineff=0.1, workers=0,
                       smear=SIGMA_YZ, vz_sigma=0.0, loopers=False):
    """Collisions at t=0 (no noise), each reproducible from its own spawned seed.  With
    ``vz_sigma`` > 0 each collision's vertex z is drawn from N(0, vz_sigma) (cm); with
    ``loopers`` the return legs of primaries that turn back inside the chamber are kept."""
    ss = np.random.SeedSequence(seed)
    rng = np.random.default_rng(ss.spawn(1)[0])
    mult = rng.integers(mult_range[0], mult_range[1] + 1, n_collisions)
    kids = ss.spawn(n_collisions + 1)[1:]
    args = [(kids[i], int(mult[i]), ineff, smear, vz_sigma, loopers) for i in range(n_collisions)]
    if workers and workers > 1 and n_collisions > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(min(workers, n_collisions)) as p:
            return p.map(_pool_collision, args, chunksize=1)
    return [_pool_collision(a) for a in args]


def _pool_collision(args):
    kid, mult, ineff, smear, vz_sigma, loopers = args
    r = np.random.default_rng(kid)
    vz = float(r.normal(0.0, vz_sigma)) if vz_sigma > 0 else None
    parts, (ti, sec, row, y, z) = _signal_clusters(r, mult, eta_range=(-0.9, 0.9),
                                                   phi_range=(0, 2 * math.pi), ineff=ineff,
                                                   smear=smear, vertex_z=vz, loopers=loopers)
    return dict(parts=parts, ti=ti, sec=sec.astype(np.uint8), row=row.astype(np.int16),
                y=y, z=z, vz=vz or 0.0)


def assemble_timeframe(seed, pool, coll_ids, window_us, noise=0.05, mean_spacing_us=20.0,
                       shuffle=True):
    """A time-frame slice: collisions placed at cumulative Exp(mean spacing) times.

    A cluster of a collision at time t_k and true z drifts for (250-|z|)/v_d, so it arrives
    at t = t_k + (250-|z|)/v_d; clusters arriving at or after the window end are dropped.
    The measured z is the arrival time mapped back to a drift distance, which is z shifted
    by v_d t_k towards the central membrane's opposite side (z - v_d t_k on side A,
    z + v_d t_k on side C).  Uniform noise fills the whole window.
    """
    rng = np.random.default_rng(seed)
    tk = np.cumsum(rng.exponential(mean_spacing_us, len(coll_ids)))
    secs, rows, ys, zs, ts, labs = [], [], [], [], [], []
    pts, etas, phis, qs = [], [], [], []
    poff = 0
    for k, cid in enumerate(coll_ids):
        c = pool[int(cid)]
        t = tk[k] + (DRIFT_LENGTH - np.abs(c["z"])) / V_DRIFT
        keep = t < window_us
        zsh = np.where(c["sec"] < 18, c["z"] - V_DRIFT * tk[k], c["z"] + V_DRIFT * tk[k])
        secs.append(c["sec"][keep]); rows.append(c["row"][keep]); ys.append(c["y"][keep])
        zs.append(zsh[keep]); ts.append(t[keep]); labs.append(c["ti"][keep] + poff)
        pt, eta, phi, q = c["parts"]
        pts.append(pt); etas.append(eta); phis.append(phi); qs.append(q)
        poff += len(pt)
    sig = tuple(np.concatenate(a) if a else np.zeros(0) for a in (labs, secs, rows, ys, zs, ts))
    n_noise = int(round(noise * len(sig[0])))
    nz = _noise_clusters(rng, n_noise, window_us=window_us)
    parts = tuple(np.concatenate(a) for a in (pts, etas, phis, qs))
    coll_part_off = np.concatenate([[0], np.cumsum([len(p) for p in pts])]).astype(np.int64)
    return _finish_job(rng, sig, nz, parts, shuffle,
                       dict(kind="timeframe", seed=seed, n_collisions=len(coll_ids),
                            window_us=window_us, t_collisions=tk.tolist(),
                            coll_part_off=coll_part_off.tolist(),
                            vertex_z=[float(pool[int(c)].get("vz", 0.0)) for c in coll_ids]))


# --------------------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------------------

def c4_job_sizes(seed, n_jobs=512, lo=100, hi=20000):
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), n_jobs))).astype(np.int64)


def _c4_job(args):
    seed, j, n = args
    kid = np.random.SeedSequence([seed, j])
    return gen_event(kid, int(n), sector=int(j % N_SECTORS))


def make_config(cfg: str, seed: int, *, workers: int = 0, n_jobs: int = 512,
                jobs=None, scale: float = 1.0, vz_sigma: float = 0.0,
                loopers: bool = False) -> ClusterSet:
    """Build one of the workloads.  ``scale`` shrinks multiplicities (tests only);
    ``jobs`` selects a subset of the c4 job list; ``workers`` > 1 uses a process pool.
    ``vz_sigma`` > 0 (c2, c3): collision vertices at z ~ N(0, vz_sigma) cm instead of z = 0,
    so that primaries near eta 0 cross the central membrane.  ``loopers`` (c2, c3): the return
    legs of primaries that turn back inside the chamber are generated too."""
    if cfg == "c1":
        cs = gen_event(seed, max(1, int(round(200 * scale))), sector=0)
    elif cfg == "c2":
        vz = float(np.random.default_rng([seed, 7]).normal(0.0, vz_sigma)) if vz_sigma > 0 else None
        cs = gen_event(seed, max(1, int(round(8000 * scale))), noise=0.05, ineff=0.1, vertex_z=vz,
                       loopers=loopers)
    elif cfg == "c3":
        rng = np.random.default_rng(seed)
        n_coll = 50 if scale >= 1 else max(1, int(round(50 * scale)))
        pool = gen_collision_pool(int(rng.integers(1 << 31)), n_coll, workers=workers,
                                  vz_sigma=vz_sigma, loopers=loopers)
        window = 1000.0 * n_coll / 50.0
        cs = assemble_timeframe(int(rng.integers(1 << 31)), pool, np.arange(n_coll), window)
    elif cfg == "c4":
        sizes = c4_job_sizes(seed, n_jobs)
        sizes = np.maximum(1, np.rint(sizes * scale).astype(np.int64))
        sel = range(n_jobs) if jobs is None else jobs
        args = [(seed, int(j), int(sizes[j])) for j in sel]
        if workers and workers > 1 and len(args) > 1:
            import multiprocessing as mp
            with mp.get_context("fork").Pool(workers) as p:
                parts = p.map(_c4_job, args, chunksize=1)
        else:
            parts = [_c4_job(a) for a in args]
        cs = concat(parts, {})
    else:
        raise ValueError(f"unknown workload {cfg!r}")
    cs.meta.update(dict(workload=cfg, seed=seed, generator_version=GENERATOR_VERSION,
                        scale=scale, vz_sigma=vz_sigma, loopers=loopers))
    return cs


def default_workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# --------------------------------------------------------------------------------------
# Inputs with exact ties (test inputs for the method's index tie-breaks)
# --------------------------------------------------------------------------------------

def with_exact_ties(cs: ClusterSet, q: float, dup_frac: float, seed: int) -> ClusterSet:
    """A copy of ``cs`` whose y and z are rounded to multiples of ``q`` (a power of two,
    so the lattice values are exact in FP32; 1/32 cm is the decoded compression step)
    and in which a fraction ``dup_frac`` of the clusters of every job appears twice with
    identical coordinates.  Each job's clusters are shuffled afterwards, so a duplicate
    is as likely to come before its original as after it.  Returns the new set; its
    ``meta["dup_group"]`` holds, per cluster, the index of the group of identical
    clusters it belongs to (int64, every cluster in exactly one group)."""
    assert q > 0 and math.log2(q) == round(math.log2(q))
    rng = np.random.default_rng(seed)
    parts, groups, base = [], [], 0
    for j in range(cs.n_jobs):
        s = cs.job(j)
        n = s.n
        k = int(round(dup_frac * n))
        src = np.concatenate([np.arange(n), rng.choice(n, k, replace=False)]) if n else np.arange(0)
        p = rng.permutation(len(src))
        src = src[p]
        y = (np.rint(s.y.astype(np.float64) / q) * q).astype(np.float32)
        z = (np.rint(s.z.astype(np.float64) / q) * q).astype(np.float32)
        parts.append(ClusterSet(s.sector[src], s.row[src], y[src], z[src], s.time[src], s.label[src],
                                np.array([0, len(src)], np.int32), s.part_pt, s.part_eta, s.part_phi,
                                s.part_q, np.array([0, len(s.part_pt)], np.int64), {}))
        groups.append(src.astype(np.int64) + base)
        base += n
    out = concat(parts, dict(cs.meta, ties=dict(q=q, dup_frac=dup_frac, seed=seed)))
    out.meta["dup_group"] = np.concatenate(groups) if groups else np.zeros(0, np.int64)
    return out


def split_by_sector(cs: ClusterSet):
    """Every (job, sector) of ``cs`` as a job of its own: the per-sector form of a workload.

    Returns (set, perm, job_event): the clusters grouped by (job, sector), input order kept
    inside a group; perm[i] = the index in ``cs`` of cluster i of the new set; job_event[k] =
    the job of ``cs`` that new job k came from (the sector jobs of one job form one event).
    Only jobs with clusters are kept.  Particles are not split (part_off keeps every
    particle in the first sector job of its event): evaluate quality on ``cs``."""
    n = cs.n
    job_of = np.repeat(np.arange(cs.n_jobs, dtype=np.int64), np.diff(cs.job_off).astype(np.int64))
    key = job_of * N_SECTORS + cs.sector.astype(np.int64)
    perm = np.argsort(key, kind="stable")
    ks = key[perm]
    uniq, first = np.unique(ks, return_index=True)
    job_off = np.concatenate([first, [n]]).astype(np.int32)
    job_event = (uniq // N_SECTORS).astype(np.int32)
    pcount = np.diff(cs.part_off)
    part_off = np.zeros(len(uniq) + 1, np.int64)
    firsts = np.concatenate([[True], job_event[1:] != job_event[:-1]]) if len(uniq) else np.zeros(0, bool)
    part_off[1:] = np.cumsum(np.where(firsts, pcount[job_event], 0))
    out = ClusterSet(cs.sector[perm], cs.row[perm], cs.y[perm], cs.z[perm], cs.time[perm], cs.label[perm],
                     job_off, cs.part_pt, cs.part_eta, cs.part_phi, cs.part_q, part_off,
                     dict(cs.meta, split="by sector"))
    return out, perm.astype(np.int64), job_event
