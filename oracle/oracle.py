"""ctypes wrapper of the CPU oracle -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module.  The oracle is a plain single-threaded
C++ implementation of the tracking method (see the header of
``tpc_oracle.cpp`` for the steps it follows and which of them are pinned);
it shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tpc_oracle.cpp")
LIB = os.path.join(HERE, "libtpc_oracle.so")

# Strict IEEE single precision: no contraction into FMA, no fast-math.
CXXFLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
            "-fno-unsafe-math-optimizations", "-Wall"]

STAGE_GRID, STAGE_LINKS, STAGE_TRACKLETS, STAGE_SELECT, STAGE_FIT, STAGE_MERGE = range(6)


class Params(C.Structure):
    _fields_ = [(n, C.c_float) for n in (
        "win_dy_slope", "win_dy_const", "win_dz_slope", "win_dz_const", "link_cut",
        "cy0", "cz0", "cs0", "ct0", "ck0", "cy1", "cz1", "cs1", "ct1", "ck1",
        "sigma_y", "sigma_z", "nwin", "chi2_follow")] + [
        ("max_miss", C.c_int32), ("min_hits", C.c_int32)] + [
        (n, C.c_float) for n in ("smax", "bz", "merge_edge", "chi2_merge", "merge_dz", "v_drift")] + [
        ("ext_down", C.c_int32), ("merge_membrane", C.c_int32)]


# The readings of every unstated constant (windows, cuts, priors, thresholds).
DEFAULTS = dict(win_dy_slope=1.0, win_dy_const=0.5, win_dz_slope=2.0, win_dz_const=0.5,
                link_cut=1.0, cy0=1.0, cz0=1.0, cs0=0.25, ct0=0.25, ck0=100.0,
                cy1=1.0, cz1=1.0, cs1=1e-3, ct1=1e-3, ck1=1.0, sigma_y=0.1, sigma_z=0.1,
                nwin=3.0, chi2_follow=15.0, max_miss=4, min_hits=10, smax=0.95, bz=0.5,
                merge_edge=5.0, chi2_merge=50.0, merge_dz=20.0, v_drift=2.58, ext_down=0, merge_membrane=0)


# The synchronous phase's cut set (its tracks feed the compression, which attaches clusters to
# track pieces alike and codes the clusters on tracks as small residuals): no merge across
# sector edges, and the tracks extended below their innermost hits (A13); everything else as
# DEFAULTS.
SYNC = dict(DEFAULTS, merge_edge=-1.0, ext_down=1)

# The asynchronous phase's cut set: the default reading plus the merge across the central
# membrane (A21).
ASYNC = dict(DEFAULTS, merge_membrane=1)


def params(**over) -> Params:
    d = dict(DEFAULTS)
    d.update(over)
    return Params(**d)


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["g++", *CXXFLAGS, "-o", tmp, SRC])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_create.restype = P
        L.orc_create.argtypes = [C.c_int32, P, P, P, P, C.c_int32, P, P, C.POINTER(Params)]
        L.orc_destroy.argtypes = [P]
        L.orc_set_brute.argtypes = [P, C.c_int32]
        L.orc_status.argtypes = [P]
        L.orc_get_track_t0.argtypes = [P, C.c_int32, P, P]
        L.orc_get_track_ext.argtypes = [P, C.c_int32, P]
        L.orc_pair_legs.argtypes = [C.POINTER(Params), C.c_int32, P, P, P, P, P, P, C.c_int32]
        L.orc_pair_legs.restype = None
        L.orc_collision_time_f32.argtypes = [P, C.c_float, C.c_int32, C.POINTER(Params)]
        L.orc_collision_time_f32.restype = C.c_float
        L.orc_collision_time_f64.argtypes = [P, C.c_double, C.c_int32, C.POINTER(Params)]
        L.orc_collision_time_f64.restype = C.c_double
        L.orc_fp64_seconds.argtypes = [P]
        L.orc_fp64_seconds.restype = C.c_double
        L.orc_run.argtypes = [P, C.c_int32]
        L.orc_num_slot_members.restype = C.c_int64
        L.orc_num_slot_members.argtypes = [P]
        L.orc_get_rows.argtypes = [P, P, P]
        L.orc_get_links.argtypes = [P, P, P, P, P]
        L.orc_num_tracklets.argtypes = [P]
        L.orc_num_tracklet_hits.restype = C.c_int64
        L.orc_num_tracklet_hits.argtypes = [P]
        L.orc_get_tracklets.argtypes = [P] * 7
        L.orc_get_hitw.argtypes = [P, P]
        L.orc_num_tracks.argtypes = [P, C.c_int32]
        L.orc_num_track_hits.restype = C.c_int64
        L.orc_num_track_hits.argtypes = [P, C.c_int32]
        L.orc_get_tracks.argtypes = [P, C.c_int32] + [P] * 16
        L.orc_propagate_f32.argtypes = [P, P, C.c_float, C.c_float, C.POINTER(Params)]
        L.orc_propagate_f64.argtypes = [P, P, C.c_double, C.c_double, C.POINTER(Params)]
        L.orc_update_f32.argtypes = [P, P, C.c_float, C.c_float, C.POINTER(Params), P]
        L.orc_update_f64.argtypes = [P, P, C.c_double, C.c_double, C.POINTER(Params), P]
        L.orc_asinc_f32.argtypes = [C.c_float, P, P]
        L.orc_asinc_f64.argtypes = [C.c_double, P, P]
        L.orc_row_x.restype = C.c_float
        L.orc_row_x.argtypes = [C.c_int32]
        L.orc_merge_chi2.restype = C.c_float
        L.orc_merge_chi2.argtypes = [P, P, P, P]
        L.orc_fit_hits_f64.argtypes = [P, C.c_int32, P, P, P, P, P, P]
        L.orc_fit_hits_f32.argtypes = [P, C.c_int32, P, P, P, P, P, P]
        L.orc_rotate_f64.argtypes = [P, P, P, C.c_int32, C.c_int32, C.POINTER(Params)]
        L.orc_rotate_f32.argtypes = [P, P, P, C.c_int32, C.c_int32, C.POINTER(Params)]
        L.orc_compress.restype = C.c_int32
        L.orc_compress.argtypes = [C.POINTER(Params), C.c_int32, P, P, P, P, C.c_int32] + [P] * 6 + [
            C.c_float, C.c_float, P, P, P, P, P]
        L.orc_decompress.argtypes = [C.POINTER(Params), C.c_int32] + [P] * 5 + [C.c_int32, P, P, P, P] + [
            C.c_float, C.c_float, P, P, P, P]
        L.orc_predict.restype = C.c_int32
        L.orc_rans_model.argtypes = [P, C.c_int32, P]
        L.orc_rans_model.restype = None
        L.orc_rans_encode.argtypes = [P, C.c_int32, P, P, P]
        L.orc_rans_encode.restype = C.c_int32
        L.orc_rans_decode.argtypes = [P, P, P, C.c_int32, P]
        L.orc_rans_decode.restype = None
        L.orc_find_clusters.restype = C.c_int32
        L.orc_find_clusters.argtypes = [C.c_int32] + [P] * 5 + [C.c_float, C.c_float, C.c_int32, C.c_int32] + [P] * 10
        L.orc_cf_pads.restype = C.c_int32
        L.orc_cf_pads.argtypes = [C.c_int32, C.c_float]
        L.orc_rans_lanes.argtypes = [C.c_int64]
        L.orc_rans_lanes.restype = C.c_int64
        L.orc_predict.argtypes = [C.POINTER(Params), P, C.c_float, C.c_int32, C.c_int32, C.c_int32, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


class Run:
    """Runs the oracle over a cluster list grouped into jobs and exposes stage outputs."""

    def __init__(self, sector, row, y, z, job_off, prm: Params | None = None,
                 last_stage: int = STAGE_MERGE, brute: bool = False, job_event=None):
        L = lib()
        self.prm = prm or params()
        self.sector = np.ascontiguousarray(sector, np.uint8)
        self.row = np.ascontiguousarray(row, np.int16)
        self.y = np.ascontiguousarray(y, np.float32)
        self.z = np.ascontiguousarray(z, np.float32)
        self.job_off = np.ascontiguousarray(job_off, np.int32)
        self.n = int(self.y.shape[0])
        self.job_event = None if job_event is None else np.ascontiguousarray(job_event, np.int32)
        self.h = L.orc_create(self.n, _p(self.sector), _p(self.row), _p(self.y), _p(self.z),
                              int(self.job_off.shape[0] - 1), _p(self.job_off),
                              None if self.job_event is None else _p(self.job_event),
                              C.byref(self.prm))
        L.orc_set_brute(self.h, int(brute))
        L.orc_run(self.h, last_stage)
        self.last_stage = last_stage

    @classmethod
    def from_set(cls, cs, prm=None, last_stage=STAGE_MERGE, brute=False, job_event=None):
        return cls(cs.sector, cs.row, cs.y, cs.z, cs.job_off, prm, last_stage, brute, job_event)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.orc_destroy(self.h)
            self.h = None

    @property
    def status(self) -> int:
        return lib().orc_status(self.h)

    @property
    def fp64_seconds(self) -> float:
        """Wall time the last run spent in its FP64 refits."""
        return float(lib().orc_fp64_seconds(self.h))

    def rows(self):
        """(slot_off[J*36*152+1], members) with members of each slot in ascending index."""
        L = lib()
        J = self.job_off.shape[0] - 1
        off = np.zeros(J * 36 * 152 + 1, np.int64)
        mem = np.zeros(L.orc_num_slot_members(self.h), np.int32)
        L.orc_get_rows(self.h, _p(off), _p(mem))
        return off, mem

    def links(self):
        a = [np.zeros(self.n, np.int32) for _ in range(4)]
        lib().orc_get_links(self.h, *map(_p, a))
        return dict(up_raw=a[0], down_raw=a[1], up=a[2], down=a[3])

    def tracklets(self):
        L = lib()
        T = L.orc_num_tracklets(self.h)
        H = L.orc_num_tracklet_hits(self.h)
        start = np.zeros(T, np.int32)
        off = np.zeros(T + 1, np.int32)
        hits = np.zeros(H, np.int32)
        P = np.zeros((T, 5), np.float32)
        Cv = np.zeros((T, 15), np.float32)
        x = np.zeros(T, np.float32)
        L.orc_get_tracklets(self.h, _p(start), _p(off), _p(hits), _p(P), _p(Cv), _p(x))
        w = np.zeros(self.n, np.uint64)
        L.orc_get_hitw(self.h, _p(w))
        return dict(start=start, off=off, hits=hits, P=P, C=Cv, x=x, hitw=w)

    def tracks(self, merged: bool | None = None):
        L = lib()
        if merged is None:
            merged = self.last_stage >= STAGE_MERGE
        K = L.orc_num_tracks(self.h, int(merged))
        H = L.orc_num_track_hits(self.h, int(merged))
        out = dict(tracklet=np.zeros(K, np.int32), job=np.zeros(K, np.int32),
                   sector=np.zeros(K, np.int32), sector2=np.zeros(K, np.int32),
                   off=np.zeros(K + 1, np.int32), hits=np.zeros(H, np.int32),
                   P=np.zeros((K, 5), np.float32), C=np.zeros((K, 15), np.float32),
                   x=np.zeros(K, np.float32), chi2=np.zeros(K, np.float32),
                   ndf=np.zeros(K, np.int32), Pd=np.zeros((K, 5), np.float64),
                   Cd=np.zeros((K, 15), np.float64), xd=np.zeros(K, np.float64),
                   chi2d=np.zeros(K, np.float64), ndfd=np.zeros(K, np.int32))
        keys = ["tracklet", "job", "sector", "sector2", "off", "hits", "P", "C", "x", "chi2",
                "ndf", "Pd", "Cd", "xd", "chi2d", "ndfd"]
        L.orc_get_tracks(self.h, int(merged), *[_p(out[k]) for k in keys])
        out["t0"] = np.zeros(K, np.float32)
        out["t0d"] = np.zeros(K, np.float64)
        L.orc_get_track_t0(self.h, int(merged), _p(out["t0"]), _p(out["t0d"]))
        out["n_ext"] = np.zeros(K, np.int32)
        L.orc_get_track_ext(self.h, int(merged), _p(out["n_ext"]))
        return out

    def fit_hits(self, hits, stk, fp64=True):
        L = lib()
        hits = np.ascontiguousarray(hits, np.int32)
        stk = np.ascontiguousarray(stk, np.float32)
        dt = np.float64 if fp64 else np.float32
        P = np.zeros(5, dt)
        Cv = np.zeros(15, dt)
        x = np.zeros(1, dt)
        c2 = np.zeros(1, dt)
        fn = L.orc_fit_hits_f64 if fp64 else L.orc_fit_hits_f32
        ok = fn(self.h, len(hits), _p(hits), _p(stk), _p(P), _p(Cv), _p(x), _p(c2))
        return bool(ok), P, Cv, float(x[0]), float(c2[0])


def pair_legs(tracks, event, prm=None, brute=False):
    """A25: the output index of each track's other looper leg, or -1 (tracks as returned by
    Run.tracks(); event: the event id of each track; brute: compare every pair of tracks
    instead of the neighbouring centre cells)."""
    K = len(tracks["ndf"])
    leg = np.full(K, -1, np.int32)
    if K:
        P = np.ascontiguousarray(tracks["P"], np.float32)
        x = np.ascontiguousarray(tracks["x"], np.float32)
        sec = np.ascontiguousarray(tracks["sector"], np.int32)
        ev = np.ascontiguousarray(event, np.int32)
        ndf = np.ascontiguousarray(tracks["ndf"], np.int32)
        lib().orc_pair_legs(C.byref(prm or params()), K, _p(P), _p(x), _p(sec), _p(ev), _p(ndf), _p(leg),
                            int(brute))
    return leg


# ----------------------------------------------------------------- unit hooks (pins)

def _state(P, dt):
    """5 values (hi) or 10 values (hi, lo) of the compensated state -> 10 values."""
    P = np.asarray(P, dt).ravel()
    return np.concatenate([P, np.zeros(5, dt)]) if P.size == 5 else P.copy()


def propagate(P, Cv, x1, x2, prm=None, fp64=False):
    """Returns (ok, state[10] = hi[5] + lo[5], C[15])."""
    dt = np.float64 if fp64 else np.float32
    P = _state(P, dt)
    Cv = np.array(Cv, dt)
    prm = prm or params()
    fn = lib().orc_propagate_f64 if fp64 else lib().orc_propagate_f32
    ok = fn(_p(P), _p(Cv), x1, x2, C.byref(prm))
    return bool(ok), P, Cv


def rotate(P, Cv, x, sec_from, sec_to, prm=None, fp64=False):
    """Sector rotation of a state at plane x (O10).  Returns (ok, state[10], C[15], x')."""
    dt = np.float64 if fp64 else np.float32
    P = _state(P, dt)
    Cv = np.array(Cv, dt)
    xx = np.array([x], dt)
    prm = prm or params()
    fn = lib().orc_rotate_f64 if fp64 else lib().orc_rotate_f32
    ok = fn(_p(P), _p(Cv), _p(xx), int(sec_from), int(sec_to), C.byref(prm))
    return bool(ok), P, Cv, float(xx[0])


def update(P, Cv, my, mz, prm=None, fp64=False):
    dt = np.float64 if fp64 else np.float32
    P = _state(P, dt)
    Cv = np.array(Cv, dt)
    c2 = np.zeros(1, dt)
    prm = prm or params()
    fn = lib().orc_update_f64 if fp64 else lib().orc_update_f32
    ok = fn(_p(P), _p(Cv), my, mz, C.byref(prm), _p(c2))
    return bool(ok), P, Cv, float(c2[0])


def collision_time(P, x, sector, prm=None, fp64=False):
    """T1: the collision time (us) of a track state P at plane x of `sector`."""
    dt = np.float64 if fp64 else np.float32
    P = np.ascontiguousarray(P, dt)
    fn = lib().orc_collision_time_f64 if fp64 else lib().orc_collision_time_f32
    return float(fn(_p(P), float(x), int(sector), C.byref(prm or params())))


def asinc(u, fp64=False):
    dt = np.float64 if fp64 else np.float32
    A = np.zeros(1, dt)
    B = np.zeros(1, dt)
    (lib().orc_asinc_f64 if fp64 else lib().orc_asinc_f32)(u, _p(A), _p(B))
    return A[0], B[0]


def row_x(r: int) -> float:
    return lib().orc_row_x(r)


def merge_chi2(PA, CA, PB, CB) -> float:
    a = [np.ascontiguousarray(v, np.float32) for v in (PA, CA, PB, CB)]
    return lib().orc_merge_chi2(*map(_p, a))


def tri_to_full(Cv):
    """Lower-triangle (15) -> symmetric 5x5."""
    M = np.zeros((5, 5), dtype=np.asarray(Cv).dtype)
    k = 0
    for i in range(5):
        for j in range(i + 1):
            M[i, j] = M[j, i] = Cv[k]
            k += 1
    return M


def full_to_tri(M):
    return np.array([M[i, j] for i in range(5) for j in range(i + 1)], dtype=M.dtype)


# ----------------------------------------------------------------- track-model compression

def _headers(tracks):
    K = len(tracks["off"]) - 1
    g = lambda k, dt: np.ascontiguousarray(tracks[k], dt)
    return K, g("off", np.int32), g("P", np.float32), g("x", np.float32), g("sector", np.int32), g("ndf", np.int32)


def compress(sector, row, y, z, tracks, q_y, q_z, prm=None, wide_z=False):
    """C2-C4: records (rs, ey, ez) of every track hit in track order, then of the clusters in
    no track in input order; returns dict(rs, ey, ez, n_attached, status), plus ez_hi (C7:
    24-bit absolute z codes) with wide_z.  `tracks` has the keys of Run.tracks(): off, hits,
    P, x, sector, ndf."""
    prm = prm or params()
    sector = np.ascontiguousarray(sector, np.uint8)
    row = np.ascontiguousarray(row, np.int16)
    y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32)
    K, off, P, x, ts, ndf = _headers(tracks)
    hits = np.ascontiguousarray(tracks["hits"], np.int32)
    n = len(y)
    cap = int(off[-1]) + n
    rs = np.zeros(cap, np.uint16)
    ey = np.zeros(cap, np.int16)
    ez = np.zeros(cap, np.int16)
    ezh = np.zeros(cap, np.int8) if wide_z else None
    st = np.zeros(1, np.int32)
    m = lib().orc_compress(C.byref(prm), n, _p(sector), _p(row), _p(y), _p(z), K, _p(off), _p(hits), _p(P),
                           _p(x), _p(ts), _p(ndf), q_y, q_z, _p(rs), _p(ey), _p(ez),
                           None if ezh is None else _p(ezh), _p(st))
    out = dict(rs=rs[:m], ey=ey[:m], ez=ez[:m], n_attached=int(off[-1]), status=int(st[0]))
    if wide_z:
        out["ez_hi"] = ezh[:m]
    return out


def decompress(tracks, codes, q_y, q_z, prm=None):
    """C5: (sector, row, y, z) of every record, in stream order."""
    prm = prm or params()
    K, off, P, x, ts, ndf = _headers(tracks)
    rs = np.ascontiguousarray(codes["rs"], np.uint16)
    ey = np.ascontiguousarray(codes["ey"], np.int16)
    ez = np.ascontiguousarray(codes["ez"], np.int16)
    ezh = codes.get("ez_hi")
    ezh = None if ezh is None else np.ascontiguousarray(ezh, np.int8)
    m = len(rs)
    out = dict(sector=np.zeros(m, np.uint8), row=np.zeros(m, np.int16), y=np.zeros(m, np.float32),
               z=np.zeros(m, np.float32))
    lib().orc_decompress(C.byref(prm), K, _p(off), _p(P), _p(x), _p(ts), _p(ndf), m, _p(rs), _p(ey), _p(ez),
                         None if ezh is None else _p(ezh), q_y, q_z,
                         *[_p(out[k]) for k in ("sector", "row", "y", "z")])
    return out


def predict(P, x_ref, sector_ref, sector, row, prm=None):
    """C1: (ok, py, pz) for a cluster at (sector, row) of a track with state P at x_ref."""
    prm = prm or params()
    P = np.ascontiguousarray(P, np.float32)
    yz = np.zeros(2, np.float32)
    ok = lib().orc_predict(C.byref(prm), _p(P), x_ref, sector_ref, sector, row, _p(yz))
    return bool(ok), yz[0], yz[1]


# ----------------------------------------------------------------- rANS entropy coding

RANS_LANE_SYMBOLS = 512


def rans_lanes(n: int) -> int:
    return int(lib().orc_rans_lanes(n))


def rans_model(sym):
    """E1: normalised frequencies (uint32[65536], sum 2^16 unless the stream is empty)."""
    sym = np.ascontiguousarray(sym, np.uint16)
    f = np.zeros(1 << 16, np.uint32)
    lib().orc_rans_model(_p(sym), len(sym), _p(f))
    return f


def rans_encode(sym, freq=None):
    """E2, E4, E5: dict(freq, lane_off, words)."""
    sym = np.ascontiguousarray(sym, np.uint16)
    n = len(sym)
    freq = rans_model(sym) if freq is None else np.ascontiguousarray(freq, np.uint32)
    lanes = rans_lanes(n)
    off = np.zeros(lanes + 1, np.uint32)
    words = np.zeros(max(1, lanes * (RANS_LANE_SYMBOLS + 2)), np.uint16)
    m = lib().orc_rans_encode(_p(sym), n, _p(freq), _p(off), _p(words))
    return dict(freq=freq, lane_off=off, words=words[:m])


def rans_decode(enc, n):
    """E3: the n symbols back."""
    out = np.zeros(max(n, 1), np.uint16)
    f = np.ascontiguousarray(enc["freq"], np.uint32)
    off = np.ascontiguousarray(enc["lane_off"], np.uint32)
    w = np.ascontiguousarray(enc["words"], np.uint16)
    if len(w) == 0:
        w = np.zeros(1, np.uint16)
    lib().orc_rans_decode(_p(f), _p(off), _p(w), n, _p(out))
    return out[:n]


# ----------------------------------------------------------------- cluster finding

CF_DEFAULTS = dict(pitch=0.5, bin=0.5, n_time=500, q_min=10)


def cf_pads(r: int, pitch: float = 0.5) -> int:
    return int(lib().orc_cf_pads(r, pitch))


def find_clusters(sector, row, pad, time, adc, pitch=0.5, bin=0.5, n_time=500, q_min=10):
    """F1-F6: dict(digit, sector, row, y, z, q_tot, q_max, sigma_pad, sigma_time, status)."""
    a = [np.ascontiguousarray(sector, np.uint8), np.ascontiguousarray(row, np.int16),
         np.ascontiguousarray(pad, np.int16), np.ascontiguousarray(time, np.int16),
         np.ascontiguousarray(adc, np.uint16)]
    n = len(a[0])
    m0 = max(n, 1)
    out = dict(digit=np.zeros(m0, np.int32), sector=np.zeros(m0, np.uint8), row=np.zeros(m0, np.int16),
               y=np.zeros(m0, np.float32), z=np.zeros(m0, np.float32), q_tot=np.zeros(m0, np.uint32),
               q_max=np.zeros(m0, np.uint32), sigma_pad=np.zeros(m0, np.float32),
               sigma_time=np.zeros(m0, np.float32))
    st = np.zeros(1, np.int32)
    keys = ["digit", "sector", "row", "y", "z", "q_tot", "q_max", "sigma_pad", "sigma_time"]
    m = lib().orc_find_clusters(n, *map(_p, a), pitch, bin, n_time, q_min, *[_p(out[k]) for k in keys], _p(st))
    res = {k: v[:m] for k, v in out.items()}
    res["status"] = int(st[0])
    return res
