"""Python binding of libtpc.so (the C ABI in include/tpc.h).

Argument marshalling only: every step of the tracking runs in the HIP kernels
of the library.  PyTorch supplies device memory (workspace, inputs, outputs)
and the HIP stream.  If the library is not built, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtpc.so")

TPC_OK, TPC_E_ARG, TPC_E_RANGE, TPC_E_CAPACITY, TPC_E_HIP = 0, -1, -2, -3, -4
MODES = {"plain": 0, "batched": 1, "persistent": 2}
N_SECTORS, N_ROWS = 36, 152


class TpcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tpc error {code}: {msg}")
        self.code = code


class tpc_params(C.Structure):
    _fields_ = [(n, C.c_float) for n in (
        "win_dy_slope", "win_dy_const", "win_dz_slope", "win_dz_const", "link_cut",
        "cy0", "cz0", "cs0", "ct0", "ck0", "cy1", "cz1", "cs1", "ct1", "ck1",
        "sigma_y", "sigma_z", "nwin", "chi2_follow")] + [
        ("max_miss", C.c_int32), ("min_hits", C.c_int32)] + [
        (n, C.c_float) for n in ("smax", "bz", "merge_edge", "chi2_merge", "merge_dz", "v_drift")] + [
        ("ext_down", C.c_int32), ("merge_membrane", C.c_int32)]


class tpc_tuning(C.Structure):
    _fields_ = [("cells_per_cluster", C.c_float), ("block_links", C.c_int32),
                ("block_tracklets", C.c_int32), ("persistent_waves", C.c_int32),
                ("use_graph", C.c_int32), ("tracklet_order", C.c_int32),
                ("persistent_refill", C.c_int32)]


class tpc_clusters(C.Structure):
    _fields_ = [("n", C.c_int32), ("sector", C.c_void_p), ("row", C.c_void_p), ("y", C.c_void_p),
                ("z", C.c_void_p), ("time", C.c_void_p)]


class tpc_jobs(C.Structure):
    _fields_ = [("n_jobs", C.c_int32), ("job_off", C.c_void_p), ("job_off_host", C.c_void_p),
                ("job_event", C.c_void_p)]


class tpc_tracks(C.Structure):
    _fields_ = [("cap_tracks", C.c_int32), ("cap_hits", C.c_int32)] + [
        (n, C.c_void_p) for n in ("n_tracks", "hit_off", "hits", "param", "cov", "x_ref", "chi2",
                                  "ndf", "sector", "job", "tracklet", "t0")]


class tpc_codes(C.Structure):
    _fields_ = [("cap", C.c_int32)] + [(n, C.c_void_p) for n in ("n_codes", "n_attached", "rs", "ey", "ez",
                                                              "ez_hi")]


class tpc_rans(C.Structure):
    _fields_ = [("cap_words", C.c_int32)] + [(n, C.c_void_p) for n in ("n_words", "freq", "lane_off", "words")]


RANS_LANE_SYMBOLS = 512


class tpc_cf_params(C.Structure):
    _fields_ = [("pad_pitch", C.c_float), ("time_bin", C.c_float), ("n_time", C.c_int32), ("q_min", C.c_int32)]


class tpc_digits(C.Structure):
    _fields_ = [("n", C.c_int32)] + [(k, C.c_void_p) for k in ("sector", "row", "pad", "time", "adc")]


CF_KEYS = ("digit", "sector", "row", "y", "z", "q_tot", "q_max", "sigma_pad", "sigma_time")


class tpc_cf_clusters(C.Structure):
    _fields_ = [("cap", C.c_int32), ("n_clusters", C.c_void_p), ("status", C.c_void_p)] + [
        (k, C.c_void_p) for k in CF_KEYS]

# Default quantisation step of the compressed coordinates (cm): a power of two, so that
# 1/q and e*q are exact in FP32; q/sqrt(12) = 0.009 cm against 0.1 cm cluster errors.
Q_STEP = 1.0 / 32.0

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2402_01205_amd/build.py")
        # torch's HIP runtime is loaded and initialised before the library is, so the
        # library binds to that runtime; loaded the other way round, two runtimes can end
        # up in the process and the library's finds no device.
        import torch
        if torch.cuda.is_available():
            torch.cuda.init()
        L = C.CDLL(LIB_PATH)
        V, P, I = C.c_void_p, C.POINTER, C.c_int
        L.tpc_params_default.argtypes = [P(tpc_params)]
        L.tpc_params_preset.argtypes = [P(tpc_params), I]
        L.tpc_tuning_default.argtypes = [P(tpc_tuning)]
        L.tpc_ctx_create.argtypes = [P(V), I, V, P(tpc_params)]
        L.tpc_ctx_destroy.argtypes = [V]
        L.tpc_ctx_destroy.restype = None
        L.tpc_set_stream.argtypes = [V, V]
        L.tpc_set_mode.argtypes = [V, I]
        L.tpc_set_tuning.argtypes = [V, P(tpc_tuning)]
        L.tpc_last_error.argtypes = [V]
        L.tpc_last_error.restype = C.c_char_p
        L.tpc_workspace_size.argtypes = [V, C.c_int64, C.c_int32]
        L.tpc_workspace_size.restype = C.c_size_t
        L.tpc_bind_workspace.argtypes = [V, V, C.c_size_t]
        L.tpc_grid_build.argtypes = [V, P(tpc_clusters), P(tpc_jobs)]
        L.tpc_find_neighbours.argtypes = [V, V, V]
        L.tpc_construct_tracklets.argtypes = [V, V]
        L.tpc_select_tracks.argtypes = [V, V]
        L.tpc_fit_merge.argtypes = [V, P(tpc_tracks)]
        L.tpc_run.argtypes = [V, P(tpc_clusters), P(tpc_jobs), P(tpc_tracks)]
        L.tpc_sync.argtypes = [V]
        L.tpc_counts.argtypes = [V, V]
        L.tpc_get_links_raw.argtypes = [V, V, V]
        L.tpc_get_rows.argtypes = [V, V, V]
        L.tpc_get_tracklet_counts.argtypes = [V, P(C.c_int32), P(C.c_int64)]
        L.tpc_get_tracklets.argtypes = [V, V, V, V, V, V]
        L.tpc_get_selected_counts.argtypes = [V, P(C.c_int32), P(C.c_int64)]
        L.tpc_get_selected.argtypes = [V, V, V, V]
        L.tpc_debug_propagate.argtypes = [V, V, V, C.c_int32]
        L.tpc_debug_update.argtypes = [V, V, V, C.c_int32]
        L.tpc_profile.argtypes = [V, I]
        L.tpc_copy_probe.argtypes = [V, V, V, C.c_size_t]
        L.tpc_profile_read.argtypes = [V, V, V, C.c_int32, C.c_int32]
        L.tpc_compress.argtypes = [V, P(tpc_clusters), P(tpc_tracks), C.c_float, C.c_float, P(tpc_codes)]
        L.tpc_decompress.argtypes = [V, P(tpc_tracks), P(tpc_codes), C.c_float, C.c_float, V, V, V, V]
        L.tpc_cf_params_default.argtypes = [P(tpc_cf_params)]
        L.tpc_cf_workspace_size.argtypes = [P(tpc_cf_params), C.c_int32]
        L.tpc_cf_workspace_size.restype = C.c_size_t
        L.tpc_find_clusters.argtypes = [V, P(tpc_cf_params), P(tpc_digits), V, C.c_size_t, P(tpc_cf_clusters)]
        L.tpc_pair_legs_workspace_size.argtypes = [C.c_int32]
        L.tpc_pair_legs_workspace_size.restype = C.c_size_t
        L.tpc_pair_legs.argtypes = [V, P(tpc_tracks), V, V, C.c_size_t, V]
        L.tpc_rans_lanes.argtypes = [C.c_int64]
        L.tpc_rans_lanes.restype = C.c_int64
        L.tpc_rans_encode.argtypes = [V, V, C.c_int32, P(tpc_rans)]
        L.tpc_rans_decode.argtypes = [V, P(tpc_rans), C.c_int32, V]
        L.tpc_rans_encode_static.argtypes = [V, V, C.c_int32, P(tpc_rans)]
        _lib = L
    return _lib


EXPORTED = ["tpc_params_default", "tpc_params_preset", "tpc_tuning_default", "tpc_ctx_create", "tpc_ctx_destroy",
            "tpc_set_stream", "tpc_set_mode", "tpc_set_tuning", "tpc_last_error",
            "tpc_workspace_size", "tpc_bind_workspace", "tpc_grid_build", "tpc_find_neighbours", "tpc_counts",
            "tpc_construct_tracklets", "tpc_select_tracks", "tpc_fit_merge", "tpc_run", "tpc_sync",
            "tpc_get_links_raw", "tpc_get_rows", "tpc_get_tracklet_counts", "tpc_get_tracklets",
            "tpc_get_selected_counts", "tpc_get_selected", "tpc_debug_propagate", "tpc_debug_update",
            "tpc_profile", "tpc_profile_read", "tpc_copy_probe", "tpc_compress", "tpc_decompress",
            "tpc_rans_lanes", "tpc_rans_encode", "tpc_rans_decode", "tpc_rans_encode_static",
            "tpc_cf_params_default",
            "tpc_cf_workspace_size", "tpc_find_clusters", "tpc_pair_legs_workspace_size", "tpc_pair_legs"]
PROF_NAMES = ["k_links", "k_tracklets", "grid_build", "select", "fit_merge", "compress", "decompress",
              "rans_encode", "rans_decode", "find_clusters", "pair_legs"]


def default_params(**over) -> tpc_params:
    p = tpc_params()
    lib().tpc_params_default(C.byref(p))
    for k, v in over.items():
        setattr(p, k, v)
    return p


PRESETS = {"async": 0, "sync": 1}


def preset_params(name: str, **over) -> tpc_params:
    """The cut set of a processing phase ("async": the defaults plus the membrane merge,
    "sync"), then overrides."""
    p = tpc_params()
    if lib().tpc_params_preset(C.byref(p), PRESETS[name]) != TPC_OK:
        raise TpcError(TPC_E_ARG, f"unknown preset {name!r}")
    for k, v in over.items():
        setattr(p, k, v)
    return p


def default_tuning(**over) -> tpc_tuning:
    t = tpc_tuning()
    lib().tpc_tuning_default(C.byref(t))
    for k, v in over.items():
        setattr(t, k, v)
    return t


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


@dataclass
class DeviceClusters:
    """Cluster SoA and job table resident on the GPU (torch tensors)."""
    sector: "object"
    row: "object"
    y: "object"
    z: "object"
    time: "object"
    job_off: "object"          # device int32 [J+1]
    job_off_host: np.ndarray   # host int32 [J+1]
    job_event: "object" = None  # device int32 [J] or None

    @property
    def n(self) -> int:
        return int(self.y.shape[0])

    @property
    def n_jobs(self) -> int:
        return int(self.job_off_host.shape[0] - 1)

    @classmethod
    def from_set(cls, cs, device="cuda", job_event=None):
        import torch
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dt)).to(device, non_blocking=False)
        jo = np.ascontiguousarray(cs.job_off, np.int32)
        ev = None if job_event is None else t(job_event, np.int32)
        return cls(t(cs.sector, np.uint8), t(cs.row, np.int16), t(cs.y, np.float32),
                   t(cs.z, np.float32), t(cs.time, np.float32), t(jo, np.int32), jo, ev)


class Tracker:
    """One library context on one GPU, its workspace and output buffers."""

    def __init__(self, device: int = 0, params: tpc_params | None = None, mode: str = "batched",
                 tuning: tpc_tuning | None = None, stream=None):
        import torch
        self.torch = torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.ctx = C.c_void_p()
        self.params = params or default_params()
        self._check(lib().tpc_ctx_create(C.byref(self.ctx), device, C.c_void_p(self.stream.cuda_stream),
                                         C.byref(self.params)), "tpc_ctx_create")
        self.set_mode(mode)
        if tuning is not None:
            self.set_tuning(tuning)
        self.ws = None
        self.out = None
        self._keep = None

    def __del__(self):
        if getattr(self, "ctx", None) and self.ctx.value and _lib is not None:
            _lib.tpc_ctx_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def _check(self, rc, what=""):
        if rc != TPC_OK:
            msg = lib().tpc_last_error(self.ctx if self.ctx.value else None).decode()
            raise TpcError(rc, f"{what}: {msg}")

    def set_mode(self, mode: str):
        self.mode = mode
        self._check(lib().tpc_set_mode(self.ctx, MODES[mode]), "tpc_set_mode")

    def set_tuning(self, t: tpc_tuning):
        self.tuning = t
        self._check(lib().tpc_set_tuning(self.ctx, C.byref(t)), "tpc_set_tuning")
        self.ws = None

    def set_stream(self, stream):
        self.stream = stream
        self._check(lib().tpc_set_stream(self.ctx, C.c_void_p(stream.cuda_stream)), "tpc_set_stream")

    def workspace_size(self, n: int, n_jobs: int) -> int:
        return int(lib().tpc_workspace_size(self.ctx, n, n_jobs))

    def reserve(self, n: int, n_jobs: int):
        """Allocates the workspace and the output buffers for inputs of up to n clusters in
        n_jobs jobs now, so that later runs of that size allocate nothing."""
        self._ensure(n, n_jobs)

    def _ensure(self, n: int, n_jobs: int):
        torch = self.torch
        need = self.workspace_size(n, n_jobs)
        if self.ws is None or self.ws.numel() < need:
            self.ws = None
            self.ws = torch.empty(need, dtype=torch.uint8, device=f"cuda:{self.device}")
            self._check(lib().tpc_bind_workspace(self.ctx, _ptr(self.ws), need), "tpc_bind_workspace")
        capT = min(n // 8 + 1024, n + 1024)
        capH = n + 1
        if self.out is None or self.out["cap_tracks"] < capT or self.out["cap_hits"] < capH:
            dev = f"cuda:{self.device}"
            i32, f32 = torch.int32, torch.float32
            self.out = dict(cap_tracks=capT, cap_hits=capH,
                            n_tracks=torch.zeros(1, dtype=i32, device=dev),
                            hit_off=torch.zeros(capT + 1, dtype=i32, device=dev),
                            hits=torch.zeros(capH, dtype=i32, device=dev),
                            param=torch.zeros(capT, 5, dtype=f32, device=dev),
                            cov=torch.zeros(capT, 15, dtype=f32, device=dev),
                            x_ref=torch.zeros(capT, dtype=f32, device=dev),
                            chi2=torch.zeros(capT, dtype=f32, device=dev),
                            ndf=torch.zeros(capT, dtype=i32, device=dev),
                            sector=torch.zeros(capT, dtype=i32, device=dev),
                            job=torch.zeros(capT, dtype=i32, device=dev),
                            tracklet=torch.zeros(capT, dtype=i32, device=dev),
                            t0=torch.zeros(capT, dtype=f32, device=dev))

    def _prepare(self, ev: DeviceClusters):
        self._ensure(ev.n, ev.n_jobs)
        o = self.out
        self._tracks = tpc_tracks(o["cap_tracks"], o["cap_hits"], *[
            _ptr(o[k]) for k in ("n_tracks", "hit_off", "hits", "param", "cov", "x_ref", "chi2", "ndf",
                                 "sector", "job", "tracklet", "t0")])
        self._cl = tpc_clusters(ev.n, _ptr(ev.sector), _ptr(ev.row), _ptr(ev.y), _ptr(ev.z), _ptr(ev.time))
        self._jobs_host = np.ascontiguousarray(ev.job_off_host, np.int32)
        self._jb = tpc_jobs(ev.n_jobs, _ptr(ev.job_off), self._jobs_host.ctypes.data_as(C.c_void_p),
                            _ptr(ev.job_event))
        self._keep = ev

    # ---- the five stages (same names as the C ABI)
    def tpc_grid_build(self, ev: DeviceClusters):
        self._prepare(ev)
        self._check(lib().tpc_grid_build(self.ctx, C.byref(self._cl), C.byref(self._jb)), "tpc_grid_build")

    def tpc_find_neighbours(self, up=None, down=None):
        self._check(lib().tpc_find_neighbours(self.ctx, _ptr(up), _ptr(down)), "tpc_find_neighbours")

    def tpc_construct_tracklets(self, n_tracklets=None):
        self._check(lib().tpc_construct_tracklets(self.ctx, _ptr(n_tracklets)), "tpc_construct_tracklets")

    def tpc_select_tracks(self, n_selected=None):
        self._check(lib().tpc_select_tracks(self.ctx, _ptr(n_selected)), "tpc_select_tracks")

    def tpc_fit_merge(self):
        self._check(lib().tpc_fit_merge(self.ctx, C.byref(self._tracks)), "tpc_fit_merge")

    def tpc_run(self, ev: DeviceClusters):
        self._prepare(ev)
        self._check(lib().tpc_run(self.ctx, C.byref(self._cl), C.byref(self._jb), C.byref(self._tracks)),
                    "tpc_run")

    def tpc_sync(self):
        self._check(lib().tpc_sync(self.ctx), "tpc_sync")

    def tpc_counts(self, dst):
        """Enqueues the copy of the last run's six counters (status bits, tracklets,
        selected tracks and hits, output tracks and hits) into `dst` (int32 tensor of 6,
        device or pinned host)."""
        assert dst.dtype == self.torch.int32 and dst.numel() >= 6 and dst.is_contiguous()
        self._check(lib().tpc_counts(self.ctx, _ptr(dst)), "tpc_counts")

    # ---- track-model compression of the current clusters against the current tracks
    def tpc_compress(self, q_y: float = Q_STEP, q_z: float = Q_STEP, cap: int | None = None,
                     wide_z: bool = False) -> dict:
        """Enqueues tpc_compress; returns the record buffers (device tensors, rs stored as int16);
        wide_z: 24-bit absolute z codes (the high bytes in ez_hi), for time frames."""
        torch = self.torch
        dev = f"cuda:{self.device}"
        cap = max(self._keep.n, 1) if cap is None else cap
        cd = getattr(self, "codes", None)
        if cd is None or cd["cap"] != cap or (cd["ez_hi"] is not None) != wide_z:
            i32, i16 = torch.int32, torch.int16
            cd = dict(cap=cap, n_codes=torch.zeros(1, dtype=i32, device=dev),
                      n_attached=torch.zeros(1, dtype=i32, device=dev),
                      rs=torch.zeros(max(cap, 1), dtype=i16, device=dev),
                      ey=torch.zeros(max(cap, 1), dtype=i16, device=dev),
                      ez=torch.zeros(max(cap, 1), dtype=i16, device=dev),
                      ez_hi=torch.zeros(max(cap, 1), dtype=torch.int8, device=dev) if wide_z else None)
            self.codes = cd
        cd["q"] = (q_y, q_z)
        self._codes = tpc_codes(cap, *[_ptr(cd[k]) for k in ("n_codes", "n_attached", "rs", "ey", "ez", "ez_hi")])
        self._check(lib().tpc_compress(self.ctx, C.byref(self._cl), C.byref(self._tracks), q_y, q_z,
                                       C.byref(self._codes)), "tpc_compress")
        return cd

    def tpc_decompress(self, out: dict | None = None) -> dict:
        """Enqueues tpc_decompress of the last records against the current tracks into device
        tensors sector, row, y, z [cap]."""
        torch = self.torch
        dev = f"cuda:{self.device}"
        cd = self.codes
        cap = max(cd["cap"], 1)
        if out is None:
            out = dict(sector=torch.zeros(cap, dtype=torch.uint8, device=dev),
                       row=torch.zeros(cap, dtype=torch.int16, device=dev),
                       y=torch.zeros(cap, dtype=torch.float32, device=dev),
                       z=torch.zeros(cap, dtype=torch.float32, device=dev))
        q_y, q_z = cd["q"]
        self._check(lib().tpc_decompress(self.ctx, C.byref(self._tracks), C.byref(self._codes), q_y, q_z,
                                         *[_ptr(out[k]) for k in ("sector", "row", "y", "z")]),
                    "tpc_decompress")
        return out

    # ---- the two legs of loopers among the current tracks
    def tpc_pair_legs(self, job_event=None):
        """Enqueues tpc_pair_legs on the current tracks (job_event: device int32 [n_jobs] or
        None); returns the device int32 tensor leg [cap_tracks], kept until the next call:
        the index of each track's other leg, or -1."""
        torch = self.torch
        dev = f"cuda:{self.device}"
        cap = self.out["cap_tracks"]
        need = int(lib().tpc_pair_legs_workspace_size(cap))
        if need == 0:
            raise TpcError(TPC_E_ARG, "tpc_pair_legs_workspace_size: too many track slots")
        if getattr(self, "leg_ws", None) is None or self.leg_ws.numel() < need:
            self.leg_ws = torch.empty(need, dtype=torch.uint8, device=dev)
        if getattr(self, "legs", None) is None or self.legs.numel() != max(cap, 1):
            self.legs = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        ev = None if job_event is None else _ptr(job_event)
        self._check(lib().tpc_pair_legs(self.ctx, C.byref(self._tracks), ev, _ptr(self.leg_ws), need,
                                        _ptr(self.legs)), "tpc_pair_legs")
        return self.legs

    # ---- rANS entropy coding of a device stream of 16-bit symbols
    def tpc_rans_encode(self, sym, cap_words: int | None = None) -> dict:
        """Enqueues tpc_rans_encode of `sym` (device tensor of 2-byte elements); returns the
        coded stream's device buffers."""
        torch = self.torch
        dev = f"cuda:{self.device}"
        n = int(sym.numel())
        lanes = int(lib().tpc_rans_lanes(n))
        cap = n + 2 * lanes if cap_words is None else cap_words
        enc = dict(n=n, cap_words=cap, n_words=torch.zeros(1, dtype=torch.int32, device=dev),
                   freq=torch.zeros(1 << 16, dtype=torch.int32, device=dev),
                   lane_off=torch.zeros(lanes + 1, dtype=torch.int32, device=dev),
                   words=torch.zeros(max(cap, 1), dtype=torch.int16, device=dev))
        enc["_s"] = tpc_rans(cap, *[_ptr(enc[k]) for k in ("n_words", "freq", "lane_off", "words")])
        self._check(lib().tpc_rans_encode(self.ctx, _ptr(sym), n, C.byref(enc["_s"])), "tpc_rans_encode")
        return enc

    def rans_outputs(self, n: int, cap_words: int | None = None) -> dict:
        """Device output buffers of a coded stream of n symbols (words for the worst case
        unless cap_words is given)."""
        torch = self.torch
        dev = f"cuda:{self.device}"
        lanes = int(lib().tpc_rans_lanes(n))
        cap = n + 2 * lanes if cap_words is None else cap_words
        enc = dict(n=n, cap_words=cap, n_words=torch.zeros(1, dtype=torch.int32, device=dev),
                   freq=torch.zeros(1 << 16, dtype=torch.int32, device=dev),
                   lane_off=torch.zeros(lanes + 1, dtype=torch.int32, device=dev),
                   words=torch.zeros(max(cap, 1), dtype=torch.int16, device=dev))
        enc["_s"] = tpc_rans(cap, *[_ptr(enc[k]) for k in ("n_words", "freq", "lane_off", "words")])
        return enc

    def tpc_rans_encode_static(self, sym, enc: dict) -> dict:
        """Enqueues tpc_rans_encode_static of `sym` (device tensor of 2-byte elements) into the
        caller's buffers `enc` (from rans_outputs, for at least sym.numel() symbols)."""
        n = int(sym.numel())
        if int(lib().tpc_rans_lanes(n)) + 1 > enc["lane_off"].numel():
            raise ValueError("lane offset buffer too small for the stream")
        enc["n"] = n
        self._check(lib().tpc_rans_encode_static(self.ctx, _ptr(sym), n, C.byref(enc["_s"])),
                    "tpc_rans_encode_static")
        return enc

    def tpc_rans_decode(self, enc: dict, out=None):
        """Enqueues tpc_rans_decode of a stream from tpc_rans_encode into `out` (device, int16)."""
        torch = self.torch
        n = enc["n"]
        if out is None:
            out = torch.zeros(max(n, 1), dtype=torch.int16, device=f"cuda:{self.device}")
        self._check(lib().tpc_rans_decode(self.ctx, C.byref(enc["_s"]), n, _ptr(out)), "tpc_rans_decode")
        return out

    def rans_numpy(self, enc: dict) -> dict:
        self.torch.cuda.synchronize(self.device)
        m = min(int(enc["n_words"].item()), enc["cap_words"])
        return dict(n_words=int(enc["n_words"].item()), freq=enc["freq"].cpu().numpy().view(np.uint32),
                    lane_off=enc["lane_off"].cpu().numpy().view(np.uint32),
                    words=enc["words"][:m].cpu().numpy().view(np.uint16))

    # ---- cluster finding from digits (device tensors)
    def tpc_find_clusters(self, digits: dict, params: tpc_cf_params | None = None, cap: int | None = None) -> dict:
        """Enqueues tpc_find_clusters on digits {sector u8, row i16, pad i16, time i16, adc i16
        (read as uint16)}; returns the output device tensors (kept until the next call)."""
        torch = self.torch
        dev = f"cuda:{self.device}"
        if params is None:
            params = tpc_cf_params()
            lib().tpc_cf_params_default(C.byref(params))
        n = int(digits["adc"].numel())
        need = int(lib().tpc_cf_workspace_size(C.byref(params), n))
        if need == 0:
            raise TpcError(TPC_E_ARG, "tpc_cf_workspace_size: invalid parameters")
        if getattr(self, "cf_ws", None) is None or self.cf_ws.numel() < need:
            self.cf_ws = torch.empty(need, dtype=torch.uint8, device=dev)
        cap = max(n, 1) if cap is None else cap
        i32, f32 = torch.int32, torch.float32
        o = dict(cap=cap, n_clusters=torch.zeros(1, dtype=i32, device=dev), status=torch.zeros(1, dtype=i32, device=dev),
                 digit=torch.zeros(max(cap, 1), dtype=i32, device=dev),
                 sector=torch.zeros(max(cap, 1), dtype=torch.uint8, device=dev),
                 row=torch.zeros(max(cap, 1), dtype=torch.int16, device=dev),
                 y=torch.zeros(max(cap, 1), dtype=f32, device=dev), z=torch.zeros(max(cap, 1), dtype=f32, device=dev),
                 q_tot=torch.zeros(max(cap, 1), dtype=i32, device=dev),
                 q_max=torch.zeros(max(cap, 1), dtype=i32, device=dev),
                 sigma_pad=torch.zeros(max(cap, 1), dtype=f32, device=dev),
                 sigma_time=torch.zeros(max(cap, 1), dtype=f32, device=dev))
        dg = tpc_digits(n, *[_ptr(digits[k]) for k in ("sector", "row", "pad", "time", "adc")])
        cl = tpc_cf_clusters(cap, _ptr(o["n_clusters"]), _ptr(o["status"]), *[_ptr(o[k]) for k in CF_KEYS])
        self._check(lib().tpc_find_clusters(self.ctx, C.byref(params), C.byref(dg), _ptr(self.cf_ws), need,
                                            C.byref(cl)), "tpc_find_clusters")
        return o

    def clusters_numpy(self, o: dict) -> dict:
        """The found clusters as numpy arrays (waits for the stream); status as TPC_STATUS_* bits."""
        self.torch.cuda.synchronize(self.device)
        m = min(int(o["n_clusters"].item()), o["cap"])
        r = {k: o[k][:m].cpu().numpy() for k in CF_KEYS}
        r["q_tot"] = r["q_tot"].view(np.uint32)
        r["q_max"] = r["q_max"].view(np.uint32)
        r["n"] = int(o["n_clusters"].item())
        r["status"] = int(o["status"].item())
        return r

    def codes_numpy(self) -> dict:
        """The records of the last tpc_compress (waits for the stream; no error check)."""
        self.torch.cuda.synchronize(self.device)
        cd = self.codes
        m = min(int(cd["n_codes"].item()), cd["cap"])
        out = dict(n_codes=int(cd["n_codes"].item()), n_attached=int(cd["n_attached"].item()),
                   rs=cd["rs"][:m].cpu().numpy().view(np.uint16), ey=cd["ey"][:m].cpu().numpy(),
                   ez=cd["ez"][:m].cpu().numpy())
        if cd["ez_hi"] is not None:
            out["ez_hi"] = cd["ez_hi"][:m].cpu().numpy()
        return out

    run = tpc_run
    sync = tpc_sync

    def copy_probe(self, src, dst):
        """Streaming copy src -> dst (torch tensors of equal byte size, multiple of 16)."""
        nbytes = src.numel() * src.element_size()
        self._check(lib().tpc_copy_probe(self.ctx, _ptr(src), _ptr(dst), nbytes), "tpc_copy_probe")

    def profile(self, enable: bool = True):
        self._check(lib().tpc_profile(self.ctx, int(enable)), "tpc_profile")

    def profile_read(self, reset: bool = True) -> dict:
        ms = (C.c_double * len(PROF_NAMES))()
        n = (C.c_int32 * len(PROF_NAMES))()
        self._check(lib().tpc_profile_read(self.ctx, ms, n, len(PROF_NAMES), int(reset)), "tpc_profile_read")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(PROF_NAMES)}

    # ---- results
    def tracks(self) -> dict:
        """Final tracks as numpy arrays (synchronises; raises on a reported error)."""
        self.sync()
        return self.tracks_nosync()

    def tracks_nosync(self) -> dict:
        """Final tracks after waiting for the stream, without raising on a data error."""
        self.torch.cuda.synchronize(self.device)
        o = self.out
        K = int(o["n_tracks"].item())
        K = min(K, o["cap_tracks"])
        off = o["hit_off"][:K + 1].cpu().numpy()
        return dict(n=K, off=off, hits=o["hits"][:int(off[-1]) if K else 0].cpu().numpy(),
                    param=o["param"][:K].cpu().numpy(), cov=o["cov"][:K].cpu().numpy(),
                    x_ref=o["x_ref"][:K].cpu().numpy(), chi2=o["chi2"][:K].cpu().numpy(),
                    ndf=o["ndf"][:K].cpu().numpy(), sector=o["sector"][:K].cpu().numpy(),
                    job=o["job"][:K].cpu().numpy(), tracklet=o["tracklet"][:K].cpu().numpy(),
                    t0=o["t0"][:K].cpu().numpy())

    def links_raw(self) -> dict:
        """Raw (uncleaned) links as input indices; the clean links come from tpc_find_neighbours."""
        torch = self.torch
        n = self._keep.n
        dev = f"cuda:{self.device}"
        a = [torch.full((max(n, 1),), -1, dtype=torch.int32, device=dev) for _ in range(2)]
        self._check(lib().tpc_get_links_raw(self.ctx, _ptr(a[0]), _ptr(a[1])), "tpc_get_links_raw")
        self.torch.cuda.synchronize(self.device)
        return dict(up_raw=a[0][:n].cpu().numpy(), down_raw=a[1][:n].cpu().numpy())

    def debug_propagate(self, states: np.ndarray) -> np.ndarray:
        """rows [P5, C15, x1, x2] -> rows [ok, P5(hi), L5(lo), C15] through the device model."""
        torch = self.torch
        dev = f"cuda:{self.device}"
        a = torch.from_numpy(np.ascontiguousarray(states, np.float32)).to(dev)
        out = torch.zeros(a.shape[0], 26, dtype=torch.float32, device=dev)
        self._check(lib().tpc_debug_propagate(self.ctx, _ptr(a), _ptr(out), a.shape[0]), "debug")
        self.torch.cuda.synchronize(self.device)
        return out.cpu().numpy()

    def debug_update(self, rows: np.ndarray) -> np.ndarray:
        """rows [P5, L5, C15, my, mz] -> rows [ok, P5, L5, C15, chi2] through the device model."""
        torch = self.torch
        dev = f"cuda:{self.device}"
        a = torch.from_numpy(np.ascontiguousarray(rows, np.float32)).to(dev)
        out = torch.zeros(a.shape[0], 27, dtype=torch.float32, device=dev)
        self._check(lib().tpc_debug_update(self.ctx, _ptr(a), _ptr(out), a.shape[0]), "debug")
        self.torch.cuda.synchronize(self.device)
        return out.cpu().numpy()

    def rows(self):
        torch = self.torch
        dev = f"cuda:{self.device}"
        J = self._keep.n_jobs
        off = torch.zeros(J * N_SECTORS * N_ROWS + 1, dtype=torch.int32, device=dev)
        mem = torch.full((max(1, self._keep.n),), -1, dtype=torch.int32, device=dev)
        self._check(lib().tpc_get_rows(self.ctx, _ptr(off), _ptr(mem)), "tpc_get_rows")
        self.torch.cuda.synchronize(self.device)
        o = off.cpu().numpy()
        return o, mem.cpu().numpy()[:int(o[-1])]

    def tracklet_counts(self):
        T = C.c_int32()
        H = C.c_int64()
        self._check(lib().tpc_get_tracklet_counts(self.ctx, C.byref(T), C.byref(H)), "counts")
        return T.value, H.value

    def tracklets(self) -> dict:
        torch = self.torch
        dev = f"cuda:{self.device}"
        T = C.c_int32()
        H = C.c_int64()
        self._check(lib().tpc_get_tracklet_counts(self.ctx, C.byref(T), C.byref(H)), "counts")
        T, H = T.value, H.value
        start = torch.zeros(max(T, 1), dtype=torch.int32, device=dev)
        off = torch.zeros(T + 1, dtype=torch.int32, device=dev)
        hits = torch.zeros(max(H, 1), dtype=torch.int32, device=dev)
        state = torch.zeros(max(T, 1), 21, dtype=torch.float32, device=dev)
        w = torch.zeros(max(1, self._keep.n), dtype=torch.int64, device=dev)
        self._check(lib().tpc_get_tracklets(self.ctx, _ptr(start), _ptr(off), _ptr(hits), _ptr(state), _ptr(w)),
                    "tpc_get_tracklets")
        st = state[:T].cpu().numpy()
        return dict(start=start[:T].cpu().numpy(), off=off.cpu().numpy(), hits=hits[:H].cpu().numpy(),
                    P=st[:, :5], C=st[:, 5:20], x=st[:, 20], hitw=w.cpu().numpy().view(np.uint64))

    def selected(self) -> dict:
        torch = self.torch
        dev = f"cuda:{self.device}"
        K = C.c_int32()
        H = C.c_int64()
        self._check(lib().tpc_get_selected_counts(self.ctx, C.byref(K), C.byref(H)), "counts")
        K, H = K.value, H.value
        tr = torch.zeros(max(K, 1), dtype=torch.int32, device=dev)
        off = torch.zeros(K + 1, dtype=torch.int32, device=dev)
        hits = torch.zeros(max(H, 1), dtype=torch.int32, device=dev)
        self._check(lib().tpc_get_selected(self.ctx, _ptr(tr), _ptr(off), _ptr(hits)), "tpc_get_selected")
        return dict(tracklet=tr[:K].cpu().numpy(), off=off.cpu().numpy(), hits=hits[:H].cpu().numpy())
