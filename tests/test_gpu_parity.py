"""HIP path against the CPU oracle, stage by stage, through the C ABI (needs a gfx950 GPU).

Bit-exact: row membership, raw and clean links, tracklet starts/hits/states/hit weights,
selected tracks, final track hit lists, and the FP32 fitted parameters (the oracle's FP32
path uses the same operation order).  FP32 fit vs the FP64 oracle refit: 1e-4 relative on
q/pT (floor 0.1 GeV^-1) and 1e-3 cm on y, z.
"""
import numpy as np
import pytest

import oracle.oracle as O
import tpcsynth as g
from tests.gpu_helpers import bits, compare_all, gpu_run, oracle_run, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2402_01205_amd import tpc
    tpc.lib()  # fails loudly if the HIP library is missing


def test_device_math_bit_exact():
    """Propagation and Kalman update of the device model against the oracle's FP32 path."""
    import oracle.oracle as O
    from paper_2402_01205_amd.tpc import Tracker
    rng = np.random.default_rng(7)
    n = 4000
    P = np.stack([rng.uniform(-40, 40, n), rng.uniform(-300, 300, n), rng.uniform(-0.9, 0.9, n),
                  rng.uniform(-1.1, 1.1, n), rng.uniform(-10, 10, n)], 1).astype(np.float32)
    A = rng.normal(size=(n, 5, 5))
    Cf = np.einsum("nij,nkj->nik", A, A) * 0.05 + np.eye(5) * 0.01
    Ct = np.stack([O.full_to_tri(c) for c in Cf]).astype(np.float32)
    r1 = rng.integers(0, 152, n)
    r2 = np.clip(r1 + rng.integers(-30, 30, n), 0, 151)
    x1 = np.array([O.row_x(int(r)) for r in r1], np.float32)
    x2 = np.array([O.row_x(int(r)) for r in r2], np.float32)
    tr = Tracker(0)
    out = tr.debug_propagate(np.concatenate([P, Ct, x1[:, None], x2[:, None]], 1))
    n_ok = 0
    for i in range(n):
        ok, Pn, Cn = O.propagate(P[i], Ct[i], float(x1[i]), float(x2[i]))
        assert bool(out[i, 0]) == ok, i
        if ok:
            n_ok += 1
            assert np.array_equal(out[i, 1:11].view(np.uint32), Pn.view(np.uint32)), i
            assert np.array_equal(out[i, 11:].view(np.uint32), Cn.view(np.uint32)), i
    assert n_ok > n // 2
    L = (rng.normal(size=(n, 5)) * 1e-7).astype(np.float32)
    m = (P[:, :2] + rng.normal(size=(n, 2)) * 0.3).astype(np.float32)
    out = tr.debug_update(np.concatenate([P, L, Ct, m], 1))
    for i in range(n):
        ok, Pn, Cn, c2 = O.update(np.concatenate([P[i], L[i]]), Ct[i], float(m[i, 0]), float(m[i, 1]))
        assert bool(out[i, 0]) == ok
        if ok:
            assert np.array_equal(out[i, 1:11].view(np.uint32), Pn.view(np.uint32)), i
            assert np.array_equal(out[i, 11:26].view(np.uint32), Cn.view(np.uint32)), i
            assert np.float32(out[i, 26]) == np.float32(c2)


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_single_sector_event(seed):
    cs = g.make_config("c1", seed)
    say("c1 seed", seed, "n", cs.n)
    s = compare_all(gpu_run(cs), oracle_run(cs))
    assert s["n_tracks"] > 50


@pytest.mark.parametrize("seed,scale", [(21, 0.25), (22, 1.0)])
def test_full_tpc_event(seed, scale):
    cs = g.make_config("c2", seed, scale=scale)
    say("c2 seed", seed, "scale", scale, "n", cs.n)
    o = oracle_run(cs)
    s = compare_all(gpu_run(cs), o)
    assert s["merged"] > 100
    if scale == 1.0:
        # one job of more tracklets than the ownership count keeps in LDS: the per-cluster
        # atomic path; the smaller event takes the LDS path
        assert len(o["trk"]["start"]) > 65536


def test_timeframe_slice():
    cs = g.make_config("c3", 31, scale=0.06)
    say("c3 slice n", cs.n)
    compare_all(gpu_run(cs), oracle_run(cs))


def test_batched_uneven_jobs():
    sizes = g.c4_job_sizes(41)
    jobs = sorted(set(list(range(0, 512, 64)) + [int(np.argmax(sizes)), int(np.argmin(sizes))]))
    cs = g.make_config("c4", 41, jobs=jobs)
    say("c4 jobs", jobs, "n", cs.n)
    compare_all(gpu_run(cs), oracle_run(cs))


def test_sector_jobs_of_one_event_merge_across_jobs():
    """An event split into per-sector jobs with a shared event id tracks and merges exactly
    like the oracle given the same grouping."""
    cs = g.make_config("c2", 23, scale=0.2)
    order = np.argsort(cs.sector, kind="stable")
    cuts = np.searchsorted(cs.sector[order], np.arange(37)).astype(np.int32)
    split = g.ClusterSet(cs.sector[order], cs.row[order], cs.y[order], cs.z[order], cs.time[order],
                         cs.label[order], cuts, cs.part_pt, cs.part_eta, cs.part_phi, cs.part_q,
                         np.array([0, len(cs.part_pt)]), {})
    ev = np.zeros(36, np.int32)
    s = compare_all(gpu_run(split, job_event=ev), oracle_run(split, job_event=ev))
    assert s["merged"] > 50


@pytest.mark.parametrize("cfg,seed,scale", [("c2", 21, 0.5), ("c3", 31, 0.1)])
def test_sync_preset_bit_exact(cfg, seed, scale):
    """The synchronous phase's cut set (no merge across sector edges): every stage equals the
    oracle's with the same reading, and no track is merged."""
    from paper_2402_01205_amd.tpc import preset_params
    cs = g.make_config(cfg, seed, scale=scale)
    o = oracle_run(cs, O.params(**O.SYNC))
    s = compare_all(gpu_run(cs, params=preset_params("sync")), o)
    assert s["merged"] == 0 and s["n_tracks"] > 500
    say(cfg, "sync preset: tracks", s["n_tracks"])


@pytest.mark.parametrize("mode,tune", [
    ("plain", {}), ("batched", dict(tracklet_order=0)),
    ("persistent", dict(persistent_refill=1, tracklet_order=0)),
    ("persistent", dict(persistent_refill=0, tracklet_order=0)),
    ("persistent", dict(persistent_refill=1, tracklet_order=1)),
    ("persistent", dict(persistent_refill=0, tracklet_order=0, persistent_waves=32))])
def test_launch_modes_identical(mode, tune):
    """Every launch mode and tuning choice gives the default batched form's result."""
    from paper_2402_01205_amd.tpc import default_tuning
    sizes = g.c4_job_sizes(41)
    cs = g.make_config("c4", 41, jobs=[3, 100, 200, int(np.argmax(sizes))])
    a = gpu_run(cs, mode="batched")
    b = gpu_run(cs, mode=mode, tuning=default_tuning(**tune))
    for k in ("up", "down"):
        assert np.array_equal(a[k], b[k])
    for k in ("off", "hits", "tracklet", "ndf"):
        assert np.array_equal(a["tracks"][k], b["tracks"][k])
    assert np.array_equal(a["tracks"]["param"].view(np.uint32), b["tracks"]["param"].view(np.uint32))


@pytest.mark.parametrize("cpc", [0.125, 1.0, 3.0, 8.0])
def test_grid_cell_size_invariance(cpc):
    from paper_2402_01205_amd.tpc import default_tuning
    cs = g.make_config("c2", 21, scale=0.2)
    a = gpu_run(cs)
    b = gpu_run(cs, tuning=default_tuning(cells_per_cluster=cpc))
    assert np.array_equal(a["raw"]["up_raw"], b["raw"]["up_raw"])
    for k in ("off", "hits", "tracklet"):
        assert np.array_equal(a["tracks"][k], b["tracks"][k])


def test_repeatable():
    cs = g.make_config("c2", 22, scale=0.2)
    a = gpu_run(cs)
    b = gpu_run(cs)
    assert np.array_equal(a["trk"]["hitw"], b["trk"]["hitw"])
    assert np.array_equal(a["tracks"]["hits"], b["tracks"]["hits"])


def test_invalid_clusters_reported_and_excluded():
    from paper_2402_01205_amd.tpc import TPC_E_RANGE
    cs = g.make_config("c1", 11)
    cs.row = cs.row.copy(); cs.sector = cs.sector.copy(); cs.y = cs.y.copy()
    cs.row[5] = 200
    cs.sector[6] = 40
    cs.y[7] = np.nan
    gres = gpu_run(cs)
    assert gres["status"] == TPC_E_RANGE
    compare_all(gres, oracle_run(cs))


def test_empty_and_tiny_inputs():
    cs = g.make_config("c1", 11)
    empty = cs.job(0)
    idx = np.arange(0)
    tiny = g.ClusterSet(cs.sector[:2], cs.row[:2], cs.y[:2], cs.z[:2], cs.time[:2], cs.label[:2],
                        np.array([0, 2], np.int32), cs.part_pt, cs.part_eta, cs.part_phi, cs.part_q,
                        np.array([0, len(cs.part_pt)]), {})
    r = gpu_run(tiny)
    assert r["tracks"]["n"] == 0
    nothing = g.ClusterSet(cs.sector[idx], cs.row[idx], cs.y[idx], cs.z[idx], cs.time[idx],
                           cs.label[idx], np.array([0, 0], np.int32), cs.part_pt, cs.part_eta,
                           cs.part_phi, cs.part_q, np.array([0, len(cs.part_pt)]), {})
    r = gpu_run(nothing, stages=False)
    assert r["tracks"]["n"] == 0
    # an empty job between two real ones
    both = g.concat([cs, nothing, cs])
    compare_all(gpu_run(both), oracle_run(both))


def test_dense_rows_beyond_the_per_slot_counter_range():
    """Rows far denser than any workload's: 70,000 noise clusters in one row (past the 16-bit
    cell counters of the per-slot cell sort) and 12,000 in another (more cells than one LDS
    range at the default cell size), on top of a single-sector event; same results as the
    oracle."""
    cs = g.make_config("c1", 11)
    rng = np.random.default_rng(5)
    rows = np.concatenate([np.full(70000, 60), np.full(12000, 100)]).astype(np.int16)
    m = len(rows)
    y = (rng.uniform(-1.0, 1.0, m) * g.ROW_X[rows] * g.TAN_HALF).astype(np.float32)
    z = rng.uniform(0.0, g.DRIFT_LENGTH, m).astype(np.float32)
    cat = lambda a, b: np.concatenate([a, b.astype(a.dtype)])
    dense = g.ClusterSet(cat(cs.sector, np.zeros(m)), cat(cs.row, rows), cat(cs.y, y), cat(cs.z, z),
                         cat(cs.time, (g.DRIFT_LENGTH - z) / g.V_DRIFT), cat(cs.label, np.full(m, -1)),
                         np.array([0, cs.n + m], np.int32), cs.part_pt, cs.part_eta, cs.part_phi, cs.part_q,
                         np.array([0, len(cs.part_pt)]), {})
    say("dense rows n", dense.n)
    compare_all(gpu_run(dense), oracle_run(dense))


def test_graph_replays_match_eager():
    """The captured stage chain, replayed several times with eager work and synchronisations
    in between, reproduces the eager result every time."""
    import torch

    from paper_2402_01205_amd.tpc import DeviceClusters, Tracker, default_tuning
    sizes = g.c4_job_sizes(41)
    cs = g.make_config("c4", 41, jobs=[7, 77, int(np.argmax(sizes))])
    ev = DeviceClusters.from_set(cs, "cuda:0")
    eager = Tracker(0, mode="batched", tuning=default_tuning(use_graph=0))
    eager.run(ev)
    ref = eager.tracks()
    for mode in ("batched", "persistent"):
        gr = Tracker(0, mode=mode, tuning=default_tuning(use_graph=1))
        for rep in range(4):
            gr.run(ev)
            got = gr.tracks()
            assert got["n"] == ref["n"], (mode, rep)
            assert np.array_equal(got["hits"], ref["hits"]), (mode, rep)
            assert np.array_equal(got["param"].view(np.uint32), ref["param"].view(np.uint32)), (mode, rep)
            x = torch.randn(1 << 20, device="cuda:0")
            (x * 2).sum().item()   # eager work between replays
            torch.cuda.synchronize()
        assert gr.ctx.value


def test_autotune_candidates_are_bit_identical():
    from paper_2402_01205_amd.autotune import tune
    from paper_2402_01205_amd.tpc import DeviceClusters
    cs = g.make_config("c2", 21, scale=0.1)
    best, rep = tune(DeviceClusters.from_set(cs, "cuda:0"), 0, reps=1)
    assert rep["verified"] and len(rep["trials"]) >= 8


@pytest.mark.parametrize("preset", [None, "sync"])
def test_serving_chunk_alone_equals_chunk_in_mix(preset):
    """Each chunk's full result from the concurrent Server (three slots busy at once,
    batches of up to two chunks, results copied back from overlapping streams) equals
    the same chunk tracked alone, bit for bit: hit lists, parameters, covariance,
    x_ref, chi2, ndf and sector; with the default reading and with the synchronous cut
    set (whose downward extension claims clusters within each chunk's job only)."""
    import torch

    from paper_2402_01205_amd.serve import Pool, Server, assemble, make_stream
    from paper_2402_01205_amd.tpc import Tracker, preset_params
    prm = preset_params(preset) if preset else None
    cols = g.gen_collision_pool(61, 8, mult_range=(100, 400))
    pool = Pool.from_collisions(cols)
    got = {}

    def keep(cid, res):
        got[cid] = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in res.items()}

    srv = Server(pool, 0, n_slots=3, max_batch=2, params=prm)
    chunks = make_stream(8, 14, rate_hz=1e5, coll_range=(2, 6), seed=63)
    res = srv.run(chunks, realtime=True, on_result=keep)
    say("server", {k: v for k, v in res.items() if k not in ("tracks", "latencies")})
    assert res["n_chunks"] == 14 and res["p99_ms"] >= res["p50_ms"] > 0 and res["errors"] == 0
    assert res["max_concurrent"] == 3 and res["batches"] < 14      # overlap and shared batches
    assert sorted(got) == list(range(14))
    s = torch.cuda.current_stream()
    tr = Tracker(0, params=prm, mode="batched")
    n_cmp = 0
    for ch in chunks:
        ev = assemble(pool, [ch], s)
        tr.run(ev)
        t = tr.tracks()
        m = got[ch.cid]
        assert m["status"] == 0 and m["n_tracks"] == t["n"], ch.cid
        assert np.array_equal(m["hit_off"], t["off"]), ch.cid
        assert np.array_equal(m["hits"], t["hits"]), ch.cid
        for k, tk in (("param", "param"), ("cov", "cov"), ("x_ref", "x_ref"), ("chi2", "chi2"), ("t0", "t0")):
            assert np.array_equal(m[k].view(np.uint32), t[tk].view(np.uint32)), (ch.cid, k)
        for k in ("ndf", "sector"):
            assert np.array_equal(m[k], t[k]), (ch.cid, k)
        n_cmp += t["n"]
    say("tracks compared", n_cmp)
    assert n_cmp > 100


def test_output_capacity_reports_required_sizes_and_truncates():
    """Outputs smaller than needed: TPC_E_CAPACITY, n_tracks = the required count, the
    tracks and hits that fit equal the full result's, nothing beyond the capacities is
    written (guard values survive)."""
    import ctypes as C

    import torch

    from paper_2402_01205_amd import tpc as T
    cs = g.make_config("c1", 12)
    full = gpu_run(cs, stages=False)["tracks"]
    K, H = full["n"], int(full["off"][-1])
    assert K > 40
    for cap_t, cap_h in ((40, H + 10), (K + 5, 1000)):
        tr = T.Tracker(0)
        ev = T.DeviceClusters.from_set(cs, "cuda:0")
        tr.tpc_grid_build(ev)
        tr.tpc_find_neighbours()
        tr.tpc_construct_tracklets()
        tr.tpc_select_tracks()
        dev = "cuda:0"
        guard = 7
        o = dict(n_tracks=torch.zeros(1, dtype=torch.int32, device=dev),
                 hit_off=torch.full((cap_t + 1 + guard,), -7, dtype=torch.int32, device=dev),
                 hits=torch.full((cap_h + guard,), -7, dtype=torch.int32, device=dev),
                 param=torch.full((cap_t + guard, 5), -7.0, device=dev),
                 cov=torch.full((cap_t + guard, 15), -7.0, device=dev),
                 x_ref=torch.full((cap_t + guard,), -7.0, device=dev),
                 chi2=torch.full((cap_t + guard,), -7.0, device=dev),
                 ndf=torch.full((cap_t + guard,), -7, dtype=torch.int32, device=dev),
                 sector=torch.full((cap_t + guard,), -7, dtype=torch.int32, device=dev),
                 job=torch.full((cap_t + guard,), -7, dtype=torch.int32, device=dev),
                 tracklet=torch.full((cap_t + guard,), -7, dtype=torch.int32, device=dev),
                 t0=torch.full((cap_t + guard,), -7.0, device=dev))
        out = T.tpc_tracks(cap_t, cap_h, *[C.c_void_p(o[k].data_ptr()) for k in (
            "n_tracks", "hit_off", "hits", "param", "cov", "x_ref", "chi2", "ndf", "sector", "job", "tracklet",
            "t0")])
        assert T.lib().tpc_fit_merge(tr.ctx, C.byref(out)) == T.TPC_OK
        assert T.lib().tpc_sync(tr.ctx) == T.TPC_E_CAPACITY
        torch.cuda.synchronize()
        assert int(o["n_tracks"].item()) == K
        kt = min(K, cap_t)
        assert np.array_equal(o["param"][:kt].cpu().numpy().view(np.uint32), full["param"][:kt].view(np.uint32))
        assert np.array_equal(o["hit_off"][:kt].cpu().numpy(), full["off"][:kt])
        if K <= cap_t:
            assert int(o["hit_off"][K].item()) == H
        hits = o["hits"].cpu().numpy()
        nh = min(cap_h, int(full["off"][kt]))
        assert np.array_equal(hits[:nh], full["hits"][:nh])
        for k in ("param", "cov", "x_ref", "chi2", "ndf", "sector", "job", "tracklet", "t0"):
            assert bool((o[k][cap_t:] == -7).all()), k
        assert bool((o["hit_off"][cap_t + 1:] == -7).all())
        assert (hits[cap_h:] == -7).all()


def test_tracklet_capacity_overflow_is_reported_without_faults():
    """More chain starts than the workspace holds (capT = N/8 + 1024): straight
    five-cluster tracks, well apart, give one start per five clusters.  The library
    reports TPC_E_CAPACITY, drops the tracklets beyond its capacity and stays within
    bounds."""
    from paper_2402_01205_amd.tpc import TPC_E_CAPACITY, default_tuning
    x = 85 + np.arange(152) * 160 / 151
    sec, row, y, z = [], [], [], []
    for t, r0 in enumerate(range(0, 147, 6)):          # five rows, then one empty row
        zs = np.arange(4.0, 246.0, 8.0) + (4.0 if t % 2 else 0.0)
        half = x[r0] * np.tan(np.radians(10)) - 0.5
        y0 = np.arange(-half, half, 4.0)
        for k in range(5):
            r = r0 + k
            Y, Z = np.meshgrid(y0 * (x[r] / x[r0]), zs)   # radial lines: y proportional to x
            sec.append(np.zeros(Y.size, np.uint8)); row.append(np.full(Y.size, r, np.int16))
            y.append(Y.ravel().astype(np.float32)); z.append(Z.ravel().astype(np.float32))
    n = sum(len(a) for a in y)
    assert n // 5 > n // 8 + 1024
    cs = g.ClusterSet(np.concatenate(sec), np.concatenate(row), np.concatenate(y), np.concatenate(z),
                      np.zeros(n, np.float32), np.full(n, -1, np.int32), np.array([0, n], np.int32),
                      np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32),
                      np.zeros(0, np.int8), np.array([0, 0]), {})
    o = oracle_run(cs)
    ot = o["trk"]
    # five-hit tracklets are below the ten hits of a track: no tracks
    assert len(o["tracks"]["tracklet"]) == 0
    for mode, tune in (("batched", None), ("persistent", dict(tracklet_order=0)),
                       ("persistent", dict(persistent_refill=1))):
        say("mode", mode, tune)
        r = gpu_run(cs, mode=mode, tuning=tune and default_tuning(**tune))
        assert r["status"] == TPC_E_CAPACITY
        assert np.array_equal(r["up"], o["links"]["up"]) and np.array_equal(r["down"], o["links"]["down"])
        gt = r["trk"]
        T = len(gt["start"])
        assert T == n // 8 + 1024 < len(ot["start"])        # the oracle has no such capacity
        # the tracklets kept are the first ones in start order, and equal the oracle's
        assert np.array_equal(gt["start"], ot["start"][:T])
        assert np.array_equal(gt["off"], ot["off"][:T + 1])
        assert np.array_equal(gt["hits"], ot["hits"][:gt["off"][-1]])
        assert np.array_equal(bits(gt["P"]), bits(ot["P"][:T]))
        assert r["tracks"]["n"] == 0
