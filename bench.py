#!/usr/bin/env python3
"""Benchmark: TPC clusters tracked per second on one MI355X, batched vs plain.

One step = the whole tracking path (grid build, neighbour links, tracklets,
selection, fit and sector merge) over the workload's clusters, already resident
in HBM.  The default workload is the batched form: 512 single-sector jobs of
100..20000 primaries (log-uniform), ~89M clusters, tracked by one chain of
persistent launches captured in a hipGraph; the same data is also run through
the plain path (one launch sequence per sector-job) for comparison.  After the
tracking, the track-model compression of the same clusters against the tracks
found (and its decoding) is timed on its own; it is not part of the step.

Prints one JSON line (see the keys below).  Only --gpus 1 is supported.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "TPC clusters tracked/sec at 1 MI355X (batched vs plain); p50/p99 chunk latency"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "c1": "single TPC sector, 1 event: 200 primaries, no noise",
    "c2": "full TPC, 1 central Pb-Pb-like event: 36 sectors, 8000 primaries, 5% noise, 10% inefficiency",
    "c3": "time-frame slice: 50 collisions at 50 kHz, 500-8000 primaries each, drift-shifted z",
    "c4": "batched form: 512 single-sector jobs, 100-20000 primaries each (log-uniform)",
}
SEEDS = {"c1": 11, "c2": 21, "c3": 31, "c4": 41}
# Algorithmic bytes (unique bytes each kernel must move), as the method's plan prices them:
#  neighbour kernel: per cluster y, z (8) + cell offsets (2) + raw up/down links written (8)
#                    = 18 B
#  tracklet kernel : per tracklet hit: next link (4) + y, z (8) + hit written (4) + hit-weight
#                    read-modify-write (16) = 32 B; per tracklet: state written = 80 B
LINK_BYTES_PER_CLUSTER = 18
TRK_BYTES_PER_HIT = 32
TRK_BYTES_PER_TRACKLET = 80
#  compression     : per cluster: sector, row, y, z read (11) + record written (6); per track
#                    hit: its cluster index (4); per track: hit offset, state, x_ref, sector,
#                    ndf (36)
#  decompression   : per cluster: record read (6) + sector, row, y, z written (11); per track 36
CMP_BYTES_PER_CLUSTER = 17
CMP_BYTES_PER_HIT = 4
CMP_BYTES_PER_TRACK = 36
Q_STEP = 1.0 / 32.0
#  rANS encode     : per symbol 2 B read; per coded word 2 B written; per lane 4 B (offset)
#  rANS decode     : per coded word 2 B read; per symbol 2 B written; per lane 8 B (offsets)
#  cluster finding : per digit 9 B read (sector, row, pad, time, adc); per cluster 35 B written
CF_BYTES_PER_DIGIT = 9
CF_BYTES_PER_CLUSTER = 35


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("paper_2402_01205_amd/csrc/tpc.hip", "paper_2402_01205_amd/csrc/tpc_math.h",
                  "paper_2402_01205_amd/csrc/tpc_kernels.h")


def source_digest() -> str:
    """sha256 over the kernel sources: a traffic record holds only for the code it was taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_record(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the rocprofv3 counter summaries under profiles/
    (a line `<!-- traffic-record {json} -->`), or None when there is none for the current
    kernel sources."""
    import glob
    import re
    digest = source_digest()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for m in re.finditer(r"<!-- traffic-record (\{.*?\}) -->", open(f).read()):
            rec = json.loads(m.group(1))
            if rec.get("kernel") == kernel and rec.get("workload") == workload and rec.get("sources") == digest:
                rec["file"] = os.path.relpath(f, ROOT)
                return rec
    return None


def host_cpu() -> dict:
    """The host the oracle runs on: logical CPUs, the CPUs this process may use, model, clock."""
    info = {"nproc": os.cpu_count(), "cpus_available": len(os.sched_getaffinity(0))}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k = k.strip()
                if k == "model name" and "model" not in info:
                    info["model"] = v.strip()
                elif k == "cpu MHz" and "mhz" not in info:
                    info["mhz"] = float(v)
    except OSError:
        pass
    return info


def c4_sample_jobs(cs):
    """Every 16th job plus the largest one."""
    jobs = list(range(0, cs.n_jobs, 16))
    big = int(np.argmax(np.diff(cs.job_off)))
    return sorted(set(jobs) | {big})


def _oracle_job(sub):
    """One job of a sample through the oracle (in a worker process): (tracks, seconds)."""
    import oracle.oracle as O
    t0 = time.perf_counter()
    r = O.Run.from_set(sub)
    return len(r.tracks()["tracklet"]), time.perf_counter() - t0


def cpu_parallel(subs, workers, desc):
    """The oracle over independent jobs, one job per worker process.  Run before any GPU use,
    so the pool may fork."""
    import multiprocessing as mp
    n = sum(s.n for s in subs)
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_job, sorted(subs, key=lambda s: -s.n), chunksize=1)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "clusters/s", "cores": workers, "kind": "oracle",
            "sample": f"{desc} ({n} clusters), one job per process; {sum(r[0] for r in res)} tracks; "
                      f"{dt:.1f} s wall, {sum(r[1] for r in res):.1f} s summed over the processes"}


def cpu_single(cs, desc):
    """The oracle (single thread, as it stands) on one cluster set: rate, FP64 refit share."""
    import oracle.oracle as O
    t0 = time.perf_counter()
    r = O.Run.from_set(cs)
    dt = time.perf_counter() - t0
    ntr = len(r.tracks()["tracklet"])
    f64 = r.fp64_seconds
    return r, {"value": cs.n / dt, "unit": "clusters/s", "cores": 1, "kind": "oracle", "seconds": dt,
               "fp64_refit_seconds": f64, "without_fp64_refit": cs.n / max(dt - f64, 1e-9),
               "sample": f"{desc} ({cs.n} clusters); {ntr} tracks; {dt:.1f} s single-threaded, "
                         f"of which {f64:.2f} s FP64 refit"}


def cpu_baseline(cs, others, workers):
    """The oracle on the host: the headline workload's sample on one core (every 16th job plus
    the largest, with the rate extrapolated to all jobs by cluster count), the smaller
    workloads in full on one core, and the same samples over `workers` processes."""
    import tpcsynth as g
    host = host_cpu()
    if cs.n_jobs > 1:
        jobs = c4_sample_jobs(cs)
        sample = cs.subset_jobs(jobs)
        desc = f"jobs 0..{cs.n_jobs - 1} step 16 plus the largest ({len(jobs)} of {cs.n_jobs} sector-jobs)"
    else:
        jobs, sample, desc = [0], cs, "whole workload"
    r, out = cpu_single(sample, desc)
    out["host"] = host
    if cs.n_jobs > 1:
        out["extrapolated"] = True
        out["extrapolation"] = ("cluster-weighted: the sample's clusters/s applied to all "
                                f"{cs.n} clusters ({cs.n / out['value']:.0f} s estimated for the whole workload)")
    full = {}
    for name, ocs in [("c1", g.make_config("c1", 11))] + [(k, v) for k, v in others.items() if k == "c2"]:
        _, full[name] = cpu_single(ocs, f"{name} in full")
        log(f"cpu baseline {name} (1 core): {full[name]['value']:.3e} clusters/s")
    out["full_runs"] = full
    par = {}
    if cs.n_jobs > 1:
        par[cs.meta.get("workload", "main")] = cpu_parallel([cs.job(j) for j in jobs], workers, "the same sample")
    if "c3" in others:
        split, _, _ = g.split_by_sector(others["c3"])
        par["c3"] = cpu_parallel([split.job(j) for j in range(split.n_jobs)], workers,
                                 "c3 in full as 36 sector jobs (no merge across sectors in this leg)")
    for k, v in par.items():
        v["host"] = host
        v["note"] = f"{workers} worker processes: this GPU's share of the host's CPUs"
        log(f"cpu baseline {k} ({workers} processes): {v['value']:.3e} clusters/s")
    return r, sample, out, par


def cpu_chain_baseline(r, sample):
    """The compression and rANS oracles on the sample, against its own oracle tracks."""
    import oracle.oracle as O
    t = r.tracks()
    t0 = time.perf_counter()
    c = O.compress(sample.sector, sample.row, sample.y, sample.z, t, Q_STEP, Q_STEP)
    dc = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.decompress(t, c, Q_STEP, Q_STEP)
    dd = time.perf_counter() - t0
    H = c["n_attached"]
    streams = [np.ascontiguousarray(c[k][a:b]).view(np.uint16) for k in ("rs", "ey", "ez")
               for a, b in ((0, H), (H, len(c["rs"])))]
    t0 = time.perf_counter()
    encs = [O.rans_encode(v) for v in streams]
    de = time.perf_counter() - t0
    t0 = time.perf_counter()
    for v, e in zip(streams, encs):
        O.rans_decode(e, len(v))
    dr = time.perf_counter() - t0
    nsym = sum(len(v) for v in streams)
    comp = {"value": sample.n / dc, "unit": "clusters/s", "cores": 1, "kind": "oracle",
            "decompress_clusters_per_s": sample.n / dd,
            "sample": f"the same sample and its oracle tracks; {dc:.2f} s encode, {dd:.2f} s decode"}
    rans = {"value": nsym / de, "unit": "symbols/s", "cores": 1, "kind": "oracle",
            "decode_symbols_per_s": nsym / dr,
            "sample": f"the six record streams of that sample ({nsym} symbols); {de:.2f} s encode, "
                      f"{dr:.2f} s decode"}
    return comp, rans


def copy_probe(tr, torch, mib, reps):
    """Achieved GB/s of the library's streaming copy kernel (read + write bytes)."""
    n = (mib << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    tr.copy_probe(a, b)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        tr.copy_probe(a, b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return 2.0 * a.numel() * 4 / ms / 1e6


def serve_pool(args, log):
    """The serving workload's collision pool (host), generated before any GPU use."""
    import tpcsynth as g
    t0 = time.perf_counter()
    cols = g.gen_collision_pool(51, args.serve_pool, workers=args.workers)
    log(f"serving pool of {args.serve_pool} collisions generated in {time.perf_counter() - t0:.1f}s")
    return cols


def serve_run(args, cols, tuning, log):
    """Continuous-batching serving of time-frame chunks (Poisson arrivals) at the stated rate;
    when that rate saturates the GPU, a second run at 0.8x the measured capacity."""
    from paper_2402_01205_amd.serve import Pool, Server, make_stream, plan_chunk, n_noise
    pool = Pool.from_collisions(cols)
    srv = Server(pool, 0, tuning=default_tuning_from(tuning))

    def one(n_chunks, rate, seed):
        chunks = make_stream(args.serve_pool, n_chunks, rate_hz=rate, seed=seed)
        res = srv.run(chunks, realtime=True, log=log)
        res.pop("tracks")
        res.pop("latencies")
        res["saturated"] = res["clusters_per_s"] < 0.95 * res["offered_clusters_per_s"]
        res.update(rate_hz=rate, arrival_seed=seed, pool_collisions=args.serve_pool, pool_seed=51)
        log("serving: " + json.dumps(res))
        return res

    res = one(args.serve_chunks, args.serve_rate, 52)
    if res["saturated"] and args.serve_context_chunks > 0:
        # the mean chunk size of the stream, for the rate that offers 0.8x the measured capacity
        probe = make_stream(args.serve_pool, args.serve_chunks, rate_hz=args.serve_rate, seed=52)
        mean_cl = np.mean([plan_chunk(pool, c).n_signal + n_noise(c) for c in probe])
        rate = 0.8 * res["clusters_per_s"] / mean_cl
        res["at_0.8x_capacity"] = one(args.serve_context_chunks, rate, 53)
    return res


def default_tuning_from(t):
    from paper_2402_01205_amd.tpc import default_tuning
    return default_tuning(**{k: getattr(t, k) for k, _ in t._fields_})


def _entropy_bits(v) -> float:
    """Order-0 entropy (bits per value) of an int16 stream."""
    if len(v) == 0:
        return 0.0
    c = np.bincount(v.astype(np.int64) + 32768, minlength=65536)
    p = c[c > 0] / len(v)
    return float(-(p * np.log2(p)).sum())


def compression_run(tr, cs, tracks, steps, log):
    """Track-model compression of the clusters against the tracks just found, and decoding:
    times (HIP events on the library's stream), roofline of the compression call, and the
    order-0 entropy of the record streams against all-absolute records at the same step."""
    tr.profile(True)
    tr.profile_read(reset=True)
    for _ in range(steps):
        tr.tpc_compress(Q_STEP, Q_STEP)
    for _ in range(steps):
        tr.tpc_decompress()
    prof = tr.profile_read(reset=True)
    tr.profile(False)
    tr.sync()
    c_ms = prof["compress"][0] / max(1, prof["compress"][1])
    d_ms = prof["decompress"][0] / max(1, prof["decompress"][1])
    rec = tr.codes_numpy()
    n, H, K = cs.n, rec["n_attached"], int(tracks["n"])
    c_bytes = CMP_BYTES_PER_CLUSTER * n + CMP_BYTES_PER_HIT * H + CMP_BYTES_PER_TRACK * K
    d_bytes = CMP_BYTES_PER_CLUSTER * n + CMP_BYTES_PER_TRACK * K
    rs, ey, ez = rec["rs"], rec["ey"], rec["ez"]
    res = (rs >> 15) == 0
    streams = [rs.view(np.int16), ey[res], ez[res], ey[~res], ez[~res]]
    bits = sum(_entropy_bits(v) * len(v) for v in streams) / max(n, 1)
    iq = np.float32(1.0) / np.float32(Q_STEP)
    ay = np.clip(np.rint(cs.y * iq), -32767, 32767).astype(np.int16)
    az = np.clip(np.rint(cs.z * iq), -32767, 32767).astype(np.int16)
    ars = (cs.row.astype(np.uint16) | (cs.sector.astype(np.uint16) << 8) | np.uint16(1 << 15)).view(np.int16)
    bits_abs = _entropy_bits(ars) + _entropy_bits(ay) + _entropy_bits(az)
    gbs = c_bytes / c_ms / 1e6
    out = {"q_cm": Q_STEP, "ms": c_ms, "clusters_per_s": n / (c_ms / 1e3), "decompress_ms": d_ms,
           "decompress_clusters_per_s": n / (d_ms / 1e3), "records": rec["n_codes"], "track_hit_records": H,
           "residual_records": int(res.sum()),
           "roofline": {"bound": "hbm", "kernel": "tpc_compress (all its kernels)", "achieved": gbs,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                        "algorithmic_bytes": c_bytes, "traffic": None},
           "decompress_GBs": d_bytes / d_ms / 1e6,
           "entropy_bits_per_cluster": bits, "entropy_bits_per_cluster_absolute": bits_abs,
           "entropy_ratio": bits_abs / bits if bits else None}
    out["rans"] = rans_run(tr, rec["n_attached"], n, steps)
    log("compression: " + json.dumps(out))
    return out


def sync_preset_run(ev, cs, tracks, tuning, args, timed, log, torch):
    """The synchronous phase's cut set on the same workload (no merge across sector edges,
    tracks extended below their innermost hits): step time, per-stage times, tracking quality,
    the share of clusters on tracks and what that does to the compression."""
    from paper_2402_01205_amd.evaluate import quality
    from paper_2402_01205_amd.tpc import Tracker, preset_params
    ts = Tracker(0, params=preset_params("sync"), mode=args.mode, tuning=tuning)
    ts.run(ev)
    ts.sync()
    sms = timed(ts, args.steps)
    ts.sync()
    st = ts.tracks()
    ts.profile(True)
    ts.profile_read(reset=True)
    for _ in range(args.steps):
        ts.run(ev)
    sprof = ts.profile_read(reset=True)
    ts.profile(False)
    sq = quality(cs.label, cs.job_off, cs.sector, st["off"], st["hits"], cs.part_off, cs.part_pt,
                 by_job=cs.n_jobs > 1)
    if "per_job" in sq:
        sq["by_job_size_decile"] = by_decile(sq.pop("per_job"), np.diff(cs.job_off))
    sc = compression_run(ts, cs, st, args.steps, lambda m: None)
    sig = cs.label >= 0

    def attached_signal(t):
        a = np.zeros(cs.n, bool)
        a[t["hits"]] = True
        return float(a[sig].mean())

    row = {"params": "TPC_PRESET_SYNC (merge_edge < 0, ext_down = 1)", "ms_per_step": sms,
           "clusters_per_s": cs.n / (sms / 1e3), "tracks": int(st["n"]),
           "stages_ms": {k: v[0] / max(1, v[1]) for k, v in sprof.items() if v[1]},
           "attached_clusters": int(st["off"][-1]) / cs.n,
           "async_attached_clusters": int(tracks["off"][-1]) / cs.n,
           "attached_signal_clusters": attached_signal(st),
           "async_attached_signal_clusters": attached_signal(tracks),
           "quality": sq,
           "compression": {k: sc[k] for k in ("ms", "track_hit_records", "residual_records",
                                             "entropy_bits_per_cluster")},
           "rans_coded_bits_per_cluster": sc["rans"]["coded_bits_per_cluster"]}
    log("sync preset: " + json.dumps({k: v for k, v in row.items() if k != "quality"}))
    del ts
    return row


def _majority(cs, t):
    """Majority particle, its share and the hit count of every output track."""
    off, hits = t["off"], t["hits"]
    nh = np.diff(off)
    tid = np.repeat(np.arange(len(nh)), nh)
    lab = cs.label[hits].astype(np.int64)
    ok = lab >= 0
    big = int(lab.max()) + 1 if lab.size else 1
    u, c = np.unique(tid[ok] * big + lab[ok], return_counts=True)
    trk, part = u // big, u % big
    order = np.lexsort((-c, trk))
    first = np.concatenate([[True], trk[order][1:] != trk[order][:-1]]) if len(order) else np.zeros(0, bool)
    maj = np.full(len(nh), -1, np.int64)
    cnt = np.zeros(len(nh), np.int64)
    maj[trk[order][first]] = part[order][first]
    cnt[trk[order][first]] = c[order][first]
    return maj, cnt, nh


def membrane_run(cs, args, tuning, time_run, log, dev):
    """The time-frame slice with its collision vertices spread in z: the default reading
    against the asynchronous cut set, which merges pieces across the central membrane; the
    collision times of the tracks joined across it against the generator's, beside the
    vertex-based times of the other good tracks (off by the vertex z over v_drift)."""
    from paper_2402_01205_amd.tpc import DeviceClusters, Tracker, preset_params
    ev = DeviceClusters.from_set(cs, dev)
    off_c = np.asarray(cs.meta["coll_part_off"], np.int64)
    coll = np.repeat(np.arange(len(off_c) - 1), np.diff(off_c))
    t_true = np.asarray(cs.meta["t_collisions"])[coll]
    out = {"workload": f"c3: {WORKLOADS['c3']}, vertices at z ~ N(0, {args.vz_sigma} cm)",
           "n_clusters": cs.n}
    for name, prm in (("default", None), ("async_preset", preset_params("async"))):
        tr = Tracker(0, params=prm, mode=args.mode, tuning=tuning)
        ms = time_run(tr, ev, args.steps)
        t = tr.tracks()
        maj, cnt, nh = _majority(cs, t)
        good = (maj >= 0) & (cnt >= 0.9 * nh) & (nh >= 30) & ~np.isnan(t["t0"])
        tid = np.repeat(np.arange(len(nh)), nh)
        side = (cs.sector[t["hits"]] < 18).astype(np.int64)
        both = np.zeros(len(nh), np.int64)
        np.bitwise_or.at(both, tid, 1 << side)
        across = both == 3
        row = {"ms_per_step": ms, "clusters_per_s": cs.n / (ms / 1e3), "tracks": int(t["n"]),
               "tracks_across_membrane": int(across.sum())}
        for key, m in (("across_membrane", good & across), ("vertex_based", good & ~across)):
            if m.any():
                d = np.abs(t["t0"][m] - t_true[maj[m]])
                row[f"t0_abs_err_us_{key}"] = {"tracks": int(m.sum()), "median": float(np.median(d)),
                                               "p95": float(np.percentile(d, 95))}
        out[name] = row
        del tr
    log("membrane merge: " + json.dumps(out))
    return out


def looper_run(cs, args, tuning, time_run, log, dev):
    """The full TPC event with the return legs of its loopers: step time, and how many of the
    return-leg clusters end on tracks (each return leg is tracked on its own, described
    against its momentum)."""
    from paper_2402_01205_amd.tpc import DeviceClusters, Tracker
    ev = DeviceClusters.from_set(cs, dev)
    tr = Tracker(0, mode=args.mode, tuning=tuning)
    ms = time_run(tr, ev, args.steps)
    t = tr.tracks()
    leg = cs.meta["leg"]
    att = np.zeros(cs.n, bool)
    att[t["hits"]] = True
    nh = np.diff(t["off"])
    tid = np.repeat(np.arange(len(nh)), nh)
    lg = leg[t["hits"]].astype(np.int64)
    n1 = np.bincount(tid, weights=(lg == 1), minlength=len(nh))
    n0 = np.bincount(tid, weights=(lg == 0), minlength=len(nh))
    # the pairing of the two legs: time per call (HIP events on the library's stream) and how
    # many pairs join both legs of one particle
    tr.profile(True)
    tr.profile_read(reset=True)
    for _ in range(max(args.steps, 1)):
        legs = tr.tpc_pair_legs()
    prof = tr.profile_read(reset=True)
    tr.profile(False)
    legs = legs[:t["n"]].cpu().numpy()
    maj = _majority(cs, t)[0]
    kind = np.where(n1 > n0, 1, 0)
    i = np.flatnonzero(legs > np.arange(len(legs)))
    j = legs[i]
    pairs = len(i)
    right = int(((maj[i] == maj[j]) & (maj[i] >= 0) & (kind[i] != kind[j])).sum())
    out = {"workload": f"c2: {WORKLOADS['c2']}, with the return legs of its loopers",
           "n_clusters": cs.n, "return_leg_clusters": int((leg == 1).sum()),
           "ms_per_step": ms, "clusters_per_s": cs.n / (ms / 1e3), "tracks": int(t["n"]),
           "return_leg_tracks": int(((n1 > 0) & (n0 == 0)).sum()),
           "tracks_mixing_legs": int(((n1 > 0) & (n0 > 0)).sum()),
           "attached_outgoing_leg_clusters": float(att[leg == 0].mean()),
           "attached_return_leg_clusters": float(att[leg == 1].mean()),
           "leg_pairs": pairs, "leg_pairs_of_one_particle": right,
           "pair_legs_ms": prof["pair_legs"][0] / max(prof["pair_legs"][1], 1)}
    log("return legs: " + json.dumps(out))
    del tr
    return out


def cf_cpu_baseline(dg):
    """The oracle's cluster finder on the digits of sectors 0-3 of the digit workload."""
    import oracle.oracle as O
    m = dg.sector < 4
    args = [dg.sector[m], dg.row[m], dg.pad[m], dg.time[m], dg.adc[m]]
    t0 = time.perf_counter()
    c = O.find_clusters(*args, n_time=dg.n_time)
    dt = time.perf_counter() - t0
    return {"value": int(m.sum()) / dt, "unit": "digits/s", "cores": 1, "kind": "oracle",
            "sample": f"sectors 0-3 of the digit workload ({int(m.sum())} digits, {len(c['y'])} clusters); "
                      f"{dt:.1f} s single-threaded"}


def cf_run(tr, dg, steps, torch):
    """Cluster finding on the digit workload: time per call (HIP events on the library's
    stream, on a workspace the previous call left clean), roofline."""
    from paper_2402_01205_amd.tpc import lib, tpc_cf_params
    import ctypes as C
    p = tpc_cf_params()
    lib().tpc_cf_params_default(C.byref(p))
    p.n_time = dg.n_time
    f = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dt)).to("cuda:0")
    dd = dict(sector=f(dg.sector, np.uint8), row=f(dg.row, np.int16), pad=f(dg.pad, np.int16),
              time=f(dg.time, np.int16), adc=f(dg.adc.view(np.int16), np.int16))
    out = tr.tpc_find_clusters(dd, p)           # warm-up: clears the map once
    torch.cuda.synchronize()
    tr.profile(True)
    tr.profile_read(reset=True)
    for _ in range(steps):
        out = tr.tpc_find_clusters(dd, p)
    prof = tr.profile_read(reset=True)
    tr.profile(False)
    res = tr.clusters_numpy(out)
    ms = prof["find_clusters"][0] / max(1, prof["find_clusters"][1])
    nb = CF_BYTES_PER_DIGIT * dg.n + CF_BYTES_PER_CLUSTER * res["n"]
    gbs = nb / ms / 1e6
    r = {"workload": dg.desc, "digits": dg.n, "clusters": res["n"], "status": res["status"], "ms": ms,
         "digits_per_s": dg.n / (ms / 1e3), "clusters_per_s": res["n"] / (ms / 1e3),
         "roofline": {"bound": "hbm", "kernel": "tpc_find_clusters (all its kernels)", "achieved": gbs,
                      "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes": nb}}
    log("cluster finding: " + json.dumps(r))
    return r


def record_streams(tr, H, n):
    """The six fields of the compression records as device streams: rs, ey, ez, each split
    into the track hits (residual codes) and the clusters in no track (absolute codes)."""
    cd = tr.codes
    return {f"{k}_{part}": cd[k][a:b].contiguous()
            for k in ("rs", "ey", "ez") for part, a, b in (("tracks", 0, H), ("free", H, n))}


def rans_run(tr, H, n, steps):
    """rANS coding of the compression records, field by field: time per pass over the six
    streams (HIP events on the library's stream), coded size and roofline."""
    streams = record_streams(tr, H, n)
    tr.profile(True)
    tr.profile_read(reset=True)
    encs = {}
    for _ in range(steps):
        for k, v in streams.items():
            encs[k] = tr.tpc_rans_encode(v)
    outs = {k: None for k in streams}
    for _ in range(steps):
        for k in streams:
            outs[k] = tr.tpc_rans_decode(encs[k], outs[k])
    prof = tr.profile_read(reset=True)
    tr.profile(False)
    tr.sync()
    e_ms = prof["rans_encode"][0] / steps
    d_ms = prof["rans_decode"][0] / steps
    per, words, lanes, model = {}, 0, 0, 0
    exact = True
    for k, v in streams.items():
        r = tr.rans_numpy(encs[k])
        nl = len(r["lane_off"]) - 1
        nz = int((r["freq"] > 0).sum())
        words += r["n_words"]
        lanes += nl
        model += nz
        exact &= bool(outs[k][:v.numel()].equal(v))
        per[k] = {"symbols": int(v.numel()), "words": r["n_words"], "symbols_in_model": nz,
                  "bits_per_symbol": 16.0 * r["n_words"] / max(1, v.numel())}
    sym = 3 * n
    coded_bytes = 2 * words + 4 * lanes + 4 * model   # words, lane offsets, sparse model
    e_bytes = 2 * sym + 2 * words + 4 * lanes
    d_bytes = 2 * sym + 2 * words + 8 * lanes
    return {"encode_ms": e_ms, "decode_ms": d_ms, "symbols": sym,
            "encode_symbols_per_s": sym / (e_ms / 1e3), "decode_symbols_per_s": sym / (d_ms / 1e3),
            "round_trip_exact": exact, "coded_bytes": coded_bytes,
            "coded_bits_per_cluster": 8.0 * coded_bytes / max(n, 1),
            "record_bits_per_cluster": 48.0, "ratio_vs_records": 48.0 * n / max(8.0 * coded_bytes, 1),
            "ratio_vs_float_clusters": 88.0 * n / max(8.0 * coded_bytes, 1),
            "roofline_encode": {"bound": "hbm", "achieved": e_bytes / e_ms / 1e6, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": e_bytes / e_ms / 1e6 / HBM_PEAK_GBS},
            "roofline_decode": {"bound": "hbm", "achieved": d_bytes / d_ms / 1e6, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": d_bytes / d_ms / 1e6 / HBM_PEAK_GBS},
            "streams": per}


def kernel_rows(prof, n, T, H):
    """Time, algorithmic bytes and GB/s of the two hot kernels from a profiled pass."""
    ms = lambda k: prof[k][0] / max(1, prof[k][1])
    lb = LINK_BYTES_PER_CLUSTER * n
    tb = TRK_BYTES_PER_HIT * H + TRK_BYTES_PER_TRACKLET * T
    return {"k_links": dict(ms=ms("k_links"), bytes=lb, gbs=lb / ms("k_links") / 1e6),
            "k_tracklets": dict(ms=ms("k_tracklets"), bytes=tb, gbs=tb / ms("k_tracklets") / 1e6,
                                tracklets=int(T), tracklet_hits=int(H))}


def kernel_json(kern):
    return {k: {"ms": v["ms"], "GB/s": v["gbs"], "frac": v["gbs"] / HBM_PEAK_GBS, "algorithmic_bytes": v["bytes"],
                **({"tracklets": v["tracklets"], "tracklet_hits": v["tracklet_hits"]} if "tracklets" in v else {})}
            for k, v in kern.items()}


def by_decile(pj, sizes):
    """Efficiency and fake rate over the jobs sorted by size (clusters), in ten groups."""
    order = np.argsort(sizes, kind="stable")
    out = []
    for grp in np.array_split(order, 10):
        f, fd = int(pj["findable"][grp].sum()), int(pj["found"][grp].sum())
        t, fk = int(pj["tracks"][grp].sum()), int(pj["fakes"][grp].sum())
        out.append({"jobs": len(grp), "clusters_per_job": [int(sizes[grp].min()), int(sizes[grp].max())],
                    "clusters": int(sizes[grp].sum()), "efficiency": fd / f if f else None,
                    "fake_rate": fk / t if t else None})
    return out


def same_tracks(a, b, perm=None):
    """Two track outputs hold the same tracks (as sets of hit lists); perm maps b's cluster
    indices to a's."""
    def lists(t, p):
        off, hits = t["off"], t["hits"] if p is None else p[t["hits"]]
        return sorted(tuple(hits[off[i]:off[i + 1]].tolist()) for i in range(int(t["n"])))
    return int(a["n"]) == int(b["n"]) and lists(a, None) == lists(b, perm)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--seed", type=int, default=None)
    ap.add_argument("--mode", default="persistent", choices=["batched", "persistent"])
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--profile-only", action="store_true",
                    help="run warmup+steps of the batched path only (for rocprofv3)")
    ap.add_argument("--probe-only", action="store_true",
                    help="run only the streaming-copy probe (counter calibration)")
    ap.add_argument("--probe-mib", type=int, default=2048)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--serve-chunks", type=int, default=2000, help="chunks of the serving run (0 = skip)")
    ap.add_argument("--serve-pool", type=int, default=512, help="collisions in the serving pool")
    ap.add_argument("--serve-rate", type=float, default=20.0)
    ap.add_argument("--serve-context-chunks", type=int, default=1000,
                    help="chunks of the run at 0.8x the measured capacity when the stated rate saturates")
    ap.add_argument("--cf-config", default="d3", choices=["d1", "d2", "d3", ""],
                    help="digit workload of the cluster-finding row ('' = skip)")
    ap.add_argument("--no-loopers", dest="loopers", action="store_false",
                    help="skip the full event with its loopers' return legs")
    ap.add_argument("--vz-sigma", type=float, default=5.0,
                    help="vertex z spread (cm) of the extra time frame for the membrane merge (0: skip)")
    ap.add_argument("--also", default="c2,c3",
                    help="other workloads timed in the same launch configuration (comma list, '' = none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "only one GPU is measured; run with --gpus 1"}))
        sys.exit(2)

    if args.probe_only:
        import torch
        from paper_2402_01205_amd.tpc import Tracker
        gbs = copy_probe(Tracker(0), torch, args.probe_mib, args.steps)
        print(json.dumps({"copy_probe_GBs": gbs, "bytes_per_launch": 2 * args.probe_mib << 20}), flush=True)
        return

    import tpcsynth as g
    seed = args.seed if args.seed is not None else SEEDS[args.config]
    t0 = time.perf_counter()
    cs = g.make_config(args.config, seed, workers=args.workers)  # before any GPU use
    log(f"generated {args.config} seed {seed}: {cs.n} clusters, {cs.n_jobs} jobs "
        f"in {time.perf_counter() - t0:.1f}s")
    others = {}
    vz_set = loop_set = None
    if not args.profile_only:
        for name in [x for x in args.also.split(",") if x and x != args.config]:
            others[name] = g.make_config(name, SEEDS[name], workers=args.workers)
            log(f"generated {name}: {others[name].n} clusters")
        if args.vz_sigma > 0:
            vz_set = g.make_config("c3", SEEDS["c3"], workers=args.workers, vz_sigma=args.vz_sigma)
            log(f"generated c3 with vertices spread in z ({args.vz_sigma} cm): {vz_set.n} clusters")
        loop_set = g.make_config("c2", SEEDS["c2"], loopers=True) if args.loopers else None
    # the oracle baselines first, before any GPU use
    cpu = cpu_par = cpu_chain = None
    if not args.no_cpu and not args.profile_only:
        r_cpu, sample, cpu, cpu_par = cpu_baseline(cs, others, args.workers)
        log(f"cpu baseline (1 core): {cpu['value']:.3e} clusters/s")
        cpu_chain = cpu_chain_baseline(r_cpu, sample)
        del r_cpu, sample
    dg = None
    if args.cf_config:
        from tpcsynth import digits as D
        t0 = time.perf_counter()
        _, dg, nt = D.digit_config(args.cf_config, 7)
        dg.n_time = nt
        dg.desc = {"d1": "one sector of one event", "d2": "one full-TPC event (8000 primaries)",
                   "d3": "8 full-TPC events at uniform times over two drift lengths (1000 time bins)"}[args.cf_config]
        log(f"digits {args.cf_config}: {dg.n} in {time.perf_counter() - t0:.1f}s")
    cf_cpu = cf_cpu_baseline(dg) if (dg is not None and not args.no_cpu and not args.profile_only) else None
    serve_cols = serve_pool(args, log) if (args.serve_chunks > 0 and not args.profile_only) else None

    import torch

    from paper_2402_01205_amd.evaluate import quality
    from paper_2402_01205_amd.tpc import DeviceClusters, Tracker, default_tuning
    dev = "cuda:0"
    ev = DeviceClusters.from_set(cs, dev)
    torch.cuda.synchronize()

    tune_report = None
    if args.no_autotune:
        tuning = default_tuning(use_graph=0 if args.no_graph else 1)
    else:
        from paper_2402_01205_amd.autotune import tune
        sample = cs.subset_jobs(range(0, cs.n_jobs, 8)) if cs.n_jobs >= 64 else cs
        t1 = time.perf_counter()
        tuning, tune_report = tune(DeviceClusters.from_set(sample, dev), 0, reps=2)
        tuning.use_graph = 0 if args.no_graph else 1
        log(f"autotune on {sample.n} clusters: {tune_report['best']} "
            f"({len(tune_report['trials'])} candidates, all bit-identical) in {time.perf_counter() - t1:.1f}s")
    args.mode = "persistent" if tuning.persistent_waves > 0 else "batched"
    tr = Tracker(0, mode=args.mode, tuning=tuning)

    def timed(tracker, steps):
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            tracker.run(ev)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    for i in range(args.warmup):
        tr.run(ev)
        log(f"warmup {i + 1}/{args.warmup}")
    tr.sync()
    ms = timed(tr, args.steps)
    tr.sync()
    log(f"batched ({args.mode}{'' if args.no_graph else ' + graph'}): {ms:.2f} ms/step")
    if args.profile_only and args.config == "c4":
        # the compression kernels in the same trace, after the tracking steps (the batched
        # workload's z fits the compression's absolute codes; a time frame's does not)
        for _ in range(args.steps):
            tr.tpc_compress(Q_STEP, Q_STEP)
        for _ in range(args.steps):
            tr.tpc_decompress()
        tr.sync()
        H = int(tr.codes["n_attached"].item())
        streams = record_streams(tr, H, cs.n)
        for _ in range(args.steps):
            encs = {k: tr.tpc_rans_encode(v) for k, v in streams.items()}
        for _ in range(args.steps):
            for e in encs.values():
                tr.tpc_rans_decode(e)
        tr.sync()
        log(f"compression: {args.steps} encode and {args.steps} decode calls, then rANS of its six streams")
    if args.profile_only:
        if dg is not None:
            cf_run(tr, dg, args.steps, torch)
        print(json.dumps({"ms_per_step": ms, "sources": source_digest(),
                          "tuning": {k: getattr(tuning, k) for k, _ in tuning._fields_}}), flush=True)
        return
    tracks = tr.tracks()

    # per-kernel times with HIP events on the tracker's stream (same launch configuration)
    tr.profile(True)
    tr.profile_read(reset=True)
    for _ in range(args.steps):
        tr.run(ev)
    prof = tr.profile_read(reset=True)
    tr.profile(False)
    T, H = tr.tracklet_counts()
    kern = kernel_rows(prof, cs.n, T, H)
    dom = max(kern, key=lambda k: kern[k]["ms"])
    trec = traffic_record(dom, args.config)
    traffic = None
    if trec and trec.get("read_bytes") is not None and trec.get("write_bytes") is not None:
        traffic = trec["read_bytes"] + trec["write_bytes"]
    log("stage ms/step: " + ", ".join(f"{k} {v[0] / max(1, v[1]):.3f}" for k, v in prof.items() if v[1]))
    log("kernels: " + json.dumps(kern))
    compression = compression_run(tr, cs, tracks, args.steps, log)
    sync_row = sync_preset_run(ev, cs, tracks, tuning, args, timed, log, torch)
    clusters_row = cf_run(tr, dg, args.steps, torch) if dg is not None else None
    if clusters_row is not None:
        clusters_row["cpu_baseline"] = cf_cpu

    # plain path on the same data
    plain_ms = None
    if args.plain_steps > 0:
        tp = Tracker(0, mode="plain")
        tp.run(ev)
        tp.sync()
        plain_ms = timed(tp, args.plain_steps)
        tp.sync()
        pt = tp.tracks()
        same = (pt["n"] == tracks["n"] and np.array_equal(pt["hits"], tracks["hits"]))
        log(f"plain: {plain_ms:.2f} ms/step; identical to batched: {same}")
        del tp

    probe = copy_probe(tr, torch, 1024, 5)
    log(f"copy probe: {probe:.0f} GB/s")
    q = quality(cs.label, cs.job_off, cs.sector, tracks["off"], tracks["hits"], cs.part_off, cs.part_pt,
                by_job=cs.n_jobs > 1)
    if "per_job" in q:
        q["by_job_size_decile"] = by_decile(q.pop("per_job"), np.diff(cs.job_off))
    log("quality: " + json.dumps(q))
    also = {}
    def time_run(tracker, dev_set, steps):
        tracker.run(dev_set)
        tracker.sync()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            tracker.run(dev_set)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    for name, ocs in others.items():
        oev = DeviceClusters.from_set(ocs, dev)
        otr = Tracker(0, mode=args.mode, tuning=tuning)
        oms = time_run(otr, oev, args.steps)
        ot = otr.tracks()
        otr.profile(True)
        otr.profile_read(reset=True)
        for _ in range(args.steps):
            otr.run(oev)
        oprof = otr.profile_read(reset=True)
        otr.profile(False)
        oT, oH = otr.tracklet_counts()
        oq = quality(ocs.label, ocs.job_off, ocs.sector, ot["off"], ot["hits"], ocs.part_off, ocs.part_pt)
        also[name] = {"workload": WORKLOADS[name], "n_clusters": ocs.n, "ms_per_step": oms,
                      "clusters_per_s": ocs.n / (oms / 1e3), "tracks": int(ot["n"]), "quality": oq,
                      "kernels": kernel_json(kernel_rows(oprof, ocs.n, oT, oH)),
                      "stages_ms": {k: v[0] / max(1, v[1]) for k, v in oprof.items() if v[1]}}
        log(f"{name}: {oms:.3f} ms/step, {ocs.n / (oms / 1e3):.3e} clusters/s, quality {oq}")
        if name == "c3":
            # the time frame's compression: drift-shifted z needs the 24-bit absolute z codes
            otr.tpc_compress(Q_STEP, Q_STEP, wide_z=True)
            otr.sync()
            otr.profile(True)
            otr.profile_read(reset=True)
            for _ in range(args.steps):
                otr.tpc_compress(Q_STEP, Q_STEP, wide_z=True)
            cprof = otr.profile_read(reset=True)
            otr.profile(False)
            otr.sync()
            cms = cprof["compress"][0] / max(1, cprof["compress"][1])
            rec = otr.codes_numpy()
            nt = np.isnan(ot["t0"]).sum()
            also[name]["compression_24bit_z"] = {
                "ms": cms, "clusters_per_s": ocs.n / (cms / 1e3), "records": rec["n_codes"],
                "max_abs_z_code": int(np.abs((rec["ez_hi"].astype(np.int64) * 65536 + rec["ez"].view(np.uint16))
                                             [(rec["rs"] >> 15) == 1]).max())}
            also[name]["collision_times"] = {"tracks": int(ot["n"]), "without_t0": int(nt)}
            log(f"{name} compression (24-bit z codes): {cms:.3f} ms")
        del otr, oev
        if name == "c3":
            # the synchronous phase's cut set on the same time frame
            from paper_2402_01205_amd.tpc import preset_params
            sev = DeviceClusters.from_set(ocs, dev)
            str_ = Tracker(0, params=preset_params("sync"), mode=args.mode, tuning=tuning)
            sms = time_run(str_, sev, args.steps)
            st = str_.tracks()
            sq = quality(ocs.label, ocs.job_off, ocs.sector, st["off"], st["hits"], ocs.part_off, ocs.part_pt)
            also[name]["sync_preset"] = {"ms_per_step": sms, "clusters_per_s": ocs.n / (sms / 1e3),
                                         "tracks": int(st["n"]), "quality": sq,
                                         "attached_clusters": int(st["off"][-1]) / ocs.n,
                                         "async_attached_clusters": int(ot["off"][-1]) / ocs.n}
            log(f"{name} sync preset: {sms:.3f} ms/step, quality {sq}")
            del str_, sev
        if name == "c3" and args.plain_steps > 0:
            # the per-sector form: every sector its own job, launched one after the other
            split, perm, jev = g.split_by_sector(ocs)
            sev = DeviceClusters.from_set(split, dev, jev)
            ptr = Tracker(0, mode="plain")
            pms = time_run(ptr, sev, args.plain_steps)
            same = same_tracks(ot, ptr.tracks(), perm)
            also[name].update({"plain_per_sector_ms_per_step": pms,
                               "plain_per_sector_clusters_per_s": ocs.n / (pms / 1e3),
                               "batched_over_plain": pms / oms, "plain_jobs": split.n_jobs,
                               "plain_identical_tracks": same})
            log(f"{name} plain per sector ({split.n_jobs} jobs): {pms:.3f} ms/step; identical tracks: {same}")
            del ptr, sev
    membrane = membrane_run(vz_set, args, tuning, time_run, log, dev) if vz_set is not None else None
    loopers = looper_run(loop_set, args, tuning, time_run, log, dev) if loop_set is not None else None
    serving = None
    if args.serve_chunks > 0:
        del tr, ev                 # the serving run sizes its admission by free HBM
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        serving = serve_run(args, serve_cols, tuning, log)
    value = cs.n / (ms / 1e3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "clusters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {WORKLOADS[args.config]}", "seed": seed,
                   "n_clusters": cs.n, "n_jobs": cs.n_jobs,
                   "mode": f"{args.mode}{'' if args.no_graph else '+hipGraph'}"},
        "plain_value": (cs.n / (plain_ms / 1e3)) if plain_ms else None,
        "plain_ms_per_step": plain_ms,
        "batched_over_plain": (plain_ms / ms) if plain_ms else None,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": kern[dom]["gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": kern[dom]["gbs"] / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_ratio": (traffic / kern[dom]["bytes"]) if traffic else None,
                     "kernel_ms": kern[dom]["ms"], "algorithmic_bytes": kern[dom]["bytes"],
                     "bytes_per_unit": ({"cluster": LINK_BYTES_PER_CLUSTER} if dom == "k_links" else
                                        {"tracklet_hit": TRK_BYTES_PER_HIT, "tracklet": TRK_BYTES_PER_TRACKLET}),
                     "traffic_source": trec["file"] if trec else None},
        "kernels": kernel_json(kern),
        "copy_probe_GBs": probe,
        "p50_chunk_latency_ms": serving["p50_ms"] if serving else None,
        "p99_chunk_latency_ms": serving["p99_ms"] if serving else None,
        "serving": serving,
        "other_workloads": also,
        "tuning": tune_report["best"] if tune_report else None,
        "stages_ms": {k: v[0] / max(1, v[1]) for k, v in prof.items() if v[1]},
        "compression": compression,
        "sync_preset": sync_row,
        "membrane_merge": membrane,
        "return_legs": loopers,
        "cluster_finding": clusters_row,
        "tracks": int(tracks["n"]),
        "tracklets": int(T),
        "quality": q,
    }
    if cpu is not None:
        compression["cpu_baseline"], compression["rans"]["cpu_baseline"] = cpu_chain
        out["cpu_baseline"] = cpu
        out["cpu_baseline_all_cores"] = cpu_par
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
