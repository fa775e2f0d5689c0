"""Shared helpers of the GPU tests: run the HIP path stage by stage through the C ABI and
compare every stage output with the oracle."""
import sys

import numpy as np

import oracle.oracle as O


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_run(cs, mode="batched", tuning=None, params=None, job_event=None, stages=True, legs=False):
    import torch

    from paper_2402_01205_amd.tpc import DeviceClusters, Tracker
    tr = Tracker(0, params=params, mode=mode, tuning=tuning)
    ev = DeviceClusters.from_set(cs, "cuda:0", job_event)
    n = max(cs.n, 1)
    up = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
    dn = torch.full((n,), -1, dtype=torch.int32, device="cuda:0")
    tr.tpc_grid_build(ev)
    tr.tpc_find_neighbours(up, dn)
    tr.tpc_construct_tracklets()
    tr.tpc_select_tracks()
    tr.tpc_fit_merge()
    if legs:
        tr.tpc_pair_legs(ev.job_event)
    status = None
    try:
        tr.sync()
    except Exception as e:  # range errors are reported at sync; outputs stay valid
        status = getattr(e, "code", None)
    res = dict(status=status, tracks=tr.tracks_nosync() if status else tr.tracks())
    if legs:
        res["legs"] = tr.legs[:tr.out["cap_tracks"]].cpu().numpy()
    if stages:
        res.update(up=up.cpu().numpy()[:cs.n], down=dn.cpu().numpy()[:cs.n], raw=tr.links_raw(),
                   rows=tr.rows(), trk=tr.tracklets(), sel=tr.selected())
    return res


def oracle_run(cs, params=None, job_event=None):
    r = O.Run.from_set(cs, params, job_event=job_event)
    return dict(r=r, links=r.links(), trk=r.tracklets(), sel=O.Run.from_set(
        cs, params, last_stage=O.STAGE_SELECT, job_event=job_event).tracks(merged=False),
        tracks=r.tracks(merged=True), rows=r.rows())


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def compare_rows(g, o):
    goff, gmem = g
    ooff, omem = o
    assert np.array_equal(goff.astype(np.int64), ooff)
    # members per slot as sets (order inside a slot is the grid's cell order)
    s = np.repeat(np.arange(len(goff) - 1), np.diff(goff))
    gk = np.lexsort((gmem, s))
    assert np.array_equal(gmem[gk], omem)


def compare_all(g, o, fp_check=True):
    """Bit-exact comparison of every stage; returns a short summary."""
    L = o["links"]
    assert np.array_equal(g["raw"]["up_raw"], L["up_raw"]), "raw up links differ"
    assert np.array_equal(g["raw"]["down_raw"], L["down_raw"]), "raw down links differ"
    assert np.array_equal(g["up"], L["up"]), "clean up links differ"
    assert np.array_equal(g["down"], L["down"]), "clean down links differ"
    compare_rows(g["rows"], o["rows"])
    gt, ot = g["trk"], o["trk"]
    assert np.array_equal(gt["start"], ot["start"]), "tracklet starts differ"
    assert np.array_equal(gt["off"], ot["off"]), "tracklet lengths differ"
    assert np.array_equal(gt["hits"], ot["hits"]), "tracklet hits differ"
    assert np.array_equal(bits(gt["P"]), bits(ot["P"])), "tracklet states differ"
    assert np.array_equal(bits(gt["C"]), bits(ot["C"])), "tracklet covariances differ"
    assert np.array_equal(bits(gt["x"]), bits(ot["x"]))
    assert np.array_equal(gt["hitw"], ot["hitw"]), "hit weights differ"
    gs, os_ = g["sel"], o["sel"]
    assert np.array_equal(gs["tracklet"], os_["tracklet"]), "selected tracklets differ"
    assert np.array_equal(gs["off"], os_["off"])
    assert np.array_equal(gs["hits"], os_["hits"]), "selected hits differ"
    gk, ok = g["tracks"], o["tracks"]
    assert gk["n"] == len(ok["tracklet"]), (gk["n"], len(ok["tracklet"]))
    assert np.array_equal(gk["tracklet"], ok["tracklet"]), "track ids differ"
    assert np.array_equal(gk["off"], ok["off"]), "track lengths differ"
    assert np.array_equal(gk["hits"], ok["hits"]), "track hits differ"
    assert np.array_equal(gk["ndf"], ok["ndf"])
    assert np.array_equal(gk["sector"], ok["sector"])
    good = gk["ndf"] >= 0
    assert np.array_equal(bits(gk["param"][good]), bits(ok["P"][good])), "fitted params differ from FP32 oracle"
    assert np.array_equal(bits(gk["cov"][good]), bits(ok["C"][good]))
    assert np.array_equal(bits(gk["x_ref"][good]), bits(ok["x"][good]))
    nan = np.isnan(ok["t0"])
    assert np.array_equal(np.isnan(gk["t0"]), nan), "collision times fail on different tracks"
    assert np.array_equal(bits(gk["t0"][~nan]), bits(ok["t0"][~nan])), "collision times differ from FP32 oracle"
    if fp_check:
        check_fp64(gk, ok)
    return dict(n_tracks=gk["n"], n_tracklets=len(gt["start"]), merged=int((ok["sector2"] >= 0).sum()))


def check_fp64(gk, ok):
    """FP32 GPU fit against the FP64 oracle refit: 1e-4 relative on q/pT (floor 0.1 GeV^-1),
    1e-3 cm on y and z."""
    g32 = gk["ndf"] >= 0
    g64 = ok["ndfd"] >= 0
    assert np.array_equal(g32, g64), "fit failures differ between FP32 and FP64"
    P = gk["param"][g32].astype(np.float64)
    Pd = ok["Pd"][g32]
    assert np.all(np.abs(P[:, 4] - Pd[:, 4]) <= 1e-4 * np.maximum(np.abs(Pd[:, 4]), 0.1))
    assert np.all(np.abs(P[:, 0] - Pd[:, 0]) <= 1e-3)
    assert np.all(np.abs(P[:, 1] - Pd[:, 1]) <= 1e-3)
    # collision time: the position tolerance (1e-3 cm of z) at the beam line, over v_drift
    t0, t0d = gk["t0"][g32].astype(np.float64), ok["t0d"][g32]
    assert np.array_equal(np.isnan(t0), np.isnan(t0d)), "collision times fail on different tracks"
    f = ~np.isnan(t0)
    assert np.all(np.abs(t0[f] - t0d[f]) <= 1e-3 / 2.58)
