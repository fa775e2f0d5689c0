"""Track-model compression on the GPU against the oracle, through the C ABI (needs a gfx950 GPU).

The records (row/sector/absolute word and two int16 codes) are integers that both sides decide
in FP32 with the same operations: bit-exact.  The decoded clusters are FP32 sums and products
in the same order on both sides: bit-exact, NaN markers included; and within half a
quantisation step (plus FP32 rounding) of the input clusters.
"""
import ctypes as C

import numpy as np
import pytest

import oracle.oracle as O
import tpcsynth as g
from tests.gpu_helpers import bits, say

pytestmark = pytest.mark.gpu

Q = 1.0 / 32.0


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2402_01205_amd import tpc
    tpc.lib()


def _status(tr):
    from paper_2402_01205_amd.tpc import TpcError
    try:
        tr.sync()
        return 0
    except TpcError as e:
        return e.code


def _track(cs, mode="batched"):
    from paper_2402_01205_amd.tpc import DeviceClusters, Tracker
    tr = Tracker(0, mode=mode)
    ev = DeviceClusters.from_set(cs, "cuda:0")
    tr.run(ev)
    return tr, ev, _status(tr)


def _decoded(tr, m):
    d = tr.tpc_decompress()
    st = _status(tr)
    return {k: v[:m].cpu().numpy() for k, v in d.items()}, st


def _oracle(cs, qy, qz, tracks=None):
    t = O.Run.from_set(cs).tracks(merged=True) if tracks is None else tracks
    c = O.compress(cs.sector, cs.row, cs.y, cs.z, t, qy, qz)
    return t, c, O.decompress(t, c, qy, qz)


def _compare(gc, oc, gd, od):
    assert gc["n_codes"] == len(oc["rs"]), (gc["n_codes"], len(oc["rs"]))
    assert gc["n_attached"] == oc["n_attached"]
    assert np.array_equal(gc["rs"], oc["rs"]), "records differ"
    assert np.array_equal(gc["ey"], oc["ey"]), "y codes differ"
    assert np.array_equal(gc["ez"], oc["ez"]), "z codes differ"
    assert np.array_equal(gd["sector"], od["sector"]) and np.array_equal(gd["row"], od["row"])
    assert np.array_equal(bits(gd["y"]), bits(od["y"])), "decoded y differs"
    assert np.array_equal(bits(gd["z"]), bits(od["z"])), "decoded z differs"


def _round_trip(cs, t, d, qy, qz):
    rest = np.setdiff1d(np.arange(cs.n), t["hits"])
    perm = np.concatenate([t["hits"], rest]).astype(np.int64)
    assert np.array_equal(d["sector"], cs.sector[perm]) and np.array_equal(d["row"], cs.row[perm])
    assert np.abs(d["y"] - cs.y[perm]).max() <= qy / 2 + 1e-4
    assert np.abs(d["z"] - cs.z[perm]).max() <= qz / 2 + 1e-4


@pytest.mark.parametrize("cfg,seed,qy,qz", [("c1", 11, Q, Q), ("c1", 12, 0.5, 1.0 / 64.0),
                                            ("c2", 21, Q, Q), ("c2", 22, 0.1, 0.5)])
def test_codes_and_decoding_bit_exact(cfg, seed, qy, qz):
    cs = g.make_config(cfg, seed)
    say(cfg, seed, "clusters", cs.n, "q", qy, qz)
    tr, ev, st = _track(cs)
    assert st == 0
    tr.tpc_compress(qy, qz)
    assert _status(tr) == 0
    gc = tr.codes_numpy()
    gd, st = _decoded(tr, gc["n_codes"])
    assert st == 0
    ot, oc, od = _oracle(cs, qy, qz)
    assert np.array_equal(tr.tracks()["hits"], ot["hits"])
    _compare(gc, oc, gd, od)
    _round_trip(cs, ot, gd, qy, qz)
    H = gc["n_attached"]
    say("records", gc["n_codes"], "track hits", H, "residual", int(((gc["rs"][:H] >> 15) == 0).sum()))


@pytest.mark.parametrize("qy,qz", [(Q, Q), (0.25, 1.0 / 64.0)])
def test_time_frame_wide_codes_bit_exact(qy, qz):
    """A time frame spread over 1 ms (six collisions, drift-shifted z beyond +-1024 cm): the
    24-bit absolute z codes, their high bytes, the tracks' collision times and the decoded
    clusters equal the oracle's bit for bit; 16-bit codes saturate there."""
    pool = g.gen_collision_pool(73, 6, mult_range=(500, 1500))
    cs = g.assemble_timeframe(74, pool, np.arange(6), 1000.0, mean_spacing_us=150.0)
    assert np.abs(cs.z).max() > 1100.0
    tr, ev, st = _track(cs)
    assert st == 0
    t = tr.tracks()
    ot = O.Run.from_set(cs).tracks(merged=True)
    assert np.array_equal(t["hits"], ot["hits"]) and np.array_equal(t["off"], ot["off"])
    nan = np.isnan(ot["t0"])
    assert np.array_equal(np.isnan(t["t0"]), nan) and np.array_equal(bits(t["t0"][~nan]), bits(ot["t0"][~nan]))
    tr.tpc_compress(qy, qz, wide_z=True)
    assert _status(tr) == 0
    gc = tr.codes_numpy()
    gd, st = _decoded(tr, gc["n_codes"])
    assert st == 0
    oc = O.compress(cs.sector, cs.row, cs.y, cs.z, ot, qy, qz, wide_z=True)
    od = O.decompress(ot, oc, qy, qz)
    _compare(gc, oc, gd, od)
    assert np.array_equal(gc["ez_hi"], oc["ez_hi"]), "high bytes differ"
    assert np.abs(gc["ez_hi"]).max() > 0
    rest = np.setdiff1d(np.arange(cs.n), ot["hits"])
    perm = np.concatenate([ot["hits"], rest]).astype(np.int64)
    assert np.abs(gd["z"] - cs.z[perm]).max() <= qz / 2 + 2e-4
    tr.tpc_compress(qy, qz)
    assert _status(tr) == TPC_E_RANGE_CODE
    say("time frame", cs.n, "clusters, wide codes bit-exact; max |z|", float(np.abs(cs.z).max()))


TPC_E_RANGE_CODE = -2


def test_invalid_and_saturated_clusters():
    from paper_2402_01205_amd.tpc import TPC_E_RANGE
    cs = g.make_config("c1", 11)
    cs.row = cs.row.copy(); cs.sector = cs.sector.copy(); cs.y = cs.y.copy(); cs.z = cs.z.copy()
    cs.row[5] = 200
    cs.sector[6] = 40
    cs.y[7] = np.nan
    cs.z[8] = 5000.0
    tr, ev, st = _track(cs)
    assert st == TPC_E_RANGE
    tr.tpc_compress(Q, Q)
    assert _status(tr) == TPC_E_RANGE
    gc = tr.codes_numpy()
    gd, _ = _decoded(tr, gc["n_codes"])
    ot, oc, od = _oracle(cs, Q, Q)
    assert oc["status"] == 1
    _compare(gc, oc, gd, od)
    assert (gc["rs"] == 0x7FFF).sum() == 3


def test_empty_input():
    cs = g.make_config("c1", 11)
    idx = np.arange(0)
    nothing = g.ClusterSet(cs.sector[idx], cs.row[idx], cs.y[idx], cs.z[idx], cs.time[idx], cs.label[idx],
                           np.array([0, 0], np.int32), cs.part_pt, cs.part_eta, cs.part_phi, cs.part_q,
                           np.array([0, len(cs.part_pt)]), {})
    tr, ev, st = _track(nothing)
    assert st == 0
    tr.tpc_compress(Q, Q)
    assert _status(tr) == 0
    gc = tr.codes_numpy()
    assert gc["n_codes"] == 0 and gc["n_attached"] == 0
    gd, st = _decoded(tr, 0)
    assert st == 0


def _device_tracks(t, torch):
    """Device copies of a track list (oracle output, possibly edited) as a tpc_tracks."""
    from paper_2402_01205_amd.tpc import tpc_tracks
    dev = "cuda:0"
    K = len(t["off"]) - 1
    arr = dict(n_tracks=np.array([K], np.int32), hit_off=np.ascontiguousarray(t["off"], np.int32),
               hits=np.ascontiguousarray(t["hits"], np.int32), param=np.ascontiguousarray(t["P"], np.float32),
               x_ref=np.ascontiguousarray(t["x"], np.float32), ndf=np.ascontiguousarray(t["ndf"], np.int32),
               sector=np.ascontiguousarray(t["sector"], np.int32))
    d = {k: torch.from_numpy(v).to(dev) for k, v in arr.items()}
    p = lambda k: C.c_void_p(d[k].data_ptr())
    s = tpc_tracks(K, max(len(t["hits"]), 1), p("n_tracks"), p("hit_off"), p("hits"), p("param"), None,
                   p("x_ref"), None, p("ndf"), p("sector"), None, None)
    return s, d


def _device_codes(cap, guard, torch):
    from paper_2402_01205_amd.tpc import tpc_codes
    dev = "cuda:0"
    d = dict(n_codes=torch.zeros(1, dtype=torch.int32, device=dev),
             n_attached=torch.zeros(1, dtype=torch.int32, device=dev),
             rs=torch.full((cap + guard,), 0x5A5A, dtype=torch.int16, device=dev),
             ey=torch.full((cap + guard,), 0x5A5A, dtype=torch.int16, device=dev),
             ez=torch.full((cap + guard,), 0x5A5A, dtype=torch.int16, device=dev))
    p = lambda k: C.c_void_p(d[k].data_ptr())
    return tpc_codes(cap, p("n_codes"), p("n_attached"), p("rs"), p("ey"), p("ez")), d


def test_caller_tracks_with_failed_fits_and_bad_indices():
    """Tracks handed in by the caller (here the oracle's, edited): a failed fit takes absolute
    codes, a hit index outside the cluster list gives the invalid record and TPC_E_RANGE."""
    import torch
    from paper_2402_01205_amd.tpc import TPC_E_RANGE, lib
    cs = g.make_config("c2", 21, scale=0.25)
    tr, ev, st = _track(cs)
    assert st == 0
    t = dict(O.Run.from_set(cs).tracks(merged=True))
    t["ndf"] = t["ndf"].copy(); t["hits"] = t["hits"].copy()
    t["ndf"][0] = -1
    t["ndf"][3] = -1
    t["hits"][t["off"][2] + 1] = cs.n + 7
    ts, keep_t = _device_tracks(t, torch)
    cap = int(t["off"][-1]) + cs.n
    cd, keep_c = _device_codes(cap, 0, torch)
    assert lib().tpc_compress(tr.ctx, C.byref(tr._cl), C.byref(ts), Q, Q, C.byref(cd)) == 0
    assert _status(tr) == TPC_E_RANGE
    m = int(keep_c["n_codes"].item())
    gc = dict(n_codes=m, n_attached=int(keep_c["n_attached"].item()),
              rs=keep_c["rs"][:m].cpu().numpy().view(np.uint16), ey=keep_c["ey"][:m].cpu().numpy(),
              ez=keep_c["ez"][:m].cpu().numpy())
    out = dict(sector=torch.zeros(cap, dtype=torch.uint8, device="cuda:0"),
               row=torch.zeros(cap, dtype=torch.int16, device="cuda:0"),
               y=torch.zeros(cap, dtype=torch.float32, device="cuda:0"),
               z=torch.zeros(cap, dtype=torch.float32, device="cuda:0"))
    assert lib().tpc_decompress(tr.ctx, C.byref(ts), C.byref(cd), Q, Q,
                                *[C.c_void_p(out[k].data_ptr()) for k in ("sector", "row", "y", "z")]) == 0
    _status(tr)
    gd = {k: v[:m].cpu().numpy() for k, v in out.items()}
    oc = O.compress(cs.sector, cs.row, cs.y, cs.z, t, Q, Q)
    od = O.decompress(t, oc, Q, Q)
    assert oc["status"] == 1
    _compare(gc, oc, gd, od)
    a, b = t["off"][0], t["off"][1]
    assert np.all(gc["rs"][a:b] >> 15 == 1)
    assert gc["rs"][t["off"][2] + 1] == 0x7FFF


def test_record_capacity_reports_required_count_and_writes_nothing_beyond():
    import torch
    from paper_2402_01205_amd.tpc import TPC_E_CAPACITY, lib
    cs = g.make_config("c1", 13)
    tr, ev, st = _track(cs)
    assert st == 0
    ot, oc, od = _oracle(cs, Q, Q)
    for cap in (cs.n - 1, oc["n_attached"] // 2, 0):
        cd, keep = _device_codes(cap, 64, torch)
        assert lib().tpc_compress(tr.ctx, C.byref(tr._cl), C.byref(tr._tracks), Q, Q, C.byref(cd)) == 0
        assert _status(tr) == TPC_E_CAPACITY
        assert int(keep["n_codes"].item()) == cs.n
        rs = keep["rs"].cpu().numpy().view(np.uint16)
        ey, ez = keep["ey"].cpu().numpy(), keep["ez"].cpu().numpy()
        assert np.array_equal(rs[:cap], oc["rs"][:cap]) and np.array_equal(ey[:cap], oc["ey"][:cap])
        assert np.array_equal(ez[:cap], oc["ez"][:cap])
        assert np.all(rs[cap:] == 0x5A5A) and np.all(ey[cap:] == 0x5A5A) and np.all(ez[cap:] == 0x5A5A)


def test_arguments_are_checked():
    from paper_2402_01205_amd.tpc import TPC_E_ARG, Tracker, lib, tpc_codes
    cs = g.make_config("c1", 11)
    tr, ev, st = _track(cs)
    cd = tpc_codes(0, None, None, None, None, None)
    assert lib().tpc_compress(tr.ctx, C.byref(tr._cl), C.byref(tr._tracks), Q, Q, C.byref(cd)) == TPC_E_ARG
    with pytest.raises(Exception):
        tr.tpc_compress(0.0, Q)
    with pytest.raises(Exception):
        tr.tpc_compress(Q, float("nan"))
    fresh = Tracker(0)
    with pytest.raises(Exception):   # no tracking run: no workspace
        fresh._cl = tr._cl
        fresh._tracks = tr._tracks
        fresh._keep = tr._keep
        fresh.tpc_compress(Q, Q)


def test_compression_between_graph_replays():
    """Compression reuses scratch of the tracking workspace: a tracking run replayed from its
    captured graph after it gives the same tracks, and compressing again the same records."""
    from paper_2402_01205_amd.tpc import DeviceClusters, Tracker, default_tuning
    cs = g.make_config("c2", 21, scale=0.5)
    tr = Tracker(0, mode="persistent", tuning=default_tuning(use_graph=1))
    ev = DeviceClusters.from_set(cs, "cuda:0")
    tr.run(ev)
    t0 = tr.tracks()
    tr.tpc_compress(Q, Q)
    c0 = tr.codes_numpy()
    tr.run(ev)
    tr.run(ev)
    t1 = tr.tracks()
    assert np.array_equal(t0["hits"], t1["hits"]) and np.array_equal(bits(t0["param"]), bits(t1["param"]))
    tr.tpc_compress(Q, Q)
    c1 = tr.codes_numpy()
    for k in ("rs", "ey", "ez"):
        assert np.array_equal(c0[k], c1[k])
