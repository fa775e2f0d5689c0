"""The whole time-frame workload (50 collisions, 21.9M clusters, drift-shifted z) on the GPU,
through the C ABI (needs a gfx950 GPU).

Tracks (hit lists, FP32 parameters), collision times and the 24-bit compression records are
compared bit for bit with the oracle through the digests in tests/golden (written by
make_golden.py from the oracle alone; the oracle needs minutes for this workload).  The
collision times are also checked against the generator's: the tracks of a time frame come
from 50 collisions at known times.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import tpcsynth as g
from tests.golden.make_golden import HERE, Q_STEP, TIMEFRAME, f32_bits
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def tf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2402_01205_amd.tpc import DeviceClusters, Tracker
    with open(os.path.join(HERE, f"oracle_{TIMEFRAME[0]}_seed{TIMEFRAME[1]}_full.json")) as f:
        ref = json.load(f)
    cs = g.make_config(*TIMEFRAME, workers=16)
    assert cs.n == ref["n_clusters"]
    assert digest(np.concatenate([cs.y, cs.z]).view(np.uint32)) == ref["input_sha256"]
    say("time frame", cs.n, "clusters")
    tr = Tracker(0)
    tr.run(DeviceClusters.from_set(cs, "cuda:0"))
    t = tr.tracks()
    return cs, tr, t, ref


def test_timeframe_tracks_bit_exact(tf):
    cs, tr, t, ref = tf
    assert t["n"] == ref["n_tracks"] and int(t["off"][-1]) == ref["n_hits"]
    assert digest(t["off"]) == ref["track_off_sha256"], "track lengths differ"
    assert digest(t["hits"]) == ref["track_hits_sha256"], "track hits differ"
    good = t["ndf"] >= 0
    assert int((~good).sum()) == ref["n_fit_failed"]
    assert digest(f32_bits(t["param"][good])) == ref["params_sha256"], "fitted parameters differ"
    assert int(np.isnan(t["t0"]).sum()) == ref["n_t0_nan"]
    assert digest(f32_bits(t["t0"])) == ref["t0_sha256"], "collision times differ"
    say("tracks", t["n"], "hits", int(t["off"][-1]), "bit-exact with the oracle")


def test_timeframe_collision_times_against_the_generator(tf):
    """Good tracks (purity >= 0.9, >= 30 hits) carry their collision's time: median error
    below 0.03 us, 95% within 0.2 us (0.5 cm of drift)."""
    cs, tr, t, ref = tf
    off, hits = t["off"], t["hits"]
    lab = cs.label[hits]
    tid = np.repeat(np.arange(t["n"]), np.diff(off))
    ok = lab >= 0
    # majority label per track
    key = tid[ok].astype(np.int64) * (int(lab.max()) + 1) + lab[ok]
    u, c = np.unique(key, return_counts=True)
    trk, part = u // (int(lab.max()) + 1), u % (int(lab.max()) + 1)
    order = np.lexsort((-c, trk))
    first = np.concatenate([[True], trk[order][1:] != trk[order][:-1]])
    maj_t, maj_p, maj_c = trk[order][first], part[order][first], c[order][first]
    nh = np.diff(off)[maj_t]
    sel = (maj_c >= 0.9 * nh) & (nh >= 30) & ~np.isnan(t["t0"][maj_t])
    coll_off = np.asarray(cs.meta["coll_part_off"], np.int64)
    tk = np.asarray(cs.meta["t_collisions"])
    coll = np.searchsorted(coll_off, maj_p[sel], side="right") - 1
    d = np.abs(t["t0"][maj_t[sel]] - tk[coll])
    say("collision times of", int(sel.sum()), "tracks: median", float(np.median(d)), "95%", float(np.percentile(d, 95)))
    assert sel.sum() > 100000
    assert np.median(d) < 0.03 and np.percentile(d, 95) < 0.2


def test_timeframe_compression_24bit_codes_bit_exact(tf):
    """The time frame's drift-shifted z saturates 16-bit absolute codes (range status) and
    fits 24-bit ones, whose records equal the oracle's; every cluster decodes within half a
    step (plus FP32 rounding of z up to ~2600 cm)."""
    from paper_2402_01205_amd.tpc import TPC_E_RANGE, TpcError
    cs, tr, t, ref = tf
    tr.tpc_compress(Q_STEP, Q_STEP, wide_z=True)
    tr.sync()
    gc = tr.codes_numpy()
    assert gc["n_codes"] == cs.n and gc["n_attached"] == ref["cmp_n_attached"] and ref["cmp_status"] == 0
    for k in ("rs", "ey", "ez", "ez_hi"):
        assert digest(gc[k]) == ref[f"cmp_{k}_sha256"], f"records differ: {k}"
    d = tr.tpc_decompress()
    tr.sync()
    free = np.ones(cs.n, bool)
    free[t["hits"]] = False
    perm = np.concatenate([t["hits"], np.nonzero(free)[0]]).astype(np.int64)
    for k, v in (("sector", cs.sector), ("row", cs.row)):
        assert np.array_equal(d[k][:cs.n].cpu().numpy(), v[perm])
    for k, v in (("y", cs.y), ("z", cs.z)):
        assert np.abs(d[k][:cs.n].cpu().numpy() - v[perm]).max() <= Q_STEP / 2 + 3e-4
    ab = (gc["rs"] >> 15) == 1
    say("records", gc["n_codes"], "bit-exact; absolute z codes up to",
        int(np.abs(gc["ez_hi"].astype(np.int64) * 65536 + gc["ez"].view(np.uint16))[ab].max()))
    # 16-bit codes saturate here (the range status stays set until the next tracking run)
    tr.tpc_compress(Q_STEP, Q_STEP)
    with pytest.raises(TpcError) as e:
        tr.sync()
    assert e.value.code == TPC_E_RANGE
