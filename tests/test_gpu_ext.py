"""The downward extension of the tracks on the GPU (needs a gfx950 GPU): every stage bit
for bit with the oracle's extension (reading A13) through the C ABI, on realistic workloads
(merge on), on the pin geometries (thinned lower rows, a contested pair), in every launch
mode and in replays of the captured chain."""
import numpy as np
import pytest

import oracle.oracle as O
import tpcsynth as g
from tests.gpu_helpers import compare_all, gpu_run, oracle_run, say
from tests.test_ext_pins import R_CUT, _cluster_set, _particle_clusters, _thinned_event

pytestmark = pytest.mark.gpu


class _Set:
    """The cluster-set fields the GPU helpers read, from a pin event."""
    def __init__(self, ev):
        self.sector, self.row, self.y, self.z = ev["sector"], ev["row"], ev["y"], ev["z"]
        self.job_off = ev["job_off"]
        self.n = len(self.y)
        self.n_jobs = 1
        self.time = np.zeros(self.n, np.float32)


def _ext_params():
    from paper_2402_01205_amd.tpc import default_params
    return default_params(ext_down=1)


@pytest.mark.parametrize("cfg,seed,scale,jobs", [
    ("c2", 21, 0.5, None), ("c3", 31, 0.1, None), ("c4", 41, 1.0, "dense")])
def test_extension_bit_exact(cfg, seed, scale, jobs):
    if jobs == "dense":
        sizes = g.c4_job_sizes(seed)
        cs = g.make_config(cfg, seed, jobs=[5, 60, int(np.argmax(sizes))])
    else:
        cs = g.make_config(cfg, seed, scale=scale)
    prm = O.params(ext_down=1)
    o = oracle_run(cs, prm)
    s = compare_all(gpu_run(cs, params=_ext_params()), o)
    n_ext = int(o["tracks"]["n_ext"].sum())
    say(cfg, "extension: tracks", s["n_tracks"], "merged", s["merged"], "extension hits (heads)", n_ext)
    assert n_ext > 100


@pytest.mark.parametrize("step", [3, 6])
def test_extension_pin_geometry_bit_exact(step):
    ev, _ = _thinned_event(3, 25, step)
    cs = _Set(ev)
    o = oracle_run(cs, O.params(ext_down=1))
    compare_all(gpu_run(cs, params=_ext_params()), o)
    assert (o["tracks"]["n_ext"].sum() > 0) == (step == 3)


def test_extension_of_tracks_beyond_the_list_room_bit_exact():
    """Tracks that start at row 130 with their lower clusters every third row: the rows
    below the tracks outnumber the clusters, so the later tracks keep no list of found
    clusters and their searches are replayed; every stage still equals the oracle."""
    ev, _ = _thinned_event(5, 30, 3, r_cut=130)
    cs = _Set(ev)
    o = oracle_run(cs, O.params(ext_down=1))
    sel = o["sel"]
    rows_below = sum(int(cs.row[sel["hits"][sel["off"][i]]]) for i in range(len(sel["tracklet"])))
    assert rows_below > cs.n + 1, (rows_below, cs.n)
    compare_all(gpu_run(cs, params=_ext_params()), o)
    assert o["tracks"]["n_ext"].sum() > 300


@pytest.mark.parametrize("longer", ["A", "B"])
def test_contested_pair_bit_exact(longer):
    a = float(g.sector_alpha(0))
    top_a, top_b = (151, 130) if longer == "A" else (130, 151)
    ca = _particle_clusters(2.0, 0.3, a, 1.0, list(range(R_CUT, top_a + 1)) + list(range(R_CUT - 3, -1, -3)))
    cb = _particle_clusters(2.0, 0.3, a + 0.0015, 1.0, list(range(R_CUT, top_b + 1)))
    cs = _Set(_cluster_set([(0, ca), (1, cb)]))
    o = oracle_run(cs, O.params(ext_down=1))
    compare_all(gpu_run(cs, params=_ext_params()), o)
    n_low = len(range(R_CUT - 3, -1, -3))
    assert sorted(o["tracks"]["n_ext"].tolist()) == [0, n_low]


@pytest.mark.parametrize("mode,tune", [
    ("plain", {}), ("batched", dict(use_graph=0)), ("batched", {}),
    ("persistent", dict(persistent_refill=1)), ("persistent", {})])
def test_extension_launch_modes_and_replays_identical(mode, tune):
    """Every launch mode gives the eager batched result, also over three runs of the
    captured chain (eager work between them)."""
    import torch

    from paper_2402_01205_amd.tpc import DeviceClusters, Tracker, default_tuning
    sizes = g.c4_job_sizes(41)
    cs = g.make_config("c4", 41, jobs=[3, 100, 200, int(np.argmax(sizes))])
    ev = DeviceClusters.from_set(cs, "cuda:0")
    ref_t = Tracker(0, params=_ext_params(), mode="batched", tuning=default_tuning(use_graph=0))
    ref_t.run(ev)
    ref = ref_t.tracks()
    tr = Tracker(0, params=_ext_params(), mode=mode, tuning=default_tuning(**tune))
    for rep in range(3):
        tr.run(ev)
        got = tr.tracks()
        for k in ("off", "hits", "tracklet", "ndf"):
            assert np.array_equal(got[k], ref[k]), (mode, rep, k)
        for k in ("param", "cov", "x_ref", "t0"):
            assert np.array_equal(got[k].view(np.uint32), ref[k].view(np.uint32)), (mode, rep, k)
        x = torch.randn(1 << 20, device="cuda:0")
        (x * 2).sum().item()
        torch.cuda.synchronize()
    say(mode, tune, "tracks", ref["n"], "hits", int(ref["off"][-1]))


def test_sync_preset_extends_and_does_not_merge():
    from paper_2402_01205_amd.tpc import preset_params
    cs = g.make_config("c3", 31, scale=0.1)
    o = oracle_run(cs, O.params(**O.SYNC))
    s = compare_all(gpu_run(cs, params=preset_params("sync")), o)
    assert s["merged"] == 0 and int(o["tracks"]["n_ext"].sum()) > 100
