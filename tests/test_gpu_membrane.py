"""The merge across the central membrane on the GPU (needs a gfx950 GPU): every stage bit for
bit with the oracle's reading A21 through the C ABI, on exact crossers (collision at 0 and at
123.4 us), on the negative cases, on a full event and a time frame whose vertices are spread
in z, in every launch mode and over replays of the captured chain, alone and with the
downward extension."""
import numpy as np
import pytest

import oracle.oracle as O
import tpcsynth as g
from tests.gpu_helpers import compare_all, gpu_run, oracle_run, say
from tests.test_membrane_pins import CROSSERS, PHI0, _crosser, _set

pytestmark = pytest.mark.gpu


class _Set:
    def __init__(self, ev):
        self.sector, self.row, self.y, self.z = ev["sector"], ev["row"], ev["y"], ev["z"]
        self.job_off = ev["job_off"]
        self.n = len(self.y)
        self.n_jobs = 1
        self.time = np.zeros(self.n, np.float32)


def _params(**over):
    from paper_2402_01205_amd.tpc import default_params
    return default_params(merge_membrane=1, **over)


def _membrane_links(tracks):
    return int(((tracks["sector2"] >= 0) & ((tracks["sector"] < 18) != (tracks["sector2"] < 18))).sum())


@pytest.mark.parametrize("t0", [0.0, 123.4])
@pytest.mark.parametrize("pt,eta,z0,dphi", CROSSERS)
def test_exact_crosser_bit_exact(pt, eta, z0, dphi, t0):
    sec, row, y, z = _crosser(pt, eta, PHI0 + dphi, 1.0, z0)
    cs = _Set(_set([(sec, row, y, z)], t0))
    o = oracle_run(cs, O.params(merge_membrane=1))
    g_ = gpu_run(cs, params=_params())
    compare_all(g_, o)
    assert g_["tracks"]["n"] == 1 and _membrane_links(o["tracks"]) == 1


def test_negative_cases_bit_exact():
    sec, row, y, z = _crosser(1.5, -0.045, PHI0 + 0.06, 1.0, 6.0)
    sa, ra, ya, za = _crosser(1.5, 0.02, PHI0 + 0.06, 1.0, 0.5)
    s2, r2, y2, z2 = _crosser(1.5, -0.045, PHI0 - 0.06, -1.0, 6.0)
    c, a, m = sec >= 18, sa < 18, s2 >= 18
    cs = _Set(_set([(sec[c], row[c], y[c], z[c]), (sa[a], ra[a], ya[a], za[a]),
                    (s2[m], r2[m], y2[m], z2[m])]))
    o = oracle_run(cs, O.params(merge_membrane=1))
    compare_all(gpu_run(cs, params=_params()), o)
    assert _membrane_links(o["tracks"]) == 0


def _timeframe():
    pool = g.gen_collision_pool(77, 6, vz_sigma=8.0)
    return g.assemble_timeframe(78, pool, np.arange(6), 500.0)


@pytest.mark.parametrize("case", ["event", "timeframe", "timeframe+ext"])
def test_vertex_spread_workloads_bit_exact(case):
    cs = g.make_config("c2", 21, scale=0.5, vz_sigma=8.0) if case == "event" else _timeframe()
    ext = int(case.endswith("+ext"))
    o = oracle_run(cs, O.params(merge_membrane=1, ext_down=ext))
    s = compare_all(gpu_run(cs, params=_params(ext_down=ext)), o)
    n = _membrane_links(o["tracks"])
    say(case, "tracks", s["n_tracks"], "merged", s["merged"], "across the membrane", n)
    assert n > 50


@pytest.mark.parametrize("mode,tune", [
    ("plain", {}), ("batched", dict(use_graph=0)), ("batched", {}), ("persistent", {})])
def test_membrane_launch_modes_and_replays_identical(mode, tune):
    import torch

    from paper_2402_01205_amd.tpc import DeviceClusters, Tracker, default_tuning
    cs = _timeframe()
    ev = DeviceClusters.from_set(cs, "cuda:0")
    rt = Tracker(0, params=_params(), mode="batched", tuning=default_tuning(use_graph=0))
    rt.run(ev)
    ref = rt.tracks()
    tr = Tracker(0, params=_params(), mode=mode, tuning=default_tuning(**tune))
    for rep in range(3):
        tr.run(ev)
        got = tr.tracks()
        for k in ("off", "hits", "tracklet", "ndf", "sector"):
            assert np.array_equal(got[k], ref[k]), (mode, rep, k)
        for k in ("param", "cov", "x_ref", "t0"):
            assert np.array_equal(got[k].view(np.uint32), ref[k].view(np.uint32)), (mode, rep, k)
        x = torch.randn(1 << 20, device="cuda:0")
        (x * 2).sum().item()
        torch.cuda.synchronize()
