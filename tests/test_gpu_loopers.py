"""Loopers' return legs on the GPU (needs a gfx950 GPU): events and time frames whose
primaries that turn back inside the chamber also leave their return legs, tracked bit for bit
with the oracle through the C ABI (the default reading, the asynchronous and synchronous cut
sets), and the exact loopers of the pins."""
import numpy as np
import pytest

import oracle.oracle as O
import tpcsynth as g
from tests.gpu_helpers import compare_all, gpu_run, oracle_run, say
from tests.test_looper_pins import LOOPERS, _looper

pytestmark = pytest.mark.gpu


class _Set:
    def __init__(self, ev):
        self.sector, self.row, self.y, self.z = ev["sector"], ev["row"], ev["y"], ev["z"]
        self.job_off = ev["job_off"]
        self.n = len(self.y)
        self.n_jobs = 1
        self.time = np.zeros(self.n, np.float32)


@pytest.mark.parametrize("pt,eta,phi,q", LOOPERS)
def test_exact_looper_bit_exact(pt, eta, phi, q):
    cs = _Set(_looper(pt, eta, phi, q))
    compare_all(gpu_run(cs), oracle_run(cs))


@pytest.mark.parametrize("cfg,preset", [("c2", None), ("c2", "async"), ("c3", "sync")])
def test_return_legs_bit_exact(cfg, preset):
    from paper_2402_01205_amd.tpc import preset_params
    cs = (g.make_config("c2", 21, scale=0.4, loopers=True) if cfg == "c2" else
          g.make_config("c3", 31, scale=0.1, loopers=True, vz_sigma=5.0))
    prm = {None: O.DEFAULTS, "async": O.ASYNC, "sync": O.SYNC}[preset]
    o = oracle_run(cs, O.params(**prm))
    s = compare_all(gpu_run(cs, params=preset_params(preset) if preset else None), o)
    say(cfg, preset, "tracks", s["n_tracks"], "merged", s["merged"])
