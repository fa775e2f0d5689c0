"""Cluster finding on the GPU against the oracle, through the C ABI (needs a gfx950 GPU).

Peaks (integers) and the FP32 centroids, widths and charges computed from exact integer
moments in the same operation order: bit-exact with the oracle, on the digits of a
single-sector event and of a full TPC event, in read-out order and shuffled, with other
parameters, invalid and duplicated digits, an empty list and a too small output.
"""
import numpy as np
import pytest

import oracle.oracle as O
from tests.gpu_helpers import bits, say
from tpcsynth import digits as D

pytestmark = pytest.mark.gpu

KEYS = ("digit", "sector", "row", "q_tot", "q_max")
FKEYS = ("y", "z", "sigma_pad", "sigma_time")


@pytest.fixture(scope="module")
def tracker():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2402_01205_amd.tpc import Tracker
    return Tracker(0)


def _dev(d):
    import torch
    f = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a, dt)).to("cuda:0")
    return dict(sector=f(d[0], np.uint8), row=f(d[1], np.int16), pad=f(d[2], np.int16), time=f(d[3], np.int16),
                adc=f(np.asarray(d[4], np.uint16).view(np.int16), np.int16))


def _gpu(tr, d, params=None, cap=None):
    o = tr.tpc_find_clusters(_dev(d), params, cap)
    return tr.clusters_numpy(o)


def _params(**kw):
    from paper_2402_01205_amd.tpc import lib, tpc_cf_params
    import ctypes as C
    p = tpc_cf_params()
    lib().tpc_cf_params_default(C.byref(p))
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def _compare(g, o):
    assert g["n"] == len(o["y"]), (g["n"], len(o["y"]))
    for k in KEYS:
        assert np.array_equal(g[k], o[k]), k
    for k in FKEYS:
        assert np.array_equal(bits(g[k]), bits(o[k])), k


def _arrays(d):
    return [d.sector, d.row, d.pad, d.time, d.adc]


@pytest.mark.parametrize("cfg,seed", [("d1", 11), ("d1", 12), ("d2", 21)])
def test_digits_of_generated_events_bit_exact(tracker, cfg, seed):
    cs, d, _ = D.digit_config(cfg, seed)
    say(cfg, seed, "digits", d.n)
    g = _gpu(tracker, _arrays(d))
    assert g["status"] == 0
    o = O.find_clusters(*_arrays(d))
    _compare(g, o)
    say("clusters", g["n"], "from", cs.n, "generated")


def test_shuffled_digits_and_other_parameters(tracker):
    cs, d, _ = D.digit_config("d1", 13)
    a = _arrays(d)
    perm = np.random.default_rng(1).permutation(d.n)
    sh = [x[perm] for x in a]
    g = _gpu(tracker, sh)
    _compare(g, O.find_clusters(*sh))
    # the same clusters as in read-out order, in the shuffled order of their peaks
    base = O.find_clusters(*a)
    assert np.array_equal(np.sort(perm[g["digit"]]), np.sort(base["digit"]))
    g = _gpu(tracker, a, _params(q_min=25, n_time=600))
    _compare(g, O.find_clusters(*a, q_min=25, n_time=600))


def test_invalid_duplicated_and_empty(tracker):
    from paper_2402_01205_amd.tpc import TPC_E_RANGE
    cs, d, _ = D.digit_config("d1", 11)
    a = [x.copy() for x in _arrays(d)]
    a[1][3] = 152
    a[2][4] = 500
    a[3][5] = -1
    a[0][6] = 40
    dup = [np.concatenate([x, x[100:400]]) for x in a]        # duplicated digits add up
    g = _gpu(tracker, dup)
    assert g["status"] == 1 and TPC_E_RANGE < 0
    o = O.find_clusters(*dup)
    assert o["status"] == 1
    _compare(g, o)
    g = _gpu(tracker, [x[:0] for x in a])
    assert g["n"] == 0 and g["status"] == 0


def test_output_capacity(tracker):
    """Too small an output: TPC_STATUS_CAPACITY, the number found reported, the first cap
    clusters written and nothing beyond them (guard values)."""
    import ctypes as C
    import torch
    from paper_2402_01205_amd.tpc import CF_KEYS, lib, tpc_cf_clusters, tpc_cf_params, tpc_digits
    cs, d, _ = D.digit_config("d1", 12)
    o = O.find_clusters(*_arrays(d))
    n = len(o["y"])
    dd = _dev(_arrays(d))
    p = tpc_cf_params()
    lib().tpc_cf_params_default(C.byref(p))
    need = int(lib().tpc_cf_workspace_size(C.byref(p), d.n))
    ws = torch.empty(need, dtype=torch.uint8, device="cuda:0")
    dg = tpc_digits(d.n, *[C.c_void_p(dd[k].data_ptr()) for k in ("sector", "row", "pad", "time", "adc")])
    types = dict(digit=torch.int32, sector=torch.uint8, row=torch.int16, y=torch.float32, z=torch.float32,
                 q_tot=torch.int32, q_max=torch.int32, sigma_pad=torch.float32, sigma_time=torch.float32)
    for cap in (n - 1, n // 2, 0):
        guard = 64
        out = {k: torch.full((cap + guard,), 7, dtype=t, device="cuda:0") for k, t in types.items()}
        cnt = torch.zeros(2, dtype=torch.int32, device="cuda:0")
        cl = tpc_cf_clusters(cap, C.c_void_p(cnt.data_ptr()), C.c_void_p(cnt.data_ptr() + 4),
                             *[C.c_void_p(out[k].data_ptr()) for k in CF_KEYS])
        assert lib().tpc_find_clusters(tracker.ctx, C.byref(p), C.byref(dg), C.c_void_p(ws.data_ptr()), need,
                                       C.byref(cl)) == 0
        torch.cuda.synchronize()
        assert int(cnt[0]) == n and int(cnt[1]) == 2
        g = {k: v.cpu().numpy() for k, v in out.items()}
        for k in ("digit", "sector", "row"):
            assert np.array_equal(g[k][:cap], o[k][:cap]), k
            assert np.all(g[k][cap:] == 7), k
        for k in FKEYS:
            assert np.array_equal(bits(g[k][:cap]), bits(o[k][:cap])), k
            assert np.all(g[k][cap:] == 7), k


def test_workspace_reuse_across_digit_sets(tracker):
    """The charge map is left clean after each call: different digit sets one after the other
    on the same workspace each give the oracle's clusters."""
    sets = []
    for seed in (11, 12, 13):
        _, d, _ = D.digit_config("d1", seed)
        sets.append(_arrays(d))
    for a in (sets[0], sets[1], sets[2], sets[0]):
        g = _gpu(tracker, a)
        assert g["status"] == 0
        _compare(g, O.find_clusters(*a))
