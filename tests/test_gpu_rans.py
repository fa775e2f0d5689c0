"""rANS entropy coding on the GPU against the oracle, through the C ABI (needs a gfx950 GPU).

Model, lane offsets and words are integers: bit-exact with the oracle's coder on the same
streams; decoding restores every symbol.  Streams: the fields of the oracle's compression
records of a full TPC event (the coder's real input), synthetic distributions, lane and chunk
boundaries, an empty stream and a constant one (a stream of the batched workload's size is
in the full-size tests).
"""
import ctypes as C

import numpy as np
import pytest

import oracle.oracle as O
import tpcsynth as g
from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu

CHUNK = 64 * 512


@pytest.fixture(scope="module")
def tracker():
    """A context whose workspace (from one tracking run) holds streams of up to 4M symbols."""
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2402_01205_amd.tpc import DeviceClusters, Tracker
    cs = g.make_config("c2", 21, scale=4.0)
    tr = Tracker(0)
    tr.run(DeviceClusters.from_set(cs, "cuda:0"))
    tr.sync()
    say("context for streams up to", cs.n, "symbols")
    return tr, cs


def _gpu(tr, s, cap=None):
    import torch
    from paper_2402_01205_amd.tpc import TpcError
    d = torch.from_numpy(np.ascontiguousarray(s, np.uint16).view(np.int16)).to("cuda:0")
    enc = tr.tpc_rans_encode(d, cap)
    st = 0
    try:
        tr.sync()
    except TpcError as e:
        st = e.code
    out = tr.tpc_rans_decode(enc)
    tr.sync()
    return tr.rans_numpy(enc), out[:len(s)].cpu().numpy().view(np.uint16), st


def _compare(gr, ref):
    assert np.array_equal(gr["freq"], ref["freq"]), "models differ"
    assert np.array_equal(gr["lane_off"], ref["lane_off"]), "lane offsets differ"
    assert gr["n_words"] == len(ref["words"])
    assert np.array_equal(gr["words"], ref["words"]), "words differ"


def _record_streams():
    cs = g.make_config("c2", 22)
    t = O.Run.from_set(cs).tracks(merged=True)
    c = O.compress(cs.sector, cs.row, cs.y, cs.z, t, 1.0 / 32.0, 1.0 / 32.0)
    H = c["n_attached"]
    as16 = lambda a: np.ascontiguousarray(a).view(np.uint16)
    return {"rs_tracks": as16(c["rs"][:H]), "rs_free": as16(c["rs"][H:]), "ey_tracks": as16(c["ey"][:H]),
            "ey_free": as16(c["ey"][H:]), "ez_tracks": as16(c["ez"][:H]), "ez_free": as16(c["ez"][H:])}


def test_compression_record_streams_bit_exact(tracker):
    tr, _ = tracker
    for name, s in _record_streams().items():
        gr, dec, st = _gpu(tr, s)
        assert st == 0
        ref = O.rans_encode(s)
        _compare(gr, ref)
        assert np.array_equal(dec, s)
        say(name, len(s), "symbols", 16 * gr["n_words"] / max(len(s), 1), "bits/symbol")


@pytest.mark.parametrize("n", [0, 1, 63, 64, 65, CHUNK - 1, CHUNK, CHUNK + 1, 3 * CHUNK + 17])
def test_lane_and_chunk_boundaries(tracker, n):
    tr, _ = tracker
    s = np.random.default_rng(n).integers(0, 40, n).astype(np.uint16)
    gr, dec, st = _gpu(tr, s)
    assert st == 0
    _compare(gr, O.rans_encode(s))
    assert np.array_equal(dec, s)


@pytest.mark.parametrize("kind", ["uniform", "const", "two", "all_symbols"])
def test_extreme_distributions(tracker, kind):
    tr, _ = tracker
    rng = np.random.default_rng(9)
    s = {"uniform": lambda: rng.integers(0, 65536, 300000).astype(np.uint16),
         "const": lambda: np.full(100001, 65535, np.uint16),
         "two": lambda: rng.choice(np.array([0, 65535], np.uint16), 200000, p=[0.999, 0.001]),
         "all_symbols": lambda: rng.permutation(65536 * 3).astype(np.uint32).astype(np.uint16)}[kind]()
    gr, dec, st = _gpu(tr, s)
    assert st == 0
    _compare(gr, O.rans_encode(s))
    assert np.array_equal(dec, s)


def test_word_capacity(tracker):
    """Too small a word buffer: TPC_E_CAPACITY, the words needed reported, nothing written
    beyond the capacity."""
    import torch
    from paper_2402_01205_amd.tpc import TPC_E_CAPACITY, TpcError, lib, tpc_rans
    tr, _ = tracker
    s = np.clip(np.rint(np.random.default_rng(4).normal(0, 5, 200000)), -99, 99).astype(np.int16).view(np.uint16)
    ref = O.rans_encode(s)
    need = len(ref["words"])
    dev = "cuda:0"
    for cap in (need - 1, need // 3, 0):
        guard = 64
        buf = dict(n_words=torch.zeros(1, dtype=torch.int32, device=dev),
                   freq=torch.zeros(1 << 16, dtype=torch.int32, device=dev),
                   lane_off=torch.zeros(O.rans_lanes(len(s)) + 1, dtype=torch.int32, device=dev),
                   words=torch.full((cap + guard,), 0x5A5A, dtype=torch.int16, device=dev))
        st = tpc_rans(cap, *[C.c_void_p(buf[k].data_ptr()) for k in ("n_words", "freq", "lane_off", "words")])
        d = torch.from_numpy(s.view(np.int16)).to(dev)
        assert lib().tpc_rans_encode(tr.ctx, C.c_void_p(d.data_ptr()), len(s), C.byref(st)) == 0
        with pytest.raises(TpcError) as e:
            tr.sync()
        assert e.value.code == TPC_E_CAPACITY
        assert int(buf["n_words"].item()) == need
        w = buf["words"].cpu().numpy().view(np.uint16)
        assert np.array_equal(w[:cap], ref["words"][:cap])
        assert np.all(w[cap:] == 0x5A5A)
        assert np.array_equal(buf["lane_off"].cpu().numpy().view(np.uint32), ref["lane_off"])
