"""The rANS encoder that allocates nothing (tpc_rans_encode_static) against tpc_rans_encode,
through the C ABI (needs a gfx950 GPU).

Both entry points run the same kernels; the static one keeps its intermediate buffers in the
library's fixed device array instead of a context workspace.  Model, lane offsets, word count
and words must be identical, bit for bit, on two calls in a row (the second on a smaller
stream, so that leftovers of the first in the shared array would show), on a context that
never ran a tracking stage, and at the size limit; beyond it the call fails on the host.
"""
import numpy as np
import pytest

from tests.gpu_helpers import say

pytestmark = pytest.mark.gpu


def _stream(rng, n, kind):
    if kind == "geometric":
        v = np.minimum(rng.geometric(0.05, n), 3000) * np.where(rng.random(n) < 0.5, -1, 1)
        return v.astype(np.int16).view(np.uint16)
    return rng.integers(0, 1 << 16, n, dtype=np.uint16)


def _dev(s):
    import torch
    return torch.from_numpy(np.ascontiguousarray(s).view(np.int16)).to("cuda:0")


def _host(enc):
    """Word count, model, the stream's lane offsets and the words written."""
    import torch

    from paper_2402_01205_amd.tpc import lib
    torch.cuda.synchronize()
    m = min(int(enc["n_words"].item()), enc["cap_words"])
    lanes = int(lib().tpc_rans_lanes(enc["n"]))
    return (int(enc["n_words"].item()), enc["freq"].cpu().numpy().view(np.uint32).copy(),
            enc["lane_off"][:lanes + 1].cpu().numpy().view(np.uint32).copy(),
            enc["words"][:m].cpu().numpy().view(np.uint16).copy())


def _same(a, b, what):
    assert a[0] == b[0], f"{what}: word counts differ"
    assert np.array_equal(a[1], b[1]), f"{what}: models differ"
    assert np.array_equal(a[2], b[2]), f"{what}: lane offsets differ"
    assert np.array_equal(a[3], b[3]), f"{what}: words differ"


@pytest.fixture(scope="module")
def trackers():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import tpcsynth as g
    from paper_2402_01205_amd.tpc import DeviceClusters, Tracker
    cs = g.make_config("c2", 21, scale=4.5)         # > 4194304 clusters: streams up to the limit
    assert cs.n >= 4194304
    ref = Tracker(0)
    ref.run(DeviceClusters.from_set(cs, "cuda:0"))    # workspace for streams of up to cs.n symbols
    ref.sync()
    fresh = Tracker(0)                                 # no tracking run: no workspace at all
    say("reference context for streams up to", cs.n, "symbols")
    return ref, fresh, cs.n


def test_static_encoder_equals_workspace_encoder_on_two_calls(trackers):
    ref, fresh, nmax = trackers
    rng = np.random.default_rng(77)
    big = min(nmax, 2_500_001)
    outs = fresh.rans_outputs(big)                     # caller-owned outputs, allocated once
    for n, kind in ((big, "geometric"), (123_457, "uniform")):
        s = _stream(rng, n, kind)
        d = _dev(s)
        say("static encode", kind, n, "symbols")
        a = _host(ref.tpc_rans_encode(d))
        ref.sync()
        b = _host(fresh.tpc_rans_encode_static(d, outs))
        fresh.sync()
        _same(a, b, f"{kind} stream of {n}")
        dec = ref.tpc_rans_decode(outs)
        ref.sync()
        assert np.array_equal(dec[:n].cpu().numpy().view(np.uint16), s)


def test_static_encoder_on_the_context_that_tracked(trackers):
    """The same context may use both entry points; the static call leaves its workspace alone."""
    ref, _, _ = trackers
    rng = np.random.default_rng(78)
    s = _stream(rng, 70_000, "geometric")
    d = _dev(s)
    a = _host(ref.tpc_rans_encode(d))
    b = _host(ref.tpc_rans_encode_static(d, ref.rans_outputs(len(s))))
    ref.sync()
    _same(a, b, "same context")


def test_static_encoder_at_its_limit_and_beyond(trackers):
    import torch

    from paper_2402_01205_amd.tpc import TPC_E_ARG, lib
    ref, fresh, _ = trackers
    nmax = 4194304
    s = _stream(np.random.default_rng(79), nmax, "geometric")
    d = _dev(s)
    say("static encode at the limit:", nmax, "symbols")
    a = _host(ref.tpc_rans_encode(d))
    ref.sync()
    enc = fresh.rans_outputs(nmax)
    b = _host(fresh.tpc_rans_encode_static(d, enc))
    fresh.sync()
    _same(a, b, "stream at the limit")
    dec = torch.zeros(nmax, dtype=torch.int16, device="cuda:0")
    ref.tpc_rans_decode(enc, dec)
    ref.sync()
    assert np.array_equal(dec.cpu().numpy().view(np.uint16), s)
    tr = fresh
    # one symbol over the limit: rejected on the host before anything is enqueued
    import ctypes as C
    small = tr.rans_outputs(1)
    rc = lib().tpc_rans_encode_static(tr.ctx, C.c_void_p(_dev(s[:1]).data_ptr()), nmax + 1, C.byref(small["_s"]))
    assert rc == TPC_E_ARG
    assert b"TPC_RANS_STATIC_MAX_SYMBOLS" in lib().tpc_last_error(tr.ctx)


def test_static_encoder_reports_capacity(trackers):
    from paper_2402_01205_amd.tpc import TPC_E_CAPACITY, TpcError
    _, fresh, _ = trackers
    s = _stream(np.random.default_rng(80), 50_000, "uniform")
    d = _dev(s)
    full = _host(fresh.tpc_rans_encode_static(d, fresh.rans_outputs(len(s))))
    fresh.sync()
    small = fresh.rans_outputs(len(s), cap_words=1000)
    fresh.tpc_rans_encode_static(d, small)
    with pytest.raises(TpcError) as e:
        fresh.sync()
    assert e.value.code == TPC_E_CAPACITY
    got = _host(small)
    assert got[0] == full[0] and np.array_equal(got[3], full[3][:1000])
    # the next call clears the status word
    fresh.tpc_rans_encode_static(d, fresh.rans_outputs(len(s)))
    fresh.sync()
