"""Pins of the oracle's rANS entropy coder (section 5: the common ANS compression that every
detector's data goes through; Tables 1 and 2 time its TPC encoding and decoding).

Checked against what the definition of range ANS fixes: exact round trips; the model's
normalisation (sum 2^16, every symbol that occurs keeps a slot, the remainder to the most
frequent symbol); per-lane sizes within a few words of the information content of the lane
under the model (a coder that drops or misuses the model cannot meet both bounds); and closed
forms: a constant stream costs only the final states, a stream using all 65536 symbols once
costs exactly one word per symbol.
"""
import numpy as np
import pytest

import oracle.oracle as O

S = O.RANS_LANE_SYMBOLS
CHUNK = 64 * S


def _streams():
    rng = np.random.default_rng(3)
    g = np.clip(np.rint(rng.normal(0, 3, 70000)), -32768, 32767).astype(np.int16).view(np.uint16)
    heavy = (rng.geometric(0.02, 50000) % 65536).astype(np.uint16)
    uni = rng.integers(0, 65536, 40000).astype(np.uint16)
    two = rng.choice(np.array([7, 60000], np.uint16), 30001, p=[0.99, 0.01])
    return dict(gauss=g, heavy=heavy, uniform=uni, two=two, const=np.full(CHUNK + 3, 42, np.uint16))


@pytest.mark.parametrize("name", ["gauss", "heavy", "uniform", "two", "const"])
def test_round_trip_is_exact(name):
    s = _streams()[name]
    e = O.rans_encode(s)
    assert np.array_equal(O.rans_decode(e, len(s)), s)


@pytest.mark.parametrize("n", [0, 1, 2, 63, 64, 65, CHUNK - 1, CHUNK, CHUNK + 1, 3 * CHUNK + 17])
def test_round_trip_at_lane_and_chunk_boundaries(n):
    rng = np.random.default_rng(n)
    s = rng.integers(0, 40, n).astype(np.uint16)
    e = O.rans_encode(s)
    assert len(e["lane_off"]) == O.rans_lanes(n) + 1
    assert O.rans_lanes(n) == 64 * ((n + CHUNK - 1) // CHUNK)
    assert np.all(np.diff(e["lane_off"].astype(np.int64)) >= 0)
    assert np.array_equal(O.rans_decode(e, n), s)


def test_model_normalisation():
    rng = np.random.default_rng(5)
    s = np.clip(np.rint(rng.normal(100, 40, 200000)), 0, 65535).astype(np.uint16)
    f = O.rans_model(s).astype(np.int64)
    c = np.bincount(s, minlength=65536).astype(np.int64)
    assert f.sum() == 1 << 16
    assert np.array_equal(f > 0, c > 0)
    K = int((c > 0).sum())
    ideal = c * ((1 << 16) - K) // len(s)
    top = int(np.argmax(c))          # first maximum: the smaller symbol on ties
    rest = np.arange(65536) != top
    assert np.array_equal(f[rest], np.where(c[rest] > 0, np.maximum(1, ideal[rest]), 0))
    assert f[top] == (1 << 16) - f[rest].sum()


def test_model_closed_forms():
    # two symbols, equal counts: floor(n/2 (2^16 - 2) / n) = 32767 each, the 2 left over to
    # the smaller symbol
    s = np.array([9, 3] * 500, np.uint16)
    f = O.rans_model(s)
    assert f[3] == 32769 and f[9] == 32767 and f.sum() == 65536
    # one symbol: the whole range
    f = O.rans_model(np.full(10, 5, np.uint16))
    assert f[5] == 65536 and f.sum() == 65536
    # every symbol once: one slot each
    f = O.rans_model(np.arange(65536, dtype=np.uint16))
    assert np.all(f == 1)


def test_lane_sizes_track_the_information_content():
    """With I the information of a lane's symbols under the model (sum of log2(2^16 / f_s)):
    the state starts at 2^16 and ends in [2^16, 2^32) and is flushed as 32 bits, so the lane
    takes I + 16 + (32 - log2 of the final state) bits, up to the floor rounding of each
    step (a small fraction of a bit per symbol either way)."""
    for name, s in _streams().items():
        e = O.rans_encode(s)
        f = e["freq"].astype(np.float64)
        info = np.log2(65536.0 / np.where(f > 0, f, 1.0))
        n = len(s)
        for l in range(O.rans_lanes(n)):
            k, j = divmod(l, 64)
            idx = np.arange(k * CHUNK + j, min(n, (k + 1) * CHUNK), 64)
            bits = 16 * int(e["lane_off"][l + 1] - e["lane_off"][l])
            if len(idx) == 0:
                assert bits == 0
                continue
            I = float(info[s[idx]].sum())
            assert I + 8 <= bits <= I + 32 + 0.02 * len(idx), (name, l, bits, I)


def test_closed_form_sizes():
    # constant stream: no word is ever emitted, each lane holds its final state only
    n = 2 * CHUNK + 5
    e = O.rans_encode(np.full(n, 1234, np.uint16))
    active = sum(1 for l in range(O.rans_lanes(n)) if l % 64 < 64 and (l // 64) * CHUNK + l % 64 < n)
    assert len(e["words"]) == 2 * active
    # all 65536 symbols once (f = 1 each): exactly one word per symbol plus the states
    s = np.random.default_rng(8).permutation(65536).astype(np.uint16)
    e = O.rans_encode(s)
    assert len(e["words"]) == 65536 + 2 * O.rans_lanes(65536)
    assert np.array_equal(O.rans_decode(e, 65536), s)
