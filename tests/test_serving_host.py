"""Host logic of the serving loop, on the CPU: the Poisson chunk stream, which clusters of
each collision arrive inside a chunk's window, and the assembly of a batch (one job per
chunk: the kept clusters of its collisions with z moved by the drift of each collision's
time, then its noise clusters)."""
import numpy as np
import torch

from paper_2402_01205_amd import serve as S


def _pool(seed=1, n_coll=6):
    rng = np.random.default_rng(seed)
    cols = []
    for i in range(n_coll):
        n = 300 + 40 * i
        cols.append(dict(sec=rng.integers(0, 36, n).astype(np.uint8), row=rng.integers(0, 152, n).astype(np.int16),
                         y=rng.normal(0, 10, n).astype(np.float32),
                         z=rng.uniform(-250, 250, n).astype(np.float32)))
    return cols, S.Pool.from_collisions(cols, device="cpu")


def test_stream_is_poisson_with_bounded_chunks():
    chunks = S.make_stream(512, 4000, rate_hz=20.0, coll_range=(10, 200), seed=52)
    arr = np.array([c.arrival for c in chunks])
    assert np.all(np.diff(arr) > 0)
    gaps = np.diff(np.concatenate([[0.0], arr]))
    assert abs(gaps.mean() - 0.05) < 0.05 * 0.05 * 4          # mean 1/rate, 4 standard errors
    assert abs(np.std(gaps) / gaps.mean() - 1.0) < 0.1         # exponential: cv = 1
    m = np.array([len(c.colls) for c in chunks])
    assert m.min() >= 10 and m.max() <= 200
    for c in chunks[:50]:
        assert np.all(np.diff(c.t_coll) > 0) and c.window == len(c.colls) * 20.0
        assert np.all((c.colls >= 0) & (c.colls < 512))


def test_kept_clusters_are_those_that_arrive_inside_the_window():
    """A cluster at |z| of a collision at t_k arrives at t_k + (250 - |z|) / v_d; a chunk keeps
    exactly those arriving before its window ends, a prefix of the |z|-sorted collision."""
    cols, pool = _pool()
    chunks = S.make_stream(len(cols), 20, coll_range=(3, 6), mean_spacing_us=30.0, seed=7)
    for ch in chunks:
        S.plan_chunk(pool, ch)
        for i, c in enumerate(ch.colls):
            az = np.abs(cols[c]["z"]).astype(np.float64)
            arrive = ch.t_coll[i] + (S.DRIFT_LENGTH - az) / S.V_DRIFT
            assert ch.keep[i] == int((arrive < ch.window).sum())
        assert ch.n_signal == int(ch.keep.sum())
    assert any(0 < k < len(cols[c]["z"]) for ch in chunks for k, c in zip(ch.keep, ch.colls))


def test_assembly_of_a_batch():
    cols, pool = _pool(3)
    chunks = S.make_stream(len(cols), 4, coll_range=(2, 4), mean_spacing_us=40.0, seed=3)
    for ch in chunks:
        S.plan_chunk(pool, ch)
    ev = S.assemble(pool, chunks, None, device="cpu")
    jo = ev.job_off_host
    assert len(jo) == len(chunks) + 1 and jo[0] == 0
    assert np.array_equal(np.diff(jo), [c.n_signal + S.n_noise(c) for c in chunks])
    assert np.array_equal(ev.job_event.numpy(), np.arange(len(chunks)))
    sec, row = ev.sector.numpy(), ev.row.numpy()
    y, z = ev.y.numpy(), ev.z.numpy()
    for j, ch in enumerate(chunks):
        a = jo[j]
        for i, c in enumerate(ch.colls):
            o = np.argsort(-np.abs(cols[c]["z"]), kind="stable")[:ch.keep[i]]
            k = len(o)
            shift = np.float32(S.V_DRIFT * ch.t_coll[i])
            zs = cols[c]["z"][o]
            want_z = np.where(cols[c]["sec"][o] < 18, zs - shift, zs + shift)
            assert np.array_equal(sec[a:a + k], cols[c]["sec"][o])
            assert np.array_equal(row[a:a + k], cols[c]["row"][o])
            assert np.array_equal(y[a:a + k], cols[c]["y"][o])
            assert np.array_equal(z[a:a + k], want_z.astype(np.float32))
            a += k
        # noise: inside the acceptance, z within the drift length of its side
        b = jo[j + 1]
        assert b - a == S.n_noise(ch)
        x = 85.0 + row[a:b].astype(np.float64) * 160.0 / 151.0
        assert np.all(np.abs(y[a:b]) <= x * S.TAN10 + 1e-4)
        side = np.where(sec[a:b] < 18, 1.0, -1.0)
        assert np.all(side * z[a:b] <= S.DRIFT_LENGTH + 1e-4)
        assert np.all(side * z[a:b] >= S.DRIFT_LENGTH - S.V_DRIFT * ch.window - 1e-3)
    # the same chunks assemble to the same clusters (noise seeded per chunk)
    ev2 = S.assemble(pool, chunks, None, device="cpu")
    for k in ("sector", "row", "y", "z"):
        assert torch.equal(getattr(ev, k), getattr(ev2, k))
