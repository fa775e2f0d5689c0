"""Pins of the CPU oracle against what mathematics and physics fix.

Each test checks the oracle against something other than itself: the helix
closed form, finite differences, the information-form Kalman identity, libm's
asin, a brute-force neighbour search, whole-row scans in place of the window searches'
z ranges, invariants of the cellular automaton and of the ownership arbitration, and
zero-smear special cases.
"""
import math

import numpy as np
import pytest

import oracle.oracle as O
import tpcsynth as g
from paper_2402_01205_amd.evaluate import quality
from tests.truth import true_state

ROWX32 = np.array([np.float32(85.0 + r * 160.0 / 151.0) for r in range(152)], np.float32)


def test_row_geometry():
    for r in (0, 1, 75, 151):
        assert O.row_x(r) == ROWX32[r]
    assert abs(float(ROWX32[151]) - 245.0) < 1e-5


# ------------------------------------------------------------------ asin(u)/u
def test_asinc_fp32_against_libm():
    us = np.concatenate([np.linspace(-0.999, 0.999, 20001), [1e-8, -1e-8, 0.5, -0.5, 0.49999, 0.50001]])
    for u in us.astype(np.float32):
        A, B = O.asinc(float(u))
        ud = float(u)
        Aref = math.asin(ud) / ud if ud != 0 else 1.0
        # series branch: a few ulp; range-reduced branch (|u| > 1/2): within 5e-7
        assert abs(A - Aref) <= (2.5e-7 if abs(ud) <= 0.5 else 5e-7) * Aref, (u, A, Aref)
        if abs(ud) > 1e-3:
            Bref = (1.0 / math.sqrt(1 - ud * ud) - Aref) / (ud * ud)
            assert abs(B - Bref) <= 2e-5 * Bref, (u, B, Bref)


def test_asinc_fp64_series_branch():
    for u in (1e-6, 1e-3, 0.0499, 0.0501, 0.3, -0.7, 0.95):
        A, B = O.asinc(u, fp64=True)
        Aref = math.asin(u) / u
        assert abs(A - Aref) <= 4e-16 * Aref
        Bref = (1.0 / math.sqrt(1 - u * u) - Aref) / (u * u) if abs(u) > 0.02 else 1 / 3 + 0.3 * u * u
        assert abs(B - Bref) <= (1e-12 if abs(u) > 0.02 else 1e-7) * Bref


# ------------------------------------------------------------------ propagation
def _particles(n, seed):
    rng = np.random.default_rng(seed)
    pt = np.exp(rng.uniform(np.log(0.15), np.log(10.0), n))
    eta = rng.uniform(-0.9, 0.9, n)
    phi = rng.uniform(0.02, 0.33, n)  # sector 0 (A) or 18 (C) by the sign of eta
    q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return pt, eta, phi, q


@pytest.mark.parametrize("seed", [1, 2])
def test_propagation_matches_closed_form_helix(seed):
    pt, eta, phi, q = _particles(200, seed)
    prm = O.params(smax=0.999)
    n_checked = 0
    for i in range(len(pt)):
        sec = 0 if eta[i] >= 0 else 18
        for r1, r2 in ((0, 1), (10, 40), (60, 20), (100, 151), (151, 0)):
            x1, x2 = float(ROWX32[r1]), float(ROWX32[r2])
            ok1, y1, z1, s1, t1, k1 = true_state(pt[i], eta[i], phi[i], q[i], sec, x1)
            ok2, y2, z2, s2, t2, k2 = true_state(pt[i], eta[i], phi[i], q[i], sec, x2)
            if not (ok1 and ok2) or abs(s1) > 0.99 or abs(s2) > 0.99:
                continue
            P = [y1, z1, s1, t1, k1]
            ok, Pn, _ = O.propagate(P, np.eye(5)[np.tril_indices(5)], x1, x2, prm, fp64=True)
            assert ok
            hi, lo = Pn[:5], Pn[5:]
            got = hi + lo
            assert abs(got[0] - y2) < 1e-9 and abs(got[1] - z2) < 1e-9, (i, r1, r2, got, y2, z2)
            assert abs(got[2] - s2) < 1e-12 and got[3] == t1 and got[4] == k1
            n_checked += 1
    assert n_checked > 500


def test_propagation_invariants_and_failure():
    # a track turning over: |sin phi| reaching smax fails and leaves the state untouched
    P = [1.0, 2.0, 0.9, 0.3, -9.0]  # curvature C = -kappa B k > 0 turns s towards +1
    Cv = np.eye(5)[np.tril_indices(5)]
    ok, Pn, Cn = O.propagate(P, Cv, 85.0, 140.0, O.params(), fp64=True)
    assert not ok and np.allclose(Pn[:5], P) and np.allclose(Cn, Cv)
    # dx = 0 is the identity
    ok, Pn, Cn = O.propagate(P, Cv, 100.0, 100.0, O.params(), fp64=True)
    assert ok and np.allclose(Pn[:5], P) and np.allclose(Cn, Cv)


def _jac_from_transport(P, x1, x2, prm):
    """Column a of J from transporting C = e_a e_a^T (J has a unit diagonal)."""
    J = np.zeros((5, 5))
    for a in range(5):
        E = np.zeros((5, 5))
        E[a, a] = 1.0
        ok, _, Cn = O.propagate(P, O.full_to_tri(E), x1, x2, prm, fp64=True)
        assert ok
        M = O.tri_to_full(Cn)
        J[:, a] = M[:, a] / math.sqrt(M[a, a])
    return J


@pytest.mark.parametrize("state,x1,x2", [
    ([3.0, 10.0, 0.2, 0.5, 1.7], 100.0, 101.06),
    ([-5.0, -40.0, -0.6, -0.8, -6.0], 150.0, 160.6),
    ([12.0, 80.0, 0.4, 0.3, 0.1], 200.0, 180.0),
    ([1.0, 5.0, 0.05, 0.1, -9.5], 90.0, 120.0),
    ([0.0, 0.0, 0.0, 0.0, 0.0], 85.0, 245.0),
])
def test_jacobian_against_finite_differences(state, x1, x2):
    prm = O.params(smax=0.999)
    J = _jac_from_transport(state, x1, x2, prm)
    Jfd = np.zeros((5, 5))
    for a in range(5):
        hstep = 1e-6 * max(1.0, abs(state[a]))
        pp = np.array(state, float); pp[a] += hstep
        pm = np.array(state, float); pm[a] -= hstep
        okp, Pp, _ = O.propagate(pp, np.zeros(15), x1, x2, prm, fp64=True)
        okm, Pm, _ = O.propagate(pm, np.zeros(15), x1, x2, prm, fp64=True)
        assert okp and okm
        Jfd[:, a] = ((Pp[:5] + Pp[5:]) - (Pm[:5] + Pm[5:])) / (2 * hstep)
    assert np.allclose(J, Jfd, rtol=1e-6, atol=1e-7), (J, Jfd)


def test_transport_is_J_C_Jt():
    prm = O.params(smax=0.999)
    state = [2.0, 30.0, 0.3, -0.4, 2.5]
    J = _jac_from_transport(state, 120.0, 131.0, prm)
    rng = np.random.default_rng(0)
    A = rng.normal(size=(5, 5))
    Cf = A @ A.T + np.eye(5)
    ok, _, Cn = O.propagate(state, O.full_to_tri(Cf), 120.0, 131.0, prm, fp64=True)
    assert ok
    assert np.allclose(O.tri_to_full(Cn), J @ Cf @ J.T, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ sector rotation (O10)
def _rotated_at_plane(P, x, frm, to, xn0, prm):
    """Rotate into sector `to`, then move along the helix to the plane x' = xn0:
    the state map whose derivative the rotation's covariance transform must be."""
    ok, Pr, _, xn = O.rotate(P, np.zeros(15), x, frm, to, prm, fp64=True)
    assert ok
    ok, Pp, _ = O.propagate(Pr, np.zeros(15), xn, xn0, prm, fp64=True)
    assert ok
    return Pp[:5] + Pp[5:]


def _jac_from_rotation(P, x, frm, to, prm):
    """Column a of J from rotating C = e_a e_a^T (every diagonal entry of J is > 0)."""
    J = np.zeros((5, 5))
    for a in range(5):
        E = np.zeros((5, 5))
        E[a, a] = 1.0
        ok, _, Cn, _ = O.rotate(P, O.full_to_tri(E), x, frm, to, prm, fp64=True)
        assert ok
        M = O.tri_to_full(Cn)
        J[:, a] = M[:, a] / math.sqrt(M[a, a])
    return J


@pytest.mark.parametrize("state,x,frm,to", [
    ([30.0, 40.0, 0.3, 0.5, 5.0], 180.0, 0, 1),     # leaves through +y, positive curvature term
    ([30.0, 40.0, 0.3, 0.5, -5.0], 180.0, 0, 1),
    ([-35.0, -60.0, -0.4, -0.7, 8.0], 220.0, 19, 18),  # side C, through -y
    ([-20.0, 10.0, -0.2, 0.1, -9.5], 120.0, 17, 16),
    ([40.0, 100.0, 0.5, 0.9, 2.0], 240.0, 17, 0),    # wraps 17 -> 0
    ([-42.0, -5.0, -0.35, -0.2, -3.0], 238.0, 0, 17),   # wraps 0 -> 17
])
def test_rotation_jacobian_against_finite_differences(state, x, frm, to):
    """O10: the covariance transform of the sector rotation is the derivative of the
    map 'rotate, then move back along the helix to the rotated nominal plane'
    (central differences of the exact FP64 state map, propagation pinned above)."""
    prm = O.params(smax=0.999)
    ok, _, _, xn0 = O.rotate(state, np.zeros(15), x, frm, to, prm, fp64=True)
    assert ok
    J = _jac_from_rotation(state, x, frm, to, prm)
    Jfd = np.zeros((5, 5))
    for a in range(5):
        hstep = 1e-6 * max(1.0, abs(state[a]))
        pp = np.array(state, float); pp[a] += hstep
        pm = np.array(state, float); pm[a] -= hstep
        Jfd[:, a] = (_rotated_at_plane(pp, x, frm, to, xn0, prm)
                     - _rotated_at_plane(pm, x, frm, to, xn0, prm)) / (2 * hstep)
    assert np.allclose(J, Jfd, rtol=1e-6, atol=1e-8), (J, Jfd)
    # the curvature term is really there (k != 0 in every case above)
    assert abs(J[2, 0]) > 1e-4


def test_rotation_is_J_C_Jt():
    prm = O.params(smax=0.999)
    state, x = [25.0, -30.0, 0.25, -0.6, -4.0], 200.0
    J = _jac_from_rotation(state, x, 3, 4, prm)
    rng = np.random.default_rng(1)
    A = rng.normal(size=(5, 5))
    Cf = A @ A.T + np.eye(5)
    ok, _, Cn, _ = O.rotate(state, O.full_to_tri(Cf), x, 3, 4, prm, fp64=True)
    assert ok
    assert np.allclose(O.tri_to_full(Cn), J @ Cf @ J.T, rtol=1e-12, atol=1e-12)


def test_rotation_there_and_back_is_identity():
    """Turning into the neighbour sector and back returns the state (up to the FP32
    rounding of the cos 20 / sin 20 table values, ~1e-7 relative)."""
    prm = O.params(smax=0.999)
    state, x = np.array([30.0, 40.0, 0.3, 0.5, 5.0]), 180.0
    ok, P1, _, x1 = O.rotate(state, np.zeros(15), x, 5, 6, prm, fp64=True)
    ok2, P2, _, x2 = O.rotate(P1, np.zeros(15), x1, 6, 5, prm, fp64=True)
    assert ok and ok2
    assert abs(x2 - x) < 1e-6
    assert np.allclose(P2[:5] + P2[5:], state, rtol=0, atol=1e-6)


def test_rotation_rejects_non_adjacent_and_other_side():
    prm = O.params()
    for frm, to in [(0, 2), (0, 18), (3, 3), (20, 5)]:
        ok, *_ = O.rotate([1.0, 1.0, 0.1, 0.1, 1.0], np.eye(5)[np.tril_indices(5)], 150.0, frm, to, prm, fp64=True)
        assert not ok


# ------------------------------------------------------------------ Kalman update
@pytest.mark.parametrize("seed", range(5))
def test_update_equals_information_form(seed):
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(5, 5))
    Cf = A @ A.T * 0.1 + np.diag([0.5, 0.5, 0.01, 0.01, 0.3])
    P = rng.normal(size=5) * [10, 50, 0.3, 0.5, 2]
    P[2] = np.clip(P[2], -0.5, 0.5)
    m = P[:2] + rng.normal(size=2) * 0.3
    prm = O.params()
    V = np.diag([prm.sigma_y ** 2, prm.sigma_z ** 2]).astype(np.float64)
    V = np.diag([float(np.float32(prm.sigma_y)) ** 2, float(np.float32(prm.sigma_z)) ** 2])
    ok, Pn, Cn, chi2 = O.update(P, O.full_to_tri(Cf), m[0], m[1], prm, fp64=True)
    assert ok
    H = np.zeros((2, 5)); H[0, 0] = H[1, 1] = 1
    Ci = np.linalg.inv(Cf)
    Cinfo = np.linalg.inv(Ci + H.T @ np.linalg.inv(V) @ H)
    Pinfo = Cinfo @ (Ci @ P + H.T @ np.linalg.inv(V) @ m)
    r = m - H @ P
    chi2_ref = r @ np.linalg.inv(H @ Cf @ H.T + V) @ r
    assert np.allclose(Pn[:5] + Pn[5:], Pinfo, rtol=1e-10, atol=1e-10)
    assert np.allclose(O.tri_to_full(Cn), Cinfo, rtol=1e-9, atol=1e-12)
    assert abs(chi2 - chi2_ref) <= 1e-9 * max(1.0, chi2_ref)


def test_update_rejects_non_positive_innovation():
    Cv = np.zeros(15)
    Cv[0] = -1.0  # S00 = -1 + sigma^2 < 0 => det < 0
    ok, Pn, Cn, _ = O.update([0, 0, 0, 0, 0], Cv, 1.0, 1.0, O.params(), fp64=True)
    assert not ok and np.all(Pn == 0)


# ------------------------------------------------------------------ neighbours
def _slab(cs, sector, zlo, zhi, ymax=1e9):
    m = (cs.sector == sector) & (cs.z >= zlo) & (cs.z < zhi) & (np.abs(cs.y) < ymax)
    idx = np.nonzero(m)[0]
    return (cs.sector[idx], cs.row[idx], cs.y[idx], cs.z[idx], cs.label[idx])


def brute_force_links(sector, row, y, z, prm):
    """All (d, h, u) triples by exhaustive enumeration (no row lists, no z search)."""
    n = len(y)
    f32 = np.float32
    up = np.full(n, -1, np.int32)
    dn = np.full(n, -1, np.int32)
    idx = np.arange(n)
    cut2 = f32(prm.link_cut) * f32(prm.link_cut)
    for h in range(n):
        r = int(row[h])
        for d in (1, 2):
            if r - d < 0 or r + d > 151:
                break
            dxu = ROWX32[r + d] - ROWX32[r]
            wy = f32(prm.win_dy_slope) * dxu + f32(prm.win_dy_const)
            wz = f32(prm.win_dz_slope) * dxu + f32(prm.win_dz_const)
            rho = ROWX32[r + d] / ROWX32[r]
            yc = y[h] * rho
            U = idx[(sector == sector[h]) & (row == r + d)]
            U = U[(np.abs(y[U] - yc) <= wy) & (np.abs(z[U] - z[h]) <= wz)]
            D = idx[(sector == sector[h]) & (row == r - d)]
            if U.size == 0 or D.size == 0:
                continue
            uu, dd = np.meshgrid(U, D, indexing="ij")
            ry = (y[uu] + y[dd]) - (y[h] + y[h])
            rz = (z[uu] + z[dd]) - (z[h] + z[h])
            sc = ry * ry + rz * rz
            ok = sc <= cut2
            if not ok.any():
                continue
            sc, uu, dd = sc[ok], uu[ok], dd[ok]
            o = np.lexsort((dd, uu, sc))[0]
            up[h], dn[h] = uu[o], dd[o]
            break
    return up, dn


@pytest.mark.parametrize("case", ["c1", "c2", "c3", "c4dense"])
def test_neighbours_equal_brute_force(case):
    if case == "c1":
        cs = g.make_config("c1", 13)
        sec, row, y, z, _ = _slab(cs, 0, 0.0, 25.0)
    elif case == "c2":
        cs = g.make_config("c2", 22)
        sec, row, y, z, _ = _slab(cs, 5, 40.0, 54.0)
    elif case == "c3":
        pool = g.gen_collision_pool(33, 6)
        cs = g.assemble_timeframe(34, pool, np.arange(6), 120.0)
        sec, row, y, z, _ = _slab(cs, 20, -10.0, 0.0)
    else:
        cs = g.make_config("c4", 41, jobs=[int(np.argmax(g.c4_job_sizes(41)))])
        zm = float(np.median(cs.z))
        sec, row, y, z, _ = _slab(cs, int(cs.sector[0]), zm, zm + 1.2, ymax=4.0)
    assert 300 < len(y) <= 2500, len(y)
    prm = O.params()
    jo = np.array([0, len(y)], np.int32)
    ref_up, ref_dn = brute_force_links(sec, row, y, z, prm)
    for brute in (False, True):
        L = O.Run(sec, row, y, z, jo, prm, last_stage=O.STAGE_LINKS, brute=brute).links()
        assert np.array_equal(L["up_raw"], ref_up)
        assert np.array_equal(L["down_raw"], ref_dn)
    assert (ref_up >= 0).mean() > 0.5


@pytest.mark.parametrize("case,preset", [("c1", "default"), ("c2loopers", "default"), ("c2loopers", "sync"),
                                         ("c2loopers", "async"), ("c4medium", "sync")])
def test_window_searches_equal_whole_row_scans(case, preset):
    """The following's and the extension's window searches visit only the clusters of the row
    whose z lies in the window (a binary search in the z-sorted row); scanning every cluster
    of the row instead (the plain definition: the minimum chi2 inside the window) gives the
    same links, tracklets and tracks, merged and extended, bit for bit."""
    if case == "c1":
        cs = g.make_config("c1", 21)
    elif case == "c2loopers":
        cs = g.make_config("c2", 21, scale=0.05, loopers=True)
    else:
        sizes = g.c4_job_sizes(41)
        cs = g.make_config("c4", 41, jobs=[int(np.argsort(sizes)[len(sizes) // 2])])
    prm = O.params(**{"default": O.DEFAULTS, "sync": O.SYNC, "async": O.ASYNC}[preset])
    a = O.Run.from_set(cs, prm)
    b = O.Run.from_set(cs, prm, brute=True)
    ta, tb = a.tracklets(), b.tracklets()
    for k in ("start", "off", "hits", "hitw"):
        assert np.array_equal(ta[k], tb[k]), k
    ka, kb = a.tracks(), b.tracks()
    for k in ("off", "hits", "tracklet", "P", "C", "x", "ndf", "n_ext", "t0"):
        assert np.array_equal(ka[k], kb[k], equal_nan=True), k
    assert len(ka["ndf"]) > 50
    if preset == "sync":
        assert int(ka["n_ext"].sum()) > 0


# ------------------------------------------------------------------ CA invariants
@pytest.fixture(scope="module")
def c2_run():
    cs = g.make_config("c2", 23, scale=0.3)
    return cs, O.Run.from_set(cs, last_stage=O.STAGE_FIT)


def test_link_cleaning_and_starts(c2_run):
    cs, r = c2_run
    L = r.links()
    up, dn, ur, dr = L["up"], L["down"], L["up_raw"], L["down_raw"]
    n = cs.n
    h = np.nonzero(up >= 0)[0]
    assert np.all(dn[up[h]] == h)                     # mutual
    assert np.all(ur[h] == up[h]) and np.all(dr[up[h]] == h)
    k = np.nonzero((ur >= 0) & (up < 0))[0]
    assert np.all(dr[ur[k]] != k)                      # dropped links were not mutual
    assert np.all(cs.row[up[h]] > cs.row[h]) and np.all(cs.row[up[h]] - cs.row[h] <= 2)
    T = r.tracklets()
    st = T["start"]
    assert np.all(np.diff(st) > 0)                     # ids ascend with the start index
    exp = np.nonzero((dn < 0) & (up >= 0) & (np.where(up >= 0, up[np.maximum(up, 0)], -1) >= 0))[0]
    assert np.array_equal(st, exp)
    # chains are disjoint: every cluster is on at most one chain
    seen = np.zeros(n, np.int32)
    for s in st:
        c = s
        while c >= 0:
            seen[c] += 1
            c = up[c]
    assert seen.max() == 1


def test_tracklets_follow_chain_and_rows(c2_run):
    cs, r = c2_run
    L = r.links()
    T = r.tracklets()
    for i in range(0, len(T["start"]), 7):
        hits = T["hits"][T["off"][i]:T["off"][i + 1]]
        if hits.size == 0:
            continue
        st = T["start"][i]
        d = L["down_raw"][st]
        first = d if (d >= 0 and L["up_raw"][d] < 0) else st
        assert hits[0] == first
        assert np.all(np.diff(cs.row[hits]) > 0)
        assert np.all(cs.sector[hits] == cs.sector[hits[0]])
        # the chain prefix is the up-link chain from the start
        if first != st:
            hits = hits[1:]
        c, k = hits[0], 0
        while c >= 0 and k < hits.size:
            if hits[k] != c:
                break
            c, k = L["up"][c], k + 1
        assert k >= min(3, hits.size)


def test_ownership_and_selection(c2_run):
    cs, r = c2_run
    T = r.tracklets()
    K = r.tracks(merged=False)
    w = T["hitw"]
    used = np.zeros(cs.n, np.int32)
    np.add.at(used, K["hits"], 1)
    assert used.max() <= 1                             # one owner per cluster
    prm = O.params()
    for t in range(len(K["tracklet"])):
        tid = K["tracklet"][t]
        th = T["hits"][T["off"][tid]:T["off"][tid + 1]]
        kh = K["hits"][K["off"][t]:K["off"][t + 1]]
        key = (np.uint64(len(th)) << np.uint64(32)) | np.uint64(0xFFFFFFFF - int(tid))
        assert np.array_equal(kh, th[w[th] == key])
        assert len(kh) >= prm.min_hits
    # hit weights are the max key over the valid tracklets containing the hit
    ref = np.zeros(cs.n, np.uint64)
    for tid in range(len(T["start"])):
        th = T["hits"][T["off"][tid]:T["off"][tid + 1]]
        if len(th) >= prm.min_hits:
            key = (np.uint64(len(th)) << np.uint64(32)) | np.uint64(0xFFFFFFFF - int(tid))
            ref[th] = np.maximum(ref[th], key)
    assert np.array_equal(ref, w)


def test_results_invariant_under_input_permutation():
    cs = g.make_config("c2", 21, scale=0.15)
    r1 = O.Run.from_set(cs)
    rng = np.random.default_rng(9)
    p = rng.permutation(cs.n)
    r2 = O.Run(cs.sector[p], cs.row[p], cs.y[p], cs.z[p], cs.job_off)
    K1, K2 = r1.tracks(), r2.tracks()
    s1 = {tuple(sorted(K1["hits"][K1["off"][i]:K1["off"][i + 1]])) for i in range(len(K1["tracklet"]))}
    s2 = {tuple(sorted(p[K2["hits"][K2["off"][i]:K2["off"][i + 1]]])) for i in range(len(K2["tracklet"]))}
    assert s1 == s2 and len(s1) > 100


def test_invalid_clusters_are_excluded_and_flagged():
    cs = g.make_config("c1", 11)
    sec, row, y, z = cs.sector.copy(), cs.row.copy(), cs.y.copy(), cs.z.copy()
    row[5] = 200
    sec[6] = 40
    y[7] = np.nan
    r = O.Run(sec, row, y, z, cs.job_off)
    assert r.status & 1
    L = r.links()
    for i in (5, 6, 7):
        assert L["up_raw"][i] == -1 and L["down_raw"][i] == -1
        assert i not in set(L["up_raw"]) and i not in set(L["down_raw"])


# ------------------------------------------------------------------ tracking sanity
def test_zero_smear_single_sector_is_perfect():
    cs = g.gen_event(11, 200, sector=0, smear=0.0)
    r = O.Run.from_set(cs)
    K = r.tracks()
    q = quality(cs.label, cs.job_off, cs.sector, K["off"], K["hits"])
    assert q["efficiency"] == 1.0 and q["fake_rate"] == 0.0
    # every track is pure
    for t in range(len(K["tracklet"])):
        lab = cs.label[K["hits"][K["off"][t]:K["off"][t + 1]]]
        assert np.all(lab == lab[0])


def test_zero_smear_fit_recovers_truth():
    """With exact clusters and the true (s, t, k) at the outermost hit, every residual is
    zero, so the FP64 fit must reproduce the exact helix state at the innermost hit; its
    covariance must equal the batch least-squares covariance (A^T W A + prior^-1)^-1."""
    cs = g.gen_event(12, 60, sector=0, smear=0.0, shuffle=False)
    r = O.Run.from_set(cs, last_stage=O.STAGE_FIT)
    prm = O.params()
    checked = 0
    for p in range(len(cs.part_pt)):
        hits = np.nonzero(cs.label == p)[0]
        if len(hits) < 20:
            continue
        hits = hits[np.argsort(cs.row[hits])]
        xo = float(ROWX32[cs.row[hits[-1]]])
        ok, yo, zo, so, to, ko = true_state(cs.part_pt[p], cs.part_eta[p], cs.part_phi[p], cs.part_q[p], 0, xo)
        stk = np.array([so, to, ko], np.float32)
        # the generator's float32 cluster coordinates are the measurements; use them exactly
        okf, P, Cv, x, chi2 = r.fit_hits(hits, stk, fp64=True)
        assert okf
        xi = float(ROWX32[cs.row[hits[0]]])
        _, yi, zi, si, ti, ki = true_state(cs.part_pt[p], cs.part_eta[p], cs.part_phi[p], cs.part_q[p], 0, xi)
        # float32 rounding of the clusters and of (s,t,k) limits the agreement
        assert abs(P[0] - yi) < 2e-5 and abs(P[1] - zi) < 5e-5, (P, yi, zi)
        assert abs(P[2] - si) < 2e-6 and abs(P[3] - ti) < 2e-6
        assert abs(P[4] - ki) < 1e-3 * abs(ki) + 1e-4
        checked += 1
    assert checked >= 10


def test_fit_covariance_equals_batch_least_squares():
    prm = O.params()
    # one exact track in sector 0, hits on rows 20..59
    pt, eta, phi, q = 0.8, 0.3, math.radians(9.0), 1.0
    rows = np.arange(20, 60)
    xs = ROWX32[rows].astype(np.float64)
    ok, y, z, s, t, k = true_state(pt, eta, phi, q, 0, xs)
    assert np.all(ok)
    sec = np.zeros(len(rows), np.uint8)
    run = O.Run(sec, rows.astype(np.int16), y.astype(np.float32), z.astype(np.float32),
                np.array([0, len(rows)], np.int32), prm, last_stage=O.STAGE_GRID)
    stk = np.array([s[-1], float(t), float(k)], np.float32)
    okf, P, Cv, x, chi2 = run.fit_hits(np.arange(len(rows)), stk, fp64=True)
    assert okf
    # batch: linearise the measurement model around the fitted state at the innermost hit
    x0 = float(ROWX32[rows[0]])
    def meas(st):
        out = []
        for xi in xs:
            okp, Pn, _ = O.propagate(st, np.zeros(15), x0, float(np.float32(xi)), prm, fp64=True)
            out.extend((Pn[:2] + Pn[5:7]).tolist())
        return np.array(out)
    A = np.zeros((2 * len(rows), 5))
    for a in range(5):
        hs = 1e-6
        pp = P.copy(); pp[a] += hs
        pm = P.copy(); pm[a] -= hs
        A[:, a] = (meas(pp) - meas(pm)) / (2 * hs)
    sy2 = float(np.float32(prm.sigma_y)) ** 2
    W = np.eye(2 * len(rows)) / sy2
    # the prior sits at the outermost hit: transport its information to x0
    prior = np.diag([prm.cy1, prm.cz1, prm.cs1, prm.ct1, prm.ck1]).astype(np.float64)
    prior = np.diag([float(np.float32(v)) for v in (prm.cy1, prm.cz1, prm.cs1, prm.ct1, prm.ck1)])
    okp, Pout, _ = O.propagate(P, np.zeros(15), x0, float(ROWX32[rows[-1]]), prm, fp64=True)
    Jo = _jac_from_transport(P, x0, float(ROWX32[rows[-1]]), prm)   # d(state_out)/d(state_0)
    info = A.T @ W @ A + Jo.T @ np.linalg.inv(prior) @ Jo
    Cbatch = np.linalg.inv(info)
    Ck = O.tri_to_full(Cv)
    assert np.allclose(Ck, Cbatch, rtol=2e-4, atol=1e-12), (np.diag(Ck), np.diag(Cbatch))


def test_pulls_are_standard_normal():
    """Statistical pin: fitted parameters minus the exact helix state, divided by the fitted
    errors, follow N(0,1) on single-sector events (all three seeds of the workload)."""
    pulls = {2: [], 3: [], 4: []}
    for seed in (11, 12, 13):
        cs = g.make_config("c1", seed)
        r = O.Run.from_set(cs)
        K = r.tracks()
        for t in range(len(K["tracklet"])):
            hits = K["hits"][K["off"][t]:K["off"][t + 1]]
            lab = cs.label[hits]
            if not np.all(lab == lab[0]) or K["ndfd"][t] < 0:
                continue
            p = lab[0]
            ok, yi, zi, si, ti, ki = true_state(cs.part_pt[p], cs.part_eta[p], cs.part_phi[p],
                                                cs.part_q[p], 0, float(K["xd"][t]))
            if not ok:
                continue
            Cf = O.tri_to_full(K["Cd"][t])
            for a, tv in ((2, si), (3, ti), (4, ki)):
                pulls[a].append((K["Pd"][t][a] - tv) / math.sqrt(Cf[a, a]))
    for a, v in pulls.items():
        v = np.array(v)
        assert len(v) > 150
        assert abs(v.mean()) < 0.2, (a, v.mean())
        assert 0.75 < v.std() < 1.25, (a, v.std())


def test_fp32_fit_within_tolerance_of_fp64():
    """The FP32 path (which the GPU reproduces bit for bit) against the FP64 refit:
    1e-4 relative on q/pT (floor |q/pT| = 0.1, the workload's pT <= 10 GeV) and 1e-3 cm."""
    for cs in (g.make_config("c1", 11), g.make_config("c2", 22, scale=0.3)):
        K = O.Run.from_set(cs).tracks()
        ok32, ok64 = K["ndf"] >= 0, K["ndfd"] >= 0
        assert np.array_equal(ok32, ok64)
        P, Pd = K["P"][ok32].astype(np.float64), K["Pd"][ok32]
        assert np.all(np.abs(P[:, 4] - Pd[:, 4]) <= 1e-4 * np.maximum(np.abs(Pd[:, 4]), 0.1))
        assert np.all(np.abs(P[:, :2] - Pd[:, :2]) <= 1e-3)


# ------------------------------------------------------------------ merge
def test_boundary_crosser_is_merged():
    """A zero-smear track leaving sector 0 into sector 1 at mid radius yields exactly one
    merged track that holds every one of its clusters."""
    pt, eta, phi, q = np.array([0.5]), np.array([0.3]), np.array([math.radians(8.0)]), np.array([-1])
    ti, sec, row, y, z, _ = g.crossings(pt, eta, phi, q)
    assert set(np.unique(sec)) == {0, 1}
    assert (sec == 0).sum() > 20 and (sec == 1).sum() > 20
    jo = np.array([0, len(y)], np.int32)
    r = O.Run(sec.astype(np.uint8), row.astype(np.int16), y.astype(np.float32),
              z.astype(np.float32), jo)
    K = r.tracks()
    assert len(K["tracklet"]) == 1
    hits = K["hits"][K["off"][0]:K["off"][1]]
    assert sorted(hits.tolist()) == list(range(len(y)))
    assert K["sector"][0] == 0 and K["sector2"][0] == 1
    assert K["ndf"][0] == 2 * len(y) - 5
    # inner piece first, then the outer piece
    assert np.all(sec[hits[: (sec == 0).sum()]] == 0)
    # without the merge stage: two pieces
    K4 = O.Run(sec.astype(np.uint8), row.astype(np.int16), y.astype(np.float32),
               z.astype(np.float32), jo, last_stage=O.STAGE_FIT).tracks(merged=False)
    assert len(K4["tracklet"]) == 2


def test_merge_chi2_cholesky_against_solve():
    rng = np.random.default_rng(4)
    A = rng.normal(size=(5, 5)); CA = A @ A.T + np.eye(5) * 0.1
    B = rng.normal(size=(5, 5)); CB = B @ B.T + np.eye(5) * 0.1
    PA, PB = rng.normal(size=5), rng.normal(size=5)
    c = O.merge_chi2(PA, O.full_to_tri(CA), PB, O.full_to_tri(CB))
    d = PA - PB
    ref = d @ np.linalg.solve(CA + CB, d)
    assert abs(c - ref) <= 1e-4 * ref
