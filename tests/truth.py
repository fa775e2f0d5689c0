"""Exact helix states from the generator's closed form (test helper).

The true track state of a particle at a pad-row plane of a sector frame,
derived from the transverse circle (centre, radius, sense of rotation) that the
generator uses, by circle/plane intersection -- a formula independent of the
oracle's chord-based propagation.
"""
import math

import numpy as np

import tpcsynth as g


def true_state(pt, eta, phi, q, sector, x, z0=0.0):
    """(ok, y, z, s, t, k) at local plane x of `sector` on the first outgoing half turn of a
    primary from (0, 0, z0)."""
    pt, eta, phi, q, x = (np.asarray(v, np.float64) for v in (pt, eta, phi, q, x))
    R, h, xc, yc = g.helix_geometry(pt, phi, q)
    a = g.sector_alpha(sector)
    ca, sa = np.cos(a), np.sin(a)
    xcl = xc * ca + yc * sa
    ycl = -xc * sa + yc * ca
    D = R * R - (x - xcl) ** 2
    ok = D >= 0
    y = ycl - h * np.sqrt(np.where(ok, D, 0.0))
    ox, oy = -xcl, -ycl
    px, py = x - xcl, y - ycl
    dphi = np.mod(h * np.arctan2(ox * py - oy * px, ox * px + oy * py), 2 * math.pi)
    ok &= (dphi > 0) & (dphi <= math.pi)
    arc = R * dphi
    t = np.sinh(eta)
    z = z0 + t * arc
    s = h * (x - xcl) / R
    k = q / pt
    return ok, y, z, s, t, k


def true_state_return(pt, eta, phi, q, sector, x, z0=0.0):
    """(ok, y, z, s, t, k) at local plane x of `sector` on the return leg of a looper (the
    second half turn), as the tracker parametrises it: along increasing x, which is against
    the momentum there, so sin(phi), tan(lambda) and q/pT change sign."""
    pt, eta, phi, q, x = (np.asarray(v, np.float64) for v in (pt, eta, phi, q, x))
    R, h, xc, yc = g.helix_geometry(pt, phi, q)
    a = g.sector_alpha(sector)
    ca, sa = np.cos(a), np.sin(a)
    xcl = xc * ca + yc * sa
    ycl = -xc * sa + yc * ca
    D = R * R - (x - xcl) ** 2
    ok = D >= 0
    y = ycl + h * np.sqrt(np.where(ok, D, 0.0))
    ox, oy = -xcl, -ycl
    px, py = x - xcl, y - ycl
    dphi = np.mod(h * np.arctan2(ox * py - oy * px, ox * px + oy * py), 2 * math.pi)
    ok &= (dphi > math.pi) & (dphi < 2 * math.pi)
    t = np.sinh(eta)
    z = z0 + t * R * dphi
    s = -h * (x - xcl) / R
    return ok, y, z, s, -t, -q / pt


def rk4_crossing(pt, eta, phi, q, sector, x_target, step=0.02):
    """Integrate dr/dl = p/|p|, dp/dl = kappa q (p/|p| x B) from the origin (RK4) until
    the local x of `sector` reaches x_target; returns local (y, z)."""
    kap = g.KAPPA * g.B_TESLA
    a = float(g.sector_alpha(sector))
    ca, sa = math.cos(a), math.sin(a)
    p = np.array([pt * math.cos(phi), pt * math.sin(phi), pt * math.sinh(eta)])
    pn = float(np.linalg.norm(p))

    def f(st):
        u = st[3:] / pn
        # u x B with B = (0, 0, 1):  (u_y, -u_x, 0)
        return np.concatenate([u, kap * q * np.array([u[1], -u[0], 0.0])])

    def rk(st, hh):
        k1 = f(st)
        k2 = f(st + 0.5 * hh * k1)
        k3 = f(st + 0.5 * hh * k2)
        k4 = f(st + hh * k3)
        return st + hh / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)

    st = np.concatenate([[0.0, 0.0, 0.0], p])
    lx = lambda s: s[0] * ca + s[1] * sa
    for _ in range(200000):
        nxt = rk(st, step)
        if lx(nxt) >= x_target:
            break
        st = nxt
    else:
        raise RuntimeError("no crossing")
    hh = 0.0
    for _ in range(30):  # Newton on the partial step length
        s2 = rk(st, hh)
        vx = (s2[3] * ca + s2[4] * sa) / pn
        hh += (x_target - lx(s2)) / vx
    s2 = rk(st, hh)
    return -s2[0] * sa + s2[1] * ca, s2[2]
