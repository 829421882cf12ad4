"""Brute-force force stencil on tiny lattices (pure Python loops).

TEST INFRASTRUCTURE ONLY.  An independent second writing of Eq. (2) and the
two force definitions after it, used to pin the C oracle's force routine.  The
24 offsets of Fig. 1 (belts 1-2) are listed by hand, each with its belt-1 D2Q9
weight and its two-belt weight as exact fractions.
"""
from fractions import Fraction as Fr
import math

import numpy as np

# (cx, cy, belt-1 D2Q9 weight, two-belt weight)
OFFSETS = [
    # belt 1: four axis neighbours
    (1, 0, Fr(1, 9), Fr(4, 63)), (0, 1, Fr(1, 9), Fr(4, 63)),
    (-1, 0, Fr(1, 9), Fr(4, 63)), (0, -1, Fr(1, 9), Fr(4, 63)),
    # belt 1: four diagonal neighbours
    (1, 1, Fr(1, 36), Fr(4, 135)), (-1, 1, Fr(1, 36), Fr(4, 135)),
    (-1, -1, Fr(1, 36), Fr(4, 135)), (1, -1, Fr(1, 36), Fr(4, 135)),
    # belt 2: distance 2 on the axes
    (2, 0, 0, Fr(1, 180)), (0, 2, 0, Fr(1, 180)),
    (-2, 0, 0, Fr(1, 180)), (0, -2, 0, Fr(1, 180)),
    # belt 2: knight moves
    (2, 1, 0, Fr(2, 945)), (1, 2, 0, Fr(2, 945)), (-1, 2, 0, Fr(2, 945)), (-2, 1, 0, Fr(2, 945)),
    (-2, -1, 0, Fr(2, 945)), (-1, -2, 0, Fr(2, 945)), (1, -2, 0, Fr(2, 945)), (2, -1, 0, Fr(2, 945)),
    # belt 2: corners
    (2, 2, 0, Fr(1, 15120)), (-2, 2, 0, Fr(1, 15120)),
    (-2, -2, 0, Fr(1, 15120)), (2, -2, 0, Fr(1, 15120)),
]


def psi(rho, rho0):
    return rho0 * (1.0 - math.exp(-rho / rho0))


def _at(g, x, y, walls):
    ny, nx = g.shape
    x %= nx
    if walls:
        if y < 0:
            y = -1 - y
        elif y >= ny:
            y = 2 * ny - 1 - y
    else:
        y %= ny
    return g[y, x]


def force(rho_a, rho_b, rho0, g_aa1, g_aa2, g_bb1, g_bb2, g_ab, walls=False):
    """Returns (FAx, FAy, FBx, FBy) by a literal loop over sites and offsets."""
    rho = [np.asarray(rho_a, float), np.asarray(rho_b, float)]
    ny, nx = rho[0].shape
    ps = [np.vectorize(lambda r: psi(r, rho0))(r) for r in rho]
    ga = [g_aa1, g_bb1]
    gr = [g_aa2, g_bb2]
    out = [np.zeros((ny, nx)) for _ in range(4)]
    for s in range(2):
        o = 1 - s
        for y in range(ny):
            for x in range(nx):
                fx = fy = 0.0
                for cx, cy, w1, p12 in OFFSETS:
                    pn = _at(ps[s], x + cx, y + cy, walls)
                    rn = _at(rho[o], x + cx, y + cy, walls)
                    # attraction (belt 1) and repulsion (belts 1-2) on psi_s
                    fx += -ga[s] * ps[s][y, x] * float(w1) * cx * pn
                    fy += -ga[s] * ps[s][y, x] * float(w1) * cy * pn
                    fx += -gr[s] * ps[s][y, x] * float(p12) * cx * pn
                    fy += -gr[s] * ps[s][y, x] * float(p12) * cy * pn
                    # cross-species repulsion (belt 1) on rho_s'
                    fx += -(g_ab / rho0) * rho[s][y, x] * float(w1) * cx * rn
                    fy += -(g_ab / rho0) * rho[s][y, x] * float(w1) * cy * rn
                out[2 * s][y, x] = fx
                out[2 * s + 1][y, x] = fy
    return tuple(out)


# D2Q9 velocities and weights for the brute-force full step, listed by hand.
D2Q9 = [
    (0, 0, Fr(4, 9)),
    (1, 0, Fr(1, 9)), (0, 1, Fr(1, 9)), (-1, 0, Fr(1, 9)), (0, -1, Fr(1, 9)),
    (1, 1, Fr(1, 36)), (-1, 1, Fr(1, 36)), (-1, -1, Fr(1, 36)), (1, -1, Fr(1, 36)),
]


def full_step(f, rho0, tau, g_aa1, g_aa2, g_bb1, g_bb2, g_ab, walls=False, u_top=0.0, u_bot=0.0):
    """One time step of Eq. (1) by literal loops; f has shape (2, 9, ny, nx).

    Returns (f_new, F_bot_x, F_top_x): the x momentum the bottom and top walls
    receive.  The moving-wall term and the wall density follow the oracle's
    documented reading (own node, pre-collision density)."""
    f = np.asarray(f, float)
    _, _, ny, nx = f.shape
    cs2 = 1.0 / 3.0
    rho = f.sum(axis=1)                     # (2, ny, nx)
    jx = np.zeros((ny, nx))
    jy = np.zeros((ny, nx))
    for i, (cx, cy, _) in enumerate(D2Q9):
        jx += cx * (f[0, i] + f[1, i])
        jy += cy * (f[0, i] + f[1, i])
    ux = jx / (rho[0] + rho[1])
    uy = jy / (rho[0] + rho[1])
    F = force(rho[0], rho[1], rho0, g_aa1, g_aa2, g_bb1, g_bb2, g_ab, walls=walls)
    fstar = np.empty_like(f)
    for s in range(2):
        for y in range(ny):
            for x in range(nx):
                vx = ux[y, x] + tau * F[2 * s][y, x] / rho[s, y, x]
                vy = uy[y, x] + tau * F[2 * s + 1][y, x] / rho[s, y, x]
                for i, (cx, cy, w) in enumerate(D2Q9):
                    cu = cx * vx + cy * vy
                    feq = float(w) * rho[s, y, x] * (1 + cu / cs2 + cu * cu / (2 * cs2 * cs2)
                                                     - (vx * vx + vy * vy) / (2 * cs2))
                    fstar[s, i, y, x] = f[s, i, y, x] - (f[s, i, y, x] - feq) / tau
    fnew = np.full_like(f, np.nan)
    fbot = ftop = 0.0
    for s in range(2):
        for i, (cx, cy, w) in enumerate(D2Q9):
            ib = next(j for j, (ax, ay, _) in enumerate(D2Q9) if ax == -cx and ay == -cy)
            for y in range(ny):
                for x in range(nx):
                    yt, xt = y + cy, (x + cx) % nx
                    if not walls:
                        fnew[s, i, yt % ny, xt] = fstar[s, i, y, x]
                    elif 0 <= yt < ny:
                        fnew[s, i, yt, xt] = fstar[s, i, y, x]
                    else:
                        uw = u_bot if yt < 0 else u_top
                        back = fstar[s, i, y, x] + 2 * float(w) * rho[s, y, x] * (-cx * uw) / cs2
                        fnew[s, ib, y, x] = back
                        if yt < 0:
                            fbot += cx * (fstar[s, i, y, x] + back)
                        else:
                            ftop += cx * (fstar[s, i, y, x] + back)
    return fnew, fbot, ftop
