"""Seeded synthetic initial data for the 2D compressible Euler workloads.

This module only *defines inputs*: it draws seeded random numbers and turns
primitive fields (rho, v1, v2, p) into conserved fields (rho, m1, m2, E) with
the ideal-gas law of Section 1 (p = (gamma - 1)(E - rho |v|^2 / 2)).  It holds
none of the lattice Boltzmann scheme's arithmetic and imports neither the HIP
library nor the oracle, so both sides can be fed the same arrays.

Layout of every returned field: float64, shape [4, ny, nx], component-major,
component order (rho, m1 = rho v1, m2 = rho v2, E).  Cell centres are
x_i = (i + 1/2) dx on the stated domain (cell-centred grid, square cells).
"""
from __future__ import annotations

import numpy as np

GAMMA_AIR = 1.4


def prim_to_cons(rho, v1, v2, p, gamma):
    """Conserved variables from primitives (ideal gas, Section 1)."""
    rho = np.asarray(rho, dtype=np.float64)
    v1 = np.broadcast_to(np.asarray(v1, dtype=np.float64), rho.shape)
    v2 = np.broadcast_to(np.asarray(v2, dtype=np.float64), rho.shape)
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    u = np.empty((4,) + rho.shape, dtype=np.float64)
    u[0] = rho
    u[1] = rho * v1
    u[2] = rho * v2
    u[3] = p / (gamma - 1.0) + 0.5 * rho * (v1 * v1 + v2 * v2)
    return u


def cell_centres(n, lo=0.0, hi=1.0):
    dx = (hi - lo) / n
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * dx


# ---------------------------------------------------------------------------
# Workloads used for parity, benchmarks and differentiation
# ---------------------------------------------------------------------------

def quadrant_states(rng):
    """Four quadrant states (rho, v1, v2, p), drawn in the order
    (x<1/2,y<1/2), (x>=1/2,y<1/2), (x<1/2,y>=1/2), (x>=1/2,y>=1/2);
    rho ~ U[0.1,1.5], v1, v2 ~ U[-1,1], p ~ U[0.05,1.5]."""
    states = []
    for _ in range(4):
        rho = rng.uniform(0.1, 1.5)
        v1 = rng.uniform(-1.0, 1.0)
        v2 = rng.uniform(-1.0, 1.0)
        p = rng.uniform(0.05, 1.5)
        states.append((rho, v1, v2, p))
    return states


def riemann4(n=64, seed=0, gamma=GAMMA_AIR, rng=None):
    """Four-quadrant 2D Riemann problem on [0,1]^2 (the Lax-Liu family of
    Section 4.7) with seeded quadrant states, split at (1/2, 1/2)."""
    if rng is None:
        rng = np.random.default_rng(seed)
    st = quadrant_states(rng)
    x = cell_centres(n)
    X, Y = np.meshgrid(x, x, indexing="xy")  # [ny, nx]
    q = (X >= 0.5).astype(np.int64) + 2 * (Y >= 0.5).astype(np.int64)
    prim = np.array(st, dtype=np.float64)  # [4 quadrants, 4 fields]
    f = prim[q]  # [ny, nx, 4]
    return prim_to_cons(f[..., 0], f[..., 1], f[..., 2], f[..., 3], gamma)


def double_rarefaction(n=2048, seed=0, gamma=GAMMA_AIR):
    """Near-vacuum double rarefaction: (rho, v1, v2, p) = (1, -2, 0, 0.4) for
    x < 1/2 and (1, +2, 0, 0.4) for x >= 1/2, with rho += 1e-3 xi,
    xi ~ U[-1, 1) per cell."""
    rng = np.random.default_rng(seed)
    x = cell_centres(n)
    xi = rng.random((n, n)) * 2.0 - 1.0
    rho = 1.0 + 1e-3 * xi
    v1 = np.where(x[None, :] < 0.5, -2.0, 2.0) * np.ones((n, 1))
    return prim_to_cons(rho, v1, 0.0, 0.4, gamma)


def blast(n=8192, seed=0, gamma=GAMMA_AIR, p_in=1e3, p_out=1e-2, radius=0.1):
    """Blast: rho = 1 + 0.01 xi (xi ~ U[-1,1)), v = 0, p = p_in inside the
    circle of the given radius about (1/2, 1/2), p_out outside."""
    rng = np.random.default_rng(seed)
    x = cell_centres(n)
    xi = rng.random((n, n)) * 2.0 - 1.0
    rho = 1.0 + 0.01 * xi
    del xi
    r2 = (x[None, :] - 0.5) ** 2 + (x[:, None] - 0.5) ** 2
    p = np.where(r2 < radius * radius, p_in, p_out)
    del r2
    return prim_to_cons(rho, 0.0, 0.0, p, gamma)


def batch_sides(count=256, seed=0):
    """Square sides 128*k, k ~ U{1..8}."""
    rng = np.random.default_rng(seed)
    return [int(128 * k) for k in rng.integers(1, 9, size=count)]


def batch_riemann4(count=256, seed=0, gamma=GAMMA_AIR, sides=None):
    """Ensemble of four-quadrant problems of uneven size; instance i draws its
    quadrant states from default_rng([seed, i])."""
    if sides is None:
        sides = batch_sides(count, seed)
    out = []
    for i, s in enumerate(sides):
        rng = np.random.default_rng([seed, i])
        out.append(riemann4(s, gamma=gamma, rng=rng))
    return out


def gaussian_bump(n=512, seed=0, gamma=GAMMA_AIR, amp=0.1, sigma=0.05,
                  centre=None):
    """rho = 1 + amp exp(-r^2/(2 sigma^2)) with r the minimum-image distance to
    a seeded centre c ~ U[0.25, 0.75]^2 on the periodic unit square; v = 0,
    p = 1."""
    if centre is None:
        rng = np.random.default_rng(seed)
        centre = rng.uniform(0.25, 0.75, size=2)
    x = cell_centres(n)
    dxm = x[None, :] - centre[0]
    dym = x[:, None] - centre[1]
    dxm = dxm - np.round(dxm)
    dym = dym - np.round(dym)
    rho = 1.0 + amp * np.exp(-(dxm * dxm + dym * dym) / (2.0 * sigma * sigma))
    return prim_to_cons(rho, 0.0, 0.0, 1.0, gamma)


def gaussian_bump_target(n=512, seed=0, target_seed=1, gamma=GAMMA_AIR):
    """Target initial bump: the seeded centre moved by U[-0.02, 0.02]^2."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.25, 0.75, size=2)
    c2 = c + np.random.default_rng(target_seed).uniform(-0.02, 0.02, size=2)
    return gaussian_bump(n, gamma=gamma, centre=c2)


# ---------------------------------------------------------------------------
# Validation problems of Section 4
# ---------------------------------------------------------------------------

def entropy_wave(n, gamma=GAMMA_AIR):
    """Section 4.1: (rho, v1, v2, p) = (1 + 0.1 sin(2 pi (x + y)), 1, 1, 1)
    on the periodic unit square."""
    x = cell_centres(n)
    rho = 1.0 + 0.1 * np.sin(2.0 * np.pi * (x[None, :] + x[:, None]))
    return prim_to_cons(rho, 1.0, 1.0, 1.0, gamma)


def sod_y(n=100, ncols=4, gamma=GAMMA_AIR):
    """Section 4.2 Sod data laid along y (x-invariant): (1, 0, 1) for
    y < 1/2 and (0.125, 0, 0.1) above, on ncols columns."""
    y = cell_centres(n)
    rho = np.where(y < 0.5, 1.0, 0.125)[:, None] * np.ones((1, ncols))
    p = np.where(y < 0.5, 1.0, 0.1)[:, None] * np.ones((1, ncols))
    return prim_to_cons(rho, 0.0, 0.0, p, gamma)


def shu_osher(n=800, nrows=4, gamma=GAMMA_AIR):
    """Section 4.3 on [-5, 5] (1D data along x, nrows rows)."""
    x = cell_centres(n, -5.0, 5.0)
    left = x < -4.0
    rho = np.where(left, 3.857143, 1.0 + 0.2 * np.sin(5.0 * x))
    v1 = np.where(left, 2.629369, 0.0)
    p = np.where(left, 10.33333333333, 1.0)
    ones = np.ones((nrows, 1))
    return prim_to_cons(rho[None, :] * ones, v1[None, :] * ones, 0.0,
                        p[None, :] * ones, gamma)


def lax_liu3(n=400, gamma=GAMMA_AIR):
    """Section 4.7: configuration 3 of the 2D Riemann problem, split at 0.8."""
    x = cell_centres(n)
    X, Y = np.meshgrid(x, x, indexing="xy")
    rho = np.empty_like(X)
    v1 = np.empty_like(X)
    v2 = np.empty_like(X)
    p = np.empty_like(X)
    ll = (X <= 0.8) & (Y <= 0.8)
    lu = (X <= 0.8) & (Y > 0.8)
    rl = (X > 0.8) & (Y <= 0.8)
    ru = (X > 0.8) & (Y > 0.8)
    for m, s in ((ll, (0.138, 1.206, 1.206, 0.029)), (lu, (0.5323, 1.206, 0.0, 0.3)),
                 (rl, (0.5323, 0.0, 1.206, 0.3)), (ru, (1.5, 0.0, 0.0, 1.5))):
        rho[m], v1[m], v2[m], p[m] = s
    return prim_to_cons(rho, v1, v2, p, gamma)


def leblanc(n=1000, nrows=4, gamma=5.0 / 3.0):
    """Section 4.5 on [0, 9]."""
    x = cell_centres(n, 0.0, 9.0)
    left = x <= 3.0
    rho = np.where(left, 1.0, 1e-3)
    p = np.where(left, 0.1 * (gamma - 1.0), 1e-7 * (gamma - 1.0))
    ones = np.ones((nrows, 1))
    return prim_to_cons(rho[None, :] * ones, 0.0, 0.0, p[None, :] * ones, gamma)


def isentropic_vacuum(n=50, nrows=4, amp=0.9999995, gamma=3.0):
    """Section 4.4 on the periodic [-1, 1]: (1 + amp sin(pi x), 0, rho^gamma)."""
    x = cell_centres(n, -1.0, 1.0)
    rho = 1.0 + amp * np.sin(np.pi * x)
    ones = np.ones((nrows, 1))
    return prim_to_cons(rho[None, :] * ones, 0.0, 0.0,
                        (rho ** gamma)[None, :] * ones, gamma)


def random_admissible(count, seed=0, gamma=GAMMA_AIR, rho_range=(1e-3, 2.0),
                      v_range=(-3.0, 3.0), p_range=(1e-4, 2.0)):
    """Independent random admissible states, [4, count]."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(*rho_range, size=count)
    v1 = rng.uniform(*v_range, size=count)
    v2 = rng.uniform(*v_range, size=count)
    p = rng.uniform(*p_range, size=count)
    return prim_to_cons(rho, v1, v2, p, gamma)


# Side codes of the boundary descriptions (the values of the library's and the
# oracle's boundary kinds): 1 = reflective wall, 2 = Dirichlet state.
_WALL, _DIRICHLET = 1, 2


def dmr_states(gamma=GAMMA_AIR):
    """Section 4.8 double Mach reflection: post-shock (8, 8.25 cos 30deg,
    -8.25 sin 30deg, 116.5) and pre-shock (1.4, 0, 0, 1) states, [4] each."""
    post = prim_to_cons(8.0, 8.25 * np.cos(np.pi / 6.0), -8.25 * np.sin(np.pi / 6.0), 116.5, gamma)
    pre = prim_to_cons(1.4, 0.0, 0.0, 1.0, gamma)
    return post, pre


def dmr_shock_x(y, t):
    """Position on [0, 3] of the incident Mach 10 shock at height y, time t:
    it meets y = 0 at x = 1/6 at t = 0 at 60 degrees to the x axis and moves
    at speed 10 along its normal."""
    return 1.0 / 6.0 + (y + 20.0 * t) / np.sqrt(3.0)


def double_mach(nx=1500, ny=500, gamma=GAMMA_AIR):
    """Section 4.8 double Mach reflection on [0, 3] x [0, 1] (square cells,
    nx = 3 ny).  Returns (u0, kinds, states): the initial moments and, per
    side (west, east, south, north), the boundary kinds (uint8) and states
    [4, n].  Every boundary cell holds the exact solution (the shock moving
    at its Rankine-Hugoniot speed) at its centre, half a cell outside the
    domain, except the south cells with x >= 1/6, which are a reflective wall.
    On the west and on the south that state is the post-shock one at all
    times; on the east and the north it changes as the shock passes
    (`double_mach_east`, `double_mach_north` give them at time t; here t = 0)."""
    post, pre = dmr_states(gamma)
    x = cell_centres(nx, 0.0, 3.0)
    y = cell_centres(ny)
    X, Y = np.meshgrid(x, y, indexing="xy")
    u0 = np.where((X < dmr_shock_x(Y, 0.0))[None], post[:, None, None], pre[:, None, None])
    kinds = (np.full(ny, _DIRICHLET, np.uint8), np.full(ny, _DIRICHLET, np.uint8),
             np.where(x < 1.0 / 6.0, _DIRICHLET, _WALL).astype(np.uint8),
             np.full(nx, _DIRICHLET, np.uint8))
    states = (np.repeat(post[:, None], ny, 1), double_mach_east(ny, 0.0, gamma),
              np.repeat(post[:, None], nx, 1), double_mach_north(nx, 0.0, gamma))
    return (np.ascontiguousarray(u0), kinds, tuple(np.ascontiguousarray(s) for s in states))


def double_mach_north(nx, t, gamma=GAMMA_AIR):
    """North boundary states of the double Mach reflection at time t, at the
    boundary cells' centres y = 1 + dx/2: post-shock left of the moving
    shock, pre-shock right of it, [4, nx]."""
    post, pre = dmr_states(gamma)
    x = cell_centres(nx, 0.0, 3.0)
    behind = x < dmr_shock_x(1.0 + 1.5 / nx, t)
    return np.ascontiguousarray(np.where(behind[None], post[:, None], pre[:, None]))


def double_mach_east(ny, t, gamma=GAMMA_AIR):
    """East boundary states of the double Mach reflection at time t, at the
    boundary cells' centres x = 3 + dx/2: pre-shock until the shock reaches
    them (from t of about 0.19 on, top rows first), post-shock after, [4, ny]."""
    post, pre = dmr_states(gamma)
    y = cell_centres(ny)
    behind = 3.0 + 0.5 / ny < dmr_shock_x(y, t)
    return np.ascontiguousarray(np.where(behind[None], post[:, None], pre[:, None]))


def jet(mach, nx=800, ny=400, gamma=5.0 / 3.0):
    """Section 4.8 astrophysical jets: Mach 80 on [0, 2] x [-1/2, 1/2] with
    inflow (5, 30, 0, 0.4127), Mach 2000 on [0, 1] x [-1/4, 1/4] with inflow
    (5, 800, 0, 0.4127), where |y| < 0.05 on the west side; ambient gas
    (0.5, 0, 0, 0.4127) everywhere else.  Returns (u0, west, dx, t_end): the
    initial moments, the west side's Dirichlet states [4, ny] (the other
    sides are zero-gradient), the cell size and the final time of the paper
    (0.07, resp. 0.001)."""
    if mach == 80:
        lx, ly, v, t_end = 2.0, 1.0, 30.0, 0.07
    elif mach == 2000:
        lx, ly, v, t_end = 1.0, 0.5, 800.0, 0.001
    else:
        raise ValueError("mach must be 80 or 2000")
    amb = prim_to_cons(0.5, 0.0, 0.0, 0.4127, gamma)
    inflow = prim_to_cons(5.0, v, 0.0, 0.4127, gamma)
    u0 = np.repeat(np.repeat(amb[:, None, None], ny, 1), nx, 2)
    y = cell_centres(ny, -0.5 * ly, 0.5 * ly)
    west = np.where((np.abs(y) < 0.05)[None], inflow[:, None], amb[:, None])
    return np.ascontiguousarray(u0), np.ascontiguousarray(west), lx / nx, t_end
