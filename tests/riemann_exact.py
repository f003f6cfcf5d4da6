"""Exact solution of the 1D Riemann problem for the ideal-gas Euler equations.

Written from the mathematics: the star pressure p* is the root of
    f_L(p) + f_R(p) + (u_R - u_L) = 0,
where f_K(p) is the Rankine-Hugoniot velocity jump across a shock
(p > p_K) or the isentropic (Riemann-invariant) jump across a rarefaction
(p <= p_K); the solution is then sampled along x/t.  Used by the tests to pin
the oracle on x-invariant Sod data (Section 4.2).  Vacuum generation is not
handled (not needed for the data it is used on).
"""
from __future__ import annotations

import math

import numpy as np


def _fk(p, rho, pk, g):
    c = math.sqrt(g * pk / rho)
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        s = math.sqrt(A / (p + B))
        f = (p - pk) * s
        df = s * (1.0 - 0.5 * (p - pk) / (p + B))
    else:
        e = (g - 1.0) / (2.0 * g)
        f = 2.0 * c / (g - 1.0) * ((p / pk) ** e - 1.0)
        df = 1.0 / (rho * c) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(L, R, g):
    """(p*, u*) for left/right primitive states (rho, u, p)."""
    rl, ul, pl = L
    rr, ur, pr = R
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    if 2.0 * (cl + cr) / (g - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated")
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(200):
        fl, dfl = _fk(p, rl, pl, g)
        fr, dfr = _fk(p, rr, pr, g)
        F = fl + fr + (ur - ul)
        pn = p - F / (dfl + dfr)
        if pn <= 0.0:
            pn = 0.5 * p
        if abs(pn - p) <= 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fk(p, rl, pl, g)
    fr, _ = _fk(p, rr, pr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(L, R, g, xi):
    """Primitive (rho, u, p) arrays at similarity coordinates xi = (x - x0)/t."""
    rl, ul, pl = L
    rr, ur, pr = R
    ps, us = star_state(L, R, g)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for n, s in np.ndenumerate(xi):
        if s <= us:  # left of the contact
            rk, uk, pk, sgn = rl, ul, pl, -1.0
        else:
            rk, uk, pk, sgn = rr, ur, pr, 1.0
        ck = math.sqrt(g * pk / rk)
        if ps > pk:  # shock
            rs = rk * ((ps / pk + gm) / (gm * ps / pk + 1.0))
            S = uk + sgn * ck * math.sqrt((g + 1.0) / (2.0 * g) * ps / pk + (g - 1.0) / (2.0 * g))
            if sgn * (s - S) >= 0.0:
                rho[n], u[n], p[n] = rk, uk, pk
            else:
                rho[n], u[n], p[n] = rs, us, ps
        else:  # rarefaction
            rs = rk * (ps / pk) ** (1.0 / g)
            cs = ck * (ps / pk) ** ((g - 1.0) / (2.0 * g))
            head = uk + sgn * ck
            tail = us + sgn * cs
            if sgn * (s - head) >= 0.0:
                rho[n], u[n], p[n] = rk, uk, pk
            elif sgn * (s - tail) <= 0.0:
                rho[n], u[n], p[n] = rs, us, ps
            else:
                c = 2.0 / (g + 1.0) * (ck - sgn * 0.5 * (g - 1.0) * (uk - s))
                uu = 2.0 / (g + 1.0) * (-sgn * ck + 0.5 * (g - 1.0) * uk + s)
                rho[n] = rk * (c / ck) ** (2.0 / (g - 1.0))
                u[n] = uu
                p[n] = pk * (c / ck) ** (2.0 * g / (g - 1.0))
    return rho, u, p
