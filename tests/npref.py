"""Independent numpy restatements of single equations of the paper, used by
the CPU tests to pin the oracle.  Each helper is written directly from the
equation it names; none of them calls the oracle."""
from __future__ import annotations

import numpy as np


def euler_flux(u, gamma):
    """Section 1: f = (m1, m1 v1 + p, m2 v1, (E + p) v1),
    g = (m2, m1 v2, m2 v2 + p, (E + p) v2), p = (gamma - 1)(E - |m|^2/(2 rho))."""
    rho, m1, m2, E = u
    p = (gamma - 1.0) * (E - (m1 * m1 + m2 * m2) / (2.0 * rho))
    f = np.stack([m1, m1 * m1 / rho + p, m1 * m2 / rho, (E + p) * m1 / rho])
    g = np.stack([m2, m1 * m2 / rho, m2 * m2 / rho + p, (E + p) * m2 / rho])
    return f, g


def pressure(u, gamma):
    rho, m1, m2, E = u
    return (gamma - 1.0) * (E - (m1 * m1 + m2 * m2) / (2.0 * rho))


def maxwellians(u, gamma, alpha, a):
    """Example 1: M_1..M_5 as a [5, 4, ...] array."""
    f, g = euler_flux(u, gamma)
    w = (1.0 - alpha) / 4.0
    return np.stack([w * u + f / (2 * a), w * u - f / (2 * a), w * u + g / (2 * a),
                     w * u - g / (2 * a), alpha * u])


def wavespeed(u, gamma):
    """Section 4: max of |v| + sqrt(gamma p / rho)."""
    rho = u[0]
    v = np.sqrt(u[1] ** 2 + u[2] ** 2) / rho
    c = np.sqrt(gamma * pressure(u, gamma) / rho)
    return float(np.max(v + c))


# periodic neighbour shifts of a [..., ny, nx] field
def east(q):
    return np.roll(q, -1, axis=-1)


def west(q):
    return np.roll(q, 1, axis=-1)


def north(q):
    return np.roll(q, -1, axis=-2)


def south(q):
    return np.roll(q, 1, axis=-2)


def lf_first_order(u, gamma, alpha, a):
    """Proposition 4, eqs. (14)-(15): first-order finite-volume update with
    F^(1)_{i+1/2} = (f_{i+1} + f_i)/2 - a (1 - alpha)/4 (u_{i+1} - u_i) and
    dt/dx = 1/a (periodic)."""
    f, g = euler_flux(u, gamma)
    k = a * (1.0 - alpha) / 4.0
    F = 0.5 * (east(f) + f) - k * (east(u) - u)  # face i+1/2
    G = 0.5 * (north(g) + g) - k * (north(u) - u)
    return u - (1.0 / a) * (F - west(F) + G - south(G))


def faces(S, gamma, alpha, a):
    """Face quantities of a periodic state S [20, ny, nx]:
    u*_{i+1/2} (eq. (12) with 2 beta lambda = a (1 - alpha)), Delta F_{i+1/2}
    (eq. (22)), and the same for the y-faces j+1/2."""
    u = S[0:4]
    uk = [S[4:8], S[8:12], S[12:16], S[16:20]]
    f, g = euler_flux(u, gamma)
    M = maxwellians(u, gamma, alpha, a)
    two_k = a * (1.0 - alpha)
    usx = 0.5 * (east(u) + u) - (east(f) - f) / two_k
    usy = 0.5 * (north(u) + u) - (north(g) - g) / two_k
    dF = a * (M[0] - uk[0] - east(M[1]) + east(uk[1]))
    dG = a * (M[2] - uk[2] - north(M[3]) + north(uk[3]))
    return usx, usy, dF, dG


def lmp_bounds(S, gamma, alpha, a):
    """eq. (29): mu, nu = min / max of rho and rho* on the four faces (periodic)."""
    usx, usy, _, _ = faces(S, gamma, alpha, a)
    cand = np.stack([S[0], usx[0], west(usx[0]), usy[0], south(usy[0])])
    return cand.min(axis=0), cand.max(axis=0)


def second_order_kinetic(S, u5, gamma, alpha, a):
    """Example 3: u_k^{n+1} = 2 M_k(u_up) - u_{k,up}, k = 1..5, with u_5 kept
    explicitly; returns (u^{n+1}, [u_1..u_4]^{n+1}, u_5^{n+1})."""
    u = S[0:4]
    M = maxwellians(u, gamma, alpha, a)
    u1 = west(2 * M[0] - S[4:8])
    u2 = east(2 * M[1] - S[8:12])
    u3 = south(2 * M[2] - S[12:16])
    u4 = north(2 * M[3] - S[16:20])
    u5n = 2 * M[4] - u5
    return u1 + u2 + u3 + u4 + u5n, (u1, u2, u3, u4), u5n


def blended_fv(S, tx, ty, gamma, alpha, a):
    """Section 3.2 flux-limited finite-volume form:
    u^{n+1} = u - (1/a)[F_{i+1/2} - F_{i-1/2} + G_{j+1/2} - G_{j-1/2}],
    F = F^(1) + theta Delta F.  tx[j, i] is theta of face i-1/2 (periodic:
    nx + 1 entries per row), ty[j, i] of face j-1/2."""
    u = S[0:4]
    f, g = euler_flux(u, gamma)
    k = a * (1.0 - alpha) / 4.0
    _, _, dF, dG = faces(S, gamma, alpha, a)
    thx = tx[:, 1:]  # theta of face i+1/2
    thy = ty[1:, :]  # theta of face j+1/2
    F = 0.5 * (east(f) + f) - k * (east(u) - u) + thx * dF
    G = 0.5 * (north(g) + g) - k * (north(u) - u) + thy * dG
    return u - (1.0 / a) * (F - west(F) + G - south(G))


def theta_lmp(rs, D, kappa, muL, nuL, muR, nuR):
    """Section 3.3.1, final case formula, blended as min(1, .) (Section 3.2):
    1 if D = 0; kappa min(nu_R - rho*, rho* - mu_L) / D if D > 0;
    -kappa min(rho* - mu_R, nu_L - rho*) / D if D < 0."""
    with np.errstate(divide="ignore", invalid="ignore"):
        pos = kappa * np.minimum(nuR - rs, rs - muL) / D
        neg = -kappa * np.minimum(rs - muR, nuL - rs) / D
    t = np.where(D > 0, pos, np.where(D < 0, neg, 1.0))
    return np.minimum(1.0, t)


def pad(q, width, bc_x, bc_y):
    """[..., ny, nx] field extended by `width` ghost cells on every side: a
    periodic axis (bc 0) wraps, an outflow axis (bc 1) repeats the edge cell,
    the zero-gradient condition of Section 4.2 applied to every plane."""
    nd = q.ndim
    wx = [(0, 0)] * (nd - 1) + [(width, width)]
    wy = [(0, 0)] * (nd - 2) + [(width, width), (0, 0)]
    q = np.pad(q, wx, mode="wrap" if bc_x == 0 else "edge")
    return np.pad(q, wy, mode="wrap" if bc_y == 0 else "edge")
