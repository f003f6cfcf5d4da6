"""Pins of the oracle's per-cell blending (Section 3.1, eq. (naive_blending)),
the ablation that the paper states first and sets aside: each distribution
leaving a cell is blended with that cell's factor theta_ij, read here as the
smallest factor of the cell's four faces (a ghost cell takes the factor of
the cell it copies).  Checked against the five-population form of the
equation restated in numpy, the special cases theta = 1 and theta = 0, and
conservation."""
import math

import numpy as np
import pytest

import npref
from paper_2411_15001_amd import cases

GAMMA = 1.4


def percell_reference(S, tx, ty, a, bc_x=0, bc_y=0, alpha=0.5):
    """eq. (naive_blending) with u_5 = u - sum_k u_k carried explicitly:
    u_k^{n+1}(i, j) = M_k(u_U) + theta_U (M_k(u_U) - u_{k,U}), U the upwind
    cell of direction k (the cell itself for the rest population k = 5), and
    u^{n+1} = sum over the five populations."""
    th = np.minimum(np.minimum(tx[:, :-1], tx[:, 1:]), np.minimum(ty[:-1, :], ty[1:, :]))
    Sp = npref.pad(S, 1, bc_x, bc_y)
    thp = npref.pad(th, 1, bc_x, bc_y)
    u = Sp[0:4]
    uk = [Sp[4 + 4 * k:8 + 4 * k] for k in range(4)]
    u5 = u - uk[0] - uk[1] - uk[2] - uk[3]
    M = npref.maxwellians(u, GAMMA, alpha, a)
    post = [M[k] + thp * (M[k] - uk[k]) for k in range(4)]
    u1 = npref.west(post[0])
    u2 = npref.east(post[1])
    u3 = npref.south(post[2])
    u4 = npref.north(post[3])
    u5n = M[4] + thp * (M[4] - u5)
    un = u1 + u2 + u3 + u4 + u5n
    out = np.concatenate([un, u1, u2, u3, u4])[:, 1:-1, 1:-1]
    return out, th


@pytest.mark.parametrize("bc", [(0, 0), (1, 1), (1, 0)])
@pytest.mark.parametrize("lims", [1 | 8, 2 | 8, 4 | 8, 1 | 2 | 8])
def test_percell_equals_five_population_form(orc, bc, lims):
    n = 32
    cfg = orc.Config(nx=n, ny=n - 4, limiters=lims, bc_x=bc[0], bc_y=bc[1], blend=orc.BLEND_CELL)
    u0 = np.ascontiguousarray(cases.riemann4(n, seed=12)[:, :n - 4, :])
    S, _ = orc.init(cfg, u0)
    S, _, _, _ = orc.run(cfg, S, 6)
    S1, tx, ty, info = orc.step(cfg, S)
    ref, th = percell_reference(S, tx, ty, info.a, *bc)
    assert info.n_limited == int((th < 1).sum())
    assert info.n_limited > 0 or not (lims & 6)
    for q in range(20):
        err = np.abs(S1[q] - ref[q]).max() / np.abs(ref[q]).max()
        assert err <= 1e-12, (q, err)
    # the face factors are those of the face-blended scheme on the same state
    Sf, txf, tyf, _ = orc.step(orc.Config(nx=n, ny=n - 4, limiters=lims, bc_x=bc[0], bc_y=bc[1]), S)
    assert np.array_equal(tx, txf) and np.array_equal(ty, tyf)
    if info.n_limited:
        assert not np.array_equal(S1, Sf)  # the two blendings differ where theta < 1


@pytest.mark.parametrize("kw", [dict(limiters=0), dict(order=1)])
def test_percell_special_cases(orc, kw):
    """theta = 1 everywhere (unlimited) and theta = 0 (first order): the
    per-cell and face blendings are the same scheme, bit for bit (Example 3,
    and the first-order scheme of Example 2)."""
    n = 24
    S0, _ = orc.init(orc.Config(nx=n, ny=n), cases.riemann4(n, seed=3))
    for bc in ((0, 0), (1, 1)):
        cf = orc.Config(nx=n, ny=n, bc_x=bc[0], bc_y=bc[1], **kw)
        cc = orc.Config(nx=n, ny=n, bc_x=bc[0], bc_y=bc[1], blend=orc.BLEND_CELL, **kw)
        Sf, _, _, _ = orc.run(cf, S0, 5)
        Sc, _, _, _ = orc.run(cc, S0, 5)
        assert np.array_equal(Sf, Sc)


def test_percell_conserves_moments(orc):
    """Periodic grid, LMP-limited four-quadrant data: the totals of rho, m1,
    m2 and E are conserved to round-off over 100 steps (the zeroth moment of
    eq. (naive_blending) is conserved, Section 3.1)."""
    n = 48
    cfg = orc.Config(nx=n, ny=n, limiters=1 | 2 | 8, a_beta=1.1, blend=orc.BLEND_CELL)
    S0, _ = orc.init(cfg, cases.riemann4(n, seed=6))
    S, _, _, tot = orc.run(cfg, S0, 100)
    assert tot[1] > 0
    for c in range(4):
        a, b = math.fsum(S0[c].ravel()), math.fsum(S[c].ravel())
        scale = math.fsum(np.abs(S0[0]).ravel()) + math.fsum(np.abs(S0[3]).ravel())
        assert abs(a - b) <= 1e-13 * scale, (c, a, b)
