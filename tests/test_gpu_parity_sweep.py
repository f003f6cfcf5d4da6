"""Seeded sweep over the configuration space against the oracle: grid sizes
from 1 to a few hundred cells per side (ragged and partial strips), every
limiter set the scheme defines, first and second order, periodic and outflow
axes, sponge layers, rest weights alpha in [1/2, 1), speed factors beta >= 1,
a fixed kinetic speed, the RLMP relaxation constants, wall and Dirichlet
boundary cells, and strip heights, waves per workgroup, persistent grids and
strip modes of the launch.  Each case evolves a few steps in the oracle and
on the GPU from the same initial data and compares the float64 state, the
face factors of one more step and the event counts bit for bit; the
float32-state form is compared in density to 1e-5 relative L1.  The cases are
drawn from a fixed seed, so a failure names a reproducible case."""
import numpy as np
import pytest

import oracle
from paper_2411_15001_amd import binding as B
from paper_2411_15001_amd import cases

pytestmark = pytest.mark.gpu

# limiter sets: PP (1), LMP (2), RLMP (4), pressure (8); 0 = unlimited
LIMITER_SETS = [1 | 8, 2 | 8, 4 | 8, 1 | 2 | 8, 1 | 4 | 8, 1 | 2 | 4 | 8, 1, 8, 2, 0]
N_CASES = 400


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch

    assert torch.cuda.is_available()
    B.lib()
    return torch


def Solver(*a, **k):
    from paper_2411_15001_amd.solver import Solver as S

    return S(*a, **k)


def draw_case(i):
    """Configuration i of the sweep (a dict), from its own seed."""
    rng = np.random.default_rng([2411, 15001, i])
    c = {}
    # widths that are multiples of 64 take the LDS-staged march with density bounds
    c["nx"] = int(rng.choice([1, 2, 3, 17, 63, 64, 65, 100, 128, 129, 192, 200, 257]))
    c["ny"] = int(rng.choice([1, 2, 5, 16, 31, 64, 90, 150]))
    c["lims"] = int(rng.choice(LIMITER_SETS))
    c["order"] = 1 if rng.random() < 0.15 else 2
    c["bc_x"] = int(rng.integers(0, 2))
    c["bc_y"] = int(rng.integers(0, 2))
    c["sponge"] = int(rng.integers(1, 4)) if (c["bc_x"] or c["bc_y"]) and rng.random() < 0.25 else 0
    c["alpha"] = float(rng.choice([0.5, 0.5, 0.6, 0.75, 0.9]))
    c["beta"] = float(rng.choice([1.0, 1.0, 1.1, 1.5, 2.0]))
    c["fixed_a"] = bool(rng.random() < 0.2)
    c["rlmp"] = (0.999, 1.001) if rng.random() < 0.7 else (0.99, 1.01)
    c["prec"] = B.LBM_FP32_STATE if rng.random() < 0.25 else B.LBM_FP64
    c["steps"] = int(rng.integers(2, 9))
    c["launch"] = (int(rng.choice([0, 4, 8, 16, 64])), int(rng.choice([0, 1, 2, 4])))
    c["grid"] = int(rng.choice([0, 0, 0, 1, 2]))
    c["mode"] = int(rng.integers(0, 2))
    # boundary descriptions on outflow axes: none, zero-gradient, wall,
    # Dirichlet or mixed per cell
    c["bnd"] = [None] * 4
    for side in range(4):
        ax_outflow = c["bc_x"] if side < 2 else c["bc_y"]
        if ax_outflow and c["sponge"] == 0 and rng.random() < 0.5:
            c["bnd"][side] = str(rng.choice(["z", "w", "d", "m"]))
    c["seed"] = int(rng.integers(0, 1 << 30))
    return c


def build(c):
    """Initial moments, oracle configuration and the boundary arrays."""
    nx, ny = c["nx"], c["ny"]
    rng = np.random.default_rng(c["seed"])
    if c["lims"] == 0 and c["order"] == 2:
        # unlimited second order only on smooth data
        u0 = cases.gaussian_bump(max(nx, ny), seed=c["seed"] % 7, amp=0.2, sigma=0.2)
    else:
        u0 = cases.riemann4(max(nx, ny), seed=c["seed"] % 97)
    u0 = np.ascontiguousarray(u0[:, :ny, :nx])
    kinds, states = [None] * 4, [None] * 4
    for side, code in enumerate(c["bnd"]):
        if code is None:
            continue
        n = ny if side < 2 else nx
        along = nx if side < 2 else ny  # cells along the side's normal axis
        k = {"z": np.zeros(n), "w": np.ones(n), "d": np.full(n, 2),
             "m": rng.integers(0, 3, size=n)}[code].astype(np.uint8)
        if along < 2:
            k[k == 1] = 0  # a wall needs two cells along its axis
        kinds[side] = k
        if (k == 2).any():
            states[side] = np.ascontiguousarray(cases.prim_to_cons(
                rng.uniform(0.3, 1.5, n), rng.uniform(-1, 1, n), rng.uniform(-1, 1, n),
                rng.uniform(0.2, 1.5, n), 1.4))
    cfg = dict(nx=nx, ny=ny, dx=1.0 / max(nx, ny), alpha=c["alpha"], order=c["order"],
               limiters=c["lims"], a_beta=c["beta"], bc_x=c["bc_x"], bc_y=c["bc_y"],
               sponge=c["sponge"], rlmp_lo=c["rlmp"][0], rlmp_hi=c["rlmp"][1],
               bnd_kind=tuple(kinds), bnd_state=tuple(states))
    if c["fixed_a"]:
        _, info = oracle.init(oracle.Config(**cfg), u0)
        cfg.update(a_mode=1, a_fixed=1.25 * 2.0 * info.lam / (1.0 - c["alpha"]))
    return u0, oracle.Config(**cfg), kinds, states


@pytest.mark.parametrize("i", range(N_CASES))
def test_sweep_case(i, gpu):
    c = draw_case(i)
    print("sweep case", i, c, flush=True)
    u0, ocfg, kinds, states = build(c)
    S, _ = oracle.init(ocfg, u0)
    # step by step: the library's Bouchut flag is raised by any step, the
    # oracle reports it per step
    t, tot, bouchut = 0.0, np.zeros(4, np.int64), 0
    for _ in range(c["steps"]):
        S, t, info, tt = oracle.run(ocfg, S, 1, t)
        tot += tt
        bouchut |= info.bouchut
    P = ocfg.params()
    s = Solver(u0, dx=P.dx, alpha=ocfg.alpha, order=ocfg.order, limiters=ocfg.limiters,
               a_mode=ocfg.a_mode, a_beta=ocfg.a_beta, a_fixed=ocfg.a_fixed, bc_x=ocfg.bc_x,
               bc_y=ocfg.bc_y, sponge=ocfg.sponge, eps=ocfg.eps, rlmp_lo=ocfg.rlmp_lo,
               rlmp_hi=ocfg.rlmp_hi, precision=c["prec"])
    for side in range(4):
        if kinds[side] is not None:
            s.set_boundary(side, kinds[side], states[side])
    s.set_launch(*c["launch"], groups_per_cu=c["grid"], strip_mode=c["mode"])
    s.step(c["steps"])
    d = s.diagnostics()
    assert d["bouchut"] == bouchut, (d, bouchut)
    if c["prec"] == B.LBM_FP64:
        assert [d["n_guard"], d["n_limited"], d["n_bad"], d["n_lmp"]] == tot.tolist(), (d, tot)
        G = s.get_state().cpu().numpy()
        assert np.array_equal(G, S, equal_nan=True), "max abs diff %.3e" % np.nanmax(np.abs(G - S))
        S1, tx, ty, _ = oracle.step(ocfg, S)
        gtx, gty = s.step_theta()
        assert np.array_equal(gtx.cpu().numpy(), tx) and np.array_equal(gty.cpu().numpy(), ty)
        assert np.array_equal(s.get_state().cpu().numpy(), S1, equal_nan=True)
    else:
        if tot[2] == 0:
            assert d["n_bad"] == 0, d
        rho = s.moments(check=False)[0].cpu().numpy()[0]
        err = np.abs(rho - S[0]).sum() / np.abs(S[0]).sum()
        assert err < 1e-5, err
    s.close()


N_BATCH_CASES = 40


def draw_batch_case(i):
    rng = np.random.default_rng([2411, 15001, 7, i])
    c = {}
    n = int(rng.integers(1, 13))
    c["sizes"] = [(int(rng.choice([1, 5, 33, 64, 65, 128, 130, 200])),
                   int(rng.choice([1, 4, 17, 64, 100, 131]))) for _ in range(n)]
    c["lims"] = int(rng.choice(LIMITER_SETS[:6]))
    c["order"] = 1 if rng.random() < 0.1 else 2
    c["bc_x"] = int(rng.integers(0, 2))
    c["bc_y"] = int(rng.integers(0, 2))
    c["alpha"] = float(rng.choice([0.5, 0.5, 0.7]))
    c["beta"] = float(rng.choice([1.0, 1.1, 1.5]))
    c["prec"] = B.LBM_FP32_STATE if rng.random() < 0.3 else B.LBM_FP64
    c["steps"] = int(rng.integers(2, 8))
    c["graph_steps"] = int(rng.integers(0, 5))
    c["launch"] = (int(rng.choice([0, 4, 16, 64])), int(rng.choice([0, 1, 2, 4])))
    c["grid"] = int(rng.choice([0, 0, 1, 2, 4]))
    c["mode"] = int(rng.integers(0, 2))
    c["seed"] = int(rng.integers(0, 1 << 30))
    # per-instance boundary descriptions on outflow axes (half of the cases)
    c["bnd"] = []
    with_bnd = rng.random() < 0.5
    for _ in c["sizes"]:
        sides = [None] * 4
        for side in range(4):
            if with_bnd and (c["bc_x"] if side < 2 else c["bc_y"]) and rng.random() < 0.5:
                sides[side] = str(rng.choice(["z", "w", "d", "m"]))
        c["bnd"].append(sides)
    return c


@pytest.mark.parametrize("i", range(N_BATCH_CASES))
def test_batch_sweep_case(i, gpu):
    """An uneven ensemble (one launch per step, then graph replays; in half
    of the cases per-instance wall / Dirichlet / mixed boundary cells) against
    the oracle run of each instance alone (dx = 1/nx per instance): float64
    moments bit for bit, float32 state to 1e-5 relative L1 in density."""
    from paper_2411_15001_amd.solver import BatchSolver

    c = draw_batch_case(i)
    print("batch sweep case", i, c, flush=True)
    u0s, descs = [], []
    for k, (nx, ny) in enumerate(c["sizes"]):
        u = cases.riemann4(max(nx, ny), rng=np.random.default_rng([c["seed"], k]))
        u0s.append(np.ascontiguousarray(u[:, :ny, :nx]))
        # the boundary arrays of instance k, built as in the single-grid sweep
        sub = dict(nx=nx, ny=ny, lims=c["lims"], order=c["order"], bc_x=c["bc_x"], bc_y=c["bc_y"],
                   sponge=0, alpha=c["alpha"], beta=c["beta"], rlmp=(0.999, 1.001), fixed_a=False,
                   bnd=c["bnd"][k], seed=c["seed"] + k)
        _, _, kinds, states = build(sub)
        descs.append((kinds, states))
    kw = dict(limiters=c["lims"], order=c["order"], alpha=c["alpha"], a_beta=c["beta"],
              bc_x=c["bc_x"], bc_y=c["bc_y"])
    bs = BatchSolver(u0s, precision=c["prec"], **kw)
    for k, (kinds, states) in enumerate(descs):
        for side in range(4):
            if kinds[side] is not None:
                bs.set_boundary(k, side, kinds[side], states[side])
    bs.set_launch(*c["launch"], groups_per_cu=c["grid"], strip_mode=c["mode"])
    bs.step(c["steps"])
    bs.step_graph(c["graph_steps"])
    total = c["steps"] + c["graph_steps"]
    diags = [bs.diagnostics(k) for k in range(len(u0s))]  # before moments() clears the counters
    for k, u in enumerate(u0s):
        ny, nx = u.shape[1:]
        kinds, states = descs[k]
        cfg = oracle.Config(nx=nx, ny=ny, dx=1.0 / nx, bnd_kind=tuple(kinds), bnd_state=tuple(states), **kw)
        S, _ = oracle.init(cfg, u)
        S, _, _, tot = oracle.run(cfg, S, total)
        m = bs.moments(k, check=False)[0].cpu().numpy()
        if c["prec"] == B.LBM_FP64:
            assert np.array_equal(m, S[0:4], equal_nan=True), (k, nx, ny)
            d = diags[k]
            assert d["n_bad"] == tot[2] and d["n_limited"] == tot[1], (k, d, tot)
        else:
            err = np.abs(m[0] - S[0]).sum() / np.abs(S[0]).sum()
            assert err < 1e-5, (k, err)
    bs.close()


N_ADJOINT_CASES = 48


def draw_adjoint_case(i):
    rng = np.random.default_rng([2411, 15001, 13, i])
    c = {}
    c["nx"] = int(rng.choice([1, 2, 17, 64, 65, 100]))
    c["ny"] = int(rng.choice([1, 3, 16, 40, 70]))
    c["lims"] = int(rng.choice(LIMITER_SETS[:6] + [0]))
    c["order"] = 1 if rng.random() < 0.2 else 2
    c["bc_x"] = int(rng.integers(0, 2))
    c["bc_y"] = int(rng.integers(0, 2))
    c["sponge"] = int(rng.integers(1, 4)) if (c["bc_x"] or c["bc_y"]) and rng.random() < 0.3 else 0
    c["alpha"] = float(rng.choice([0.5, 0.6, 0.8]))
    c["beta"] = float(rng.choice([1.0, 1.1, 2.0]))
    c["steps"] = int(rng.integers(1, 10))
    c["seed"] = int(rng.integers(0, 1 << 30))
    c["rlmp"] = (0.999, 1.001)
    c["fixed_a"] = False
    c["bnd"] = [None] * 4
    for side in range(4):
        if (c["bc_x"] if side < 2 else c["bc_y"]) and c["sponge"] == 0 and rng.random() < 0.5:
            c["bnd"][side] = str(rng.choice(["z", "w", "d", "m"]))
    return c


@pytest.mark.parametrize("i", range(N_ADJOINT_CASES))
def test_adjoint_sweep_case(i, gpu):
    """<J v, w> from the oracle's complex-step tangent of one step (theta and a
    frozen at the forward values) equals <v, J^T w> from lbm_step_adjoint to
    1e-12, and lbm_step_adjoint_theta with the face factors of lbm_step_theta
    equals lbm_step_adjoint bit for bit, over random sizes, limiter sets,
    orders, axes, sponges, alpha, beta and wall / Dirichlet cells."""
    torch = gpu
    c = draw_adjoint_case(i)
    print("adjoint sweep case", i, c, flush=True)
    u0, cfg, kinds, states = build(c)
    kw = dict(dx=cfg.params().dx, limiters=c["lims"], order=c["order"], alpha=c["alpha"],
              a_beta=c["beta"], bc_x=c["bc_x"], bc_y=c["bc_y"], sponge=c["sponge"])
    S, _ = oracle.init(cfg, u0)
    S, _, _, tot = oracle.run(cfg, S, c["steps"])
    _, tx, ty, info = oracle.step(cfg, S)
    s = Solver(u0, **kw)
    for side in range(4):
        if kinds[side] is not None:
            s.set_boundary(side, kinds[side], states[side])
    Ut = torch.from_numpy(S).cuda()
    rng = np.random.default_rng(c["seed"])
    v = rng.normal(size=S.shape)
    w = rng.normal(size=S.shape)
    h = 1e-30
    _, im = oracle.step_frozen_cs(cfg, S, h * v, tx, ty, info.a)
    jv = im / h
    wt = torch.from_numpy(w).cuda()
    a = torch.empty_like(Ut)
    B.lbm_step_adjoint(s.ctx, Ut, wt, a)
    lhs, rhs = float(np.sum(jv * w)), float(np.sum(v * a.cpu().numpy()))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(jv) * np.linalg.norm(w), (lhs, rhs)
    # the theta-supplied adjoint with the face factors of the forward step
    s.set_state(Ut)
    gtx, gty = s.step_theta()
    assert np.array_equal(gtx.cpu().numpy(), tx) and np.array_equal(gty.cpu().numpy(), ty)
    b = torch.empty_like(Ut)
    B.lbm_step_adjoint_theta(s.ctx, Ut, gtx, gty, wt, b)
    assert torch.equal(a, b)
    s.close()
