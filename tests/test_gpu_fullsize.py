"""Parity at the benchmarked sizes, in the launch shapes bench.py times (the
committed autotune cache supplies them; a copy is used so the committed file
is never rewritten)."""
import os
import shutil

import numpy as np
import pytest

import oracle
from paper_2411_15001_amd import binding as B
from paper_2411_15001_amd import cases

pytestmark = pytest.mark.gpu

CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_2411_15001_amd", "autotune_cache.json")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch

    assert torch.cuda.is_available()
    B.lib()
    return torch


@pytest.fixture
def cache(tmp_path):
    p = str(tmp_path / "autotune_cache.json")
    shutil.copy(CACHE, p)
    return p


def okw(ocfg):
    return dict(dx=ocfg.params().dx, gamma=ocfg.gamma, alpha=ocfg.alpha, order=ocfg.order,
                limiters=ocfg.limiters, a_mode=ocfg.a_mode, a_beta=ocfg.a_beta,
                a_fixed=ocfg.a_fixed, bc_x=ocfg.bc_x, bc_y=ocfg.bc_y, sponge=ocfg.sponge,
                eps=ocfg.eps, rlmp_lo=ocfg.rlmp_lo, rlmp_hi=ocfg.rlmp_hi)


def test_c2_blast_full_size(cache):
    """8192^2 blast (p = 1e3 | 1e-2, periodic), FP64 form, PP + pressure,
    a = 4 lambda^n, in the benchmark's launch shape: two steps equal the
    oracle bit for bit over the whole 20-plane state."""
    from paper_2411_15001_amd.solver import Solver

    n = 8192
    u0 = cases.blast(n, seed=0)
    ocfg = oracle.Config(nx=n, ny=n, limiters=oracle.RHO_PP | oracle.PRESSURE)
    s = Solver(u0, **okw(ocfg))
    s.autotune(cache)
    s.step(2)
    G = s.get_state().cpu().numpy()
    d = s.diagnostics()
    s.close()
    S, _ = oracle.init(ocfg, u0)
    del u0
    S, t, info, _ = oracle.run(ocfg, S, 2)
    assert np.array_equal(G, S)
    assert d["lam"] == info.lambda_new and d["t"] == t


def test_c3_batch_full_size(cache):
    """The benchmarked ensemble (256 four-quadrant problems, sides 128 k,
    k ~ U{1..8}, outflow, PP + pressure, a = 4.4 lambda): in the FP32 form and
    the benchmark's launch shape, 20 graph-replayed steps leave the smallest,
    the largest and one mid-list instance bit-identical to their own
    single-instance runs; in the FP64 form the workload's 500 steps (graph
    replays) leave the first instance of each side 128, 256, 384 and 512 and
    the largest one bit-identical to their oracle runs, with the same lambda
    and time.  The FP32 ensemble after the same 500 steps stays admissible;
    its density error against the oracle is held to 1e-4 plus five times the
    oracle's own spread from one float32 rounding of u0 (these four-quadrant
    flows become sensitive by then: that spread reaches 2e-3 to 9e-2, while
    float32 rounds the state at every step), and to 1e-4 outright on the
    128^2 instance, which stays resolved (about a minute of oracle time)."""
    from paper_2411_15001_amd.solver import BatchSolver, Solver

    sides = cases.batch_sides(256, seed=0)
    u0s = cases.batch_riemann4(256, seed=0, sides=sides)
    kw = dict(limiters=B.LBM_RHO_PP | B.LBM_PRESSURE, a_beta=1.1, bc_x=B.LBM_BC_OUTFLOW,
              bc_y=B.LBM_BC_OUTFLOW)
    bs = BatchSolver(u0s, precision=B.LBM_FP32_STATE, **kw)
    bs.autotune(cache)
    bs.step_graph(20)
    pick = [int(np.argmin(sides)), int(np.argmax(sides)), 128]
    for i in pick:
        s = Solver(u0s[i], dx=1.0 / sides[i], precision=B.LBM_FP32_STATE, **kw)
        s.step(20)
        assert np.array_equal(bs.moments(i).cpu().numpy(), s.moments().cpu().numpy()), i
        assert bs.diagnostics(i)["lam"] == s.diagnostics()["lam"]
        s.close()
    bs.close()

    bs = BatchSolver(u0s, **kw)
    bs.step_graph(500)
    b32 = BatchSolver(u0s, precision=B.LBM_FP32_STATE, **kw)
    b32.autotune(cache)
    b32.step_graph(500)
    pick = sorted({sides.index(k) for k in (128, 256, 384, 512)} | {int(np.argmax(sides))})
    errs = {}
    for i in pick:
        n = sides[i]
        ocfg = oracle.Config(nx=n, ny=n, dx=1.0 / n, limiters=oracle.RHO_PP | oracle.PRESSURE,
                             a_beta=1.1, bc_x=1, bc_y=1)
        S, _ = oracle.init(ocfg, u0s[i])
        S, t, info, tot = oracle.run(ocfg, S, 500)
        assert tot[2] == 0, i
        d = bs.diagnostics(i)
        assert np.array_equal(bs.moments(i).cpu().numpy(), S[0:4]), (i, n)
        assert d["lam"] == info.lambda_new and d["t"] == t, (i, n)
        assert b32.diagnostics(i)["n_bad"] == 0, i
        if n > 512:
            continue
        r32 = b32.moments(i, check=False)[0].cpu().numpy()[0]
        e = float(np.abs(r32 - S[0]).sum() / np.abs(S[0]).sum())
        # the oracle's own spread from one float32 rounding of u0
        rng = np.random.default_rng(1)
        Sp, _ = oracle.init(ocfg, u0s[i] * (1 + 6e-8 * rng.uniform(-1, 1, u0s[i].shape)))
        Sp, _, _, _ = oracle.run(ocfg, Sp, 500)
        floor = float(np.abs(Sp[0] - S[0]).sum() / np.abs(S[0]).sum())
        errs[(i, n)] = (e, floor)
    bs.close()
    b32.close()
    print("FP32 ensemble, rel L1 rho vs oracle after 500 steps (error, oracle floor):", errs)
    for (i, n), (e, floor) in errs.items():
        assert e <= 1e-4 + 5 * floor, (i, n, e, floor)
    assert errs[(sides.index(128), 128)][0] <= 1e-4


@pytest.mark.parametrize("bound", ["LMP", "RLMP"])
def test_rarefaction_bounds_full_size(bound, cache):
    """8192^2 near-vacuum double rarefaction (outflow, a = 4 lambda^n) with
    PP + LMP + pressure or PP + RLMP + pressure, in the launch shapes bench.py
    times (the LDS-staged march): the FP64 form equals the oracle bit for bit
    after two steps over the whole 20-plane state, with the same lambda, time
    and counters; the FP32 form stays within 1e-6 relative L1 of the oracle's
    density and keeps every density inside its bounds."""
    import torch

    from paper_2411_15001_amd.solver import Solver

    n = 8192
    u0 = cases.double_rarefaction(n, seed=0)
    lims = oracle.RHO_PP | (oracle.RHO_LMP if bound == "LMP" else oracle.RHO_RLMP) | oracle.PRESSURE
    ocfg = oracle.Config(nx=n, ny=n, limiters=lims, bc_x=1, bc_y=1)
    res = {}
    for prec in (B.LBM_FP64, B.LBM_FP32_STATE):
        s = Solver(u0, precision=prec, **okw(ocfg))
        s.autotune(cache)
        s.step(2)
        d = s.diagnostics()
        res[prec] = (s.get_state().cpu().numpy() if prec == B.LBM_FP64 else s.moments()[0].cpu().numpy(), d)
        s.close()
        torch.cuda.empty_cache()
    S, _ = oracle.init(ocfg, u0)
    del u0
    S, t, info, tot = oracle.run(ocfg, S, 2)
    G, d = res[B.LBM_FP64]
    assert np.array_equal(G, S)
    assert d["lam"] == info.lambda_new and d["t"] == t
    assert [d["n_guard"], d["n_limited"], d["n_bad"], d["n_lmp"]] == list(tot)
    del G
    rho32, d32 = res[B.LBM_FP32_STATE]
    err = float(np.abs(rho32 - S[0]).sum() / np.abs(S[0]).sum())
    assert err <= 1e-6, err
    assert d32["n_bad"] == 0 and d32["n_guard"] == 0
    if bound == "LMP":
        assert d32["n_lmp"] == 0


@pytest.mark.skipif(os.environ.get("VLBM_LONG_TESTS") != "1",
                    reason="about four minutes of oracle time on the host cores; set VLBM_LONG_TESTS=1")
def test_c2_blast_full_horizon_window(cache, capsys):
    """The 8192^2 blast in the FP64 form (PP + pressure, a = 4 lambda^n,
    periodic) in the benchmark's launch shape, after the workload's 500 steps.

    A cell's state after n steps depends only on the cells within n of it, so
    the oracle's run on the central 3072^2 window (periodic wrap) is exact at
    more than 500 cells from the window's edges, where the wrap's influence
    has not arrived, provided lambda^n is the full grid's: it is, since the
    maximum wavespeed lies in the blast (sound speed ~37 against ~0.12 in the
    quiescent gas) and the blast, whose shock moves at most lambda^n / a^n =
    1/4 cell per step from the disk of radius 819 cells, stays inside the exact
    region (radius 1536 - n at step n).  So the central 2072^2 cells, the whole
    blast, equal the oracle's bit for bit over all 20 planes.  Beyond the
    window, outside the reach of the blast (more than 819 + 500 cells from the
    centre), the gas keeps v = 0 exactly and one energy value bit for bit: with
    uniform pressure and no velocity every term of those components is the
    same in every cell."""
    import time

    from paper_2411_15001_amd.solver import Solver

    n, steps, W = 8192, 500, 3072
    c0 = (n - W) // 2
    lo, hi = c0 + steps, c0 + W - steps
    u0 = cases.blast(n, seed=0)
    ocfg = oracle.Config(nx=n, ny=n, limiters=oracle.RHO_PP | oracle.PRESSURE)
    s = Solver(u0, **okw(ocfg))
    s.autotune(cache)
    s.step(steps)
    d = s.diagnostics()
    st = s.get_state()
    G = st[:, lo:hi, lo:hi].cpu().numpy()
    m = st[0:4].cpu().numpy()
    del st
    s.close()
    assert d["n_bad"] == 0 and d["n_guard"] == 0
    uw = np.ascontiguousarray(u0[:, c0:c0 + W, c0:c0 + W])
    del u0
    outside = np.ones((n, n), bool)
    outside[c0:c0 + W, c0:c0 + W] = False
    assert np.all(m[1][outside] == 0) and np.all(m[2][outside] == 0)
    Eq = m[3][outside]
    assert np.all(Eq == Eq[0])
    del m, outside, Eq
    wcfg = oracle.Config(nx=W, ny=W, dx=1.0 / n, limiters=oracle.RHO_PP | oracle.PRESSURE)
    S, _ = oracle.init(wcfg, uw)
    t0 = time.time()
    t = 0.0
    for k in range(0, steps, 50):
        S, t, info, tot = oracle.run(wcfg, S, 50, t)
        assert tot[2] == 0
        with capsys.disabled():
            print("  oracle C2 window: %d / %d steps, %.0f s" % (k + 50, steps, time.time() - t0), flush=True)
    assert d["t"] == t
    assert np.array_equal(G, S[:, lo - c0:hi - c0, lo - c0:hi - c0])
