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
    single-instance runs; in the FP64 form 5 steps leave the smallest
    instance bit-identical to the oracle."""
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
    bs.step(5)
    i = pick[0]
    n = sides[i]
    ocfg = oracle.Config(nx=n, ny=n, dx=1.0 / n, limiters=oracle.RHO_PP | oracle.PRESSURE,
                         a_beta=1.1, bc_x=1, bc_y=1)
    S, _ = oracle.init(ocfg, u0s[i])
    S, _, _, _ = oracle.run(ocfg, S, 5)
    assert np.array_equal(bs.moments(i).cpu().numpy(), S[0:4])
    bs.close()


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
