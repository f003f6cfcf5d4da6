"""The blocked state layout of a context's own buffers (single instance,
width a multiple of 64, face blending, no boundary descriptions), against
the planar layout that every caller buffer uses: state round trips, steps
between caller buffers, graph replays, and the switch to the planar layout
when boundary descriptions are set in the middle of a run, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2411_15001_amd import binding as B
from paper_2411_15001_amd import cases

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch

    assert torch.cuda.is_available()
    B.lib()
    return torch


def Solver(*a, **k):
    from paper_2411_15001_amd.solver import Solver as S

    return S(*a, **k)


def _u0(nx, ny, seed=4):
    return np.ascontiguousarray(cases.riemann4(max(nx, ny), seed=seed)[:, :ny, :nx])


@pytest.mark.parametrize("prec", [B.LBM_FP64, B.LBM_FP32_STATE])
@pytest.mark.parametrize("lims", [1 | 8, 1 | 2 | 8])
def test_state_round_trip_and_step_between(prec, lims, gpu):
    """A planar state set into a blocked context comes back unchanged; one
    step between caller buffers (planar kernels) equals the context's own
    step (blocked kernels), and both equal the oracle in FP64."""
    torch = gpu
    nx, ny = 192, 41
    u0 = _u0(nx, ny)
    kw = dict(precision=prec, limiters=lims, a_beta=1.1, bc_x=1, bc_y=1)
    a = Solver(u0, **kw)
    a.step(5)
    S = a.get_state()
    b = Solver(u0, **kw)
    b.set_state(S)
    assert torch.equal(b.get_state(), S)
    # the context's own step
    b.step(1)
    own = b.get_state()
    # the same step between caller buffers
    dst = torch.empty_like(S)
    B.lbm_step_between(a.ctx, S, dst)
    assert torch.equal(dst, own)
    if prec == B.LBM_FP64:
        ocfg = oracle.Config(nx=nx, ny=ny, limiters=lims, a_beta=1.1, bc_x=1, bc_y=1)
        O, _ = oracle.init(ocfg, u0)
        O, _, _, _ = oracle.run(ocfg, O, 6)
        assert np.array_equal(own.cpu().numpy(), O)
    a.close()
    b.close()


@pytest.mark.parametrize("prec", [B.LBM_FP64, B.LBM_FP32_STATE])
def test_descriptions_set_mid_run_switch_to_planar(prec, gpu):
    """Zero-gradient descriptions on every side reproduce plain outflow, so a
    run that sets them after 5 steps (its state converted to the planar
    layout then) equals a run without them and one that had them from the
    start, after 12 steps, with the same counters."""
    nx, ny = 128, 70
    u0 = _u0(nx, ny, seed=8)
    kw = dict(precision=prec, limiters=1 | 2 | 8, a_beta=1.1, bc_x=1, bc_y=1)
    runs = []
    for when in (None, 0, 5):
        s = Solver(u0, **kw)
        for k in range(12):
            if k == when:
                for side in range(4):
                    s.set_boundary(side, np.zeros(ny if side < 2 else nx, np.uint8))
            s.step(1)
        d = s.diagnostics()
        runs.append((s.get_state().cpu().numpy(), [d["n_guard"], d["n_limited"], d["n_bad"], d["n_lmp"], d["lam"]]))
        s.close()
    for G, d in runs[1:]:
        assert np.array_equal(G, runs[0][0])
        assert d == runs[0][1]


def test_graph_replay_and_reductions_on_blocked_state(gpu):
    """Graph replays of the blocked kernels equal eager steps; moments,
    totals and minima read the blocked state as the planar one."""
    nx, ny = 256, 33
    u0 = _u0(nx, ny, seed=2)
    kw = dict(precision=B.LBM_FP32_STATE, limiters=1 | 8, a_beta=1.1, bc_x=1, bc_y=1)
    a, b = Solver(u0, **kw), Solver(u0, **kw)
    a.step(12)
    for _ in range(2):
        b.step_graph(6)
        b.moments(check=False)
    assert np.array_equal(a.get_state().cpu().numpy(), b.get_state().cpu().numpy())
    S = a.get_state().cpu().numpy()
    m = a.moments().cpu().numpy()
    assert np.array_equal(m, S[0:4].astype(np.float64))
    d = a.diagnostics()
    rho = S[0].astype(np.float64)
    rhoe = S[3].astype(np.float64) - 0.5 * (S[1].astype(np.float64) ** 2 + S[2].astype(np.float64) ** 2) / rho
    assert d["min_rho"] == rho.min()
    assert abs(d["min_rhoe"] - rhoe.min()) <= 1e-15 * abs(rhoe.min())
    tot = a.totals()
    for k in range(4):
        import math

        assert abs(tot[k] - math.fsum(S[k].astype(np.float64).ravel())) <= 4e-16 * abs(tot[k]) + 1e-300
    a.close()
    b.close()


@pytest.mark.parametrize("prec", [B.LBM_FP64, B.LBM_FP32_STATE])
def test_ensemble_blocked_layout(prec, gpu):
    """An ensemble whose widths are all multiples of 64 keeps the blocked
    layout (each instance's state after the ones before it): every instance
    equals its own single-instance run (and the oracle in FP64) after 8
    steps, also when zero-gradient descriptions set on one instance after 3
    steps switch the whole ensemble to the planar layout."""
    from paper_2411_15001_amd.solver import BatchSolver

    sizes = [(64, 40), (128, 70), (192, 33)]
    u0s = [_u0(nx, ny, seed=20 + i) for i, (nx, ny) in enumerate(sizes)]
    kw = dict(precision=prec, limiters=1 | 2 | 8, a_beta=1.1, bc_x=1, bc_y=1)
    # the ensemble's state round trip through the planar caller layout
    bs = BatchSolver(u0s, **kw)
    bs.step(2)
    S = bs.get_state()
    b2 = BatchSolver(u0s, **kw)
    b2.set_state(S)
    assert gpu.equal(b2.get_state(), S)
    for i in range(len(sizes)):
        assert np.array_equal(b2.moments(i).cpu().numpy(), bs.moments(i).cpu().numpy())
    bs.close()
    b2.close()
    for switch in (False, True):
        bs = BatchSolver(u0s, **kw)
        for k in range(8):
            if switch and k == 3:
                bs.set_boundary(1, 2, np.zeros(sizes[1][0], np.uint8))
            bs.step(1)
        for i, (nx, ny) in enumerate(sizes):
            s = Solver(u0s[i], dx=1.0 / nx, **kw)
            s.step(8)
            G = bs.moments(i).cpu().numpy()
            assert np.array_equal(G, s.moments().cpu().numpy()), (switch, i)
            s.close()
            if prec == B.LBM_FP64:
                ocfg = oracle.Config(nx=nx, ny=ny, dx=1.0 / nx, limiters=1 | 2 | 8, a_beta=1.1, bc_x=1, bc_y=1)
                O, _ = oracle.init(ocfg, u0s[i])
                O, _, _, _ = oracle.run(ocfg, O, 8)
                assert np.array_equal(G, O[0:4]), (switch, i)
        bs.close()
