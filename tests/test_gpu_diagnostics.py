"""Device diagnostics: compensated totals of the conserved moments and the
LMP check of the new density (the step-diagnostics row of the hot path)."""
import math

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


def solver(*a, **k):
    from paper_2411_15001_amd.solver import Solver

    return Solver(*a, **k)


@pytest.mark.parametrize("prec", [B.LBM_FP64, B.LBM_FP32_STATE])
def test_totals_are_exact_sums(prec):
    """lbm_totals equals the correctly rounded sum (math.fsum) of the stored
    moments to within a few roundings."""
    n = 640
    s = solver(cases.blast(n, seed=0), precision=prec, limiters=1 | 8)
    s.step(20)
    tot = s.totals()
    m = s.moments().cpu().numpy()
    for k in range(4):
        ref = math.fsum(m[k].ravel().tolist())
        scale = math.fsum(np.abs(m[k]).ravel().tolist())
        assert abs(tot[k] - ref) <= 4e-16 * scale, (k, tot[k], ref)
    s.close()


@pytest.mark.parametrize("prec,tol", [(B.LBM_FP64, 1e-13), (B.LBM_FP32_STATE, 1e-6)])
def test_conservation_periodic(prec, tol):
    """Periodic blast and four-quadrant data: the totals of rho, m1, m2 and E
    are conserved over 300 steps (Section 1) to the form's rounding
    (relative to the mass + energy scale)."""
    n = 512
    for u0, kw in ((cases.blast(n, seed=0), dict(limiters=1 | 8)),
                   (cases.riemann4(n, seed=5), dict(limiters=1 | 2 | 8, a_beta=1.1))):
        s = solver(u0, precision=prec, **kw)
        t0 = np.array(s.totals())
        s.step(300)
        t1 = np.array(s.totals())
        scale = abs(t0[0]) + abs(t0[3])
        assert np.all(np.abs(t1 - t0) <= tol * scale), (t0, t1)
        s.close()


def test_batch_totals_per_instance():
    """Per-instance totals of a batch equal those of the single runs."""
    from paper_2411_15001_amd.solver import BatchSolver

    u0s = [cases.riemann4(s, rng=np.random.default_rng([2, i])) for i, s in enumerate([64, 192, 128])]
    kw = dict(limiters=1 | 8, a_beta=1.1, bc_x=1, bc_y=1)
    bs = BatchSolver(u0s, **kw)
    bs.step(15)
    for i, u in enumerate(u0s):
        s = solver(u, dx=1.0 / u.shape[2], **kw)
        s.step(15)
        assert bs.totals(i) == s.totals()
        s.close()
    bs.close()


def test_lmp_check_full_size_blast():
    """The 8192^2 blast with PP + LMP + pressure, both forms, 20 steps: no
    new density leaves its eq. (29) bounds (the convex decomposition of
    eq. (28))."""
    import torch

    u0 = torch.from_numpy(cases.blast(8192, seed=0)).cuda()
    for prec in (B.LBM_FP64, B.LBM_FP32_STATE):
        s = solver(u0, precision=prec, limiters=1 | 2 | 8)
        s.step(20)
        d = s.diagnostics()
        assert d["n_lmp"] == 0 and d["n_bad"] == 0 and d["n_guard"] == 0, (prec, d)
        s.close()
