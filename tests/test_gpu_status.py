"""Device-detected events and state diagnostics: non-finite cells reported as
LBM_ENONFINITE ahead of LBM_EPOSITIVITY, the split of the non-admissible
count into non-finite, rho <= 0 and rho e <= 0 cells, and the minima of rho
and rho e (the scheme keeps both positive, Section 2) of the current state."""
import numpy as np
import pytest

from paper_2411_15001_amd import binding as B
from paper_2411_15001_amd import cases

pytestmark = pytest.mark.gpu

GAMMA = 1.4


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch

    assert torch.cuda.is_available()
    B.lib()
    return torch


def Solver(*a, **k):
    from paper_2411_15001_amd.solver import Solver as S

    return S(*a, **k)


def classify(m):
    """Numpy restatement of the device classification of a moment field
    [4, ny, nx] (float64): wavespeed |v| + sqrt(gamma p / rho) rejected when
    rho <= 0, p <= 0 or not finite; of those, (non-finite, rho <= 0,
    rho e <= 0) with p = (gamma - 1)(E - (m1 v1 + m2 v2)/2), v = m (1/rho)."""
    rho, m1, m2, E = (m[k].astype(np.float64) for k in range(4))
    with np.errstate(all="ignore"):
        ir = 1.0 / rho
        v1, v2 = m1 * ir, m2 * ir
        p = (GAMMA - 1.0) * (E - 0.5 * (m1 * v1 + m2 * v2))
        l = np.sqrt(v1 * v1 + v2 * v2) + np.sqrt(GAMMA * p * ir)
        bad = ~(rho > 0) | ~(p > 0) | ~(l <= 1.79769313486231570e308)
        fin = np.isfinite(rho) & np.isfinite(m1) & np.isfinite(m2) & np.isfinite(E)
        nf = bad & (~fin | ((rho > 0) & (p > 0)))
        nr = bad & fin & ~(rho > 0)
        ne = bad & fin & (rho > 0) & ~(p > 0)
    return int(bad.sum()), int(nf.sum()), int(nr.sum()), int(ne.sum())


def minima(m):
    rho, m1, m2, E = (m[k].astype(np.float64) for k in range(4))
    fin = np.isfinite(rho) & np.isfinite(m1) & np.isfinite(m2) & np.isfinite(E)
    rhoe = E - 0.5 * (m1 * m1 + m2 * m2) / rho
    return rho[fin].min(), rhoe[fin].min()


@pytest.mark.parametrize("prec", [B.LBM_FP64, B.LBM_FP32_STATE])
def test_injected_states_are_classified(prec, gpu):
    """A state loaded through lbm_set_state with one NaN cell gives
    LBM_ENONFINITE, one with rho < 0 or with p < 0 (finite) LBM_EPOSITIVITY,
    and the counts split accordingly; the minima of rho and rho e equal the
    numpy minima of the stored moments bit for bit."""
    n = 48
    s = Solver(cases.riemann4(n, seed=2), precision=prec, limiters=1 | 8, a_beta=1.1,
               bc_x=B.LBM_BC_OUTFLOW, bc_y=B.LBM_BC_OUTFLOW)
    s.step(3)
    good = s.get_state()
    m = good[0:4].double().cpu().numpy()
    d = s.diagnostics()
    mr, me = minima(m)
    assert d["min_rho"] == mr and d["min_rhoe"] == me, (d, mr, me)
    assert d["n_bad"] == d["n_nonfinite"] == d["n_rho"] == d["n_rhoe"] == 0
    cases_ = [("nan", lambda q: q.__setitem__((2, 5, 7), float("nan")), B.LBM_ENONFINITE, (1, 1, 0, 0)),
              ("inf", lambda q: q.__setitem__((3, 9, 1), float("inf")), B.LBM_ENONFINITE, (1, 1, 0, 0)),
              ("rho", lambda q: q.__setitem__((0, 11, 30), -0.25), B.LBM_EPOSITIVITY, (1, 0, 1, 0)),
              ("p", lambda q: q.__setitem__((3, 20, 20), 0.25 * float(q[1, 20, 20] ** 2 + q[2, 20, 20] ** 2)
                                            / float(q[0, 20, 20])), B.LBM_EPOSITIVITY, (1, 0, 0, 1))]
    for name, edit, status, counts in cases_:
        bad = good.clone()
        edit(bad)
        s.set_state(bad)
        d = s.diagnostics()
        assert (d["n_bad"], d["n_nonfinite"], d["n_rho"], d["n_rhoe"]) == counts, (name, d)
        mb = bad[0:4].double().cpu().numpy()
        mr, me = minima(mb)
        assert d["min_rho"] == mr and d["min_rhoe"] == me, (name, d, mr, me)
        _, st = s.moments(check=False)
        assert st == status, (name, st)
        assert s.diagnostics()["n_bad"] == 0  # moments() cleared the counters
    s.close()


def test_init_rejects_nonfinite_u0(gpu):
    n = 32
    u0 = cases.riemann4(n, seed=1)
    for val, status in ((float("nan"), B.LBM_ENONFINITE), (-1.0, B.LBM_EPOSITIVITY)):
        bad = u0.copy()
        bad[0, 3, 5] = val
        with pytest.raises(B.LbmError) as e:
            Solver(bad)
        assert e.value.status == status


@pytest.mark.parametrize("prec", [B.LBM_FP64, B.LBM_FP32_STATE])
@pytest.mark.parametrize("lims", [0, 2])
def test_step_counts_match_classification(prec, lims, gpu):
    """The unlimited scheme (and LMP without the pressure limiter) leaves the
    admissible set on Lax-Liu configuration 3 (Section 4.7); the counts the
    step kernel accumulates equal the classification of every step's output
    state, and lbm_moments reports LBM_ENONFINITE exactly when a non-finite
    cell was produced."""
    n = 64
    s = Solver(cases.lax_liu3(n), precision=prec, limiters=lims, bc_x=B.LBM_BC_OUTFLOW,
               bc_y=B.LBM_BC_OUTFLOW)
    tot = np.zeros(4, np.int64)
    for _ in range(12):
        s.step(1)
        tot += classify(s.get_state()[0:4].double().cpu().numpy())
    d = s.diagnostics()
    assert (d["n_bad"], d["n_nonfinite"], d["n_rho"], d["n_rhoe"]) == tuple(tot), (d, tot)
    assert d["n_bad"] > 0
    _, st = s.moments(check=False)
    assert st == (B.LBM_ENONFINITE if tot[1] else B.LBM_EPOSITIVITY)
    s.close()


@pytest.mark.parametrize("prec", [B.LBM_FP64, B.LBM_FP32_STATE])
def test_minima_of_an_ensemble_instance(prec, gpu):
    from paper_2411_15001_amd.solver import BatchSolver

    u0s = [cases.riemann4(n, seed=n) for n in (40, 72, 24)]
    bs = BatchSolver(u0s, precision=prec, limiters=1 | 8, a_beta=1.1, bc_x=B.LBM_BC_OUTFLOW,
                     bc_y=B.LBM_BC_OUTFLOW)
    bs.step(7)
    for i in range(3):
        m = bs.moments(i).cpu().numpy()
        d = bs.diagnostics(i)
        mr, me = minima(m)
        assert d["min_rho"] == mr and d["min_rhoe"] == me, (i, d, mr, me)
        assert d["min_rho"] > 0 and d["min_rhoe"] > 0
    bs.close()
