"""The per-cell blending ablation (Section 3.1, eq. (naive_blending)) on the
GPU: bit for bit against the oracle's per-cell blending (states, face factors
and counters), its FP32 form against its FP64 form, graph replays, the
entry points that refuse it, and the ablation's outcome: where the face
blending of Section 3.2 keeps every cell admissible and every density inside
its bounds, the per-cell blending does not (the paper's reason for setting it
aside: it does not act as a flux limiter)."""
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


def okw(ocfg):
    return dict(dx=ocfg.params().dx, gamma=ocfg.gamma, alpha=ocfg.alpha, order=ocfg.order,
                limiters=ocfg.limiters, a_mode=ocfg.a_mode, a_beta=ocfg.a_beta, a_fixed=ocfg.a_fixed,
                bc_x=ocfg.bc_x, bc_y=ocfg.bc_y, sponge=ocfg.sponge, eps=ocfg.eps, rlmp_lo=ocfg.rlmp_lo,
                rlmp_hi=ocfg.rlmp_hi, blend=ocfg.blend)


def _u0(kind, nx, ny):
    m = max(nx, ny)
    u = {"r4": lambda: cases.riemann4(m, seed=5), "ll3": lambda: cases.lax_liu3(m),
         "blast": lambda: cases.blast(m, seed=0)}[kind]()
    return np.ascontiguousarray(u[:, :ny, :nx])


# kind, nx, ny, limiters, bc_x, bc_y, sponge, a_beta, steps
CASES = [
    ("r4", 48, 48, 1 | 8, 1, 1, 0, 1.1, 30),
    ("r4", 48, 48, 1 | 2 | 8, 1, 1, 0, 1.1, 30),
    ("r4", 70, 37, 4 | 8, 1, 0, 0, 1.0, 25),
    ("r4", 130, 66, 1 | 2 | 8, 1, 1, 3, 1.0, 20),
    ("r4", 5, 3, 2 | 8, 0, 1, 0, 1.0, 12),
    ("blast", 96, 96, 1 | 8, 0, 0, 0, 1.0, 40),
    ("blast", 64, 64, 1 | 2 | 8, 0, 0, 0, 1.0, 40),
    ("ll3", 64, 64, 1 | 8, 1, 1, 0, 1.0, 12),
    ("ll3", 64, 64, 0, 1, 1, 0, 1.0, 3),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "%s-%dx%d-l%d-bc%d%d-s%d" % c[:7])
def test_percell_bitwise(case, gpu):
    kind, nx, ny, lims, bx, by, sp, beta, steps = case
    u0 = _u0(kind, nx, ny)
    ocfg = oracle.Config(nx=nx, ny=ny, limiters=lims, bc_x=bx, bc_y=by, sponge=sp, a_beta=beta,
                         blend=oracle.BLEND_CELL)
    S, _ = oracle.init(ocfg, u0)
    s = Solver(u0, **okw(ocfg))
    tot = np.zeros(4, np.int64)
    for k in range(steps):
        if k == steps - 1:
            tx, ty = s.step_theta()
            S, otx, oty, info = oracle.step(ocfg, S)
            tot += (info.n_guard, info.n_limited, info.n_bad, info.n_lmp)
            assert np.array_equal(tx.cpu().numpy(), otx) and np.array_equal(ty.cpu().numpy(), oty)
        else:
            s.step(1)
            S, _, _, t = oracle.run(ocfg, S, 1)
            tot += t
    G = s.get_state().cpu().numpy()
    d = s.diagnostics()
    s.close()
    assert np.array_equal(G, S, equal_nan=True), np.nanmax(np.abs(G - S))
    assert [d["n_guard"], d["n_limited"], d["n_bad"], d["n_lmp"]] == tot.tolist(), (d, tot)


def test_percell_graph_replay_and_fp32(gpu):
    """Graph replays equal eager steps bit for bit; the FP32-state form stays
    within 1e-5 (relative L1 of the density) of the FP64 form over 20 steps
    of the four-quadrant problem with LMP."""
    n = 64
    u0 = cases.riemann4(n, seed=2)
    kw = dict(limiters=1 | 2 | 8, bc_x=1, bc_y=1, a_beta=1.1, blend=B.LBM_BLEND_CELL)
    a, b = Solver(u0, **kw), Solver(u0, **kw)
    a.step(12)
    for _ in range(2):
        b.step_graph(6)
        b.moments(check=False)  # eager work and a synchronisation between replays
    assert np.array_equal(a.get_state().cpu().numpy(), b.get_state().cpu().numpy())
    a.close()
    b.close()
    s64 = Solver(u0, **kw)
    s32 = Solver(u0, precision=B.LBM_FP32_STATE, **kw)
    s64.step(20)
    s32.step(20)
    r64 = s64.moments().cpu().numpy()[0]
    r32 = s32.moments().cpu().numpy()[0]
    e = np.abs(r32 - r64).sum() / np.abs(r64).sum()
    print("per-cell blending fp32 vs fp64 rel L1 rho: %.3e" % e)
    assert e <= 1e-5
    s64.close()
    s32.close()


def test_percell_refused_where_unsupported(gpu):
    import torch

    from paper_2411_15001_amd.solver import BatchSolver

    n = 32
    u0 = cases.riemann4(n, seed=1)
    with pytest.raises(B.LbmError) as e:
        BatchSolver([u0, u0], blend=B.LBM_BLEND_CELL)
    assert e.value.status == B.LBM_ENOTSUP
    s = Solver(u0, bc_x=1, blend=B.LBM_BLEND_CELL)
    with pytest.raises(B.LbmError) as e:
        s.set_boundary(B.LBM_WEST, np.full(n, B.LBM_BND_WALL, np.uint8))
    assert e.value.status == B.LBM_ENOTSUP
    U = s.get_state()
    with pytest.raises(B.LbmError) as e:
        B.lbm_step_adjoint(s.ctx, U.clone(), torch.zeros_like(U), torch.zeros_like(U))
    assert e.value.status == B.LBM_ENOTSUP
    st, _ = B.lbm_step_noalloc(B.make_params(n, n, blend=B.LBM_BLEND_CELL), U, torch.empty_like(U),
                               check=False)
    assert st == B.LBM_ENOTSUP
    s.close()
    assert B.lbm_workspace_bytes(B.make_params(n, n, blend=2)) == 0


@pytest.mark.parametrize("kind,n,lims,bc", [("ll3", 128, 1 | 8, 1), ("r4s0", 64, 1 | 8, 1), ("blast", 128, 1 | 8, 0),
                                            ("blast", 128, 1 | 2 | 8, 0), ("ll3", 128, 1 | 2 | 8, 1)])
def test_percell_ablation_outcome(kind, n, lims, bc, gpu):
    """The ablation's outcome, on the GPU and in the oracle alike: with the
    face blending every step stays admissible and (with LMP) every new
    density inside its eq. (29) bounds for 300 steps; with the per-cell
    blending and the same limiters a non-admissible cell appears (PP +
    pressure; the blast with LMP) or densities leave their bounds (LMP).
    Each run is compared with the oracle's step for step until the first
    event."""
    u0 = cases.riemann4(n, seed=0) if kind == "r4s0" else _u0(kind, n, n)
    beta = 1.1 if kind == "r4s0" else 1.0
    res = {}
    for blend in (B.LBM_BLEND_FACE, B.LBM_BLEND_CELL):
        s = Solver(u0, limiters=lims, bc_x=bc, bc_y=bc, a_beta=beta, blend=blend)
        first = None
        for k in range(300):
            s.step(1)
            d = s.diagnostics()
            if d["n_bad"] and first is None:
                first = k + 1
                break
        res[blend] = (first, d["n_lmp"], s.get_state().cpu().numpy(), k + 1)
        s.close()
    ocfg = oracle.Config(nx=n, ny=n, limiters=lims, bc_x=bc, bc_y=bc, a_beta=beta, blend=oracle.BLEND_CELL)
    S, _ = oracle.init(ocfg, u0)
    S, _, _, tot = oracle.run(ocfg, S, res[B.LBM_BLEND_CELL][3])
    assert np.array_equal(S, res[B.LBM_BLEND_CELL][2], equal_nan=True)
    print("%s %d^2 limiters %d: face blending first bad step %s, LMP-check cells %d; per-cell blending first "
          "bad step %s, LMP-check cells %d" % (kind, n, lims, res[0][0], res[0][1], res[1][0], res[1][1]))
    assert res[B.LBM_BLEND_FACE][0] is None and res[B.LBM_BLEND_FACE][1] == 0
    if lims & 2 and kind != "blast":
        assert res[B.LBM_BLEND_CELL][1] > 0
    else:
        assert res[B.LBM_BLEND_CELL][0] is not None
