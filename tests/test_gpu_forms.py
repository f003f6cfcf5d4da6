"""The batching and differentiation forms on the GPU, checked against
single-instance runs, the FP64 oracle (bitwise / complex-step tangents) and
finite differences."""
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


def batch(*a, **k):
    from paper_2411_15001_amd.solver import BatchSolver

    return BatchSolver(*a, **k)


# ------------------------------------------------------------------ batching
SIZES = [(128, 128), (256, 256), (384, 384), (130, 70), (61, 200), (64, 64), (3, 17), (512, 128)]


@pytest.mark.parametrize("prec", [B.LBM_FP64, B.LBM_FP32_STATE])
@pytest.mark.parametrize("lims", [1 | 8, 1 | 2 | 8])
def test_batch_equals_single_instances(prec, lims):
    """Every instance of an uneven batch advanced in one launch per step is
    bit-identical to the same instance run alone (per-instance kinetic speed,
    dx = 1/nx)."""
    u0s = []
    for i, (nx, ny) in enumerate(SIZES):
        u = cases.riemann4(max(nx, ny), rng=np.random.default_rng([7, i]))
        u0s.append(np.ascontiguousarray(u[:, :ny, :nx]))
    kw = dict(limiters=lims, a_beta=1.1, bc_x=B.LBM_BC_OUTFLOW, bc_y=B.LBM_BC_OUTFLOW,
              precision=prec)
    bs = batch(u0s, **kw)
    bs.step(12)
    bs.step_graph(9)
    for i, u in enumerate(u0s):
        ny, nx = u.shape[1:]
        s = solver(u, dx=1.0 / nx, **kw)
        s.step(21)
        a = bs.moments(i).cpu().numpy()
        b = s.moments().cpu().numpy()
        assert np.array_equal(a, b), (i, nx, ny, np.abs(a - b).max())
        assert bs.diagnostics(i)["lam"] == s.diagnostics()["lam"]
        s.close()
    bs.close()


def test_batch_fp64_against_oracle():
    sizes = [(96, 96), (70, 130), (200, 64)]
    u0s = []
    for i, (nx, ny) in enumerate(sizes):
        u = cases.riemann4(max(nx, ny), rng=np.random.default_rng([3, i]))
        u0s.append(np.ascontiguousarray(u[:, :ny, :nx]))
    bs = batch(u0s, limiters=1 | 8, a_beta=1.1, bc_x=1, bc_y=1)
    bs.step(40)
    for i, u in enumerate(u0s):
        ny, nx = u.shape[1:]
        cfg = oracle.Config(nx=nx, ny=ny, dx=1.0 / nx, limiters=1 | 8, a_beta=1.1, bc_x=1, bc_y=1)
        S, _ = oracle.init(cfg, u)
        S, _, _, _ = oracle.run(cfg, S, 40)
        assert np.array_equal(bs.moments(i).cpu().numpy(), S[0:4])
    bs.close()


def test_batch_autotune_and_cache(tmp_path):
    u0s = [cases.riemann4(s, rng=np.random.default_rng([1, i]))
           for i, s in enumerate([128, 256, 128, 384])]
    bs = batch(u0s, precision=B.LBM_FP32_STATE, a_beta=1.1, bc_x=1, bc_y=1)
    ref = batch(u0s, precision=B.LBM_FP32_STATE, a_beta=1.1, bc_x=1, bc_y=1)
    cache = str(tmp_path / "tune.json")
    rows, waves, grid, mode = bs.autotune(cache)
    assert rows >= 4 and 1 <= waves <= 4 and grid in (0, 1, 2, 4) and mode in (0, 1)
    assert open(cache).read().count("[") == 1
    # tuning does not advance the state
    bs.step(10)
    ref.step(10)
    for i in range(4):
        assert np.array_equal(bs.moments(i).cpu().numpy(), ref.moments(i).cpu().numpy())
    # a second context reads the cached entry
    again = batch(u0s, precision=B.LBM_FP32_STATE, a_beta=1.1, bc_x=1, bc_y=1)
    assert again.autotune(cache) == (rows, waves, grid, mode)
    # an ensemble with the same first instance and cell count but other
    # sides, and one with other boundary conditions, get entries of their own
    other = batch([u0s[0], u0s[3], u0s[2], u0s[1]], precision=B.LBM_FP32_STATE, a_beta=1.1, bc_x=1, bc_y=1)
    other.autotune(cache)
    assert open(cache).read().count("[") == 2
    per = batch(u0s, precision=B.LBM_FP32_STATE, a_beta=1.1)
    per.autotune(cache)
    assert open(cache).read().count("[") == 3
    for x in (bs, ref, again, other, per):
        x.close()


def test_batch_state_round_trip_and_size_checks(gpu):
    """Restoring a saved ensemble state replays the same steps bit for bit
    (lambda^n is recomputed from the restored state); the bindings refuse
    tensors whose size does not match the context before any pointer reaches
    the library."""
    u0s = [cases.riemann4(s, rng=np.random.default_rng([9, i]))
           for i, s in enumerate([64, 128, 96])]
    bs = batch(u0s, precision=B.LBM_FP32_STATE, a_beta=1.1, bc_x=1, bc_y=1)
    s0 = bs.get_state()
    assert s0.numel() == B.lbm_state_bytes(bs.ctx) == 20 * 4 * sum(s * s for s in (64, 128, 96))
    bs.step(7)
    first = [bs.moments(i).cpu().numpy() for i in range(3)]
    bs.set_state(s0)
    bs.step(7)
    for i in range(3):
        assert np.array_equal(bs.moments(i).cpu().numpy(), first[i])
    f64 = gpu.float64
    with pytest.raises(ValueError):
        B.lbm_moments(bs.ctx, 1, gpu.empty((4, 64, 64), dtype=f64, device="cuda"))
    with pytest.raises(ValueError):
        B.lbm_moments(bs.ctx, 3, gpu.empty((4, 96, 96), dtype=f64, device="cuda"))
    with pytest.raises(ValueError):
        bs.set_state(s0[:-4])
    with pytest.raises(ValueError):
        B.lbm_get_state(bs.ctx, gpu.empty(s0.numel() + 8, dtype=gpu.uint8, device="cuda"))
    bs.close()
    s = solver(cases.gaussian_bump(32), a_mode=B.LBM_A_FIXED, a_fixed=7.0)
    st = s.get_state()
    with pytest.raises(ValueError):
        B.lbm_step_adjoint(s.ctx, st, st[:, :16].contiguous(), gpu.empty_like(st))
    with pytest.raises(ValueError):
        B.lbm_step_theta(s.ctx, gpu.empty((32, 32), dtype=f64, device="cuda"),
                         gpu.empty((33, 32), dtype=f64, device="cuda"))
    s.close()


# ----------------------------------------------------------- differentiation
def _dot(a, b):
    return float(np.sum(a * b))


@pytest.mark.parametrize("prec,lims", [(B.LBM_FP64, 1 | 8), (B.LBM_FP64, 1 | 2 | 8), (B.LBM_FP32_STATE, 1 | 8)])
def test_step_between_equals_steps(gpu, prec, lims):
    """Steps between caller buffers (lbm_step_between) give the states, face
    factors and scalars of the context's own steps bit for bit; meanwhile the
    calls that read the context's own state are refused, and lbm_set_state
    takes the context back to its buffers."""
    u0 = np.ascontiguousarray(cases.riemann4(130, seed=4)[:, :70, :])
    kw = dict(precision=prec, limiters=lims, a_beta=1.1, bc_x=1, bc_y=1)
    a = solver(u0, **kw)
    b = solver(u0, **kw)
    ny, nx = 70, 130
    f64 = gpu.float64
    # a captured graph of 2 steps exists before b leaves its buffers
    a.step(2)
    b.step_graph(2)
    buf = [b.get_state()]
    for i in range(6):
        tx, ty = a.step_theta()
        if i % 2 == 0:
            bx = gpu.empty((ny, nx + 1), dtype=f64, device="cuda")
            by = gpu.empty((ny + 1, nx), dtype=f64, device="cuda")
            dst = gpu.empty_like(buf[0])
            B.lbm_step_between(b.ctx, buf[-1], dst, bx, by)
            assert gpu.equal(tx, bx) and gpu.equal(ty, by)
        else:
            dst = gpu.empty_like(buf[0])
            B.lbm_step_between(b.ctx, buf[-1], dst)
        buf.append(dst)
        assert gpu.equal(a.get_state(), dst), i
    da, db = a.diagnostics(), b.diagnostics()
    for k in ("lam", "t", "step", "n_limited", "n_guard", "n_bad"):
        assert da[k] == db[k], k
    for call in (lambda: b.get_state(), lambda: b.step(1), lambda: b.moments(),
                 lambda: b.totals(), lambda: b.step_theta(), lambda: b.step_graph(2)):
        with pytest.raises(B.LbmError) as e:
            call()
        assert e.value.status == B.LBM_EINVAL
    with pytest.raises(B.LbmError) as e:  # overlapping buffers
        B.lbm_step_between(b.ctx, buf[-1], buf[-1])
    assert e.value.status == B.LBM_EINVAL
    b.set_state(buf[-1])
    a.step(3)
    b.step(3)
    assert gpu.equal(a.get_state(), b.get_state())
    a.close()
    b.close()


@pytest.mark.parametrize("lims", [1 | 8, 1 | 2 | 8])
def test_step_adjoint_dot_product(gpu, lims):
    """<J v, w> from the oracle's complex-step tangent of the step with theta
    and a frozen equals <v, J^T w> from lbm_step_adjoint (periodic, 64^2, a
    state with limited faces)."""
    n = 64
    cfg = oracle.Config(nx=n, ny=n, limiters=lims, a_beta=1.1)
    S, _ = oracle.init(cfg, cases.riemann4(n, seed=2))
    S, _, _, _ = oracle.run(cfg, S, 15)
    _, tx, ty, info = oracle.step(cfg, S)
    rng = np.random.default_rng(4)
    for _ in range(3):
        v = rng.normal(size=S.shape)
        w = rng.normal(size=S.shape)
        h = 1e-30
        _, im = oracle.step_frozen_cs(cfg, S, h * v, tx, ty, info.a)
        jv = im / h
        s = solver(cases.riemann4(n, seed=2), limiters=lims, a_beta=1.1)
        Ut = gpu.from_numpy(S).cuda()
        wt = gpu.from_numpy(w).cuda()
        out = gpu.empty_like(wt)
        B.lbm_step_adjoint(s.ctx, Ut, wt, out)
        jtw = out.cpu().numpy()
        lhs, rhs = _dot(jv, w), _dot(v, jtw)
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.linalg.norm(jv) * np.linalg.norm(w)), (lhs, rhs)
        s.close()
    assert info.n_limited > 0


ADJ_BC_CASES = [
    # nx, ny, bc_x, bc_y, sponge, limiters
    (64, 64, 1, 1, 0, 1 | 8),
    (61, 40, 1, 0, 0, 1 | 2 | 8),
    (50, 70, 0, 1, 3, 1 | 8),
    (72, 66, 1, 1, 4, 1 | 2 | 8),
    (2, 16, 1, 1, 0, 1 | 8),
    (1, 9, 1, 0, 0, 1 | 8),
]


@pytest.mark.parametrize("case", ADJ_BC_CASES, ids=lambda c: "%dx%d-bc%d%d-s%d-l%d" % c)
def test_step_adjoint_boundaries(gpu, case):
    """Outflow boundaries (one or both axes), sponge layers, ragged and
    degenerate widths: <J v, w> from the oracle's complex-step tangent of the
    step (theta and a frozen at the forward values, its ghosts built the same
    way) equals <v, J^T w> from lbm_step_adjoint."""
    nx, ny, bcx, bcy, sponge, lims = case
    u0 = np.ascontiguousarray(cases.riemann4(max(nx, ny), seed=7)[:, :ny, :nx])
    cfg = oracle.Config(nx=nx, ny=ny, dx=1.0 / max(nx, ny), limiters=lims, a_beta=1.1,
                        bc_x=bcx, bc_y=bcy, sponge=sponge)
    S, _ = oracle.init(cfg, u0)
    S, _, _, _ = oracle.run(cfg, S, 12)
    _, tx, ty, info = oracle.step(cfg, S)
    rng = np.random.default_rng(11)
    kw = dict(dx=1.0 / max(nx, ny), limiters=lims, a_beta=1.1, bc_x=bcx, bc_y=bcy, sponge=sponge)
    s = solver(u0, **kw)
    Ut = gpu.from_numpy(S).cuda()
    for _ in range(2):
        v = rng.normal(size=S.shape)
        w = rng.normal(size=S.shape)
        h = 1e-30
        _, im = oracle.step_frozen_cs(cfg, S, h * v, tx, ty, info.a)
        jv = im / h
        out = gpu.empty_like(Ut)
        B.lbm_step_adjoint(s.ctx, Ut, gpu.from_numpy(w).cuda(), out)
        lhs, rhs = _dot(jv, w), _dot(v, out.cpu().numpy())
        assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(jv) * np.linalg.norm(w), (lhs, rhs)
    s.close()


@pytest.mark.parametrize("fixed_a", [False, True])
@pytest.mark.parametrize("lims", [1 | 8, 1 | 2 | 8])
def test_step_adjoint_theta_equals_recomputed(gpu, lims, fixed_a):
    """lbm_step_adjoint_theta with the face factors lbm_step_theta wrote for
    U_n gives the same Ubar_n, bit for bit, as lbm_step_adjoint, which
    recomputes them (adaptive and fixed kinetic speed; limited faces present
    in the LMP cases)."""
    n = 64
    u0 = cases.riemann4(n, seed=2)
    kw = dict(limiters=lims, a_beta=1.1)
    if fixed_a:
        kw = dict(limiters=lims, a_mode=B.LBM_A_FIXED,
                  a_fixed=6.0 * oracle.lam(oracle.Config(nx=n, ny=n), u0)[0])
    s = solver(u0, **kw)
    s.step(10)
    U = s.get_state()
    tx = gpu.empty((n, n + 1), dtype=gpu.float64, device="cuda")
    ty = gpu.empty((n + 1, n), dtype=gpu.float64, device="cuda")
    B.lbm_step_theta(s.ctx, tx, ty)
    if lims & 2:  # the LMP bounds limit faces at every extremum
        assert bool((tx < 1).any()) and bool((ty < 1).any())
    w = gpu.from_numpy(np.random.default_rng(8).normal(size=(20, n, n))).cuda()
    a = gpu.empty_like(w)
    b = gpu.empty_like(w)
    B.lbm_step_adjoint(s.ctx, U, w, a)
    B.lbm_step_adjoint_theta(s.ctx, U, tx, ty, w, b)
    assert gpu.equal(a, b)
    with pytest.raises(B.LbmError):
        B.lbm_step_adjoint_theta(s.ctx, U, tx, ty, w, w)
    s.close()


def test_init_adjoint_dot_product(gpu):
    n = 48
    u0 = cases.gaussian_bump(n, seed=0)
    a0 = 7.0
    cfg = oracle.Config(nx=n, ny=n, a_mode=oracle.A_FIXED, a_fixed=a0)
    rng = np.random.default_rng(1)
    v = rng.normal(size=u0.shape)
    W = rng.normal(size=(20, n, n))
    _, im = oracle.init_frozen_cs(cfg, u0, 1e-30 * v, a0)
    jv = im / 1e-30
    s = solver(u0, a_mode=B.LBM_A_FIXED, a_fixed=a0)
    out = gpu.empty((4, n, n), dtype=gpu.float64, device="cuda")
    B.lbm_init_adjoint(s.ctx, gpu.from_numpy(u0).cuda(), gpu.from_numpy(W).cuda(), out)
    lhs, rhs = _dot(jv, W), _dot(v, out.cpu().numpy())
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(jv) * np.linalg.norm(W)
    s.close()


def _c4_setup(n=512, seed=0):
    u0 = cases.gaussian_bump(n, seed=seed)
    lam0 = oracle.lam(oracle.Config(nx=n, ny=n), u0)[0]
    a_fixed = 4.4 * lam0
    return u0, a_fixed


def test_rollout_gradient_finite_differences(gpu):
    """Differentiation workload: 512^2 periodic Gaussian bump, fixed kinetic
    speed, PP + pressure, 200 steps with checkpoints every 20; loss = half the
    squared density misfit to a target made from a shifted bump.  The
    gradient from the adjoint matches central finite differences on 32
    seeded directions to 1e-6 relative."""
    from paper_2411_15001_amd.autograd import rollout

    n, steps = 512, 200
    u0, a_fixed = _c4_setup(n)
    kw = dict(a_mode=B.LBM_A_FIXED, a_fixed=a_fixed, limiters=1 | 8)
    tgt_u0 = cases.gaussian_bump_target(n)
    st = solver(tgt_u0, **kw)
    st.step(steps)
    assert st.diagnostics()["n_limited"] == 0  # read before moments() clears it
    rho_tgt = st.moments()[0].clone()
    st.close()

    def loss_of(u):
        s = solver(u, **kw)
        s.step(steps)
        lim = s.diagnostics()["n_limited"]
        m = s.moments()
        s.close()
        return 0.5 * float(((m[0] - rho_tgt) ** 2).sum()), lim

    u0t = gpu.from_numpy(u0).cuda().requires_grad_(True)
    m = rollout(u0t, steps, 20, **kw)
    L = 0.5 * ((m[0] - rho_tgt) ** 2).sum()
    L.backward()
    g = u0t.grad.cpu().numpy()
    scale = np.array([np.abs(u0[0]).max(), 1.0, 1.0, np.abs(u0[3]).max()])[:, None, None]
    worst = 0.0
    for k in range(32):
        d = np.random.default_rng(100 + k).normal(size=u0.shape) * scale
        dl = _dot(g, d)
        fd = []
        for h in (1e-6, 5e-7):
            lp, limp = loss_of(u0 + h * d)
            lm, limm = loss_of(u0 - h * d)
            assert limp == 0 and limm == 0
            fd.append((lp - lm) / (2 * h))
        # Richardson combination of the two step sizes removes the h^2 term
        est = (4 * fd[1] - fd[0]) / 3
        err = abs(dl - est) / max(abs(dl), 1e-300)
        worst = max(worst, err)
    print("rollout FD worst relative error %.3e" % worst)
    assert worst <= 1e-6


@pytest.mark.parametrize("bc", [0, 1])
def test_rollout_gradient_vs_oracle_jvp(gpu, bc):
    """<grad L, d> from the GPU adjoint equals the oracle's complex-step
    directional derivative of the same rollout (theta and a frozen at the
    oracle's forward values) on a 64^2 grid with limited faces, periodic or
    with outflow boundaries on both axes."""
    from paper_2411_15001_amd.autograd import rollout

    n, steps = 64, 30
    u0 = cases.riemann4(n, seed=6)
    lam0 = oracle.lam(oracle.Config(nx=n, ny=n), u0)[0]
    a_fixed = 6.0 * lam0  # lambda grows by ~13% over the run; keeps a >= 4 lambda
    cfg = oracle.Config(nx=n, ny=n, limiters=1 | 2 | 8, a_mode=oracle.A_FIXED, a_fixed=a_fixed,
                        bc_x=bc, bc_y=bc)
    kw = dict(a_mode=B.LBM_A_FIXED, a_fixed=a_fixed, limiters=1 | 2 | 8, bc_x=bc, bc_y=bc)
    rng = np.random.default_rng(5)
    wgt = rng.normal(size=(n, n))
    u0t = gpu.from_numpy(u0).cuda().requires_grad_(True)
    m = rollout(u0t, steps, 7, **kw)
    L = (m[0] * gpu.from_numpy(wgt).cuda()).sum()
    L.backward()
    g = u0t.grad.cpu().numpy()
    d = rng.normal(size=u0.shape)
    h = 1e-30
    S, Sim = oracle.init_frozen_cs(cfg, u0, h * d, a_fixed)
    limited = 0
    for _ in range(steps):
        Sn, tx, ty, info = oracle.step(cfg, S)
        assert info.bouchut == 0
        limited += info.n_limited
        re, Sim = oracle.step_frozen_cs(cfg, S, Sim, tx, ty, info.a)
        S = Sn
    jvp = float(np.sum(wgt * Sim[0] / h))
    assert limited > 0
    assert abs(_dot(g, d) - jvp) <= 1e-9 * abs(jvp)
