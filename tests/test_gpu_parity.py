"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

The float64 kernel evaluates every expression in the oracle's order without
contraction, so states and face factors are compared bit for bit; the 1e-11
bound on the per-plane relative error is the acceptance bar."""
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


def Solver(*a, **k):
    from paper_2411_15001_amd.solver import Solver as S

    return S(*a, **k)


def BatchSolver(*a, **k):
    from paper_2411_15001_amd.solver import BatchSolver as S

    return S(*a, **k)


def rel_err(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    scale = np.maximum(np.abs(b).max(axis=1), 1e-300)[:, None]
    return float(np.max(np.abs(a - b) / scale))


def okw(ocfg):
    """lbm_params keywords matching an oracle Config."""
    return dict(dx=ocfg.params().dx, gamma=ocfg.gamma, alpha=ocfg.alpha, order=ocfg.order,
                limiters=ocfg.limiters, a_mode=ocfg.a_mode, a_beta=ocfg.a_beta,
                a_fixed=ocfg.a_fixed, bc_x=ocfg.bc_x, bc_y=ocfg.bc_y, sponge=ocfg.sponge,
                eps=ocfg.eps, rlmp_lo=ocfg.rlmp_lo, rlmp_hi=ocfg.rlmp_hi)


def test_c0_four_quadrant_parity():
    """64x64 four-quadrant problems, seeds 0-9, outflow, alpha = 1/2,
    a^n = 4.4 lambda^n, PP + pressure, 100 steps: full state within 1e-11 and
    bit-identical."""
    n, steps = 64, 100
    for seed in range(10):
        print("c0 seed", seed, flush=True)
        u0 = cases.riemann4(n, seed=seed)
        ocfg = oracle.Config(nx=n, ny=n, limiters=1 | 8, a_beta=1.1, bc_x=1, bc_y=1)
        S, _ = oracle.init(ocfg, u0)
        S, t_ref, info, _ = oracle.run(ocfg, S, steps)
        s = Solver(u0, **okw(ocfg))
        s.step(steps)
        G = s.get_state().cpu().numpy()
        d = s.diagnostics()
        s.moments()
        assert rel_err(G, S) <= 1e-11
        assert np.array_equal(G, S), "seed %d: max rel err %.3e" % (seed, rel_err(G, S))
        assert d["lam"] == info.lambda_new
        assert abs(d["t"] - t_ref) <= 1e-14 * t_ref
        s.close()


THETA_CASES = [
    # (nx, ny, limiters, order, bc_x, bc_y, sponge, evolve_steps, u0 kind)
    (61, 37, 1 | 8, 2, 0, 0, 0, 6, "riemann"),
    (130, 70, 2 | 8, 2, 1, 1, 0, 8, "riemann"),
    (100, 45, 4 | 8, 2, 0, 1, 0, 8, "riemann"),
    (64, 64, 1 | 2 | 8, 2, 1, 1, 0, 10, "riemann"),
    (70, 33, 0, 2, 0, 0, 0, 3, "smooth"),
    (50, 50, 1 | 8, 1, 1, 0, 0, 4, "riemann"),
    (4, 100, 2 | 8, 2, 0, 1, 5, 30, "sod"),
    (3, 17, 1 | 2 | 8, 2, 0, 0, 0, 5, "riemann"),
    (300, 130, 2 | 8, 2, 1, 1, 3, 6, "riemann"),
    (257, 65, 4 | 8, 2, 0, 0, 0, 6, "laxliu"),
    (1, 9, 1 | 8, 2, 1, 0, 0, 4, "riemann"),
    (2, 16, 1 | 2 | 8, 2, 1, 1, 0, 4, "riemann"),
]


def _u0(kind, nx, ny, seed=3):
    if kind == "sod":
        return cases.sod_y(ny, ncols=nx)
    if kind == "laxliu":
        u = cases.lax_liu3(max(nx, ny))
        return np.ascontiguousarray(u[:, :ny, :nx])
    if kind == "smooth":
        u = cases.gaussian_bump(max(nx, ny), seed=seed, amp=0.3, sigma=0.1)
        u = np.ascontiguousarray(u[:, :ny, :nx])
        u[1] = 0.2 * u[0]
        u[3] += 0.5 * u[1] ** 2 / u[0]
        return u
    u = cases.riemann4(max(nx, ny), seed=seed)
    return np.ascontiguousarray(u[:, :ny, :nx])


@pytest.mark.parametrize("case", THETA_CASES, ids=lambda c: "x".join(map(str, c[:2])) + "-l%d-o%d-bc%d%d-s%d" % c[2:7])
def test_theta_and_state_bitwise(case, gpu):
    """Face factors of one step and the new state equal the oracle's bit for
    bit, over limiter sets, both boundary conditions, a sponge, sizes that
    leave ragged strips and tiny grids."""
    nx, ny, lims, order, bcx, bcy, sponge, ev, kind = case
    print("theta case", case, flush=True)
    u0 = _u0(kind, nx, ny)
    ocfg = oracle.Config(nx=nx, ny=ny, dx=1.0 / max(nx, ny), limiters=lims, order=order,
                         bc_x=bcx, bc_y=bcy, sponge=sponge)
    S, _ = oracle.init(ocfg, u0)
    S, _, _, _ = oracle.run(ocfg, S, ev)
    S1, tx, ty, info = oracle.step(ocfg, S)
    s = Solver(u0, **okw(ocfg))
    s.set_state(gpu.from_numpy(S).cuda())
    gtx, gty = s.step_theta()
    G = s.get_state().cpu().numpy()
    d = s.diagnostics()
    assert np.array_equal(gtx.cpu().numpy(), tx)
    assert np.array_equal(gty.cpu().numpy(), ty)
    assert np.array_equal(G, S1), "max rel err %.3e" % rel_err(G, S1)
    assert d["n_limited"] == info.n_limited
    assert d["n_guard"] == info.n_guard
    assert d["n_lmp"] == info.n_lmp
    s.close()


@pytest.mark.parametrize("case", THETA_CASES, ids=lambda c: "x".join(map(str, c[:2])) + "-l%d-o%d-bc%d%d-s%d" % c[2:7])
def test_fp32_state_step_shapes(case, gpu):
    """One step of the float32-state form from the oracle's state (rounded to
    float32) against the oracle's float64 step from the same rounded state,
    on every plane of the new state, over the shapes, limiter sets and
    boundaries above (ragged strips, columns past the grid's edge, tiny
    grids): only float32 rounding separates them."""
    nx, ny, lims, order, bcx, bcy, sponge, ev, kind = case
    print("fp32 case", case, flush=True)
    u0 = _u0(kind, nx, ny)
    ocfg = oracle.Config(nx=nx, ny=ny, dx=1.0 / max(nx, ny), limiters=lims, order=order,
                         bc_x=bcx, bc_y=bcy, sponge=sponge)
    S, _ = oracle.init(ocfg, u0)
    S, _, _, _ = oracle.run(ocfg, S, ev)
    S32 = S.astype(np.float32)
    S1, _, _, _ = oracle.step(ocfg, S32.astype(np.float64))
    s = Solver(u0, precision=B.LBM_FP32_STATE, **okw(ocfg))
    s.set_state(gpu.from_numpy(S32).cuda())
    s.step(1)
    G = s.get_state().cpu().numpy().astype(np.float64)
    s.close()
    err = np.abs(G - S1).max() / np.abs(S1).max()
    assert err <= 2e-5, "max abs err %.3e relative to the state's largest value" % err


@pytest.mark.parametrize("prec,lims", [(B.LBM_FP64, 1 | 8), (B.LBM_FP64, 1 | 2 | 8),
                                       (B.LBM_FP32_STATE, 1 | 8), (B.LBM_FP32_STATE, 1 | 2 | 8)])
def test_fixed_limiter_kernels(prec, lims):
    """The kernels with the limiter set fixed at compile time (PP + pressure,
    PP + LMP + pressure), with and without face output (plain steps and
    lbm_step_theta), give the same states and counters bit for bit, and in
    float64 the oracle's states, on a 200 x 131 outflow grid with ragged
    strips (the general kernels meet the oracle in the face-factor cases with
    the other limiter sets)."""
    u0 = np.ascontiguousarray(cases.riemann4(200, seed=21)[:, :131, :])
    ocfg = oracle.Config(nx=200, ny=131, dx=1.0 / 200, limiters=lims, a_beta=1.1, bc_x=1, bc_y=1)
    a = Solver(u0, precision=prec, **okw(ocfg))
    b = Solver(u0, precision=prec, **okw(ocfg))
    for _ in range(15):
        a.step(1)
        b.step_theta()
    da, db = a.diagnostics(), b.diagnostics()
    G = a.get_state().cpu().numpy()
    assert np.array_equal(G, b.get_state().cpu().numpy())
    for k in ("n_limited", "n_guard", "n_bad", "n_lmp", "lam", "t"):
        assert da[k] == db[k], k
    if prec == B.LBM_FP64:
        S, _ = oracle.init(ocfg, u0)
        S, _, info, _ = oracle.run(ocfg, S, 15)
        assert np.array_equal(G, S), "max rel err %.3e" % rel_err(G, S)
    a.close()
    b.close()


# widths that are multiples of 64 take the LDS-staged bounds-limited march
# (PP + LMP + pressure, single instance); heights, strip heights, grids and
# boundaries vary the ring's prologue and tail
LDS_CASES = [
    # nx, ny, bc_x, bc_y, strip rows, waves, groups per CU, precision, limiters, sponge
    (64, 1, 1, 1, 4, 1, 0, B.LBM_FP64, 1 | 2 | 8, 0),
    (64, 3, 0, 0, 4, 4, 0, B.LBM_FP64, 1 | 2 | 8, 0),
    (128, 70, 1, 1, 16, 4, 0, B.LBM_FP64, 1 | 2 | 8, 0),
    (192, 37, 0, 1, 64, 2, 0, B.LBM_FP64, 1 | 2 | 8, 0),
    (256, 130, 1, 0, 8, 4, 1, B.LBM_FP64, 1 | 2 | 8, 0),
    (128, 64, 1, 1, 4096, 1, 0, B.LBM_FP64, 1 | 2 | 8, 0),
    (64, 5, 1, 1, 4, 4, 0, B.LBM_FP32_STATE, 1 | 2 | 8, 0),
    (192, 99, 1, 1, 32, 4, 0, B.LBM_FP32_STATE, 1 | 2 | 8, 0),
    (256, 64, 0, 0, 16, 2, 2, B.LBM_FP32_STATE, 1 | 2 | 8, 0),
    # PP + RLMP + pressure (a set fixed at compile time)
    (128, 70, 1, 1, 16, 4, 0, B.LBM_FP64, 1 | 4 | 8, 0),
    (192, 40, 0, 0, 8, 2, 0, B.LBM_FP32_STATE, 1 | 4 | 8, 0),
    # sets read at run time, sponge layers
    (128, 66, 1, 1, 8, 4, 0, B.LBM_FP64, 2 | 8, 0),
    (192, 50, 1, 1, 16, 4, 0, B.LBM_FP64, 1 | 2 | 4 | 8, 3),
    (128, 41, 1, 0, 4, 1, 0, B.LBM_FP64, 2, 5),
    (256, 33, 0, 1, 8, 4, 0, B.LBM_FP64, 4 | 8, 2),
    (256, 33, 0, 1, 8, 4, 0, B.LBM_FP32_STATE, 4 | 8, 0),
    (128, 60, 1, 1, 16, 4, 0, B.LBM_FP32_STATE, 1 | 2 | 8, 4),
    (192, 33, 1, 0, 8, 2, 0, B.LBM_FP32_STATE, 4 | 8, 2),
]


@pytest.mark.parametrize("case", LDS_CASES, ids=lambda c: "%dx%d-bc%d%d-h%d-w%d-g%d-p%d-l%d-s%d" % c)
def test_lds_staged_lmp_march(case, gpu):
    """The LDS-staged bounds-limited march (rows brought two ahead by direct
    loads into LDS) against the register-staged one: the same states,
    counters and face factors bit for bit, and in float64 the oracle's; for
    the limiter sets fixed at compile time and for those read at run time,
    with and without sponge layers.  The register-staged march is taken by
    an ensemble of two copies, or, with sponge layers (single instance only),
    by a run whose outflow sides are described as zero-gradient cells (the
    kernels that read descriptions, bit-identical to plain outflow)."""
    nx, ny, bx, by, rows, waves, gpc, prec, lims, sponge = case
    u0 = np.ascontiguousarray(cases.riemann4(max(nx, ny), seed=nx + ny)[:, :ny, :nx])
    ocfg = oracle.Config(nx=nx, ny=ny, limiters=lims, a_beta=1.1, bc_x=bx, bc_y=by, sponge=sponge)
    a = Solver(u0, precision=prec, **okw(ocfg))
    a.set_launch(rows, waves, groups_per_cu=gpc)
    steps = 12
    for k in range(steps):
        if k % 4 == 3:
            tx, ty = a.step_theta()
        else:
            a.step(1)
    G = a.get_state().cpu().numpy()
    da = a.diagnostics()
    ma = a.moments().cpu().numpy()
    a.close()
    if not sponge:
        kw = okw(ocfg)
        kw.pop("dx")
        b = BatchSolver([u0, u0], precision=prec, dx=[1.0 / nx] * 2, **kw)
        b.step(steps)
        db = b.diagnostics(0)  # before moments(), which clears the counters
        for i in range(2):
            assert np.array_equal(ma, b.moments(i).cpu().numpy()), i
    else:
        b = Solver(u0, precision=prec, **okw(ocfg))
        for side, axis_bc in ((B.LBM_WEST, bx), (B.LBM_EAST, bx), (B.LBM_SOUTH, by), (B.LBM_NORTH, by)):
            if axis_bc == B.LBM_BC_OUTFLOW:
                b.set_boundary(side, np.zeros(ny if side < 2 else nx, np.uint8))
        b.step(steps)
        db = b.diagnostics()
        assert np.array_equal(ma, b.moments().cpu().numpy())
    for k in ("n_guard", "n_limited", "n_bad", "n_lmp", "lam"):
        assert da[k] == db[k], (k, da[k], db[k])
    b.close()
    if prec == B.LBM_FP64:
        S, _ = oracle.init(ocfg, u0)
        S, _, _, tot = oracle.run(ocfg, S, steps - 1)
        S, otx, oty, info = oracle.step(ocfg, S)
        assert np.array_equal(G, S), "max rel err %.3e" % rel_err(G, S)
        assert np.array_equal(tx.cpu().numpy(), otx) and np.array_equal(ty.cpu().numpy(), oty)
        tot = np.array(tot) + (info.n_guard, info.n_limited, info.n_bad, info.n_lmp)
        assert [da["n_guard"], da["n_limited"], da["n_bad"], da["n_lmp"]] == tot.tolist()


def _table1():
    import os

    rows = {}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_entropy_wave.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        name, n, l1, l2, li = line.split()
        rows[(name, int(n))] = (float(l1), float(l2), float(li))
    return rows


TABLE1_LIMS = {"PP": 1 | 8, "LMP": 2 | 8, "RLMP": 4 | 8}


@pytest.mark.parametrize("n", [20, 40, 80, 160, 320, 640])
@pytest.mark.parametrize("lim", ["PP", "LMP", "RLMP"])
def test_table1_on_gpu(lim, n):
    """Section 4.1, Table 1 on the GPU: the entropy wave with a fixed kinetic
    speed a = 10.7 to t = 1 (10.7/dx steps) with the pressure limiter and each
    density limiter, at every printed resolution.  The relative L1, L2 and Linf
    errors of the density match every printed digit (PP and LMP), and the L1
    and L2 columns of RLMP; the RLMP Linf column is not reproduced by the
    definition that reproduces the other two sub-tables to every digit, so the
    measured value is printed and bounded.  The LMP rows at dx = 1/320 and
    1/640 agree to 3-4 digits (bounded below).  Up to dx = 1/320 the GPU state
    also equals the oracle's bit for bit."""
    ref = _table1()[(lim, n)]
    u0 = cases.entropy_wave(n)
    steps = int(round(10.7 * n))
    ocfg = oracle.Config(nx=n, ny=n, limiters=TABLE1_LIMS[lim], a_mode=1, a_fixed=10.7)
    s = Solver(u0, **okw(ocfg))
    s.step(steps)
    d = s.diagnostics()
    G = s.get_state().cpu().numpy()
    s.close()
    assert abs(d["t"] - 1.0) < 1e-12
    if lim == "PP":
        assert d["n_limited"] == 0  # theta = 1 on every face and step (Section 4.1)
    if n <= 320:
        S, _ = oracle.init(ocfg, u0)
        S, _, _, _ = oracle.run(ocfg, S, steps)
        assert np.array_equal(G, S), "max rel err %.3e" % rel_err(G, S)
    e = G[0] - u0[0]
    l1 = np.abs(e).sum() / np.abs(u0[0]).sum()
    l2 = math.sqrt((e * e).sum() / (u0[0] ** 2).sum())
    li = np.abs(e).max() / np.abs(u0[0]).max()
    print("Table 1 %s 1/%d: L1 %.5e L2 %.5e Linf %.5e (printed %s)" % (lim, n, l1, l2, li, ref))
    got = (l1, l2, li)
    if lim == "LMP" and n >= 320:
        # the LMP factor jumps where Delta F^rho changes sign at the wave's
        # extrema, so rounding-level differences of evaluation order move
        # these finest rows: measured 3.4e-4 (1/320) and 3.2e-3 (1/640) at
        # most, relative
        tol = 5e-4 if n == 320 else 4e-3
        for v, r in zip(got, ref):
            assert abs(v - r) <= tol * r, (v, r)
        return
    assert float("%.5e" % l1) == ref[0] and float("%.5e" % l2) == ref[1]
    if lim != "RLMP":
        assert float("%.5e" % li) == ref[2]
    else:
        assert li <= 1.3 * ref[2]


def test_c1_full_size(tmp_path, capsys):
    """2048^2 near-vacuum double rarefaction, PP + LMP + pressure, a = 4
    lambda^n, outflow, in the benchmark's launch shape (from a copy of the
    committed autotune cache): after the workload's 1000 steps the state equals
    the oracle's bit for bit (the oracle runs on the host's cores meanwhile,
    about three minutes, printing its progress), every step stayed admissible
    and every new density inside its LMP bounds.  The FP32-state form of the
    same run, in its own launch shape, stays admissible and within the
    precision form's 1e-4 relative L1 of the oracle's density after the 1000
    steps."""
    import os
    import shutil
    import time

    cache = str(tmp_path / "autotune_cache.json")
    shutil.copy(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                             "paper_2411_15001_amd", "autotune_cache.json"), cache)
    n, steps = 2048, 1000
    u0 = cases.double_rarefaction(n, seed=0)
    ocfg = oracle.Config(nx=n, ny=n, limiters=1 | 2 | 8, bc_x=1, bc_y=1)
    s = Solver(u0, **okw(ocfg))
    s.autotune(cache)
    s.step(steps)
    d = s.diagnostics()  # before moments(), which clears the counters
    G = s.get_state().cpu().numpy()
    m = s.moments().cpu().numpy()  # raises on a positivity event
    s.close()
    s32 = Solver(u0, precision=B.LBM_FP32_STATE, **okw(ocfg))
    s32.autotune(cache)
    s32.step(steps)
    d32 = s32.diagnostics()
    rho32 = s32.moments().cpu().numpy()[0]
    s32.close()
    assert d32["n_bad"] == 0 and d32["n_guard"] == 0
    assert d["n_bad"] == 0 and d["n_guard"] == 0
    # the new density never left the eq. (29) bounds over the 1000 steps
    assert d["n_lmp"] == 0
    p = 0.4 * (m[3] - 0.5 * (m[1] ** 2 + m[2] ** 2) / m[0])
    assert m[0].min() > 0 and p.min() > 0
    del m
    S, _ = oracle.init(ocfg, u0)
    t0 = time.time()
    tot = np.zeros(4, np.int64)
    for k in range(0, steps, 100):
        S, _, _, tt = oracle.run(ocfg, S, 100)
        tot += tt
        with capsys.disabled():
            print("  oracle C1: %d / %d steps, %.0f s" % (k + 100, steps, time.time() - t0), flush=True)
    assert tot[2] == 0 and tot[3] == 0
    assert np.array_equal(G, S), "max rel err %.3e" % rel_err(G, S)
    assert d["n_limited"] == tot[1]
    e32 = np.abs(rho32 - S[0]).sum() / np.abs(S[0]).sum()
    with capsys.disabled():
        print("  C1 FP32 form: rel L1 rho vs oracle after %d steps %.3e, LMP check %d" % (steps, e32, d32["n_lmp"]),
              flush=True)
    assert e32 <= 1e-4


def test_fp32_form_against_oracle():
    """FP32-state form (float32 collide/stream, float64 theta solve and
    wavespeed) against the FP64 oracle, relative L1 error of the density.

    Blast (p = 1e3 | 1e-2, periodic, PP + pressure, a = 4 lambda^n) at 256^2:
    <= 1e-4 after 100 steps.  After 500 steps the PP-limited blast amplifies
    any perturbation: the oracle itself, started from data perturbed by one
    float32 rounding (6e-8 relative), moves by ~3e-2, so the bound there is a
    small multiple of that floor.  Smooth data (Section 4.1 wave, 64^2,
    685 steps): <= 1e-5.  The FP64 form stays bit-identical throughout."""
    n = 256
    u0 = cases.blast(n, seed=0)
    ocfg = oracle.Config(nx=n, ny=n, limiters=1 | 8)
    S0, _ = oracle.init(ocfg, u0)
    S100, _, _, _ = oracle.run(ocfg, S0, 100)
    S500, _, _, _ = oracle.run(ocfg, S100, 400)
    rng = np.random.default_rng(1)
    Sp, _ = oracle.init(ocfg, u0 * (1 + 6e-8 * rng.uniform(-1, 1, u0.shape)))
    Sp, _, _, _ = oracle.run(ocfg, Sp, 500)

    def l1(a, b):
        return np.abs(a[0] - b[0]).sum() / np.abs(b[0]).sum()

    floor = l1(Sp, S500)
    s32 = Solver(u0, precision=B.LBM_FP32_STATE, **okw(ocfg))
    s32.step(100)
    e100 = l1(s32.moments().cpu().numpy(), S100)
    s32.step(400)
    assert s32.diagnostics()["n_bad"] == 0  # read before moments() clears it
    e500 = l1(s32.moments().cpu().numpy(), S500)
    print("fp32 blast rel L1 rho: 100 steps %.3e, 500 steps %.3e (oracle floor %.3e)"
          % (e100, e500, floor))
    assert e100 <= 1e-4
    assert e500 <= 3 * floor + 1e-4
    s64 = Solver(u0, **okw(ocfg))
    s64.step(500)
    assert np.array_equal(s64.get_state().cpu().numpy(), S500)
    s32.close()
    s64.close()
    n = 64
    u0 = cases.entropy_wave(n)
    ocfg = oracle.Config(nx=n, ny=n, limiters=1 | 8, a_mode=1, a_fixed=10.7)
    S, _ = oracle.init(ocfg, u0)
    S, _, _, _ = oracle.run(ocfg, S, 685)
    s32 = Solver(u0, precision=B.LBM_FP32_STATE, **okw(ocfg))
    s32.step(685)
    e = l1(s32.moments().cpu().numpy(), S)
    print("fp32 entropy wave rel L1 rho %.3e" % e)
    assert e <= 1e-5
    s32.close()


def test_fp32_form_1024_against_oracle():
    """The blast at 1024^2 (the accuracy size of the 8192^2 benchmark), 500
    steps, against the FP64 oracle.  The FP64 form equals the oracle bit for
    bit after all 500 steps.  The FP32-state form's relative L1 error of the
    density is held to 1.5 times its recorded value (2.9e-3): the PP-limited
    blast has become sensitive by then, the oracle itself moving by ~4.9e-3
    from a one-float32-rounding perturbation of the initial data, so the 1e-4
    target cannot hold at this size and horizon.  Both numbers are printed."""
    n, steps = 1024, 500
    u0 = cases.blast(n, seed=0)
    ocfg = oracle.Config(nx=n, ny=n, limiters=1 | 8)
    S, _ = oracle.init(ocfg, u0)
    S, _, _, _ = oracle.run(ocfg, S, steps)
    rng = np.random.default_rng(1)
    Sp, _ = oracle.init(ocfg, u0 * (1 + 6e-8 * rng.uniform(-1, 1, u0.shape)))
    Sp, _, _, _ = oracle.run(ocfg, Sp, steps)

    def l1(a, b):
        return np.abs(a[0] - b[0]).sum() / np.abs(b[0]).sum()

    floor = l1(Sp, S)
    s64 = Solver(u0, **okw(ocfg))
    s64.step(steps)
    assert np.array_equal(s64.get_state().cpu().numpy(), S)
    s64.close()
    s32 = Solver(u0, precision=B.LBM_FP32_STATE, **okw(ocfg))
    s32.step(steps)
    assert s32.diagnostics()["n_bad"] == 0  # read before moments() clears it
    e = l1(s32.moments().cpu().numpy(), S)
    print("fp32 blast 1024^2 rel L1 rho after %d steps %.3e (oracle floor %.3e)" % (steps, e, floor))
    assert e <= 1.5 * 2.9e-3
    assert e <= floor
    s32.close()


def test_graph_replay_equals_eager(gpu):
    """lbm_step_graph replays (with eager work and syncs between them) give the
    same states as eager launches, for every slot phase."""
    n = 96
    u0 = cases.riemann4(n, seed=5)
    kw = dict(limiters=1 | 2 | 8, bc_x=1, bc_y=1)
    a = Solver(u0, **kw)
    b = Solver(u0, **kw)
    for rep in range(4):
        a.step_graph(5)
        b.step(5)
        gpu.cuda.synchronize()
        x = gpu.ones(1000, device="cuda").sum().item()
        assert x == 1000
        assert gpu.equal(a.get_state(), b.get_state()), rep
    a.step_graph(7)
    b.step(7)
    assert gpu.equal(a.get_state(), b.get_state())
    assert a.diagnostics()["t"] == b.diagnostics()["t"]
    a.close()
    b.close()


def test_graph_replay_long_runs_in_chunks(gpu):
    """A graph replay longer than one graph (2 x 1020 + 7 steps, replayed in
    chunks of 1020 launches) equals eager stepping bit for bit."""
    n = 64
    u0 = cases.riemann4(n, seed=4)
    kw = dict(limiters=1 | 8, a_beta=1.1, bc_x=1, bc_y=1)
    a = Solver(u0, **kw)
    b = Solver(u0, **kw)
    a.step_graph(2 * 1020 + 7)
    b.step(2 * 1020 + 7)
    assert gpu.equal(a.get_state(), b.get_state())
    assert a.diagnostics()["step"] == b.diagnostics()["step"] == 2 * 1020 + 7
    a.close()
    b.close()


@pytest.mark.parametrize("lims", [1 | 8, 2 | 8])
def test_determinism(lims):
    """The state after 40 steps does not depend on the launch shape (strip
    height 4..256 rows, 1..4 waves per group) on a 200 x 131 grid whose strips
    end in ragged tails in both directions."""
    u0 = np.ascontiguousarray(cases.riemann4(200, seed=8)[:, :131, :])
    kw = dict(limiters=lims, bc_x=1, bc_y=1)
    a = Solver(u0, **kw)
    a.step(40)
    ref = a.get_state().cpu().numpy()
    a.close()
    for rows, waves in [(4, 1), (8, 4), (16, 1), (64, 2), (256, 4)]:
        b = Solver(u0, **kw)
        b.set_launch(strip_rows=rows, waves_per_group=waves)
        b.step(40)
        assert np.array_equal(ref, b.get_state().cpu().numpy()), (rows, waves)
        b.close()


@pytest.mark.parametrize("prec,lims", [(B.LBM_FP64, 1 | 8), (B.LBM_FP64, 2 | 8), (B.LBM_FP32_STATE, 1 | 8)])
def test_persistent_grid_equals_one_wave_per_strip(prec, lims):
    """A persistent grid (1 or 2 workgroups per compute unit, each wave
    looping over several strips) gives the state of the one-wave-per-strip
    launch bit for bit, eagerly and from a captured graph, on a 1000 x 700
    grid cut into 4-row strips (16 x 175 strips, several per wave)."""
    u0 = np.ascontiguousarray(cases.riemann4(1000, seed=12)[:, :700, :])
    kw = dict(precision=prec, limiters=lims, bc_x=1, bc_y=1)
    a = Solver(u0, **kw)
    a.set_launch(strip_rows=4, waves_per_group=1)
    a.step(30)
    ref = a.get_state().cpu().numpy()
    a.close()
    for gpc, waves in [(1, 1), (2, 4)]:
        b = Solver(u0, **kw)
        b.set_launch(strip_rows=4, waves_per_group=waves, groups_per_cu=gpc)
        assert b.launch() == (4, waves, gpc, 0)
        groups = B.lbm_get_grid(b.ctx)[1]
        assert groups % 8 == 0 and groups * waves < 16 * 175
        b.step(13)
        b.step_graph(17)
        assert np.array_equal(ref, b.get_state().cpu().numpy()), (gpc, waves)
        b.close()


def test_persistent_grid_batch():
    """An uneven ensemble under a persistent grid (waves striding across
    instances) equals its one-wave-per-strip run instance by instance."""
    u0s = [cases.riemann4(s, rng=np.random.default_rng([5, i]))
           for i, s in enumerate([128, 640, 256, 384, 1024, 128])]
    kw = dict(precision=B.LBM_FP32_STATE, a_beta=1.1, bc_x=1, bc_y=1)
    a = BatchSolver(u0s, **kw)
    b = BatchSolver(u0s, **kw)
    a.set_launch(strip_rows=8, waves_per_group=2)
    b.set_launch(strip_rows=8, waves_per_group=2, groups_per_cu=1)
    a.step(20)
    b.step_graph(20)
    for i in range(len(u0s)):
        assert np.array_equal(a.moments(i).cpu().numpy(), b.moments(i).cpu().numpy()), i
    a.close()
    b.close()


@pytest.mark.parametrize("prec,lims", [(B.LBM_FP32_STATE, 1 | 8), (B.LBM_FP64, 1 | 2 | 8)])
def test_strip_mode_batch(prec, lims):
    """Strip heights matched to each instance (mode 1: 32 rows for the small
    and ragged instances, 64 for the others, largest first) give every
    instance of an uneven ensemble the state of the uniform 64-row launch bit
    for bit, eagerly, from a graph and under a persistent grid."""
    sides = [(128, 128), (640, 640), (256, 256), (136, 200), (1024, 1024), (200, 72), (384, 384)]
    u0s = [np.ascontiguousarray(cases.riemann4(max(nx, ny), rng=np.random.default_rng([9, i]))[:, :ny, :nx])
           for i, (nx, ny) in enumerate(sides)]
    kw = dict(precision=prec, limiters=lims, a_beta=1.1, bc_x=1, bc_y=1)
    a = BatchSolver(u0s, **kw)
    a.set_launch(strip_rows=64, waves_per_group=2)
    a.step(12)
    for gpc in (0, 1):
        b = BatchSolver(u0s, **kw)
        b.set_launch(strip_rows=64, waves_per_group=2, groups_per_cu=gpc, strip_mode=1)
        assert b.launch() == (64, 2, gpc, 1)
        b.step(5)
        b.step_graph(7)
        for i in range(len(sides)):
            assert np.array_equal(a.moments(i).cpu().numpy(), b.moments(i).cpu().numpy()), (gpc, i)
        b.close()
    with pytest.raises(B.LbmError) as e:
        B.lbm_set_strip_mode(a.ctx, 2)
    assert e.value.status == B.LBM_EINVAL
    a.close()


def test_error_statuses(gpu):
    n = 32
    u0 = cases.riemann4(n, seed=1)
    bad_p = B.make_params(n, n, alpha=0.4)
    assert B.lbm_workspace_bytes(bad_p) == 0
    ws = gpu.empty(B.lbm_workspace_bytes(B.make_params(n, n)), dtype=gpu.uint8, device="cuda")
    u0t = gpu.from_numpy(u0).cuda()
    with pytest.raises(B.LbmError) as e:
        B.lbm_init(bad_p, u0t, ws)
    assert e.value.status == B.LBM_EINVAL
    with pytest.raises(ValueError):
        Solver(u0, alpha=0.4)
    bad = u0.copy()
    bad[0, 3, 5] = -1.0
    with pytest.raises(B.LbmError) as e:
        Solver(bad)
    assert e.value.status == B.LBM_EPOSITIVITY
    # the unlimited second-order scheme leaves the admissible set on Lax-Liu 3
    s = Solver(cases.lax_liu3(64), limiters=0, bc_x=1, bc_y=1)
    s.step(5)
    d = s.diagnostics()
    assert d["n_bad"] > 0 and d["n_bad"] == d["n_nonfinite"] + d["n_rho"] + d["n_rhoe"]
    _, st = s.moments(check=False)
    assert st == (B.LBM_ENONFINITE if d["n_nonfinite"] else B.LBM_EPOSITIVITY)
    s.close()
    # a fixed kinetic speed below the Bouchut bound is flagged
    s = Solver(u0, a_mode=B.LBM_A_FIXED, a_fixed=0.5)
    s.step(1)
    assert s.diagnostics()["bouchut"] == 1
    _, st = s.moments(check=False)
    assert st in (B.LBM_EBOUCHUT, B.LBM_EPOSITIVITY, B.LBM_EGUARD)
    s.close()
    # launch shapes outside their ranges
    s = Solver(u0)
    for bad_launch in [dict(strip_rows=2), dict(strip_rows=8192), dict(waves_per_group=5)]:
        with pytest.raises(B.LbmError) as e:
            s.set_launch(**bad_launch)
        assert e.value.status == B.LBM_EINVAL
    for bad_grid in (-1, 33):
        with pytest.raises(B.LbmError) as e:
            B.lbm_set_grid(s.ctx, bad_grid)
        assert e.value.status == B.LBM_EINVAL
    assert s.launch()[2] == 0
    s.close()


@pytest.mark.parametrize("alpha,beta,lims,prec", [(0.75, 1.0, 1 | 8, B.LBM_FP64), (0.6, 2.0, 1 | 2 | 8, B.LBM_FP64),
                                                  (0.9, 1.5, 4 | 8, B.LBM_FP64), (0.5, 3.0, 2 | 8, B.LBM_FP64),
                                                  (0.75, 1.25, 1 | 8, B.LBM_FP32_STATE)])
def test_rest_weight_and_speed_factor_variants(alpha, beta, lims, prec, gpu):
    """The D2Q5 rest weight alpha in [1/2, 1) (Proposition 3) and the kinetic
    speed factor beta >= 1 of a = 2 beta lambda / (1 - alpha): face factors
    and states after 10 steps bit for bit against the oracle (float64), or
    within 1e-5 relative L1 in density (float32 state); outflow, ragged strips."""
    nx, ny = 90, 70
    u0 = np.ascontiguousarray(cases.riemann4(90, seed=11)[:, :ny, :nx])
    ocfg = oracle.Config(nx=nx, ny=ny, dx=1.0 / 90, alpha=alpha, a_beta=beta, limiters=lims,
                         bc_x=1, bc_y=1)
    S0, _ = oracle.init(ocfg, u0)
    S, _, info, tot = oracle.run(ocfg, S0, 10)
    assert tot[2] == 0 and info.bouchut == 0
    s = Solver(u0, precision=prec, **okw(ocfg))
    s.step(10)
    d = s.diagnostics()
    assert d["n_bad"] == 0 and d["n_guard"] == 0
    if prec == B.LBM_FP64:
        assert np.array_equal(s.get_state().cpu().numpy(), S)
        S1, tx, ty, _ = oracle.step(ocfg, S)
        gtx, gty = s.step_theta()
        assert np.array_equal(gtx.cpu().numpy(), tx) and np.array_equal(gty.cpu().numpy(), ty)
        assert np.array_equal(s.get_state().cpu().numpy(), S1)
    else:
        rho = s.moments().cpu().numpy()[0]
        err = np.abs(rho - S[0]).sum() / np.abs(S[0]).sum()  # slot 0: the density
        assert err < 1e-5, err
    s.close()
