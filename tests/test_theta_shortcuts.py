"""The step kernel's exact shortcuts in the face factor (the arguments are in
the comment above face_theta in csrc/step.hip), checked on the CPU in IEEE
float64 arithmetic with numpy, which rounds each operation as the kernel does
(no contraction): each test that lets a wave skip work must imply the result
the skipped formulas would give.  The samples crowd the tests' boundaries,
where a wrong margin would show.

* The square-root-free test implies the division-free test of the pressure
  factor (so skipping the square root changes nothing).
* The division-free tests imply theta^rho_PP >= 1 and theta^p >= 1 (Section
  3.3.3 and Section 3.4 formulas), so min(1, ...) is 1 without the
  divisions, for eps up to 1e-12.
"""
import numpy as np

C_FAST = 1.0 + 2.0 ** -30  # kFastMargin
M_PRE = 1.0 - 2.0 ** -26  # kPreMargin
N = 2_000_000


def _pre_test(X, g1, disc, fast_rho=True):
    tq = X * M_PRE - np.abs(g1)
    return fast_rho & (tq >= 2.0 ** -500) & (tq < 2.0 ** 500) & (disc <= (tq * tq) * M_PRE)


def _fast_test(X, g1, disc, fast_rho=True):
    Nn = np.abs(g1) + np.sqrt(disc)
    return fast_rho & (Nn * C_FAST <= X)


def test_square_root_free_test_implies_division_free_test():
    rng = np.random.default_rng(7)
    bad = 0
    hits = 0
    for scale in (-300, -40, 0, 40, 300):
        X = np.ldexp(0.5 + rng.random(N), rng.integers(scale - 20, scale + 20, N))
        g1 = np.where(rng.random(N) < 0.5, -1.0, 1.0) * X * rng.random(N) * 1.0000001
        t0 = X - np.abs(g1)
        # discriminants at, just below and just above the boundary (X - |g1|)^2
        f = 1.0 - np.ldexp(rng.random(N), -rng.integers(0, 45, N)) * np.where(rng.random(N) < 0.8, 1.0, -1.0)
        disc = np.where(t0 > 0, t0 * t0 * f, X * X * rng.random(N))
        disc = np.maximum(disc, 0.0)
        pre = _pre_test(X, g1, disc)
        fast = _fast_test(X, g1, disc)
        bad += int(np.count_nonzero(pre & ~fast))
        hits += int(np.count_nonzero(pre))
    assert bad == 0
    assert hits > N  # the test does fire on most admissible samples


def test_square_root_free_test_rejects_non_finite_values():
    X = np.array([np.inf, 1.0, 1.0, np.nan, 1.0])
    g1 = np.array([0.0, np.inf, 0.0, 0.0, np.nan])
    disc = np.array([0.0, 0.0, np.inf, 0.0, 0.0])
    assert not _pre_test(X, g1, disc).any()


def test_division_free_tests_imply_factor_one():
    rng = np.random.default_rng(11)
    u = 2.0 ** -53
    for eps in (0.0, 1e-16, 1e-12):
        kappa = np.ldexp(0.5 + rng.random(N), rng.integers(-10, 10, N))
        r0 = np.ldexp(0.5 + rng.random(N), rng.integers(-60, 20, N))
        # |D| near kappa rho* / c: the PP test's boundary
        D = kappa * r0 / C_FAST * (1.0 + np.ldexp(rng.random(N) - 0.5, -rng.integers(20, 60, N)))
        fast_rho = kappa * r0 >= np.abs(D) * C_FAST
        t_pp = kappa * r0 / np.abs(D) - eps
        assert (t_pp[fast_rho] >= 1.0).all()
        # pressure: N near kappa (-2 g0) / c
        g0 = -np.ldexp(0.5 + rng.random(N), rng.integers(-40, 40, N))
        Dn = -2.0 * g0
        Nn = kappa * Dn / C_FAST * (1.0 + np.ldexp(rng.random(N) - 0.5, -rng.integers(20, 60, N)))
        fast_p = fast_rho & (Nn * C_FAST <= kappa * Dn)
        e1 = np.abs(D) / r0
        e2 = Nn / Dn
        r = np.maximum(e1, e2)
        tp = kappa / r - eps
        assert (tp[fast_p] >= 1.0).all()
        assert np.count_nonzero(fast_p) > N // 10
        # the margin is what makes it exact: values within a few ulps of the
        # boundary exist on both sides
        assert np.count_nonzero(np.abs(t_pp - 1.0) < 64 * u) > 0
