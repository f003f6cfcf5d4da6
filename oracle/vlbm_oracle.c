/*
 * Plain FP64 CPU oracle of the blended D2Q5 vectorial lattice Boltzmann
 * scheme for the 2D Euler equations (Wissocq, Liu, Abgrall).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  Scalar loops
 * over whole-grid arrays, one step in the order of the paper: kinetic speed,
 * ghost cells, per-cell Maxwellians, per-face intermediate states and
 * anti-diffusive fluxes, density bounds, blending factors, update.  Built with
 * -O2 -ffp-contract=off and no fast-math; the optional OpenMP pragmas split
 * independent rows and leave every result bit-identical.
 *
 * Readings of points the paper leaves open are listed with the function they
 * concern.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "vlbm_oracle.h"

/* Ghost-cell source index along one axis: periodic wrap, or the nearest
 * interior cell for the zero-gradient outflow condition of Section 4.2
 * (every distribution and the moment slot are copied). */
static int map_index(int i, int n, int bc) {
  if (bc == ORC_BC_PERIODIC) {
    int r = i % n;
    return r < 0 ? r + n : r;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

static double dmin(double a, double b) { return (b < a) ? b : a; }
static double dmax(double a, double b) { return (b > a) ? b : a; }

#define CAT_(a, b) a##b
#define CAT(a, b) CAT_(a, b)
#define FN(name) CAT(name, SFX)

#define REAL double
#define SFX _d
#include "model.inc"
#undef REAL
#undef SFX

#define REAL double complex
#define SFX _c
#include "model.inc"
#undef REAL
#undef SFX

/* ------------------------------------------------------------------------ */
/* Single-state helpers exposed for the pins.                                */

void orc_flux(const double u[4], double gamma, double f[4], double g[4]) {
  double s[20] = {0};
  for (int k = 0; k < 4; ++k) s[k] = u[k];
  cell_t_d c;
  cell_terms_d(s, gamma, 0.0, 0.0, &c);
  for (int k = 0; k < 4; ++k) {
    f[k] = c.f[k];
    g[k] = c.g[k];
  }
}

void orc_maxwellians(const double u[4], double gamma, double alpha, double a,
                     double M[20]) {
  double s[20] = {0};
  for (int k = 0; k < 4; ++k) s[k] = u[k];
  cell_t_d c;
  cell_terms_d(s, gamma, 0.25 * (1.0 - alpha), 1.0 / (2.0 * a), &c);
  for (int q = 0; q < 4; ++q)
    for (int k = 0; k < 4; ++k) M[4 * q + k] = c.M[q][k];
  /* M_5 = alpha u (Example 1) */
  for (int k = 0; k < 4; ++k) M[16 + k] = alpha * u[k];
}

/* ------------------------------------------------------------------------ */
/* Blending factors (Sections 3.3 and 3.4).                                  */

/* Section 3.3.3 (PP): theta^rho = max(0, kappa rho* / |D| - eps), D the density
 * component of the face's anti-diffusive flux.  D = 0 puts no constraint on
 * the face: +inf (each face uses its own D; the indices printed in the paper's
 * formula are garbled). */
double orc_theta_rho_pp(double rho_star, double D, double kappa, double eps) {
  if (D == 0.0) return INFINITY;
  const double t = kappa * rho_star / fabs(D) - eps;
  return dmax(0.0, t);
}

/* Section 3.3.1 (LMP), the final three-case formula for the face between the
 * left cell L (bounds muL, nuL) and the right cell R (muR, nuR):
 *   D = 0: 1;  D > 0: kappa min(nuR - rho*, rho* - muL) / D;
 *   D < 0: -kappa min(rho* - muR, nuL - rho*) / D.
 * The same function serves the relaxed bounds of Section 3.3.2. */
double orc_theta_rho_lmp(double rho_star, double D, double kappa, double muL,
                         double nuL, double muR, double nuR) {
  if (D == 0.0) return 1.0;
  if (D > 0.0) return kappa * dmin(nuR - rho_star, rho_star - muL) / D;
  return -kappa * dmin(rho_star - muR, nuL - rho_star) / D;
}

/* Section 3.4: pressure positivity.  With u* = (rho*, m1*, m2*, E*) and the
 * face flux (Dr, Dm1, Dm2, DE):
 *   g0 = m1*^2 + m2*^2 - 2 rho* E*,
 *   g1 = 2 (Dr E* + DE rho* - Dm1 m1* - Dm2 m2*),
 *   g2 = Dm1^2 + Dm2^2 - 2 Dr DE,   Delta = max(0, g1^2 - 4 g0 g2),
 *   r  = max(|Dr| / rho*, (|g1| + sqrt(Delta)) / (-2 g0)),
 *   theta^p = max(0, kappa / r - eps)  (+inf when r = 0).
 * r is the spectral radius of B^{-1/2} A B^{-1/2}; the energy entry of the
 * quadratic form built from Delta F is 2 DE (the denominator of phi is read
 * with 2 Delta F^E, consistent with the matrix A).  Requires rho* > 0 and
 * g0 < 0 (checked by the caller). */
double orc_theta_p(const double us[4], const double dF[4], double kappa,
                   double eps) {
  const double r0 = us[0], m1 = us[1], m2 = us[2], E = us[3];
  const double Dr = dF[0], Dm1 = dF[1], Dm2 = dF[2], DE = dF[3];
  const double g0 = m1 * m1 + m2 * m2 - 2.0 * r0 * E;
  const double g1 = 2.0 * (Dr * E + DE * r0 - Dm1 * m1 - Dm2 * m2);
  const double g2 = Dm1 * Dm1 + Dm2 * Dm2 - 2.0 * Dr * DE;
  double disc = g1 * g1 - 4.0 * g0 * g2;
  disc = dmax(0.0, disc);
  const double e1 = fabs(Dr) / r0;
  const double e2 = (fabs(g1) + sqrt(disc)) / (-2.0 * g0);
  const double r = dmax(e1, e2);
  if (r == 0.0) return INFINITY;
  return dmax(0.0, kappa / r - eps);
}

/* ------------------------------------------------------------------------ */
/* Kinetic speed (Section 4 preamble, Proposition 3).                        */

/* Wavespeed of one state: |v| + sqrt(gamma p / rho) (the definition used in
 * the numerical section).  Returns a negative value for a state that is not
 * admissible (rho <= 0, p <= 0 or a non-finite result). */
static double cell_wavespeed(const double u[4], double gamma) {
  const double rho = u[0], m1 = u[1], m2 = u[2], E = u[3];
  const double ir = 1.0 / rho;
  const double v1 = m1 * ir;
  const double v2 = m2 * ir;
  const double ke = 0.5 * (m1 * v1 + m2 * v2);
  const double p = (gamma - 1.0) * (E - ke);
  const double l = sqrt(v1 * v1 + v2 * v2) + sqrt(gamma * p * ir);
  if (!(rho > 0.0) || !(p > 0.0) || !(l <= 1.79769313486231570e308)) return -1.0;
  return l;
}

double orc_lambda(const orc_params* P, const double* S, int64_t* nbad) {
  const size_t plane = (size_t)P->nx * (size_t)P->ny;
  double lam = 0.0;
  int64_t bad = 0;
#pragma omp parallel for schedule(static) reduction(max : lam) reduction(+ : bad)
  for (size_t c = 0; c < plane; ++c) {
    const double u[4] = {S[c], S[plane + c], S[2 * plane + c], S[3 * plane + c]};
    const double l = cell_wavespeed(u, P->gamma);
    if (l < 0.0)
      bad += 1;
    else if (l > lam)
      lam = l;
  }
  if (nbad) *nbad = bad;
  return lam;
}

/* a^n = 2 beta lambda^n / (1 - alpha) (Proposition 3; beta = 1, alpha = 1/2
 * gives the paper's a^n = 4 lambda^n), or a fixed value (Section 4.1). */
double orc_kinetic_speed(const orc_params* P, double lambda) {
  if (P->a_mode == ORC_A_FIXED) return P->a_fixed;
  return 2.0 * P->a_beta * lambda / (1.0 - P->alpha);
}

static int check_params(const orc_params* P) {
  if (!P || P->nx < 1 || P->ny < 1) return -1;
  if (!(P->gamma > 1.0) || !(P->alpha >= 0.0 && P->alpha < 1.0)) return -1;
  if (P->order != 1 && P->order != 2) return -1;
  if (P->bc_x < 0 || P->bc_x > 1 || P->bc_y < 0 || P->bc_y > 1) return -1;
  if (P->a_mode == ORC_A_FIXED && !(P->a_fixed > 0.0)) return -1;
  if (P->a_mode == ORC_A_DYNAMIC && !(P->a_beta > 0.0)) return -1;
  if (P->blend != ORC_BLEND_FACE && P->blend != ORC_BLEND_CELL) return -1;
  for (int side = 0; side < 4; ++side) {
    const uint8_t* k = P->bnd_kind[side];
    if (!k) continue;
    const int ax = side / 2, len = ax == 0 ? P->ny : P->nx, n = ax == 0 ? P->nx : P->ny;
    if ((ax == 0 ? P->bc_x : P->bc_y) != ORC_BC_OUTFLOW) return -1;
    for (int r = 0; r < len; ++r) {
      if (k[r] > ORC_BND_DIRICHLET) return -1;
      if (k[r] == ORC_BND_WALL && n < 2) return -1;
      if (k[r] == ORC_BND_DIRICHLET && !P->bnd_state[side]) return -1;
    }
  }
  return 0;
}

/* Largest wavespeed of the Dirichlet boundary states (0 if none); counts the
 * non-admissible ones. */
static double bnd_lambda(const orc_params* P, int64_t* nbad) {
  double lam = 0.0;
  for (int side = 0; side < 4; ++side) {
    const uint8_t* k = P->bnd_kind[side];
    if (!k) continue;
    const int len = side < 2 ? P->ny : P->nx;
    for (int r = 0; r < len; ++r) {
      if (k[r] != ORC_BND_DIRICHLET) continue;
      const double* st = P->bnd_state[side];
      const double u[4] = {st[r], st[len + r], st[2 * (size_t)len + r], st[3 * (size_t)len + r]};
      const double l = cell_wavespeed(u, P->gamma);
      if (l < 0.0)
        *nbad += 1;
      else if (l > lam)
        lam = l;
    }
  }
  return lam;
}

int orc_init(const orc_params* P, const double* u0, double* S, orc_info* info) {
  if (check_params(P)) return -1;
  int64_t bad = 0;
  const double lam = orc_lambda(P, u0, &bad);
  const double a = orc_kinetic_speed(P, lam);
  if (info) {
    memset(info, 0, sizeof(*info));
    info->lambda = lam;
    info->lambda_new = lam;
    info->a = a;
    info->n_bad = bad;
  }
  if (bad) return 1;
  init_map_d(P, u0, a, S);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* One step.                                                                 */

typedef struct {
  double us[4]; /* intermediate state u* (eq. (12)) */
  double dF[4]; /* anti-diffusive flux (eq. (22)) */
} face_t;

/* Sponge layer of Section 4.2: cells within `sponge` cells of an outflow wall
 * (ghost cells included); faces touching such a cell take theta = 0. */
static int in_sponge(const orc_params* P, int i, int j) {
  const int s = P->sponge;
  if (s <= 0) return 0;
  if (P->bc_x == ORC_BC_OUTFLOW && (i < s || i >= P->nx - s)) return 1;
  if (P->bc_y == ORC_BC_OUTFLOW && (j < s || j >= P->ny - s)) return 1;
  return 0;
}

/* theta of one face from its intermediate state, its flux and the bounds of
 * its two cells: theta = min(1, selected theta^rho, theta^p) (Section 3.2).
 * A face whose u* is not admissible (rho* <= 0 or g0 >= 0, impossible under
 * the Bouchut condition) is set to the first-order value theta = 0 and
 * counted. */
static double face_theta(const orc_params* P, const face_t* fc, double kappa,
                         double muL, double nuL, double muR, double nuR,
                         int* guard) {
  *guard = 0;
  if (P->order == 1) return 0.0;
  if (P->limiters == 0) return 1.0;
  const double r0 = fc->us[0], m1 = fc->us[1], m2 = fc->us[2], E = fc->us[3];
  const double g0 = m1 * m1 + m2 * m2 - 2.0 * r0 * E;
  if (!(r0 > 0.0) || !(g0 < 0.0)) {
    *guard = 1;
    return 0.0;
  }
  double t = 1.0;
  const double D = fc->dF[0];
  if (P->limiters & ORC_RHO_PP) t = dmin(t, orc_theta_rho_pp(r0, D, kappa, P->eps));
  if (P->limiters & ORC_RHO_LMP)
    t = dmin(t, orc_theta_rho_lmp(r0, D, kappa, muL, nuL, muR, nuR));
  if (P->limiters & ORC_RHO_RLMP)
    t = dmin(t, orc_theta_rho_lmp(r0, D, kappa, P->rlmp_lo * muL, P->rlmp_hi * nuL,
                                  P->rlmp_lo * muR, P->rlmp_hi * nuR));
  if (P->limiters & ORC_PRESSURE) t = dmin(t, orc_theta_p(fc->us, fc->dF, kappa, P->eps));
  return t;
}

/* Per-cell blending (Section 3.1, eq. (naive_blending)): the distribution
 * k leaving the upwind cell U = (i - alpha_k, j - beta_k) is
 * M_k(u_U) + theta_U d_k(U), and the rest population of the cell itself is
 * M_5 + theta_ij (M_5 - u_5) with u_5 = u - sum_k u_k (eq. (27)), so the
 * moment slot becomes
 *   u^{n+1} = alpha u + sum over the four faces of (incoming distribution
 *             - theta_ij times the own distribution leaving through it),
 * grouped by face in the order W, E, S, N as in the face-blended update.
 * thW .. thN are the factors of the four upwind cells, thC the cell's own. */
static void update_cell_percell(const cell_t_d* C, const cell_t_d* W, const cell_t_d* E,
                                const cell_t_d* Sth, const cell_t_d* N, double thC, double thW,
                                double thE, double thS, double thN, double alpha, double out[20]) {
  for (int c = 0; c < 4; ++c) {
    const double u1n = W->M[0][c] + thW * W->d[0][c];
    const double u2n = E->M[1][c] + thE * E->d[1][c];
    const double u3n = Sth->M[2][c] + thS * Sth->d[2][c];
    const double u4n = N->M[3][c] + thN * N->d[3][c];
    double un = alpha * C->u[c];
    un = un + (u1n - thC * C->d[1][c]);
    un = un + (u2n - thC * C->d[0][c]);
    un = un + (u3n - thC * C->d[3][c]);
    un = un + (u4n - thC * C->d[2][c]);
    out[c] = un;
    out[4 + c] = u1n;
    out[8 + c] = u2n;
    out[12 + c] = u3n;
    out[16 + c] = u4n;
  }
}

int orc_step(const orc_params* P, const double* S, double* Snew, double* theta_x,
             double* theta_y, orc_info* info) {
  if (check_params(P)) return -1;
  const int nx = P->nx, ny = P->ny;
  const int gw = 2, pw = nx + 2 * gw, ph = ny + 2 * gw;

  /* S1: lambda^n, a^n, dt^n = dx / a^n (exact streaming), kappa^n. */
  int64_t bad0 = 0;
  const double lam = dmax(orc_lambda(P, S, &bad0), bnd_lambda(P, &bad0));
  const double a = orc_kinetic_speed(P, lam);
  const double kappa = 0.5 * a * (1.0 - P->alpha);
  const double w = 0.25 * (1.0 - P->alpha);
  const double r2a = 1.0 / (2.0 * a);
  const double r2k = 1.0 / (2.0 * kappa);

  /* S2 + S3: cell terms on the grid with two ghost layers. */
  cell_t_d* T = padded_terms_d(P, S, gw, w, r2a);
  face_t* FX = (face_t*)malloc(sizeof(face_t) * (size_t)pw * (size_t)ph);
  face_t* FY = (face_t*)malloc(sizeof(face_t) * (size_t)pw * (size_t)ph);
  double* mu = (double*)malloc(sizeof(double) * (size_t)pw * (size_t)ph);
  double* nu = (double*)malloc(sizeof(double) * (size_t)pw * (size_t)ph);
  double* tx = theta_x ? theta_x : (double*)malloc(sizeof(double) * (size_t)ny * (nx + 1));
  double* ty = theta_y ? theta_y : (double*)malloc(sizeof(double) * (size_t)(ny + 1) * nx);
  if (!T || !FX || !FY || !mu || !nu || !tx || !ty) return -2;

  /* S4: faces.  FX[p] is the x-face between padded cells p and p + 1:
   * u* = (u_L + u_R)/2 - (f_R - f_L)/(2 kappa)  (eq. (12), where
   * 2 beta lambda = a (1 - alpha) = 2 kappa), Delta F = a (d_1(L) - d_2(R))
   * (eq. (22)); FY[p] the y-face between p and p + pw with g, d_3 and d_4. */
#pragma omp parallel for schedule(static)
  for (int pj = 0; pj < ph; ++pj) {
    for (int pi = 0; pi < pw; ++pi) {
      const size_t p = (size_t)pj * pw + pi;
      if (pi + 1 < pw) {
        const cell_t_d *L = &T[p], *R = &T[p + 1];
        for (int c = 0; c < 4; ++c) {
          FX[p].us[c] = 0.5 * (L->u[c] + R->u[c]) - (R->f[c] - L->f[c]) * r2k;
          FX[p].dF[c] = a * (L->d[0][c] - R->d[1][c]);
        }
      }
      if (pj + 1 < ph) {
        const cell_t_d *L = &T[p], *R = &T[p + pw];
        for (int c = 0; c < 4; ++c) {
          FY[p].us[c] = 0.5 * (L->u[c] + R->u[c]) - (R->g[c] - L->g[c]) * r2k;
          FY[p].dF[c] = a * (L->d[2][c] - R->d[3][c]);
        }
      }
    }
  }

  /* S5: local density bounds, eq. (29): min / max of rho_ij and rho* on the
   * four faces of the cell, for the interior cells and one ghost ring. */
#pragma omp parallel for schedule(static)
  for (int pj = 1; pj < ph - 1; ++pj) {
    for (int pi = 1; pi < pw - 1; ++pi) {
      const size_t p = (size_t)pj * pw + pi;
      double lo = T[p].u[0], hi = T[p].u[0];
      const double rs[4] = {FX[p - 1].us[0], FX[p].us[0], FY[p - pw].us[0], FY[p].us[0]};
      for (int q = 0; q < 4; ++q) {
        lo = dmin(lo, rs[q]);
        hi = dmax(hi, rs[q]);
      }
      mu[p] = lo;
      nu[p] = hi;
    }
  }

  /* S6: blending factor of every face adjacent to an interior cell. */
  int64_t n_guard = 0, n_limited = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_guard, n_limited)
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i <= nx; ++i) {
      /* x-face between cells (i-1, j) and (i, j) */
      const size_t pL = (size_t)(j + gw) * pw + (size_t)(i - 1 + gw);
      int guard;
      double t = face_theta(P, &FX[pL], kappa, mu[pL], nu[pL], mu[pL + 1], nu[pL + 1], &guard);
      if (in_sponge(P, i - 1, j) || in_sponge(P, i, j)) t = 0.0;
      tx[(size_t)j * (nx + 1) + i] = t;
      if (i < nx) {
        n_guard += guard;
        n_limited += (t < 1.0);
      }
    }
  }
#pragma omp parallel for schedule(static) reduction(+ : n_guard, n_limited)
  for (int j = 0; j <= ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      /* y-face between cells (i, j-1) and (i, j) */
      const size_t pL = (size_t)(j - 1 + gw) * pw + (size_t)(i + gw);
      int guard;
      double t = face_theta(P, &FY[pL], kappa, mu[pL], nu[pL], mu[pL + pw], nu[pL + pw], &guard);
      if (in_sponge(P, i, j - 1) || in_sponge(P, i, j)) t = 0.0;
      ty[(size_t)j * nx + i] = t;
      if (j < ny) {
        n_guard += guard;
        n_limited += (t < 1.0);
      }
    }
  }

  /* S7: collide and stream. */
  if (P->blend == ORC_BLEND_CELL) {
    /* theta_ij = min of the cell's four face factors, for the interior
     * cells; a ghost cell takes the factor of the cell it copies (periodic
     * wrap or the nearest cell), read through map_index */
    double* tc = (double*)malloc(sizeof(double) * (size_t)nx * ny);
    if (!tc) return -2;
    n_limited = 0;
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        double t = tx[(size_t)j * (nx + 1) + i];
        t = dmin(t, tx[(size_t)j * (nx + 1) + i + 1]);
        t = dmin(t, ty[(size_t)j * nx + i]);
        t = dmin(t, ty[(size_t)(j + 1) * nx + i]);
        tc[(size_t)j * nx + i] = t;
        n_limited += (t < 1.0);
      }
    const size_t plane = (size_t)nx * (size_t)ny;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j) {
      for (int i = 0; i < nx; ++i) {
        const size_t pc = (size_t)(j + gw) * pw + (size_t)(i + gw);
        const int iw = map_index(i - 1, nx, P->bc_x), ie = map_index(i + 1, nx, P->bc_x);
        const int js = map_index(j - 1, ny, P->bc_y), jn = map_index(j + 1, ny, P->bc_y);
        double out[20];
        update_cell_percell(&T[pc], &T[pc - 1], &T[pc + 1], &T[pc - pw], &T[pc + pw],
                            tc[(size_t)j * nx + i], tc[(size_t)j * nx + iw], tc[(size_t)j * nx + ie],
                            tc[(size_t)js * nx + i], tc[(size_t)jn * nx + i], P->alpha, out);
        for (int q = 0; q < 20; ++q) Snew[(size_t)q * plane + (size_t)j * nx + i] = out[q];
      }
    }
    free(tc);
  } else {
    update_grid_d(P, T, gw, tx, ty, Snew);
  }

  /* LMP check: the new density of every cell against its eq. (29) bounds. */
  int64_t n_lmp = 0;
  if (P->order == 2 && (P->limiters & (ORC_RHO_LMP | ORC_RHO_RLMP))) {
#pragma omp parallel for schedule(static) reduction(+ : n_lmp)
    for (int j = 0; j < ny; ++j) {
      for (int i = 0; i < nx; ++i) {
        const size_t p = (size_t)(j + gw) * pw + (size_t)(i + gw);
        const double r = Snew[(size_t)j * nx + i];
        n_lmp += (r < mu[p] - ORC_LMP_TOL * fabs(mu[p])) || (r > nu[p] + ORC_LMP_TOL * fabs(nu[p]));
      }
    }
  }

  /* S8: diagnostics of the new state. */
  int64_t bad1 = 0;
  const double lam1 = orc_lambda(P, Snew, &bad1);
  if (info) {
    info->lambda = lam;
    info->a = a;
    info->dt = P->dx / a;
    info->kappa = kappa;
    info->lambda_new = lam1;
    info->n_guard = n_guard;
    info->n_limited = n_limited;
    info->n_bad = bad1;
    info->bouchut = (a < 2.0 * lam / (1.0 - P->alpha)) ? 1 : 0;
    info->n_lmp = n_lmp;
  }
  free(T);
  free(FX);
  free(FY);
  free(mu);
  free(nu);
  if (!theta_x) free(tx);
  if (!theta_y) free(ty);
  return 0;
}

/* nsteps steps in place (S <- S^{n+nsteps}); work holds one more state.
 * totals accumulates (n_guard, n_limited, n_bad, n_lmp) over the steps. */
int orc_run(const orc_params* P, double* S, double* work, int32_t nsteps,
            double* t, orc_info* last, int64_t totals[4]) {
  const size_t n = (size_t)20 * (size_t)P->nx * (size_t)P->ny;
  orc_info info;
  memset(&info, 0, sizeof(info));
  for (int32_t s = 0; s < nsteps; ++s) {
    const int rc = orc_step(P, S, work, NULL, NULL, &info);
    if (rc) return rc;
    memcpy(S, work, n * sizeof(double));
    if (t) *t += info.dt;
    if (totals) {
      totals[0] += info.n_guard;
      totals[1] += info.n_limited;
      totals[2] += info.n_bad;
      totals[3] += info.n_lmp;
    }
  }
  if (last) *last = info;
  return 0;
}

int orc_step_frozen(const orc_params* P, const double* S, const double* theta_x,
                    const double* theta_y, double a, double* Snew) {
  if (check_params(P)) return -1;
  return step_frozen_d(P, S, theta_x, theta_y, a, Snew);
}

int orc_step_frozen_cs(const orc_params* P, const double* S, const double* Sim,
                       const double* theta_x, const double* theta_y, double a,
                       double* Snew, double* Snew_im) {
  if (check_params(P)) return -1;
  const size_t n = (size_t)20 * (size_t)P->nx * (size_t)P->ny;
  double complex* z = (double complex*)malloc(sizeof(double complex) * n);
  double complex* zn = (double complex*)malloc(sizeof(double complex) * n);
  if (!z || !zn) return -2;
  for (size_t q = 0; q < n; ++q) z[q] = CMPLX(S[q], Sim[q]);
  const int rc = step_frozen_c(P, z, theta_x, theta_y, a, zn);
  for (size_t q = 0; q < n; ++q) {
    Snew[q] = creal(zn[q]);
    Snew_im[q] = cimag(zn[q]);
  }
  free(z);
  free(zn);
  return rc;
}

int orc_init_frozen_cs(const orc_params* P, const double* u0, const double* u0_im,
                       double a, double* S, double* Sim) {
  if (check_params(P)) return -1;
  const size_t plane = (size_t)P->nx * (size_t)P->ny;
  double complex* z = (double complex*)malloc(sizeof(double complex) * 4 * plane);
  double complex* zs = (double complex*)malloc(sizeof(double complex) * 20 * plane);
  if (!z || !zs) return -2;
  for (size_t q = 0; q < 4 * plane; ++q) z[q] = CMPLX(u0[q], u0_im[q]);
  init_map_c(P, z, a, zs);
  for (size_t q = 0; q < 20 * plane; ++q) {
    S[q] = creal(zs[q]);
    Sim[q] = cimag(zs[q]);
  }
  free(z);
  free(zs);
  return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
