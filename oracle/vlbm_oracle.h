/*
 * Plain FP64 CPU oracle of the blended D2Q5 vectorial lattice Boltzmann
 * scheme (Wissocq, Liu, Abgrall, "A positive- and bound-preserving vectorial
 * lattice Boltzmann method in two dimensions").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header or constant with the HIP library and never touches a GPU.
 *
 * State layout used by every entry point: S[20][ny][nx] (float64), plane
 * s*4 + c holds slot s in {u, u_1, u_2, u_3, u_4} (the moment slot u replaces
 * u_5, eq. (27)) and component c in {rho, m1, m2, E}.
 *
 * Face arrays: theta_x[ny][nx+1], entry (j, i) is the blending factor of the
 * x-face between cells (i-1, j) and (i, j); theta_y[ny+1][nx], entry (j, i) is
 * the factor of the y-face between cells (i, j-1) and (i, j).
 *
 * Conventions the paper leaves open, each pinned by the tests: M_k of step n
 * takes the current a^n and the distributions are carried over unchanged
 * when a changes (the multistep finite-difference form of the second-order
 * scheme, Section 2 and Appendix A, holds to rounding with a changing from
 * step to step, and fails for the alternatives); the event counters of
 * orc_info (n_limited and n_guard over the west and south face of every
 * cell, n_bad and n_lmp over the cells) equal brute-force counts over the
 * face factors, numpy face states and the new state.  The two zero-gradient
 * ghost layers of outflow boundaries (a copy of the boundary cell's moment
 * slot and all four distributions), the sponge layer (theta = 0 on every face
 * touching one of the first `sponge` cells of an outflow wall, ghosts
 * included) and the Dirichlet ghosts below are pinned against numpy
 * restatements on explicitly padded fields (Example 3 with theta = 1,
 * Lax-Friedrichs with theta = 0, the LMP factors of the boundary faces from
 * two padded layers).
 *
 * Boundary cells of kind wall or Dirichlet (Section 4.8 imposes boundary
 * states through the Maxwellians of those states and uses a reflective
 * symmetry wall, without further detail):
 * ghost layer g beyond a wall holds the mirror image of interior cell g - 1
 * (normal momentum negated in the moment slot and in every distribution, the
 * two distributions moving along the wall normal exchanged); a Dirichlet
 * ghost holds the given moments u_D with u_k = M_k(u_D; a^n) in both layers.
 * A ghost cell beyond a corner reads each side's kind at that side's boundary
 * cell nearest to it; walls resolve first (the ghost is the mirror image of
 * the ghost or cell across the wall), then a Dirichlet side, x before y (its
 * state at the resolved cell, mirrored by the walls crossed), then
 * zero-gradient.  lambda^n of a step also covers the Dirichlet states (a^n
 * must satisfy Bouchut's condition for every state the stencil reads); the
 * initial a^0 of orc_init covers u0 only.  Walls, corners included, are
 * pinned by periodic runs of mirror-symmetric data (walls on two opposite
 * sides, on all four, and beside Dirichlet sides whose states are mirror
 * symmetric too); the Dirichlet ghosts, both layers, lambda^n and the
 * Dirichlet-Dirichlet corners by padded fields as above.
 */
#ifndef VLBM_ORACLE_H
#define VLBM_ORACLE_H

#include <stdint.h>

#define ORC_RHO_PP 1u
#define ORC_RHO_LMP 2u
#define ORC_RHO_RLMP 4u
#define ORC_PRESSURE 8u

#define ORC_A_DYNAMIC 0
#define ORC_A_FIXED 1

#define ORC_BC_PERIODIC 0
#define ORC_BC_OUTFLOW 1

/* Kinds of the boundary cells of a non-periodic side (Section 4.8 uses all
 * three: Dirichlet states set as Maxwellians, a reflective symmetry wall,
 * zero-gradient outflow). */
#define ORC_BND_ZERO_GRADIENT 0
#define ORC_BND_WALL 1
#define ORC_BND_DIRICHLET 2

/* Sides of the grid, the index of bnd_kind / bnd_state. */
#define ORC_WEST 0
#define ORC_EAST 1
#define ORC_SOUTH 2
#define ORC_NORTH 3

typedef struct {
  int32_t nx, ny;
  double dx;
  double gamma, alpha;
  int32_t order;     /* 1: first-order scheme (theta = 0); 2: blended scheme */
  uint32_t limiters; /* ORC_RHO_* | ORC_PRESSURE; 0 with order 2 = unlimited */
  int32_t a_mode;    /* ORC_A_DYNAMIC: a = 2 beta lambda / (1 - alpha) */
  double a_beta, a_fixed;
  int32_t bc_x, bc_y;
  int32_t sponge;    /* theta = 0 on faces touching this many cells at an outflow wall */
  double eps, rlmp_lo, rlmp_hi;
  /* Optional per-cell boundary kinds of the four sides (host arrays of ny
   * entries for west and east, nx for south and north; NULL = every cell
   * zero-gradient) and the Dirichlet moments (rho, m1, m2, E) of the same
   * cells, [4][len] (read only where the kind is ORC_BND_DIRICHLET).  Only
   * on the sides of an axis whose bc is ORC_BC_OUTFLOW; walls need at least
   * two cells along their axis. */
  const uint8_t* bnd_kind[4];
  const double* bnd_state[4];
  /* ORC_BLEND_FACE: the face blending of Section 3.2 (eqs. (25), (27)), the
   * method.  ORC_BLEND_CELL: the per-cell blending that Section 3.1 states
   * first and sets aside (eq. (naive_blending)): every distribution leaving
   * a cell is blended with that cell's factor theta_ij.  The paper leaves
   * theta_ij open; the reading here is the smallest of the factors of the
   * cell's four faces (computed as for ORC_BLEND_FACE), and a ghost cell
   * takes the factor of the cell its state is copied from.  An ablation:
   * it conserves the moments but has no positivity guarantee. */
  int32_t blend;
} orc_params;

#define ORC_BLEND_FACE 0
#define ORC_BLEND_CELL 1

typedef struct {
  double lambda;     /* lambda^n of the input state */
  double a, dt, kappa;
  double lambda_new; /* lambda^{n+1} of the output state */
  int64_t n_guard;   /* faces whose intermediate state left the admissible set */
  int64_t n_limited; /* faces with theta < 1 (left and bottom faces of every
                        cell); with ORC_BLEND_CELL, cells with theta_ij < 1 */
  int64_t n_bad;     /* output cells with rho <= 0, p <= 0 or non-finite wavespeed */
  int32_t bouchut;   /* 1 if a < 2 lambda / (1 - alpha) */
  int64_t n_lmp;     /* with LMP or RLMP limiting: output cells whose new density
                        leaves the eq. (29) bounds [mu, nu] of the cell by more
                        than ORC_LMP_TOL relative (the convex decomposition of
                        eq. (28) keeps it inside under LMP) */
} orc_info;

/* Relative slack of the LMP check above: rounding of the update only. */
#define ORC_LMP_TOL 1e-12

#ifdef __cplusplus
extern "C" {
#endif

/* Flux and Maxwellians of one state; M is [4][4] (k = 1..4, component). */
void orc_flux(const double u[4], double gamma, double f[4], double g[4]);
void orc_maxwellians(const double u[4], double gamma, double alpha, double a,
                     double M[20]);
/* Face limiters of Section 3.3 / 3.4 for a single face. */
double orc_theta_rho_pp(double rho_star, double D, double kappa, double eps);
double orc_theta_rho_lmp(double rho_star, double D, double kappa, double muL,
                         double nuL, double muR, double nuR);
double orc_theta_p(const double ustar[4], const double dF[4], double kappa,
                   double eps);

/* Maximum wavespeed over cells of the moment slot; *nbad counts cells that
 * are not admissible (they are left out of the maximum). */
double orc_lambda(const orc_params* P, const double* S, int64_t* nbad);
/* Kinetic speed a^n for a given lambda^n. */
double orc_kinetic_speed(const orc_params* P, double lambda);

int orc_init(const orc_params* P, const double* u0, double* S, orc_info* info);
int orc_step(const orc_params* P, const double* S, double* Snew,
             double* theta_x, double* theta_y, orc_info* info);
int orc_run(const orc_params* P, double* S, double* work, int32_t nsteps,
            double* t, orc_info* last, int64_t totals[4]);

/* The step map with theta and a given (frozen). */
int orc_step_frozen(const orc_params* P, const double* S, const double* theta_x,
                    const double* theta_y, double a, double* Snew);
/* Complex-step evaluation of the same frozen maps: inputs S + i*Sim, outputs
 * real and imaginary parts. */
int orc_step_frozen_cs(const orc_params* P, const double* S, const double* Sim,
                       const double* theta_x, const double* theta_y, double a,
                       double* Snew, double* Snew_im);
int orc_init_frozen_cs(const orc_params* P, const double* u0,
                       const double* u0_im, double a, double* S, double* Sim);

int orc_num_threads(void);

#ifdef __cplusplus
}
#endif

#endif
