/*
 * vlbm.h - C ABI of the MI355X (gfx950) library for the positive- and
 * bound-preserving blended D2Q5 vectorial lattice Boltzmann scheme for the 2D
 * compressible Euler equations (Wissocq, Liu, Abgrall).
 *
 * Every time step is one fused collide-limit-stream kernel launch:
 *   - Maxwellians M_k (Example 1) and non-equilibrium parts d_k = M_k - u_k;
 *   - face intermediate states u* (eq. (12)) and anti-diffusive fluxes
 *     Delta F, Delta G (eq. (22));
 *   - density limiter theta^rho (PP, LMP or RLMP, Section 3.3) and the
 *     pressure-positivity limiter theta^p (Section 3.4), theta = min(1, ...);
 *   - blended update of u_1..u_4 (eq. (25)) and of the moment slot that
 *     replaces u_5 (eq. (27));
 *   - the maximum wavespeed lambda^{n+1} of the new state, which sets the next
 *     kinetic speed a^{n+1} = 2 beta lambda / (1 - alpha) (Section 4 preamble,
 *     Proposition 3) without a host synchronisation.
 *
 * Memory: the caller owns all device memory.  It passes one workspace buffer
 * of lbm_workspace_bytes() (or lbm_batch_workspace_bytes()) bytes, 256-byte
 * aligned, that must stay allocated until lbm_destroy(); the library carves it
 * into two state buffers, per-instance scalar slots and counters.  The library
 * allocates only its small host context.  It never allocates device memory.
 *
 * State layout (every caller buffer: lbm_get_state, lbm_set_state,
 * lbm_step_between, the adjoint, lbm_step_noalloc): 20 planes, plane
 * q = s*4 + c for slot s in {u, u_1, u_2, u_3, u_4} and component c in
 * {rho, m1, m2, E}; each plane holds the instances one after the other,
 * instance i as [ny_i][nx_i] row-major.  Element type: float64 (LBM_FP64)
 * or float32 (LBM_FP32_STATE).  A context may keep the same values in
 * another order in its own workspace buffers (when every instance's width is
 * a multiple of 64, with face blending and no boundary descriptions, the 20
 * values of every 64-cell run of a row lie together, each instance's state
 * after the ones before it); the calls that copy to or from caller buffers
 * convert.
 *
 * Streams: every enqueueing call is asynchronous on the stream given to the
 * init call (a hipStream_t passed as void*; NULL = default stream).  A context
 * is bound to that stream and is not thread-safe.  Calls never abort or throw:
 * they return an lbm_status; lbm_last_error() describes the last failure.
 * Events found on the device (non-admissible cells, a face state leaving the
 * admissible set, a kinetic speed below the Bouchut bound) are counted and
 * reported by the next synchronising call (lbm_moments, lbm_diagnostics).
 */
#ifndef VLBM_H
#define VLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_BND_ZERO_GRADIENT 0
#define LBM_BND_WALL 1
#define LBM_BND_DIRICHLET 2

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = 1,      /* invalid argument (parameters, pointers, sizes) */
  LBM_ENOTSUP = 2,     /* valid but not supported by this entry point */
  LBM_EDEVICE = 3,     /* a HIP runtime call failed */
  LBM_EPOSITIVITY = 4, /* a cell with rho <= 0 or p <= 0 was produced */
  LBM_ENONFINITE = 5,  /* a cell with a non-finite value (or wavespeed) was
                          produced; takes precedence over LBM_EPOSITIVITY */
  LBM_EBOUCHUT = 6,    /* a < 2 lambda / (1 - alpha) in a fixed-a run (eq. (5)) */
  LBM_EGUARD = 7       /* a face intermediate state u* left the admissible set */
} lbm_status;

/* Density limiters (Section 3.3) and the pressure limiter (Section 3.4). */
#define LBM_RHO_PP 1u
#define LBM_RHO_LMP 2u
#define LBM_RHO_RLMP 4u
#define LBM_PRESSURE 8u

#define LBM_A_DYNAMIC 0 /* a^n = 2 beta lambda^n / (1 - alpha) */
#define LBM_A_FIXED 1   /* a^n = a_fixed (Section 4.1) */

#define LBM_BC_PERIODIC 0
#define LBM_BC_OUTFLOW 1 /* zero gradient of every distribution (Section 4.2) */

#define LBM_FP64 0
#define LBM_FP32_STATE 1 /* float32 state and collide/stream arithmetic; the
                            theta solve and the wavespeed reduction in float64 */

typedef struct {
  int32_t nx, ny;     /* cells; 1 <= nx, ny < 2^30 and nx * ny < 2^32 per instance
                         (LBM_EINVAL otherwise; the adjoint also needs ny <= 65535) */
  double dx;          /* square cells; cell centres at (i + 1/2) dx */
  double gamma;       /* ideal-gas ratio, > 1 */
  double alpha;       /* rest weight of the D2Q5 model, in [1/2, 1) (Prop. 3) */
  int32_t order;      /* 1: first-order scheme (theta = 0); 2: blended scheme */
  uint32_t limiters;  /* LBM_RHO_* | LBM_PRESSURE; 0 with order 2 = unlimited */
  int32_t a_mode;     /* LBM_A_DYNAMIC or LBM_A_FIXED */
  double a_beta;      /* beta >= 1 for LBM_A_DYNAMIC */
  double a_fixed;     /* kinetic speed for LBM_A_FIXED, > 0 */
  int32_t bc_x, bc_y; /* LBM_BC_* per axis */
  int32_t sponge;     /* theta = 0 on faces touching the first `sponge` cells
                         of an outflow wall (Section 4.2); 0 = none */
  int32_t precision;  /* LBM_FP64 or LBM_FP32_STATE */
  double eps;         /* epsilon of the PP and pressure limiters (1e-16) */
  double rlmp_lo, rlmp_hi; /* relaxed bound factors (0.999, 1.001) */
  int32_t unsafe;     /* 1 allows alpha < 1/2 or beta < 1 (no positivity
                         guarantee); 0 rejects them */
  int32_t blend;      /* LBM_BLEND_FACE (0): the face blending of Section 3.2,
                         eqs. (25), (27), the method; LBM_BLEND_CELL (1): the
                         per-cell blending that Section 3.1 states first and
                         sets aside (eq. (naive_blending)), an ablation */
} lbm_params;

/* Blending of the first- and second-order updates.  LBM_BLEND_CELL blends
 * every distribution leaving a cell with that cell's factor theta_ij, taken
 * as the smallest factor of the cell's four faces (a ghost cell takes the
 * factor of the cell it copies); it conserves the moments but guarantees no
 * positivity.  Single instance, no wall or Dirichlet cells, no adjoint
 * (LBM_ENOTSUP); every step then runs the fused kernel for the face factors
 * and a plain per-cell update kernel, and n_limited counts cells with
 * theta_ij < 1. */
#define LBM_BLEND_FACE 0
#define LBM_BLEND_CELL 1

typedef struct {
  double lambda;       /* lambda^n of the current state (instance 0 / inst) */
  double a;            /* a^n that the next step will use */
  double t;            /* accumulated time t^n */
  int64_t step;        /* steps taken since init */
  int64_t n_guard;     /* faces with u* outside the admissible set */
  int64_t n_limited;   /* faces with theta < 1 (left and bottom face of every cell) */
  int64_t n_bad;       /* non-admissible cells: n_nonfinite + n_rho + n_rhoe */
  int32_t bouchut;     /* a fixed a fell below 2 lambda / (1 - alpha) */
  int64_t n_lmp;       /* with LMP or RLMP limiting (order 2): cells whose new
                          density left the eq. (29) bounds [mu, nu] of the cell
                          by more than the update's rounding (1e-12 relative in
                          float64, 2e-6 with the float32 state).  Zero under LMP
                          (eq. (28)); RLMP relaxes the bounds, so it may count
                          there.  A check, not an error: no call fails on it. */
  int64_t n_nonfinite; /* of n_bad: a component of (rho, m1, m2, E) or the
                          wavespeed is not finite */
  int64_t n_rho;       /* of n_bad: finite, rho <= 0 */
  int64_t n_rhoe;      /* of n_bad: finite, rho > 0, internal energy
                          rho e = E - |m|^2 / (2 rho) <= 0 (p <= 0) */
  double min_rho;      /* minimum of rho over the finite cells of the current
                          state of instance inst (+inf if none; NaN after
                          lbm_step_between, whose state is in a caller buffer) */
  double min_rhoe;     /* minimum of rho e over the same cells (Section 2: the
                          scheme keeps rho > 0 and rho e > 0) */
} lbm_diag;

typedef struct lbm_ctx lbm_ctx;

/* Bytes of workspace for one instance / a batch of n instances (sizes nx[i],
 * ny[i]; all other parameters shared).  0 on invalid arguments. */
size_t lbm_workspace_bytes(const lbm_params* p);
size_t lbm_batch_workspace_bytes(const lbm_params* p, int32_t n,
                                 const int32_t* nx, const int32_t* ny);

/* Initialisation (Section 4 preamble): the moment slot takes u0 and
 * u_k = M_k(u0; a^0), k = 1..4, with lambda^0 and a^0 from u0.
 * u0_dev: float64 [4][ny][nx] (rho, m1, m2, E), device memory, read only.
 * Synchronises once to check that every cell of u0 is admissible
 * (LBM_ENONFINITE if a value is not finite, LBM_EPOSITIVITY if rho <= 0 or
 * p <= 0; no context is returned then).  On success *out owns a
 * host context bound to `stream` (free with lbm_destroy). */
lbm_status lbm_init(const lbm_params* p, const double* u0_dev, void* workspace_dev,
                    void* stream, lbm_ctx** out);

/* Batch of n independent instances sharing every parameter except nx, ny and
 * dx (dx[i] = 1/nx[i] when dx_host is NULL).  u0_packed_dev concatenates the
 * instances' float64 [4][ny_i][nx_i] blocks. */
lbm_status lbm_init_batch(const lbm_params* p, int32_t n, const int32_t* nx,
                          const int32_t* ny, const double* dx_host,
                          const double* u0_packed_dev, void* workspace_dev,
                          void* stream, lbm_ctx** out);

/* nsteps time steps (eqs. (25), (27) with the limiters of Section 3), one
 * kernel launch each, asynchronous, no host synchronisation.  The launches
 * may be recorded into a caller's hipGraph; each bakes in the step's phase
 * (lambda slot step mod 3, state buffer step mod 2) and the context counts
 * the steps once, at record time.  A recording of a multiple of 6 steps
 * returns to its starting phase, so it can be replayed any number of times
 * (the state, lambda and t follow the replays; the host-side step count
 * reported by lbm_diagnostics does not);
 * other recordings are replayed once.  lbm_step_graph does this
 * bookkeeping itself. */
lbm_status lbm_step(lbm_ctx* ctx, int32_t nsteps);

/* Same steps, replayed from a hipGraph of the launches (captured on first use
 * for each (length, phase) and cached in the context, at most 32 graphs).  A
 * graph holds at most 1020 launches; longer runs replay it (1020 is a
 * multiple of the 6-step phase period, so one graph serves every chunk).  The
 * first call for a new length synchronises with the capture; later calls are
 * asynchronous. */
lbm_status lbm_step_graph(lbm_ctx* ctx, int32_t nsteps);

/* One step that also writes the face factors: theta_x_dev float64
 * [ny][nx + 1] (x-face between cells (i-1, j) and (i, j)), theta_y_dev
 * float64 [ny + 1][nx] (y-face between (i, j-1) and (i, j)).  Single
 * instance only. */
lbm_status lbm_step_theta(lbm_ctx* ctx, double* theta_x_dev, double* theta_y_dev);

/* One step of the context whose state is read from src_dev and written to
 * dst_dev, caller buffers of lbm_state_bytes in the state layout, instead of
 * the context's own buffers; theta_x_dev / theta_y_dev as in lbm_step_theta
 * (both NULL: no face output).  The step count, lambda, t and counters
 * advance as for lbm_step, so src_dev must hold the state the context is at:
 * a copy of its current state (lbm_get_state after lbm_init, lbm_step or
 * lbm_set_state) or the dst_dev of the previous lbm_step_between.  Afterwards the context's current
 * state lives in dst_dev: lbm_step, lbm_step_graph, lbm_step_theta,
 * lbm_moments, lbm_totals, lbm_get_state and lbm_autotune return LBM_EINVAL
 * until lbm_set_state loads a state again.  For recomputing a segment of a
 * rollout step by step without copying each state out.  Single instance;
 * LBM_EINVAL if src and dst overlap or either is one of the context's own
 * state buffers.
 * Asynchronous. */
lbm_status lbm_step_between(lbm_ctx* ctx, const void* src_dev, void* dst_dev,
                            double* theta_x_dev, double* theta_y_dev);

/* Moments (rho, m1, m2, E) of instance `inst` as float64 [4][ny][nx] into
 * u_out_dev.  Synchronises the stream; returns the first device event counted
 * since the last synchronising call (LBM_EPOSITIVITY, LBM_EGUARD,
 * LBM_EBOUCHUT) or LBM_OK, and clears the counters. */
lbm_status lbm_moments(lbm_ctx* ctx, int32_t inst, double* u_out_dev);

/* Totals of the conserved moments of instance `inst` over its cells:
 * totals_host[0..3] = sum of rho, m1, m2, E of the moment slot (multiply by
 * dx^2 for the integrals), by compensated (double-double) summation, so the
 * result is within a few roundings of the exact sum of the stored values.
 * On periodic grids the scheme conserves them (Section 1), so two calls
 * bracket the conservation error of the steps between them.  totals_host is
 * host memory for 4 doubles.  Synchronises; clears no counter. */
lbm_status lbm_totals(lbm_ctx* ctx, int32_t inst, double* totals_host);

/* Diagnostics of instance `inst`: the counters accumulated since the last
 * lbm_moments, and the minima of rho and rho e of the current state (one
 * reduction kernel).  Synchronises; does not clear counters. */
lbm_status lbm_diagnostics(lbm_ctx* ctx, int32_t inst, lbm_diag* out);

/* Copy the whole current state (layout above, lbm_state_bytes bytes) to /
 * from caller device memory, converting from / to the context's own order;
 * set_state also sets lambda^n from the new state (so the next step's a^n
 * follows it) and keeps t and the step count (LBM_EINVAL if src_dev is one
 * of the context's own state buffers). */
size_t lbm_state_bytes(const lbm_ctx* ctx);
lbm_status lbm_get_state(lbm_ctx* ctx, void* dst_dev);
lbm_status lbm_set_state(lbm_ctx* ctx, const void* src_dev);

/* Adjoint of one step with the blending factors theta^n and the kinetic
 * speed a^n held fixed at the values the forward step computes from U_n
 * (they are recomputed from U_n with the forward code, bit for bit):
 *   Ubar_n = (d S^{n+1} / d S^n)^T Ubar_np1.
 * All three are float64 states in the layout above (single instance and
 * LBM_FP64, LBM_ENOTSUP otherwise; ny <= 65535).  Periodic and outflow
 * boundaries and sponge layers: with theta frozen the outflow ghosts only
 * copy the edge cells, whose adjoint takes the copied reads back.  Boundary
 * cells of lbm_set_boundary: a wall ghost mirrors its edge cell, whose
 * adjoint takes the mirrored reads back; Dirichlet ghosts are constants of
 * the map and contribute nothing, but their states enter lambda^n as in the
 * forward step, so they must be the states of step n.  Uses the context's
 * workspace as scratch; does not change the context's own state.  Fully
 * asynchronous on the context's stream (no host synchronisation); Ubar_n
 * must not alias U_n or Ubar_np1, and U_n must not be a context buffer. */
lbm_status lbm_step_adjoint(lbm_ctx* ctx, const double* U_n_dev,
                            const double* Ubar_np1_dev, double* Ubar_n_dev);

/* The same adjoint with theta^n supplied by the caller instead of recomputed:
 * theta_x_dev / theta_y_dev are the face fields that lbm_step_theta wrote for
 * the step from U_n (layouts as there), e.g. while a checkpointed segment is
 * recomputed; a^n is a_fixed or follows lambda^n of U_n.  Same restrictions
 * and aliasing rules as lbm_step_adjoint; Ubar_n must not alias the theta
 * fields.  Asynchronous; does not change the context's state. */
lbm_status lbm_step_adjoint_theta(lbm_ctx* ctx, const double* U_n_dev,
                                  const double* theta_x_dev, const double* theta_y_dev,
                                  const double* Ubar_np1_dev, double* Ubar_n_dev);

/* Adjoint of the initialisation map u0 -> (u0, M_1..M_4(u0; a^0)) with a^0
 * held fixed: u0bar = Ubar0[u] + sum_k J_{M_k}(u0)^T Ubar0[u_k].
 * u0 and u0bar: float64 [4][ny][nx]; Ubar0: float64 state. */
lbm_status lbm_init_adjoint(lbm_ctx* ctx, const double* u0_dev,
                            const double* Ubar0_dev, double* u0bar_dev);

/* Times the step kernel for the candidate strip heights, waves per workgroup,
 * grids (one wave per strip, or a persistent grid of 1, 2 or 4 workgroups
 * per compute unit) and, for ensembles, both strip modes on the context's own
 * problem and keeps the fastest: a first pass times every candidate, then the
 * four fastest are timed again three times, the median decides.  The choice is recorded in a
 * JSON cache file keyed by problem shape (NULL path = no file) as [rows,
 * waves, groups per CU, strip mode]; a cached entry is used without timing
 * (missing trailing values are 0).  The timed launches read the current state and write the
 * other buffer, and the slots (lambda, t, counters) are restored, so the
 * context's state and step count are unchanged.  Synchronises. */
lbm_status lbm_autotune(lbm_ctx* ctx, const char* cache_json_path);

/* Launch shape of the step kernel: rows per strip in [4, 4096] and waves
 * per workgroup in [1, 4] (0 keeps the current value; LBM_EINVAL outside
 * those ranges).  A new context starts with 4 waves per workgroup and the
 * tallest strip of 64, 32, 16, 8 or 4 rows that still yields at least 1024
 * (LBM_FP64) or 2048 (LBM_FP32_STATE) strips over all instances.  Changing
 * the shape drops captured graphs. */
lbm_status lbm_set_launch(lbm_ctx* ctx, int32_t strip_rows, int32_t waves_per_group);
lbm_status lbm_get_launch(const lbm_ctx* ctx, int32_t* strip_rows, int32_t* waves_per_group);

/* Strip heights of an ensemble.  Mode 0 (the default): every instance uses
 * the strip height of lbm_set_launch.  Mode 1: each instance uses the
 * tallest power of two that exceeds neither that height nor a quarter of its
 * own rows (at least 4), and the instances with the tallest strips are
 * dispatched first.  Results do not depend on the mode.  LBM_EINVAL for other
 * values; changing the mode drops captured graphs. */
lbm_status lbm_set_strip_mode(lbm_ctx* ctx, int32_t mode);
lbm_status lbm_get_strip_mode(const lbm_ctx* ctx, int32_t* mode);

/* Boundary cells of a non-periodic side (side 0 west, 1 east, 2 south, 3
 * north; the side's axis must be LBM_BC_OUTFLOW).  kind_dev: uint8 device
 * array, one entry per boundary cell (ny for west and east, nx for south and
 * north), LBM_BND_ZERO_GRADIENT (0, the outflow copy), LBM_BND_WALL (1, a
 * reflective symmetry wall: the ghost layers mirror the interior, with the
 * normal momentum negated and the two distributions moving along the normal
 * exchanged) or LBM_BND_DIRICHLET (2: the ghost layers hold the moments given
 * in state_dev with their Maxwellians at the current a^n, Section 4.8).
 * state_dev: float64 [4][len] device array of (rho, m1, m2, E) per cell, read
 * where the kind is Dirichlet (may be NULL without Dirichlet cells); those
 * states must be admissible (rho > 0, p > 0, finite: LBM_EINVAL otherwise,
 * checked here; a state the caller makes non-admissible later is skipped by
 * lambda^n, and the step's results are then unspecified).  A ghost
 * beyond a corner reads each side's kind at that side's boundary cell nearest
 * to it; walls resolve first (the ghost is the mirror image of the ghost or
 * cell across the wall), then a Dirichlet side, x before y (its state at the
 * resolved cell, mirrored by the walls crossed), then zero-gradient.  Each
 * step first raises lambda^n by the Dirichlet states, so that a^n satisfies
 * Bouchut's condition for every state the stencil reads.  The caller owns
 * both arrays and keeps them alive while the context steps.  The states may
 * change between steps (e.g. a moving inflow); the kinds are read and checked
 * by this call and must not change afterwards: call lbm_set_boundary again
 * after changing them (a kind turned Dirichlet behind the library's back on a
 * side given no state array would be read from NULL).  kind_dev = NULL
 * restores zero-gradient cells on that side.  Walls
 * need two cells along their axis.  Single-instance contexts (ensembles:
 * lbm_set_instance_boundary); the adjoint entry points cover the described
 * cells (see lbm_step_adjoint).  Synchronises; drops
 * captured graphs. */
lbm_status lbm_set_boundary(lbm_ctx* ctx, int32_t side, const uint8_t* kind_dev,
                            const double* state_dev);

/* The same description for instance inst of an ensemble (lbm_init_batch;
 * inst 0 of a single-instance context): arrays sized by that instance's
 * sides, the same checks and rules; each instance's Dirichlet states raise
 * only that instance's lambda^n.  lbm_set_boundary on an ensemble returns
 * LBM_ENOTSUP.  Synchronises; drops captured graphs. */
lbm_status lbm_set_instance_boundary(lbm_ctx* ctx, int32_t inst, int32_t side,
                                     const uint8_t* kind_dev, const double* state_dev);

/* Grid of the step kernel.  groups_per_cu = 0 (the default) launches one wave
 * per strip; k in [1, 32] launches a persistent grid of at most k workgroups
 * per compute unit of the device (rounded up to a multiple of 8, never more
 * than one wave per strip), whose waves loop over the strips of all
 * instances.  Results do not depend on the grid.  LBM_EINVAL outside [0, 32];
 * changing the grid drops captured graphs.  lbm_get_grid also returns the
 * number of workgroups a step launch uses (groups may be NULL). */
lbm_status lbm_set_grid(lbm_ctx* ctx, int32_t groups_per_cu);
lbm_status lbm_get_grid(const lbm_ctx* ctx, int32_t* groups_per_cu, int32_t* groups);

/* For callers that cannot allocate memory (code under hipGraph capture, tight
 * serving loops, harnesses that forbid allocation): one time step of a single
 * instance without a context or workspace.  src_dev holds the state (layout
 * above, 20 planes of nx * ny cells of the params' precision) and dst_dev
 * receives the next one; both are caller device buffers that must not
 * overlap.  Every parameter of lbm_params applies as in lbm_init (periodic and
 * outflow boundaries, sponge layers; no wall or Dirichlet cells).  lambda^n
 * is reduced from src_dev itself, so the call does not depend on a previous
 * one; the step is the one lbm_step_between computes for the same state
 * (bit for bit), with the time counted from 0 (diag_host->t = dt).
 * The call allocates nothing: the per-step scalars (lambda slots, time,
 * event counters) live in a static device array of LBM_NOALLOC_SCRATCH_BYTES
 * bytes that the library holds on each device it runs on until the process
 * ends (one 128-byte record is used).  It does not grow with the grid: any
 * single-instance grid the library accepts (nx, ny < 2^30, nx * ny < 2^32;
 * LBM_EINVAL beyond) runs with it.  Every call on a device shares that
 * device's array and clears it first, so calls that overlap on one device
 * (concurrent streams or threads) race and their results are unspecified.
 * Enqueued on `stream` (hipStream_t as void*; NULL = default stream).  With
 * diag_host == NULL the call is asynchronous and graph-capturable (fills,
 * reductions and the step are kernels); with a host lbm_diag it synchronises
 * the stream, fills lambda (lambda^n), a (a^n), t (dt^n), step (1) and the
 * counters of the new state (min_rho, min_rhoe: NaN), and returns the
 * step's first event as lbm_moments does. */
#define LBM_NOALLOC_SCRATCH_BYTES 256
lbm_status lbm_step_noalloc(const lbm_params* p, const void* src_dev, void* dst_dev, void* stream,
                            lbm_diag* diag_host);

const char* lbm_status_string(lbm_status s);
const char* lbm_last_error(const lbm_ctx* ctx);
void lbm_destroy(lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif
