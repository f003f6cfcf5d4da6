// Internal declarations shared by the kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vlbm.h"

namespace vlbm {

// Scheme parameters shared by every instance of a context.
struct Scheme {
  double gamma, alpha, beta, a_fixed, eps, rlmp_lo, rlmp_hi;
  int a_mode, order, limiters, bc_x, bc_y, sponge;
};

// One problem instance inside the state buffers.
struct Inst {
  long long off;   // element offset of cell (0, 0) inside every plane
  long long item0; // first work item (strip) of this instance
  double dx;
  int nx, ny;
  int xs, ys;      // strips along x and y
  int strip_h;     // rows per strip of this instance
  int pad_;
};

// Boundary description of one instance: per-cell kinds and Dirichlet moments
// of the four sides (west, east, south, north; null: zero-gradient), see
// lbm_set_boundary.
struct BndDesc {
  const uint8_t* kind[4];
  const double* state[4];
};

// Per-instance device scalars.  lam and t rotate over three slots: step n
// reads slot n % 3, writes slot (n + 1) % 3 and clears slot (n + 2) % 3.
struct alignas(128) Slots {
  unsigned long long lam[3]; // bit patterns of non-negative doubles
  double t[3];
  // guard, limited, bad, bouchut, lmp, non-finite, rho <= 0 (cumulative); of
  // the bad cells, those neither non-finite nor with rho <= 0 have p <= 0
  unsigned long long cnt[7];
};
enum {
  CNT_GUARD = 0,
  CNT_LIMITED = 1,
  CNT_BAD = 2,
  CNT_BOUCHUT = 3,
  CNT_LMP = 4,
  CNT_NONFINITE = 5,
  CNT_RHO = 6,
  CNT_N = 7
};
static_assert(sizeof(Slots) == 128, "one 128-byte record per instance");

struct StepArgs {
  const void* src;
  void* dst;
  long long plane;        // elements per plane (sum of all instances' cells)
  Slots* slots;           // [n_inst]
  const Inst* insts;      // [n_inst], device memory
  const int* item_inst;   // [n_items] instance of every item (batches), or null
  Inst inst0;             // the instance when n_inst == 1
  long long n_items;
  int n_inst;
  int slot;               // step index mod 3
  int waves_per_group;
  int xcd_remap;          // map consecutive groups onto one XCD
  int groups;             // launched workgroups
  double* theta_x;        // optional face output (single instance)
  double* theta_y;
  // boundary descriptions: a single instance's in bnd1, an ensemble's in the
  // device table bnd_table (one entry per instance)
  union {
    BndDesc bnd1;
    const BndDesc* bnd_table;
  };
  int bnd;                // 1 if any instance has a boundary description
  int blocked;            // src and dst hold the blocked layout (a context's own
                          // buffers; every width a multiple of 64, no boundary
                          // descriptions), else planar
  Scheme sc;
};

enum { BND_ZERO_GRADIENT = 0, BND_WALL = 1, BND_DIRICHLET = 2 };

// Launchers (step.hip).
hipError_t launch_step(const StepArgs& a, int precision, hipStream_t s);
// `blocked`: the state S is in the blocked layout (see step.hip), else
// planar.
hipError_t launch_init(const Scheme& sc, const Inst* insts_host, int n_inst,
                       const Inst* insts_dev, long long plane, const double* u0,
                       void* S, Slots* slots, int precision, int blocked, hipStream_t s);
hipError_t launch_lambda_state(const Scheme& sc, const Inst* insts_host, int n_inst,
                               long long plane, const void* S, Slots* slots,
                               int slot, int precision, int blocked, hipStream_t s);
hipError_t launch_moments(const Inst& in, long long plane, const void* S,
                          double* out, int precision, int blocked, hipStream_t s);
// Every instance's state (widths multiples of 64) from src to dst, planar ->
// blocked (to_blocked = 1) or blocked -> planar (0).
hipError_t launch_relayout(const Inst* insts_host, int n_inst, long long plane, const void* src, void* dst,
                           int precision, int to_blocked, hipStream_t s);
// Per-cell blending step (an ablation): state A.src -> A.dst with the face
// factors A.theta_x / A.theta_y of the same state, single instance; also
// the step's slot bookkeeping.
hipError_t launch_percell(const StepArgs& a, int precision, hipStream_t s);
// Block minima of rho and of rho e = E - |m|^2 / (2 rho) over the finite
// cells of the moment slot, part[blocks][2].
hipError_t launch_minima(const Inst& in, long long plane, const void* S, double* part,
                         int blocks, int precision, int blocked, hipStream_t s);
// Double-double partial totals of the moment slot, part[blocks][4][2]; the
// grid is `blocks` workgroups of 256 threads.
hipError_t launch_totals(const Inst& in, long long plane, const void* S, double* part,
                         int blocks, int precision, int blocked, hipStream_t s);
hipError_t launch_fill_u32(unsigned int* p, unsigned int v, long long n, hipStream_t s);
// Raises each instance's lam[slot] to the largest wavespeed of its Dirichlet
// boundary states (one workgroup per instance).
hipError_t launch_bnd_lambda(const StepArgs& a, int slot, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, long long n, hipStream_t s);
// Adjoint (adjoint.hip).  Boundary kinds per side (west, east, south,
// north), uint8 device arrays as in StepArgs; NULL: zero-gradient.
struct BndKinds {
  const uint8_t* k[4];
};
hipError_t launch_adjoint_step(const Scheme& sc, const Inst& in, long long plane,
                               const double* U, const double* Ubar1, double* Ubar0,
                               const double* theta_x, const double* theta_y,
                               const Slots* slot_src, int slot, const BndKinds& kinds,
                               hipStream_t s);
hipError_t launch_adjoint_init(const Scheme& sc, const Inst& in, const double* u0,
                               const double* Ubar0, double* u0bar,
                               const Slots* slots, int slot, hipStream_t s);

// Host helpers of the C ABI (api.hip): parameter checks (NULL when valid),
// the kernels' scheme record, and the message lbm_last_error(NULL) returns.
const char* host_check_params(const lbm_params* p);
Scheme host_make_scheme(const lbm_params* p);
void host_set_error(const char* m);

}  // namespace vlbm
