// Adjoint of one blended step and of the initialisation, FP64.
//
// With theta and a held fixed, the step (eqs. (25), (27)) is, per cell c with
// face factors tW, tE, tS, tN (faces i-1/2, i+1/2, j-1/2, j+1/2):
//   u_1'(c) = (1 + tW) M_1(u_W) - tW u_1(W),   u_2'(c) = (1 + tE) M_2(u_E) - tE u_2(E),
//   u_3'(c) = (1 + tS) M_3(u_S) - tS u_3(S),   u_4'(c) = (1 + tN) M_4(u_N) - tN u_4(N),
//   u'(c)   = alpha u + sum_k u_k'(c) - tW d_2(c) - tE d_1(c) - tS d_4(c) - tN d_3(c),
// with d_k = M_k(u) - u_k and the Maxwellian Jacobians of Example 1,
// J_{M_1,2} = w I +- A(u)/(2a), J_{M_3,4} = w I +- B(u)/(2a), A = f'(u),
// B = g'(u).  Transposing this radius-1 stencil gives the gather below for
// every cell x (g_k(c) = ubar_k'(c) + ubar'(c) is the adjoint reaching
// u_k'(c), which enters both slot k and the moment sum):
//   ubar(x)   = alpha ubar'(x) + J_{M_1}^T [(1 + tE) g_1(E) - tE ubar'(x)]
//             + J_{M_2}^T [(1 + tW) g_2(W) - tW ubar'(x)]
//             + J_{M_3}^T [(1 + tN) g_3(N) - tN ubar'(x)]
//             + J_{M_4}^T [(1 + tS) g_4(S) - tS ubar'(x)],
//   ubar_1(x) = tE (ubar'(x) - g_1(E)),  ubar_2(x) = tW (ubar'(x) - g_2(W)),
//   ubar_3(x) = tN (ubar'(x) - g_3(N)),  ubar_4(x) = tS (ubar'(x) - g_4(S)).
// The face factors come from the forward kernel run on the same state, so
// they equal the forward step's bit for bit.
//
// Outflow boundaries (zero-gradient ghosts copying the nearest cell's whole
// state): with theta frozen only the first ghost layer enters the map.  A
// ghost neighbour is not an output, so its term above drops (g_k of that
// neighbour = 0), and the edge cell reads its own state through the ghost:
// at a west edge u_1'(x) = (1 + tW) M_1(u_x) - tW u_1(x), which adds
// (1 + tW) J_{M_1}^T g_1(x) to ubar(x) and -tW g_1(x) to ubar_1(x); likewise
// M_2 / tE at an east edge, M_3 / tS at a south edge, M_4 / tN at a north
// edge.
//
// Boundary cells described per side (walls and Dirichlet states): a
// Dirichlet ghost holds given moments and their Maxwellians at the frozen a,
// so it does not depend on the state and its term drops too.  A wall ghost
// mirrors the edge cell: its moments are R u(x), with R negating the normal
// momentum, and its two distributions along the normal are the edge cell's
// other one, mirrored.  At a west wall u_1'(x) = (1 + tW) M_1(R u_x)
// - tW R u_2(x), and since the Euler flux satisfies f(R u) = -R f(u) (for an
// x-mirror; g likewise for a y-mirror), M_1(R u) = R M_2(u): the edge cell's
// own g_1(x) adds (1 + tW) J_{M_2}^T R g_1(x) to ubar(x) and -tW R g_1(x) to
// ubar_2(x).  Likewise at an east wall (M_1, slot 1, tE), a south wall (M_4,
// slot 4, tS) and a north wall (M_3, slot 3, tN).  Streaming reads no
// diagonal neighbour, so no corner ghost enters the map.

#include "vlbm_internal.h"

namespace vlbm {
namespace {

struct Jac {
  double v1, v2, q, H, gm1, gamma;
};

__device__ __forceinline__ Jac jac_of(const double u[4], double gamma) {
  Jac J;
  const double ir = 1.0 / u[0];
  J.v1 = u[1] * ir;
  J.v2 = u[2] * ir;
  J.q = 0.5 * (J.v1 * J.v1 + J.v2 * J.v2);
  J.gm1 = gamma - 1.0;
  J.gamma = gamma;
  const double p = J.gm1 * (u[3] - u[0] * J.q);
  J.H = (u[3] + p) * ir;
  return J;
}

// A(u)^T z with A = df/du of the Euler x-flux.
__device__ __forceinline__ void At(const Jac& J, const double z[4], double o[4]) {
  const double v1 = J.v1, v2 = J.v2, k = J.gm1;
  o[0] = (-v1 * v1 + k * J.q) * z[1] - v1 * v2 * z[2] + (-J.H * v1 + k * J.q * v1) * z[3];
  o[1] = z[0] + (2.0 - k) * v1 * z[1] + v2 * z[2] + (J.H - k * v1 * v1) * z[3];
  o[2] = -k * v2 * z[1] + v1 * z[2] - k * v1 * v2 * z[3];
  o[3] = k * z[1] + J.gamma * v1 * z[3];
}

// B(u)^T z with B = dg/du of the Euler y-flux.
__device__ __forceinline__ void Bt(const Jac& J, const double z[4], double o[4]) {
  const double v1 = J.v1, v2 = J.v2, k = J.gm1;
  o[0] = -v1 * v2 * z[1] + (-v2 * v2 + k * J.q) * z[2] + (-J.H * v2 + k * J.q * v2) * z[3];
  o[1] = v2 * z[1] - k * v1 * z[2] - k * v1 * v2 * z[3];
  o[2] = z[0] + v1 * z[1] + (2.0 - k) * v2 * z[2] + (J.H - k * v2 * v2) * z[3];
  o[3] = k * z[2] + J.gamma * v2 * z[3];
}

__device__ __forceinline__ double kinetic_speed(const Scheme& s, const Slots* sl, int slot) {
  const double lam = __longlong_as_double((long long)sl->lam[slot]);
  return (s.a_mode == 1) ? s.a_fixed : 2.0 * s.beta * lam / (1.0 - s.alpha);
}

// Kind of the boundary cell beyond an edge cell: the side's description, or
// zero-gradient without one.
__device__ __forceinline__ int edge_kind(const uint8_t* k, int r) {
  return k ? (int)k[r] : BND_ZERO_GRADIENT;
}

// EDGES: the context has an outflow axis (the edge terms above); periodic
// contexts run without them.  kinds: the boundary descriptions per side
// (west, east, south, north; NULL: zero-gradient).
template <bool EDGES>
__global__ __launch_bounds__(256) void adjoint_step_kernel(Scheme sc, int nx, int ny, long long P,
                                                           const double* __restrict__ U,
                                                           const double* __restrict__ B1,
                                                           double* __restrict__ B0,
                                                           const double* __restrict__ tx,
                                                           const double* __restrict__ ty,
                                                           const Slots* sl, int slot,
                                                           BndKinds kinds) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= nx || j >= ny) return;
  const double a = kinetic_speed(sc, sl, slot);
  const double w = 0.25 * (1.0 - sc.alpha);
  const double r2a = 1.0 / (2.0 * a);
  const int iw = i == 0 ? nx - 1 : i - 1, ie = i == nx - 1 ? 0 : i + 1;
  const int js = j == 0 ? ny - 1 : j - 1, jn = j == ny - 1 ? 0 : j + 1;
  // neighbours that are outflow ghosts
  const bool gw = EDGES && sc.bc_x == 1 && i == 0, ge = EDGES && sc.bc_x == 1 && i == nx - 1;
  const bool gs = EDGES && sc.bc_y == 1 && j == 0, gn = EDGES && sc.bc_y == 1 && j == ny - 1;
  const long long cX = (long long)j * nx + i;
  const long long cW = (long long)j * nx + iw, cE = (long long)j * nx + ie;
  const long long cS = (long long)js * nx + i, cN = (long long)jn * nx + i;
  const double tW = tx[(long long)j * (nx + 1) + i], tE = tx[(long long)j * (nx + 1) + i + 1];
  const double tS = ty[(long long)j * nx + i], tN = ty[(long long)(j + 1) * nx + i];
  // kinds of the ghosts beyond this cell's edges
  const int kw = gw ? edge_kind(kinds.k[0], j) : -1, ke = ge ? edge_kind(kinds.k[1], j) : -1;
  const int ks = gs ? edge_kind(kinds.k[2], i) : -1, kn = gn ? edge_kind(kinds.k[3], i) : -1;
  // g1..g4: adjoint reaching u_k' of the neighbour that reads this cell
  // (0 for a ghost); h1..h4: this cell's own g_k, read back through a
  // zero-gradient ghost; m1..m4: the same through a wall ghost, mirrored
  double u[4], ub[4], g1[4], g2[4], g3[4], g4[4], h1[4], h2[4], h3[4], h4[4];
  double m1[4], m2[4], m3[4], m4[4];
  for (int c = 0; c < 4; ++c) {
    u[c] = U[c * P + cX];
    ub[c] = B1[c * P + cX];
    g1[c] = ge ? 0.0 : B1[(4 + c) * P + cE] + B1[c * P + cE];
    g2[c] = gw ? 0.0 : B1[(8 + c) * P + cW] + B1[c * P + cW];
    g3[c] = gn ? 0.0 : B1[(12 + c) * P + cN] + B1[c * P + cN];
    g4[c] = gs ? 0.0 : B1[(16 + c) * P + cS] + B1[c * P + cS];
    const double o1 = (kw >= 0 && kw != BND_DIRICHLET) ? B1[(4 + c) * P + cX] + ub[c] : 0.0;
    const double o2 = (ke >= 0 && ke != BND_DIRICHLET) ? B1[(8 + c) * P + cX] + ub[c] : 0.0;
    const double o3 = (ks >= 0 && ks != BND_DIRICHLET) ? B1[(12 + c) * P + cX] + ub[c] : 0.0;
    const double o4 = (kn >= 0 && kn != BND_DIRICHLET) ? B1[(16 + c) * P + cX] + ub[c] : 0.0;
    h1[c] = kw == BND_ZERO_GRADIENT ? o1 : 0.0;
    h2[c] = ke == BND_ZERO_GRADIENT ? o2 : 0.0;
    h3[c] = ks == BND_ZERO_GRADIENT ? o3 : 0.0;
    h4[c] = kn == BND_ZERO_GRADIENT ? o4 : 0.0;
    // R: the x-mirror negates m_1, the y-mirror m_2
    m1[c] = kw == BND_WALL ? (c == 1 ? -o1 : o1) : 0.0;
    m2[c] = ke == BND_WALL ? (c == 1 ? -o2 : o2) : 0.0;
    m3[c] = ks == BND_WALL ? (c == 2 ? -o3 : o3) : 0.0;
    m4[c] = kn == BND_WALL ? (c == 2 ? -o4 : o4) : 0.0;
  }
  const Jac J = jac_of(u, sc.gamma);
  double z1[4], z2[4], z3[4], z4[4];
  for (int c = 0; c < 4; ++c) {
    z1[c] = (1.0 + tE) * g1[c] - tE * ub[c] + (1.0 + tW) * h1[c] + (1.0 + tE) * m2[c];
    z2[c] = (1.0 + tW) * g2[c] - tW * ub[c] + (1.0 + tE) * h2[c] + (1.0 + tW) * m1[c];
    z3[c] = (1.0 + tN) * g3[c] - tN * ub[c] + (1.0 + tS) * h3[c] + (1.0 + tN) * m4[c];
    z4[c] = (1.0 + tS) * g4[c] - tS * ub[c] + (1.0 + tN) * h4[c] + (1.0 + tS) * m3[c];
  }
  double dx[4], dy[4], ax[4], by[4];
  for (int c = 0; c < 4; ++c) {
    dx[c] = z1[c] - z2[c];
    dy[c] = z3[c] - z4[c];
  }
  At(J, dx, ax);
  Bt(J, dy, by);
  for (int c = 0; c < 4; ++c) {
    B0[c * P + cX] = sc.alpha * ub[c] + w * (z1[c] + z2[c] + z3[c] + z4[c]) + r2a * (ax[c] + by[c]);
    B0[(4 + c) * P + cX] = tE * (ub[c] - g1[c]) - tW * h1[c] - tE * m2[c];
    B0[(8 + c) * P + cX] = tW * (ub[c] - g2[c]) - tE * h2[c] - tW * m1[c];
    B0[(12 + c) * P + cX] = tN * (ub[c] - g3[c]) - tS * h3[c] - tN * m4[c];
    B0[(16 + c) * P + cX] = tS * (ub[c] - g4[c]) - tN * h4[c] - tS * m3[c];
  }
}

// u0bar = Ubar0[u] + sum_k J_{M_k}(u0)^T Ubar0[u_k] with a^0 fixed.
__global__ __launch_bounds__(256) void adjoint_init_kernel(Scheme sc, long long n,
                                                           const double* __restrict__ u0,
                                                           const double* __restrict__ B,
                                                           double* __restrict__ out,
                                                           const Slots* sl, int slot) {
  const long long c0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c0 >= n) return;
  const double a = kinetic_speed(sc, sl, slot);
  const double w = 0.25 * (1.0 - sc.alpha);
  const double r2a = 1.0 / (2.0 * a);
  double u[4], b[5][4];
  for (int c = 0; c < 4; ++c) {
    u[c] = u0[c * n + c0];
    for (int s = 0; s < 5; ++s) b[s][c] = B[(4 * s + c) * n + c0];
  }
  const Jac J = jac_of(u, sc.gamma);
  double dx[4], dy[4], ax[4], by[4];
  for (int c = 0; c < 4; ++c) {
    dx[c] = b[1][c] - b[2][c];
    dy[c] = b[3][c] - b[4][c];
  }
  At(J, dx, ax);
  Bt(J, dy, by);
  for (int c = 0; c < 4; ++c)
    out[c * n + c0] = b[0][c] + w * (b[1][c] + b[2][c] + b[3][c] + b[4][c]) + r2a * (ax[c] + by[c]);
}

}  // namespace

hipError_t launch_adjoint_step(const Scheme& sc, const Inst& in, long long plane, const double* U,
                               const double* Ub1, double* Ub0, const double* tx, const double* ty,
                               const Slots* slots, int slot, const BndKinds& kinds, hipStream_t s) {
  const dim3 block(256);
  const dim3 grid((in.nx + 255) / 256, in.ny);
  if (sc.bc_x == 1 || sc.bc_y == 1)
    hipLaunchKernelGGL(adjoint_step_kernel<true>, grid, block, 0, s, sc, in.nx, in.ny, plane, U, Ub1,
                       Ub0, tx, ty, slots, slot, kinds);
  else
    hipLaunchKernelGGL(adjoint_step_kernel<false>, grid, block, 0, s, sc, in.nx, in.ny, plane, U, Ub1,
                       Ub0, tx, ty, slots, slot, kinds);
  return hipGetLastError();
}

hipError_t launch_adjoint_init(const Scheme& sc, const Inst& in, const double* u0,
                               const double* Ub0, double* u0b, const Slots* slots, int slot,
                               hipStream_t s) {
  const long long n = (long long)in.nx * in.ny;
  hipLaunchKernelGGL(adjoint_init_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, sc, n,
                     u0, Ub0, u0b, slots, slot);
  return hipGetLastError();
}

}  // namespace vlbm
