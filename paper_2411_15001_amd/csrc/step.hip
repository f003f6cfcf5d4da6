// Fused collide-limit-stream step of the blended D2Q5 vectorial lattice
// Boltzmann scheme (Wissocq, Liu, Abgrall), gfx950.
//
// Work decomposition.  A wave owns an aligned strip of 64 consecutive
// columns (x0 = 64 xs) and H consecutive rows of one instance and marches up
// the strip one row at a time; lane l holds column x0 + l and every lane
// produces output.  x-neighbours are exchanged with wave-wide lane shifts;
// the two edge lanes also load the halo column beside the strip and evaluate
// the faces and bounds that reach across it.  y-neighbours are the rows the
// lane already holds in registers from the previous iterations.  No barrier
// is used; LDS only receives the rows of the LDS-staged marches.
//
// State layouts.  Planar: value q of cell c (row-major over the instance) at
// q * plane + c.  Blocked (a context's own buffers when every instance's
// width is a multiple of 64): each instance's state follows the ones before
// it (20 values per cell), and inside it the 20 values of every run of 64
// cells of a row lie together, value q of cell c at (c / 64) * 1280 +
// q * 64 + c % 64, so that one strip row of the state is one contiguous
// range of memory.  Caller buffers are always planar.
//
// Without density bounds (PP, pressure, unlimited, first order) both face
// factors of a row are known as soon as it arrives, so the march completes
// row L - 1 when row L arrives and reads H + 2 rows.  With LMP / RLMP bounds
// the blending factor of a face needs the bounds of both its cells, and a
// cell's bounds need its upper y-face, so the march lags two rows and reads
// H + 4.  Pipeline of one LMP iteration (newest row L loaded):
//   row L     : Maxwellians and d_k (Example 1), x-face state u*_{i+1/2} and
//               Delta F_{i+1/2} (eqs. (12), (22)), y-face L-1/2 (u*, Delta G);
//   row L - 1 : density bounds (eq. (29)), theta of its x-face i+1/2 and of
//               the y-face L-3/2 (Sections 3.3, 3.4), streamed distributions
//               u_1, u_2 (eq. (25)) and u_3, and the moment sum of eq. (27)
//               up to its face L-3/2;
//   row L - 2 : last face term of eq. (27) and u_4; the row is complete.
// Each cell's moment update adds, in this order, alpha u and the terms of its
// faces i-1/2, i+1/2, j-1/2, j+1/2 (incoming distribution minus theta times
// its own distribution leaving through that face): the evaluation order of
// the oracle, so the FP64 path reproduces it bit for bit.
//
// The wavespeed of every new cell (Section 4 preamble) is reduced over the
// wave with lane shuffles and merged with one 64-bit atomic max per strip
// into the instance's next lambda slot; the next launch derives a^{n+1} from
// it on the device.

#include <math.h>

#include <atomic>

#include "vlbm_internal.h"

namespace vlbm {
namespace {

constexpr double kHuge = __builtin_huge_val();

template <class X>
__device__ __forceinline__ X vmin(X a, X b) { return (b < a) ? b : a; }
template <class X>
__device__ __forceinline__ X vmax(X a, X b) { return (b > a) ? b : a; }

// Value held by lane - 1 / lane + 1 through DPP whole-wave shifts
// (wave_shr:1 = 0x138, wave_shl:1 = 0x130): one VALU move per dword, no LDS
// traffic.  The lane without a source (63 for from_right_or, 0 for
// from_left_or) receives `edge`: the DPP move leaves that lane's destination
// untouched, and the destination starts as `edge`.
__device__ __forceinline__ int dpp_right_or(int v, int e) {
  return __builtin_amdgcn_update_dpp(e, v, 0x130, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_left_or(int v, int e) {
  return __builtin_amdgcn_update_dpp(e, v, 0x138, 0xf, 0xf, false);
}
__device__ __forceinline__ float from_right_or(float v, float e) {
  return __int_as_float(dpp_right_or(__float_as_int(v), __float_as_int(e)));
}
__device__ __forceinline__ float from_left_or(float v, float e) {
  return __int_as_float(dpp_left_or(__float_as_int(v), __float_as_int(e)));
}
__device__ __forceinline__ double from_right_or(double v, double e) {
  const long long b = __double_as_longlong(v), x = __double_as_longlong(e);
  const int lo = dpp_right_or((int)(b & 0xffffffffll), (int)(x & 0xffffffffll));
  const int hi = dpp_right_or((int)(b >> 32), (int)(x >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double from_left_or(double v, double e) {
  const long long b = __double_as_longlong(v), x = __double_as_longlong(e);
  const int lo = dpp_left_or((int)(b & 0xffffffffll), (int)(x & 0xffffffffll));
  const int hi = dpp_left_or((int)(b >> 32), (int)(x >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int map_index(int i, int n, int bc) {
  if (bc == 0) {
    int r = i % n;
    return r < 0 ? r + n : r;
  }
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

// Element index of value q of cell c of one instance, from the instance's
// first value, in a state of `plane` cells per plane, planar or blocked (see
// the layouts above).
__device__ __forceinline__ long long sidx(int q, long long c, long long plane, int blocked) {
  return blocked ? ((c >> 6) * 1280 + q * 64 + (c & 63)) : q * plane + c;
}

__device__ __forceinline__ bool in_sponge(const Scheme& s, int i, int j, int nx, int ny) {
  const int w = s.sponge;
  if (s.bc_x == 1 && (i < w || i >= nx - w)) return true;
  if (s.bc_y == 1 && (j < w || j >= ny - w)) return true;
  return false;
}

// Section 3.3.3
__device__ __forceinline__ double theta_rho_pp(double rs, double D, double kappa, double eps) {
  if (D == 0.0) return kHuge;
  const double t = kappa * rs / fabs(D) - eps;
  return vmax(0.0, t);
}

// Section 3.3.1, final case formula (L = left/bottom cell, R = right/top cell)
__device__ __forceinline__ double theta_rho_lmp(double rs, double D, double kappa, double muL,
                                                double nuL, double muR, double nuR) {
  if (D == 0.0) return 1.0;
  // the caller takes min(1, .): when the dividend already reaches D (in the
  // direction of its sign) the rounded quotient is >= 1, and 1 stands in for
  // it without the division
  const bool pos = D > 0.0;
  const double num = pos ? kappa * vmin(nuR - rs, rs - muL) : -kappa * vmin(rs - muR, nuL - rs);
  const bool one = pos ? (num >= D) : (num <= D);
  double q = 1.0;
  if (!one) {
    // an empty volatile statement keeps the division inside the branch, so
    // that a wave with no limited face skips it instead of evaluating it on
    // every lane and selecting
    __asm__ volatile("");
    q = num / D;
  }
  return q;
}

// Relative slack of the LMP check: the rounding of the update (float64
// state: the slack the oracle uses; float32 state: a few float32 roundings).
template <class T>
constexpr double kLmpTol = sizeof(T) == 8 ? 1e-12 : 2e-6;

// Margin of the division-free test below: c = 1 + 2^-30.
constexpr double kFastMargin = 1.0 + 0x1p-30;
// Margin of the square-root-free test in front of it: m = 1 - 2^-26.
constexpr double kPreMargin = 1.0 - 0x1p-26;

// theta = min(1, selected theta^rho, theta^p) of one face (Section 3.2).  A
// face state outside the admissible set takes the first-order value 0.
//
// Division-free shortcut, exact: theta^rho_PP = fl(fl(kappa rho*)/|D|) - eps
// is >= 1 whenever fl(kappa rho*) >= fl(|D| c), and theta^p = fl(kappa/r) - eps
// is >= 1 whenever, in addition, fl(N c) <= fl(kappa (-2 g0)) with
// N = fl(|g1| + sqrt(Delta)) (both quotients behind r are then at most
// kappa (1 + u)^2 / (c (1 - u)), u = 2^-53, and eps <= 1e-12 < 2^-32 cannot
// bring a value above 1 + 2^-32 below 1).  In that case min(1, ...) over those
// two limiters is exactly 1 and the four divisions are skipped; every other
// lane evaluates the formulas in full, so the result is bit-identical.
//
// The square root behind N is skipped as well where a test without it
// already implies the one above: with X = fl(kappa (-2 g0)), a = fl(X m) and
// t = fl(a - |g1|) in [2^-500, 2^500), disc <= fl(fl(t t) m) gives
// fl(sqrt(disc)) <= t sqrt(m) (1 + u)^2 <= (a - |g1|) sqrt(m) (1 + u)^3 <
// a - |g1|, so |g1| + sqrt < a <= X m (1 + u) and fl(N c) <= X m c (1 + u)^3
// < X (m c < 1 - 2^-27).  The range of t keeps every product normal and
// finite; a NaN or an infinity fails the test and takes the full path.
//
// LIMS != 0 fixes the limiter set at compile time (the launcher selects such
// a kernel only for the second-order scheme without sponge layers and with
// eps <= 1e-12), which folds the limiter tests away; LIMS = 0 reads the set
// from the scheme.
template <int LIMS, class C>
__device__ __forceinline__ double face_theta(const Scheme& s, const C us[4], const C dF[4],
                                             double kappa, C muL, C nuL, C muR, C nuR,
                                             int& guard) {
  guard = 0;
  const unsigned lims = LIMS ? (unsigned)LIMS : (unsigned)s.limiters;
  if (LIMS == 0) {
    if (s.order == 1) return 0.0;
    if (s.limiters == 0) return 1.0;
  }
  const double r0 = us[0], m1 = us[1], m2 = us[2], E = us[3];
  const double g0 = m1 * m1 + m2 * m2 - 2.0 * r0 * E;
  if (!(r0 > 0.0) || !(g0 < 0.0)) {
    guard = 1;
    return 0.0;
  }
  const double D = dF[0];
  const bool fast_ok = LIMS != 0 || s.eps <= 1e-12;  // the launcher checks eps for LIMS != 0
  const bool fast_rho = fast_ok && (D == 0.0 || kappa * r0 >= fabs(D) * kFastMargin);
  double t = 1.0;
  if ((lims & 1u) && !fast_rho) t = vmin(t, theta_rho_pp(r0, D, kappa, s.eps));
  if (lims & 2u)
    t = vmin(t, theta_rho_lmp(r0, D, kappa, (double)muL, (double)nuL, (double)muR, (double)nuR));
  if (lims & 4u)
    t = vmin(t, theta_rho_lmp(r0, D, kappa, s.rlmp_lo * (double)muL, s.rlmp_hi * (double)nuL,
                              s.rlmp_lo * (double)muR, s.rlmp_hi * (double)nuR));
  if (lims & 8u) {
    const double Dm1 = dF[1], Dm2 = dF[2], DE = dF[3];
    const double g1 = 2.0 * (D * E + DE * r0 - Dm1 * m1 - Dm2 * m2);
    const double g2 = Dm1 * Dm1 + Dm2 * Dm2 - 2.0 * D * DE;
    double disc = g1 * g1 - 4.0 * g0 * g2;
    disc = vmax(0.0, disc);
    const double Dn = -2.0 * g0;
    const double X = kappa * Dn;
    const double tq = X * kPreMargin - fabs(g1);
    const bool pre = fast_rho && tq >= 0x1p-500 && tq < 0x1p500 && disc <= (tq * tq) * kPreMargin;
    if (!pre) {
      __asm__ volatile("");  // keeps the square root inside the branch
      const double N = fabs(g1) + sqrt(disc);
      const bool fast_p = fast_rho && N * kFastMargin <= X;
      if (!fast_p) {
        // theta^p = max(0, kappa / r - eps) with r the larger of |D| / rho*
        // and (|g1| + sqrt(disc)) / (-2 g0) (Section 3.4), reusing g0, g1,
        // disc, N
        const double e1 = fabs(D) / r0;
        const double e2 = N / Dn;
        const double r = vmax(e1, e2);
        const double tp = (r == 0.0) ? kHuge : vmax(0.0, kappa / r - s.eps);
        t = vmin(t, tp);
      }
    }
  }
  return t;
}

// Store of the new state.  With the float32 state the stores bypass cache
// allocation (non-temporal): the state is written once and read by the next
// launch from HBM anyway, and this measured 2% faster on the 8192^2 blast;
// with float64 it measured 3% slower, so plain stores are kept there.
template <class T>
__device__ __forceinline__ void put(T* p, T v) {
  if constexpr (sizeof(T) == 4)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// Store of value v at byte offset voff of the row that starts at the
// wave-uniform address `row` and holds `bytes` bytes, through a buffer
// resource: the hardware drops the lanes whose offset lies beyond the row
// (columns past the instance's edge, which pass 0xFFFFFFFF) and every lane
// when bytes = 0 (a row the strip does not produce).  The store is thus issued on every path, and the
// wait for the next prefetched row, which the compiler otherwise extends over
// stores issued under a condition, leaves these in flight.  Non-temporal, as
// put() with the float32 state.  Used by the short march with the float32
// state (0.6% faster on the 8192^2 blast, 1.3% on the 256-instance ensemble;
// with float64, and in the bounds-limited march, it measured slower).
constexpr int kRsrcWord3 = 0x00020000;  // 32-bit data format, raw access
__device__ __forceinline__ void put_row(float* row, unsigned bytes, unsigned voff, float v) {
  const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(row, (short)0, (int)bytes, kRsrcWord3);
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, voff, 0, 2);
}

// Raise lambda slot `slot` to at least lmax (>= 0; the bit patterns of
// non-negative doubles order like the integers).  Within one step a slot only
// grows from the zero the previous step stored, so an agent-scope read that
// already shows lmax or more makes the read-modify-write redundant: most
// waves skip it, which keeps same-address atomics off the critical path of
// short launches.
__device__ __forceinline__ void raise_lambda(unsigned long long* p, double lmax) {
  const unsigned long long v = (unsigned long long)__double_as_longlong(lmax);
  const unsigned long long seen = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (v > seen) atomicMax(p, v);
}

// One lane per wave publishes the wave's wavespeed maximum and event counts;
// n_cls packs the non-finite count (bits 16 and up) and the rho <= 0 count
// (low 16 bits) of the non-admissible cells.
__device__ __forceinline__ void publish(Slots* sl, int slot, double lmax, unsigned n_bad,
                                       unsigned n_guard, unsigned n_lim, unsigned n_lmp,
                                       unsigned n_nf, unsigned n_rho) {
  raise_lambda(&sl->lam[slot], lmax);
  if (n_bad) atomicAdd(&sl->cnt[CNT_BAD], (unsigned long long)n_bad);
  if (n_nf) atomicAdd(&sl->cnt[CNT_NONFINITE], (unsigned long long)n_nf);
  if (n_rho) atomicAdd(&sl->cnt[CNT_RHO], (unsigned long long)n_rho);
  if (n_guard) atomicAdd(&sl->cnt[CNT_GUARD], (unsigned long long)n_guard);
  if (n_lim) atomicAdd(&sl->cnt[CNT_LIMITED], (unsigned long long)n_lim);
  if (n_lmp) atomicAdd(&sl->cnt[CNT_LMP], (unsigned long long)n_lmp);
}

// Wavespeed |v| + sqrt(gamma p / rho) of one state, or -1 if it is not
// admissible (rho <= 0, p <= 0 or a non-finite result).
__device__ __forceinline__ double cell_wavespeed(double rho, double m1, double m2, double E,
                                                 double gamma) {
  const double ir = 1.0 / rho;
  const double v1 = m1 * ir;
  const double v2 = m2 * ir;
  const double ke = 0.5 * (m1 * v1 + m2 * v2);
  const double p = (gamma - 1.0) * (E - ke);
  const double l = sqrt(v1 * v1 + v2 * v2) + sqrt(gamma * p * ir);
  if (!(rho > 0.0) || !(p > 0.0) || !(l <= 1.79769313486231570e308)) return -1.0;
  return l;
}

// Class of a state that cell_wavespeed rejects, added to a lane's packed
// count: 1 << 16 when a component, or else the wavespeed, is not finite; 1
// when rho <= 0; 0 when rho > 0 and p <= 0 (p evaluated as in
// cell_wavespeed).  Each lane counts at most 4096 rows of a strip, so the two
// 16-bit fields do not overflow before the wave reduction unpacks them.
__device__ __forceinline__ unsigned bad_class(double rho, double m1, double m2, double E,
                                              double gamma) {
  if (!isfinite(rho) || !isfinite(m1) || !isfinite(m2) || !isfinite(E)) return 1u << 16;
  if (!(rho > 0.0)) return 1u;
  const double ir = 1.0 / rho;
  const double v1 = m1 * ir;
  const double v2 = m2 * ir;
  const double p = (gamma - 1.0) * (E - 0.5 * (m1 * v1 + m2 * v2));
  return p > 0.0 ? (1u << 16) : 0u;
}

// Reduction over the wave of the packed class counts: (non-finite, rho <= 0).
__device__ __forceinline__ void reduce_classes(unsigned cls, unsigned& n_nf, unsigned& n_rho) {
  n_nf = cls >> 16;
  n_rho = cls & 0xffffu;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    n_nf += __shfl_xor(n_nf, off, 64);
    n_rho += __shfl_xor(n_rho, off, 64);
  }
}

// Euler fluxes (Section 1) of one state.
template <class C>
__device__ __forceinline__ void fluxes(const C u[4], C gm1, C f[4], C g[4]) {
  const C rho = u[0], m1 = u[1], m2 = u[2], E = u[3];
  const C ir = C(1.0) / rho;
  const C v1 = m1 * ir;
  const C v2 = m2 * ir;
  const C ke = C(0.5) * (m1 * v1 + m2 * v2);
  const C p = gm1 * (E - ke);
  f[0] = m1;
  f[1] = m1 * v1 + p;
  f[2] = m2 * v1;
  f[3] = (E + p) * v1;
  g[0] = m2;
  g[1] = m1 * v2;
  g[2] = m2 * v2 + p;
  g[3] = (E + p) * v2;
}

// Maxwellians of Example 1, k = 0..3 for M_1..M_4: w u +- flux / (2a).
template <class C>
__device__ __forceinline__ C maxw(int k, C u, C f, C g, C w, C r2a) {
  const C wu = w * u;
  switch (k) {
    case 0: return wu + f * r2a;
    case 1: return wu - f * r2a;
    case 2: return wu + g * r2a;
    default: return wu - g * r2a;
  }
}

template <class T, class C>
struct StepConst {
  double a, kappa, lam;
  C w, r2a, r2k, ac, alpha, gm1;
};

template <class T, class C>
__device__ __forceinline__ StepConst<T, C> step_const(const Scheme& s, double lam) {
  StepConst<T, C> k;
  k.lam = lam;
  k.a = (s.a_mode == 1) ? s.a_fixed : 2.0 * s.beta * lam / (1.0 - s.alpha);
  k.kappa = 0.5 * k.a * (1.0 - s.alpha);
  k.w = (C)(0.25 * (1.0 - s.alpha));
  k.r2a = (C)(1.0 / (2.0 * k.a));
  k.r2k = (C)(1.0 / (2.0 * k.kappa));
  k.ac = (C)k.a;
  k.alpha = (C)s.alpha;
  k.gm1 = (C)(s.gamma - 1.0);
  return k;
}

// Boundary cells with a kind per cell (reflective wall, Dirichlet state,
// zero-gradient): the state of cell (i, j) of the grid extended by two ghost
// layers, -2 <= i <= nx + 1 and -2 <= j <= ny + 1.  The x sides act first (at
// the row facing the ghost, wrapped or nearest), then the y sides.  A wall
// ghost is the mirror image of the interior cell as far inside as the ghost
// is outside (the normal momentum changes sign in every slot, and the two
// distributions moving along the normal trade places); a Dirichlet ghost is
// the given moments u_D with u_k = M_k(u_D; a^n) (Example 1), the state the
// boundary is set to in Section 4.8; zero-gradient copies the boundary cell
// (Section 4.2).  Walls need two cells along their axis.
template <class T>
__device__ __forceinline__ void reflect_slots(T s[20], int ax) {
  const int c = 1 + ax, k0 = 1 + 2 * ax;
#pragma unroll
  for (int q = 0; q < 5; ++q) s[4 * q + c] = -s[4 * q + c];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const T t = s[4 * k0 + k];
    s[4 * k0 + k] = s[4 * (k0 + 1) + k];
    s[4 * (k0 + 1) + k] = t;
  }
}

// Boundary description of the instance whose slots are sl.
__device__ __forceinline__ BndDesc bnd_desc(const StepArgs& A, const Slots* sl) {
  return A.n_inst > 1 ? A.bnd_table[sl - A.slots] : A.bnd1;
}

// State of the ghost cell (i, j) of an instance with boundary descriptions.
// Each side the cell lies beyond has its kind read at its boundary cell
// nearest to the ghost.  Walls resolve first (the ghost is the mirror image
// of the cell it faces, so a corner ghost beside a wall is the mirror image
// of the ghost or cell across it), then a Dirichlet side, x before y (the
// given state at the resolved cell along that side and its Maxwellians,
// mirrored by the walls crossed), then zero-gradient sides (the nearest
// cell).  Periodic axes wrap.
template <class T, class C>
__device__ void bnd_cell(const StepArgs& A, const BndDesc& bd, const Inst& in, const T* __restrict__ sbase,
                         long long P, int i, int j, const StepConst<T, C>& K, T out[20]) {
  const Scheme& sc = A.sc;
  const int nx = in.nx, ny = in.ny;
  if (sc.bc_x == 0) i = map_index(i, nx, 0);
  if (sc.bc_y == 0) j = map_index(j, ny, 0);
  const bool out_x = i < 0 || i >= nx, out_y = j < 0 || j >= ny;
  const int side_x = i < 0 ? 0 : 1, side_y = j < 0 ? 2 : 3;
  const int kind_x = out_x && bd.kind[side_x] ? (int)bd.kind[side_x][map_index(j, ny, sc.bc_y)] : BND_ZERO_GRADIENT;
  const int kind_y = out_y && bd.kind[side_y] ? (int)bd.kind[side_y][map_index(i, nx, sc.bc_x)] : BND_ZERO_GRADIENT;
  const bool refl_x = out_x && kind_x == BND_WALL, refl_y = out_y && kind_y == BND_WALL;
  if (refl_x) i = i < 0 ? -1 - i : 2 * nx - 1 - i;
  if (refl_y) j = j < 0 ? -1 - j : 2 * ny - 1 - j;
  for (int ax = 0; ax < 2; ++ax) {
    if (!(ax == 0 ? out_x : out_y) || (ax == 0 ? kind_x : kind_y) != BND_DIRICHLET) continue;
    const int len = ax == 0 ? ny : nx;
    const int at = ax == 0 ? map_index(j, ny, sc.bc_y) : map_index(i, nx, sc.bc_x);
    const double* st = bd.state[ax == 0 ? side_x : side_y];
    C u[4], f[4], g[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) u[c] = (C)st[(long long)c * len + at];
    fluxes(u, K.gm1, f, g);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      out[c] = (T)u[c];
#pragma unroll
      for (int k = 0; k < 4; ++k) out[4 + 4 * k + c] = (T)maxw(k, u[c], f[c], g[c], K.w, K.r2a);
    }
    if (refl_y) reflect_slots(out, 1);
    if (refl_x) reflect_slots(out, 0);
    return;
  }
  i = map_index(i, nx, sc.bc_x);
  j = map_index(j, ny, sc.bc_y);
  const unsigned o = (unsigned)j * (unsigned)nx + (unsigned)i;
#pragma unroll
  for (int q = 0; q < 20; ++q) out[q] = (sbase + q * P)[o];
  if (refl_y) reflect_slots(out, 1);
  if (refl_x) reflect_slots(out, 0);
}

// Strip march for limiter sets without density bounds (PP, pressure,
// unlimited, first order).  Both face factors of row L are known as soon as
// the row arrives, so iteration L completes row L - 1.  Strips are 64 columns
// wide and aligned (x0 = 64 xs), every lane produces output: lane 0 loads the
// state of column x0 - 1 and lane 63 that of column x0 + 64 (the halo).
// Lane 63 evaluates its east face x0 + 63 + 1/2 from the halo like any other
// face, and lane 0 evaluates the west face x0 - 1/2 from its halo (a third
// face evaluation per row).  The strip to the west evaluates that same face
// with the same inputs and code, so both cells of a strip-edge face see the
// same theta.
template <class T, class C, int LIMS, bool TH, bool BND>
__device__ __forceinline__ void march_short(const StepArgs& A, const Inst& in, Slots* sl, int xs,
                                            int ys, int lane) {
  const Scheme& sc = A.sc;
  const int nx = in.nx, ny = in.ny;
  const int x0 = xs * 64;
  const int gi = x0 + lane;
  const int ci = map_index(gi, nx, sc.bc_x);
  const bool lane_out = gi < nx;
  const bool first = lane == 0, last = lane == 63;
  // halo column: west of lane 0 (its u and u_1), east of lane 63 (u and u_2)
  const int hcol = first ? map_index(x0 - 1, nx, sc.bc_x) : map_index(x0 + 64, nx, sc.bc_x);
  const int hslot = first ? 4 : 8;
  const int y0 = ys * in.strip_h;
  const int y1 = min(y0 + in.strip_h, ny);
  const bool sponge = LIMS == 0 && sc.sponge > 0;

  const double lam = __longlong_as_double((long long)sl->lam[A.slot]);
  const StepConst<T, C> K = step_const<T, C>(sc, lam);

  if (xs == 0 && ys == 0 && lane == 0) {
    sl->lam[(A.slot + 2) % 3] = 0ull;
    sl->t[(A.slot + 1) % 3] = sl->t[A.slot] + in.dx / K.a;
    if (sc.a_mode == 1 && K.a < 2.0 * lam / (1.0 - sc.alpha)) atomicOr(&sl->cnt[CNT_BOUCHUT], 1ull);
  }

  // plane q of this instance starts at base + q P; a cell is addressed by a
  // 32-bit offset row * nx + column from that uniform base
  const T* __restrict__ sbase = (const T*)A.src + in.off;
  T* __restrict__ dbase = (T*)A.dst + in.off;
  const long long P = A.plane;
  const unsigned unx = (unsigned)nx;

  // carried from row L - 1
  C pu[4] = {}, pg[4] = {}, pM3[4] = {}, pd3[4] = {}, pP[4] = {};

  double lmax = 0.0;
  unsigned n_bad = 0, n_guard = 0, n_lim = 0, n_cls = 0;

  T raw[20], hraw[8];
  // with boundary descriptions, ghost rows, columns past the edge and the
  // halo columns come from bnd_cell
  BndDesc bd{};
  if constexpr (BND) bd = bnd_desc(A, sl);
  auto bnd_load = [&](const int R) {
    if (R < 0 || R >= ny || !lane_out) {
      bnd_cell<T, C>(A, bd, in, sbase, P, gi < nx + 1 ? gi : nx + 1, R, K, raw);
    } else {
      const unsigned o = (unsigned)R * unx + (unsigned)ci;
#pragma unroll
      for (int q = 0; q < 20; ++q) raw[q] = (sbase + q * P)[o];
    }
    if (first || last) {
      T h[20];
      bnd_cell<T, C>(A, bd, in, sbase, P, first ? x0 - 1 : min(x0 + 64, nx + 1), R, K, h);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        hraw[q] = h[q];
        hraw[4 + q] = first ? h[4 + q] : h[8 + q];
      }
    }
  };
  if constexpr (BND) {
    bnd_load(y0 - 1);
  } else {
    const unsigned ro = (unsigned)map_index(y0 - 1, ny, sc.bc_y) * unx;
    const unsigned o = ro + (unsigned)ci;
#pragma unroll
    for (int q = 0; q < 20; ++q) raw[q] = (sbase + q * P)[o];
    if (first || last) {
      const unsigned oh = ro + (unsigned)hcol;
#pragma unroll
      for (int q = 0; q < 4; ++q) hraw[q] = (sbase + q * P)[oh];
#pragma unroll
      for (int q = 0; q < 4; ++q) hraw[4 + q] = (sbase + (hslot + q) * P)[oh];
    }
  }

  for (int L = y0 - 1; L <= y1; ++L) {
    C u[4], uk[4][4], hu[4], hk[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) u[c] = (C)raw[c];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) uk[k][c] = (C)raw[4 + 4 * k + c];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      hu[c] = (C)hraw[c];
      hk[c] = (C)hraw[4 + c];
    }
    if (BND && L < y1) {
      bnd_load(L + 1);
    } else if (L < y1) {  // prefetch row L + 1
      const unsigned ro = (unsigned)map_index(L + 1, ny, sc.bc_y) * unx;
      const unsigned o = ro + (unsigned)ci;
#pragma unroll
      for (int q = 0; q < 20; ++q) raw[q] = (sbase + q * P)[o];
      if (first || last) {
        const unsigned oh = ro + (unsigned)hcol;
#pragma unroll
        for (int q = 0; q < 4; ++q) hraw[q] = (sbase + q * P)[oh];
#pragma unroll
        for (int q = 0; q < 4; ++q) hraw[4 + q] = (sbase + (hslot + q) * P)[oh];
      }
    }

    C f[4], g[4], hf[4], hg[4];
    fluxes(u, K.gm1, f, g);
    fluxes(hu, K.gm1, hf, hg);
    C M[4][4], d[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        M[k][c] = maxw(k, u[c], f[c], g[c], K.w, K.r2a);
        d[k][c] = M[k][c] - uk[k][c];
      }
    // x-face i+1/2: the east neighbour's M_2, d_2 from its u, f and u_2
    C usx[4], dF[4], M2E[4], d2E[4], usy[4], dG[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      // lanes 0..62 take lane + 1; lane 63 takes its halo (the east column)
      const C uE = from_right_or(u[c], hu[c]);
      const C fE = from_right_or(f[c], hf[c]);
      const C u2E = from_right_or(uk[1][c], hk[c]);
      M2E[c] = maxw(1, uE, fE, fE, K.w, K.r2a);
      d2E[c] = M2E[c] - u2E;
      usx[c] = C(0.5) * (u[c] + uE) - (fE - f[c]) * K.r2k;
      dF[c] = K.ac * (d[0][c] - d2E[c]);
      // y-face L-1/2 between row L - 1 (below) and row L
      usy[c] = C(0.5) * (pu[c] + u[c]) - (g[c] - pg[c]) * K.r2k;
      dG[c] = K.ac * (pd3[c] - d[3][c]);
    }
    // west edge face x0 - 1/2 (meaningful in lane 0, whose halo is the west
    // column): the expressions of the east face of the western neighbour
    C usw[4], dFw[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const C hd1 = maxw(0, hu[c], hf[c], hg[c], K.w, K.r2a) - hk[c];
      usw[c] = C(0.5) * (hu[c] + u[c]) - (f[c] - hf[c]) * K.r2k;
      dFw[c] = K.ac * (hd1 - d[1][c]);
    }
    int gx, gy, gw;
    const C zero = C(0);
    double thx = face_theta<LIMS>(sc, usx, dF, K.kappa, zero, zero, zero, zero, gx);
    double thy = face_theta<LIMS>(sc, usy, dG, K.kappa, zero, zero, zero, zero, gy);
    double th_edge = face_theta<LIMS>(sc, usw, dFw, K.kappa, zero, zero, zero, zero, gw);
    if (sponge) {
      if (in_sponge(sc, gi, L, nx, ny) || in_sponge(sc, gi + 1, L, nx, ny)) thx = 0.0;
      if (in_sponge(sc, gi, L - 1, nx, ny) || in_sponge(sc, gi, L, nx, ny)) thy = 0.0;
      if (in_sponge(sc, x0 - 1, L, nx, ny) || in_sponge(sc, x0, L, nx, ny)) th_edge = 0.0;
    }
    const bool row0 = L >= y0 && L < y1;          // row L is produced by this strip
    const bool row1 = L - 1 >= y0 && L - 1 < y1;  // row L - 1 is completed now
    // faces counted here: the x-face i+1/2 of lanes 0..62, the west edge
    // face (lane 0) and the y-face L-1/2 of every lane
    if (row0 && !last && gi + 1 < nx) {
      n_guard += gx;
      n_lim += (thx < 1.0);
    }
    if (row0 && lane_out) {
      n_guard += gy;
      n_lim += (thy < 1.0);
    }
    if (row0 && first) {  // face x0 - 1/2 belongs to output cell x0
      n_guard += gw;
      n_lim += (th_edge < 1.0);
    }
    if (TH || (LIMS == 0 && A.theta_x)) {
      if (row0 && first) A.theta_x[(long long)L * (nx + 1) + x0] = th_edge;
      if (row0 && gi + 1 <= nx) A.theta_x[(long long)L * (nx + 1) + gi + 1] = thx;
      if (lane_out && (row0 || row1) && L >= 0 && L <= ny) A.theta_y[(long long)L * nx + gi] = thy;
    }

    const C tR = (C)thx;
    const C tL = from_left_or(tR, (C)th_edge);  // lane 0: the west edge face
    const C tB = (C)thy;
    C fin[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      // M_1(u_W) + theta_W d_1(W): from lane - 1, or from the halo for lane 0
      const C o1n = M[0][c] + tR * d[0][c];
      const C hM1 = maxw(0, hu[c], hf[c], hg[c], K.w, K.r2a);
      const C hd1 = hM1 - hk[c];
      const C u1n = from_left_or(o1n, hM1 + tL * hd1);
      const C u2n = M2E[c] + tR * d2E[c];
      const C u3n = pM3[c] + tB * pd3[c];
      C s = K.alpha * u[c];
      s = s + (u1n - tL * d[1][c]);
      s = s + (u2n - tR * d[0][c]);
      s = s + (u3n - tB * d[3][c]);
      // row L - 1 completes with its face j+1/2 (= L - 1/2)
      const C u4n = M[3][c] + tB * d[3][c];
      fin[c] = pP[c] + (u4n - tB * pd3[c]);
      if constexpr (sizeof(T) == 4) {
        // rows L (if produced) and L - 1 (if completed): element offset of
        // the row from the plane base and its size in bytes (0: no store)
        const long long r0 = row0 ? (long long)L * nx : 0, r1 = row1 ? (long long)(L - 1) * nx : 0;
        const unsigned rb0 = row0 ? unx * 4u : 0u, rb1 = row1 ? unx * 4u : 0u;
        // columns past the edge get an offset beyond any row (4 gi itself
        // could wrap around 2^32 when nx is close to 2^30)
        const unsigned voff = lane_out ? (unsigned)gi * 4u : 0xFFFFFFFFu;
        put_row(dbase + (4 + c) * P + r0, rb0, voff, (T)u1n);
        put_row(dbase + (8 + c) * P + r0, rb0, voff, (T)u2n);
        put_row(dbase + (12 + c) * P + r0, rb0, voff, (T)u3n);
        put_row(dbase + c * P + r1, rb1, voff, (T)fin[c]);
        put_row(dbase + (16 + c) * P + r1, rb1, voff, (T)u4n);
      } else {
        if (row0 && lane_out) {
          const unsigned o = (unsigned)L * unx + (unsigned)gi;
          put(&(dbase + (4 + c) * P)[o], (T)u1n);
          put(&(dbase + (8 + c) * P)[o], (T)u2n);
          put(&(dbase + (12 + c) * P)[o], (T)u3n);
        }
        if (row1 && lane_out) {
          const unsigned o = (unsigned)(L - 1) * unx + (unsigned)gi;
          put(&(dbase + c * P)[o], (T)fin[c]);
          put(&(dbase + (16 + c) * P)[o], (T)u4n);
        }
      }
      pP[c] = s;
    }
    if (row1 && lane_out) {
      const double l = cell_wavespeed((double)(T)fin[0], (double)(T)fin[1], (double)(T)fin[2],
                                      (double)(T)fin[3], sc.gamma);
      if (l < 0.0) {
        n_bad += 1;
        n_cls += bad_class((double)(T)fin[0], (double)(T)fin[1], (double)(T)fin[2], (double)(T)fin[3],
                           sc.gamma);
      } else {
        lmax = vmax(lmax, l);
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      pu[c] = u[c];
      pg[c] = g[c];
      pM3[c] = M[2][c];
      pd3[c] = d[2][c];
    }
  }

#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lmax = vmax(lmax, __shfl_xor(lmax, off, 64));
    n_bad += __shfl_xor(n_bad, off, 64);
    n_guard += __shfl_xor(n_guard, off, 64);
    n_lim += __shfl_xor(n_lim, off, 64);
  }
  unsigned n_nf, n_rho;
  reduce_classes(n_cls, n_nf, n_rho);
  if (lane == 0) publish(sl, (A.slot + 1) % 3, lmax, n_bad, n_guard, n_lim, 0, n_nf, n_rho);
}

// One aligned strip of the bounds-limited scheme (LMP / RLMP, eq. (29)):
// columns x0 .. x0 + 63, output rows [y0, y1).  A face's theta needs the
// density bounds of both its cells, and a cell's bounds need its upper y-face,
// so row L - 1's faces get their theta when row L arrives and row L - 2
// completes then (rows y0 - 2 .. y1 + 1 are read).  The edge lanes look one
// cell further out: lane 0 loads the west halo column x0 - 1 (u, u_1) and
// rho, m_1 of x0 - 2; lane 63 loads the east halo column x0 + 64 (u, u_2) and
// rho, m_1 of x0 + 65.  From them each evaluates the bounds of its halo cell,
// and lane 0 the west edge face x0 - 1/2, with the same expressions as every
// other lane, so both strips beside an edge face see the same theta.
template <class T, class C, int LIMS, bool TH, bool BND>
__device__ __forceinline__ void march_lmp(const StepArgs& A, const Inst& in, Slots* sl, int xs,
                                          int ys, int lane) {
  const Scheme& sc = A.sc;
  const int nx = in.nx, ny = in.ny;
  const int x0 = xs * 64;
  const int gi = x0 + lane;
  const int ci = map_index(gi, nx, sc.bc_x);
  const bool lane_out = gi < nx;
  const bool first = lane == 0, last = lane == 63;
  const int hcol = first ? map_index(x0 - 1, nx, sc.bc_x) : map_index(x0 + 64, nx, sc.bc_x);
  const int ocol = first ? map_index(x0 - 2, nx, sc.bc_x) : map_index(x0 + 65, nx, sc.bc_x);
  const int hslot = first ? 4 : 8;
  const int y0 = ys * in.strip_h;
  const int y1 = min(y0 + in.strip_h, ny);
  const bool sponge = LIMS == 0 && sc.sponge > 0;

  const double lam = __longlong_as_double((long long)sl->lam[A.slot]);
  const StepConst<T, C> K = step_const<T, C>(sc, lam);

  if (xs == 0 && ys == 0 && lane == 0) {
    sl->lam[(A.slot + 2) % 3] = 0ull;
    sl->t[(A.slot + 1) % 3] = sl->t[A.slot] + in.dx / K.a;
    if (sc.a_mode == 1 && K.a < 2.0 * lam / (1.0 - sc.alpha)) atomicOr(&sl->cnt[CNT_BOUCHUT], 1ull);
  }

  const T* __restrict__ sbase = (const T*)A.src + in.off;
  T* __restrict__ dbase = (T*)A.dst + in.off;
  const long long P = A.plane;
  const unsigned unx = (unsigned)nx;

  // carried state (zero before the first rows arrive)
  C pu[4] = {}, pf[4] = {}, pg[4] = {}, puk[4][4] = {};  // row L - 1
  C pusx[4] = {}, pdF[4] = {};                          // x-face i+1/2 of row L - 1
  C pusy[4] = {}, pdG[4] = {};                          // y-face L - 3/2
  C pmu = C(0), pnu = C(0);                             // bounds of row L - 2
  C qM3[4] = {}, qd3[4] = {}, qP[4] = {};               // row L - 2
  // edge lanes: the halo column's u and u_1 / u_2 of row L - 1, rho and m_1
  // of the outer column in row L - 1, the halo cell's y-face density at L - 3/2
  C hpu[4] = {}, hpk[4] = {}, hpf[4] = {}, hpg[4] = {};
  C opr = C(0), opm = C(0), hpy = C(0);

  double lmax = 0.0;
  unsigned n_bad = 0, n_guard = 0, n_lim = 0, n_lmp = 0, n_cls = 0;
  // float64 state: the stores of a row are issued at the top of the next
  // iteration, right after its prefetch, so that they complete under that
  // iteration's compute rather than ahead of its wait for the prefetched
  // row (measured 3% faster on the 2048^2 rarefaction; with the float32
  // state, and in the short march, the plain order measured faster)
  constexpr bool kDefer = sizeof(T) == 8;
  T sv[20];
  unsigned so1 = 0, so2 = 0;
  bool sw1 = false, sw2 = false;
  auto flush = [&]() {
    if (sw1) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        put(&(dbase + (4 + c) * P)[so1], sv[c]);
        put(&(dbase + (8 + c) * P)[so1], sv[4 + c]);
        put(&(dbase + (12 + c) * P)[so1], sv[8 + c]);
      }
    }
    if (sw2) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        put(&(dbase + c * P)[so2], sv[12 + c]);
        put(&(dbase + (16 + c) * P)[so2], sv[16 + c]);
      }
    }
  };

  T raw[20], hraw[8] = {}, oraw[2] = {};
  // with boundary descriptions, ghost rows, columns past the edge and the
  // halo columns come from bnd_cell
  BndDesc bd{};
  if constexpr (BND) bd = bnd_desc(A, sl);
  auto bnd_load = [&](const int R) {
    if (R < 0 || R >= ny || !lane_out) {
      bnd_cell<T, C>(A, bd, in, sbase, P, gi < nx + 1 ? gi : nx + 1, R, K, raw);
    } else {
      const unsigned o = (unsigned)R * unx + (unsigned)ci;
#pragma unroll
      for (int q = 0; q < 20; ++q) raw[q] = (sbase + q * P)[o];
    }
    if (first || last) {
      T h[20];
      bnd_cell<T, C>(A, bd, in, sbase, P, first ? x0 - 1 : min(x0 + 64, nx + 1), R, K, h);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        hraw[q] = h[q];
        hraw[4 + q] = first ? h[4 + q] : h[8 + q];
      }
      bnd_cell<T, C>(A, bd, in, sbase, P, first ? x0 - 2 : min(x0 + 65, nx + 1), R, K, h);
      oraw[0] = h[0];
      oraw[1] = h[1];
    }
  };
  if constexpr (BND) {
    bnd_load(y0 - 2);
  } else {
    const unsigned ro = (unsigned)map_index(y0 - 2, ny, sc.bc_y) * unx;
    const unsigned o = ro + (unsigned)ci;
#pragma unroll
    for (int q = 0; q < 20; ++q) raw[q] = (sbase + q * P)[o];
    if (first || last) {
      const unsigned oh = ro + (unsigned)hcol;
#pragma unroll
      for (int q = 0; q < 4; ++q) hraw[q] = (sbase + q * P)[oh];
#pragma unroll
      for (int q = 0; q < 4; ++q) hraw[4 + q] = (sbase + (hslot + q) * P)[oh];
      const unsigned oo = ro + (unsigned)ocol;
      oraw[0] = sbase[oo];
      oraw[1] = (sbase + P)[oo];
    }
  }

  for (int L = y0 - 2; L <= y1 + 1; ++L) {
    C u[4], uk[4][4], hu[4], hk[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) u[c] = (C)raw[c];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) uk[k][c] = (C)raw[4 + 4 * k + c];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      hu[c] = (C)hraw[c];
      hk[c] = (C)hraw[4 + c];
    }
    const C orr = (C)oraw[0], om = (C)oraw[1];
    if (BND && L <= y1) {
      bnd_load(L + 1);
    } else if (L <= y1) {  // prefetch row L + 1
      const unsigned ro = (unsigned)map_index(L + 1, ny, sc.bc_y) * unx;
      const unsigned o = ro + (unsigned)ci;
#pragma unroll
      for (int q = 0; q < 20; ++q) raw[q] = (sbase + q * P)[o];
      if (first || last) {
        const unsigned oh = ro + (unsigned)hcol;
#pragma unroll
        for (int q = 0; q < 4; ++q) hraw[q] = (sbase + q * P)[oh];
#pragma unroll
        for (int q = 0; q < 4; ++q) hraw[4 + q] = (sbase + (hslot + q) * P)[oh];
        const unsigned oo = ro + (unsigned)ocol;
        oraw[0] = sbase[oo];
        oraw[1] = (sbase + P)[oo];
      }
    }
    if constexpr (kDefer) {
      flush();
      __builtin_amdgcn_sched_barrier(0);
    }

    // ---- row L: fluxes, the x-face i+1/2 and the y-face L - 1/2
    C f[4], g[4];
    fluxes(u, K.gm1, f, g);
    C hf[4], hg[4];
    fluxes(hu, K.gm1, hf, hg);
    C usx[4], dF[4], usy[4], dG[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const C d1 = maxw(0, u[c], f[c], g[c], K.w, K.r2a) - uk[0][c];
      const C d4 = maxw(3, u[c], f[c], g[c], K.w, K.r2a) - uk[3][c];
      // lanes 0..62 take lane + 1; lane 63 takes its halo (the east column)
      const C uE = from_right_or(u[c], hu[c]);
      const C fE = from_right_or(f[c], hf[c]);
      const C u2E = from_right_or(uk[1][c], hk[c]);
      const C d2E = maxw(1, uE, fE, fE, K.w, K.r2a) - u2E;
      usx[c] = C(0.5) * (u[c] + uE) - (fE - f[c]) * K.r2k;
      dF[c] = K.ac * (d1 - d2E);
      const C pd3 = maxw(2, pu[c], pf[c], pg[c], K.w, K.r2a) - puk[2][c];
      usy[c] = C(0.5) * (pu[c] + u[c]) - (g[c] - pg[c]) * K.r2k;
      dG[c] = K.ac * (pd3 - d4);
    }

    // ---- row L - 1: the halo column's Maxwellians, the west edge face
    C hM[4], hd[4], usw[4], dFw[4], pd2[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      // lane 0: M_1 of the west column; lane 63: M_2 of the east column
      const C hM1 = maxw(0, hpu[c], hpf[c], hpg[c], K.w, K.r2a);
      const C hM2 = maxw(1, hpu[c], hpf[c], hpg[c], K.w, K.r2a);
      hM[c] = first ? hM1 : hM2;
      hd[c] = hM[c] - hpk[c];
      pd2[c] = maxw(1, pu[c], pf[c], pg[c], K.w, K.r2a) - puk[1][c];
      usw[c] = C(0.5) * (hpu[c] + pu[c]) - (pf[c] - hpf[c]) * K.r2k;
      dFw[c] = K.ac * (hd[c] - pd2[c]);
    }

    // ---- row L - 1: density bounds (eq. (29)) of the own cell and of the
    // halo cell (edge lanes)
    const C rW = from_left_or(pusx[0], usw[0]);
    C mu1 = pu[0], nu1 = pu[0];
    mu1 = vmin(mu1, rW);
    nu1 = vmax(nu1, rW);
    mu1 = vmin(mu1, pusx[0]);
    nu1 = vmax(nu1, pusx[0]);
    mu1 = vmin(mu1, pusy[0]);
    nu1 = vmax(nu1, pusy[0]);
    mu1 = vmin(mu1, usy[0]);
    nu1 = vmax(nu1, usy[0]);
    // halo cell: its inner x-face (lane 0: the west edge face; lane 63: its
    // own east face), its outer x-face and its y-faces L - 3/2 and L - 1/2
    const C xin = first ? usw[0] : pusx[0];
    const C rwo = first ? opr : hpu[0], rwe = first ? hpu[0] : opr;
    const C mwo = first ? opm : hpu[1], mwe = first ? hpu[1] : opm;
    const C xout = C(0.5) * (rwo + rwe) - (mwe - mwo) * K.r2k;
    const C hy = C(0.5) * (hpu[0] + hu[0]) - (hu[2] - hpu[2]) * K.r2k;
    C hmu = hpu[0], hnu = hpu[0];
    hmu = vmin(hmu, first ? xout : xin);
    hnu = vmax(hnu, first ? xout : xin);
    hmu = vmin(hmu, first ? xin : xout);
    hnu = vmax(hnu, first ? xin : xout);
    hmu = vmin(hmu, hpy);
    hnu = vmax(hnu, hpy);
    hmu = vmin(hmu, hy);
    hnu = vmax(hnu, hy);

    // ---- theta of the x-face i+1/2 and the west edge face of row L - 1,
    // and of the y-face L - 3/2
    const C muE = from_right_or(mu1, hmu);
    const C nuE = from_right_or(nu1, hnu);
    int gx, gy, gw;
    double thx = face_theta<LIMS>(sc, pusx, pdF, K.kappa, mu1, nu1, muE, nuE, gx);
    double thy = face_theta<LIMS>(sc, pusy, pdG, K.kappa, pmu, pnu, mu1, nu1, gy);
    double th_edge = face_theta<LIMS>(sc, usw, dFw, K.kappa, hmu, hnu, mu1, nu1, gw);
    if (sponge) {
      if (in_sponge(sc, gi, L - 1, nx, ny) || in_sponge(sc, gi + 1, L - 1, nx, ny)) thx = 0.0;
      if (in_sponge(sc, gi, L - 2, nx, ny) || in_sponge(sc, gi, L - 1, nx, ny)) thy = 0.0;
      if (in_sponge(sc, x0 - 1, L - 1, nx, ny) || in_sponge(sc, x0, L - 1, nx, ny)) th_edge = 0.0;
    }
    const bool row1 = L - 1 >= y0 && L - 1 < y1;  // row L - 1 is produced by this strip
    const bool row2 = L - 2 >= y0 && L - 2 < y1;  // row L - 2 is completed now
    // faces counted here: the x-face i+1/2 of lanes 0..62, the west edge
    // face (lane 0) and the y-face L - 3/2 of every lane
    if (row1 && !last && gi + 1 < nx) {
      n_guard += gx;
      n_lim += (thx < 1.0);
    }
    if (row1 && lane_out) {
      n_guard += gy;
      n_lim += (thy < 1.0);
    }
    if (row1 && first) {
      n_guard += gw;
      n_lim += (th_edge < 1.0);
    }
    if (TH || (LIMS == 0 && A.theta_x)) {
      if (row1 && first) A.theta_x[(long long)(L - 1) * (nx + 1) + x0] = th_edge;
      if (row1 && gi + 1 <= nx) A.theta_x[(long long)(L - 1) * (nx + 1) + gi + 1] = thx;
      if (lane_out && (row1 || row2) && L - 1 >= 0 && L - 1 <= ny)
        A.theta_y[(long long)(L - 1) * nx + gi] = thy;
    }

    // ---- rows L - 1 and L - 2: streaming and the moment slot (eqs. (25), (27))
    const C tR = (C)thx;
    const C tL = from_left_or(tR, (C)th_edge);  // lane 0: the west edge face
    const C tB = (C)thy;
    C fin[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const C pM1 = maxw(0, pu[c], pf[c], pg[c], K.w, K.r2a);
      const C pM3 = maxw(2, pu[c], pf[c], pg[c], K.w, K.r2a);
      const C pM4 = maxw(3, pu[c], pf[c], pg[c], K.w, K.r2a);
      const C pd1 = pM1 - puk[0][c];
      const C pd4 = pM4 - puk[3][c];
      // M_1 + theta d_1 of the west neighbour (lane 0: the halo column)
      const C u1n = from_left_or(pM1 + tR * pd1, hM[c] + tL * hd[c]);
      // M_2 + theta d_2 of the east neighbour (lane 63: the halo column)
      const C M2E = from_right_or(maxw(1, pu[c], pf[c], pg[c], K.w, K.r2a), hM[c]);
      const C d2E = from_right_or(pd2[c], hd[c]);
      const C u2n = M2E + tR * d2E;
      const C u3n = qM3[c] + tB * qd3[c];
      C s = K.alpha * pu[c];
      s = s + (u1n - tL * pd2[c]);
      s = s + (u2n - tR * pd1);
      s = s + (u3n - tB * pd4);
      // row L - 2 completes with its face j+1/2 (= L - 3/2)
      const C u4n = pM4 + tB * pd4;
      fin[c] = qP[c] + (u4n - tB * qd3[c]);
      if constexpr (kDefer) {
        sv[c] = (T)u1n;
        sv[4 + c] = (T)u2n;
        sv[8 + c] = (T)u3n;
        sv[12 + c] = (T)fin[c];
        sv[16 + c] = (T)u4n;
      } else {
        if (row1 && lane_out) {
          const unsigned o = (unsigned)(L - 1) * unx + (unsigned)gi;
          put(&(dbase + (4 + c) * P)[o], (T)u1n);
          put(&(dbase + (8 + c) * P)[o], (T)u2n);
          put(&(dbase + (12 + c) * P)[o], (T)u3n);
        }
        if (row2 && lane_out) {
          const unsigned o = (unsigned)(L - 2) * unx + (unsigned)gi;
          put(&(dbase + c * P)[o], (T)fin[c]);
          put(&(dbase + (16 + c) * P)[o], (T)u4n);
        }
      }
      qP[c] = s;
      qM3[c] = pM3;
      qd3[c] = pM3 - puk[2][c];
    }
    if constexpr (kDefer) {
      sw1 = row1 && lane_out;
      so1 = (unsigned)(L - 1) * unx + (unsigned)gi;
      sw2 = row2 && lane_out;
      so2 = (unsigned)(L - 2) * unx + (unsigned)gi;
    }
    if (row2 && lane_out) {
      // wavespeed of the stored new state, in float64
      const double l = cell_wavespeed((double)(T)fin[0], (double)(T)fin[1], (double)(T)fin[2],
                                      (double)(T)fin[3], sc.gamma);
      if (l < 0.0) {
        n_bad += 1;
        n_cls += bad_class((double)(T)fin[0], (double)(T)fin[1], (double)(T)fin[2], (double)(T)fin[3],
                           sc.gamma);
      } else {
        lmax = vmax(lmax, l);
      }
      // LMP check: the stored density against the eq. (29) bounds of the
      // cell (pmu, pnu: row L - 2), beyond the rounding of the update
      const double r = (double)(T)fin[0], lo = (double)pmu, hi = (double)pnu;
      n_lmp += (r < lo - kLmpTol<T> * fabs(lo)) || (r > hi + kLmpTol<T> * fabs(hi));
    }
    pmu = mu1;
    pnu = nu1;
    hpy = hy;
    opr = orr;
    opm = om;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      pu[c] = u[c];
      pf[c] = f[c];
      pg[c] = g[c];
      pusx[c] = usx[c];
      pdF[c] = dF[c];
      pusy[c] = usy[c];
      pdG[c] = dG[c];
      hpu[c] = hu[c];
      hpk[c] = hk[c];
      hpf[c] = hf[c];
      hpg[c] = hg[c];
#pragma unroll
      for (int k = 0; k < 4; ++k) puk[k][c] = uk[k][c];
    }
  }

  if constexpr (kDefer) flush();

#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lmax = vmax(lmax, __shfl_xor(lmax, off, 64));
    n_lmp += __shfl_xor(n_lmp, off, 64);
    n_bad += __shfl_xor(n_bad, off, 64);
    n_guard += __shfl_xor(n_guard, off, 64);
    n_lim += __shfl_xor(n_lim, off, 64);
  }
  unsigned n_nf, n_rho;
  reduce_classes(n_cls, n_nf, n_rho);
  if (lane == 0) publish(sl, (A.slot + 1) % 3, lmax, n_bad, n_guard, n_lim, n_lmp, n_nf, n_rho);
}

// ------------------------------------------ bounds-limited march, LDS-staged

// Row buffers per wave of the LDS-staged march: the row being consumed and
// the two requested after it.  Each row occupies 20 planes x 64 columns of T
// followed by the 16 halo loads of 16 bytes each.
constexpr int kDmaRing = 3;
constexpr int kDmaHaloBytes = 16 * 16;
template <class T>
constexpr int dma_row_bytes() { return 20 * 64 * (int)sizeof(T) + kDmaHaloBytes; }
template <class T>
constexpr int dma_lds_bytes(int waves) { return waves * kDmaRing * dma_row_bytes<T>(); }

typedef __attribute__((address_space(3))) void lds_void;

// The bounds-limited march of march_lmp with the state rows brought in by
// direct loads into LDS (global_load_lds_dwordx4: each lane moves 16 bytes,
// so one instruction carries 1024 bytes, two planes' rows in float64 or four
// in float32) two rows ahead of the row being consumed, instead of through
// registers one row ahead.  The halo values of the edge lanes (the columns
// x0 - 1, x0 - 2, x0 + 64, x0 + 65) come in the same way, 16 bytes per lane
// from 16 lanes.
// Arithmetic, evaluation order and results are those of march_lmp; only where
// the loaded values wait differs.  Used for single instances whose width is a
// multiple of 64 (every strip full) and that have no boundary descriptions.
// The loads into LDS are not tracked by the compiler's wait counters:
// the march waits on the vector-memory counter itself (see the loop head).
template <class T, class C, int LIMS, bool TH, bool BLK>
__device__ __forceinline__ void march_lmp_dma(const StepArgs& A, const Inst& in, Slots* sl, int xs,
                                              int ys, int lane, int wave) {
  const Scheme& sc = A.sc;
  const int nx = in.nx, ny = in.ny;
  const int x0 = xs * 64;
  const int gi = x0 + lane;
  const bool first = lane == 0, last = lane == 63;
  const int y0 = ys * in.strip_h;
  const int y1 = min(y0 + in.strip_h, ny);

  const double lam = __longlong_as_double((long long)sl->lam[A.slot]);
  const StepConst<T, C> K = step_const<T, C>(sc, lam);
  const bool sponge = LIMS == 0 && sc.sponge > 0;

  if (xs == 0 && ys == 0 && lane == 0) {
    sl->lam[(A.slot + 2) % 3] = 0ull;
    sl->t[(A.slot + 1) % 3] = sl->t[A.slot] + in.dx / K.a;
    if (sc.a_mode == 1 && K.a < 2.0 * lam / (1.0 - sc.alpha)) atomicOr(&sl->cnt[CNT_BOUCHUT], 1ull);
  }

  // the instance's first value: planar, cell (0, 0) of plane 0; blocked,
  // its whole state follows the instances before it
  const T* __restrict__ sbase = (const T*)A.src + in.off * (BLK ? 20 : 1);
  T* __restrict__ dbase = (T*)A.dst + in.off * (BLK ? 20 : 1);
  const long long P = A.plane;
  const unsigned unx = (unsigned)nx;
  // where value q of this lane's cell in row R goes
  auto out_at = [&](int q, int R) -> T* {
    if constexpr (BLK)
      return dbase + ((long long)R * nx + x0) * 20 + q * 64 + lane;
    else
      return &(dbase + q * P)[(unsigned)R * unx + (unsigned)gi];
  };

  extern __shared__ __align__(16) unsigned char dma_lds[];
  unsigned char* ring = dma_lds + wave * kDmaRing * dma_row_bytes<T>();
  // lane's byte offset inside one load of 1024 bytes: planes per load
  constexpr int kPpl = 1024 / (64 * (int)sizeof(T));  // 2 (float64) or 4 (float32)
  constexpr int kLanesPerPlane = 64 / kPpl;
  // planar: plane q + lane / kLanesPerPlane of the group; blocked: the
  // group's kPpl planes of the strip row lie together
  const long long lane_elem = BLK ? (long long)lane * (16 / (int)sizeof(T))
                                  : (long long)(lane / kLanesPerPlane) * P + (lane % kLanesPerPlane) * (16 / (int)sizeof(T));
  // halo: lanes 0-7 bring 16 bytes of planes 0-7 (u, u_1) that hold the
  // west columns x0 - 2 and x0 - 1, lanes 8-15 16 bytes of planes 0-3 and
  // 8-11 (u, u_2) that hold the east columns x0 + 64 and x0 + 65.  Each pair
  // of columns is wrapped or clamped first; the two are then adjacent or
  // equal (x0 is a multiple of 64 and so is nx), and the 16 bytes start at the
  // aligned element at or below the smaller one; west2 .. east1 are the
  // columns' positions inside the 16 bytes.
  constexpr int kVpl = 16 / (int)sizeof(T);  // values per 16 bytes
  const bool hlane = lane < 16;
  int wstart, west2, west1, estart, east0, east1;
  {
    const int a2 = map_index(x0 - 2, nx, sc.bc_x), a1 = map_index(x0 - 1, nx, sc.bc_x);
    wstart = min(a2, a1) / kVpl * kVpl;
    west2 = a2 - wstart;
    west1 = a1 - wstart;
    const int b0 = map_index(x0 + 64, nx, sc.bc_x), b1 = map_index(x0 + 65, nx, sc.bc_x);
    estart = min(b0, b1) / kVpl * kVpl;
    east0 = b0 - estart;
    east1 = b1 - estart;
  }
  const int hq = lane < 8 ? lane : (lane < 12 ? lane - 8 : lane - 4);
  const int hcol = lane < 8 ? wstart : estart;
  const long long halo_elem = BLK ? (long long)(hcol >> 6) * 1280 + hq * 64 + (hcol & 63) : (long long)hq * P + hcol;

  // bring row R (wrapped or clamped) into ring buffer b
  auto issue = [&](int R, int b) {
    // row offset: the row's first cell of every plane (planar), or its first
    // 64-cell block (blocked)
    const long long ro = (long long)map_index(R, ny, sc.bc_y) * nx * (BLK ? 20 : 1);
    unsigned char* dst = ring + b * dma_row_bytes<T>();
#pragma unroll
    for (int q = 0; q < 20; q += kPpl) {
      const T* g = BLK ? sbase + ro + (long long)xs * 1280 + q * 64 + lane_elem
                       : sbase + (long long)q * P + ro + x0 + lane_elem;
      __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)(dst + q * 64 * (int)sizeof(T)), 16, 0, 0);
    }
    if (hlane) {
      const T* g = sbase + halo_elem + ro;
      __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)(dst + 20 * 64 * (int)sizeof(T)), 16, 0, 0);
    }
  };
  // vector-memory operations of one row's loads
  constexpr int kRowOps = 20 / kPpl + 1;

  // carried state (zero before the first rows arrive)
  C pu[4] = {}, pf[4] = {}, pg[4] = {}, puk[4][4] = {};
  C pusx[4] = {}, pdF[4] = {};
  C pusy[4] = {}, pdG[4] = {};
  C pmu = C(0), pnu = C(0);
  C qM3[4] = {}, qd3[4] = {}, qP[4] = {};
  C hpu[4] = {}, hpk[4] = {}, hpf[4] = {}, hpg[4] = {};
  C opr = C(0), opm = C(0), hpy = C(0);

  double lmax = 0.0;
  unsigned n_bad = 0, n_guard = 0, n_lim = 0, n_lmp = 0, n_cls = 0;

  issue(y0 - 2, 0);
  issue(y0 - 1, 1);
  int b = 0;
  for (int L = y0 - 2; L <= y1 + 1; ++L) {
    // Row L's loads were issued at the top of iteration L - 2.  The vector
    // memory counter drains in issue order, so row L has arrived when no more
    // operations are outstanding than were issued after it: the 20 stores of
    // iteration L - 2, row L + 1's loads and the 20 stores of iteration L - 1.
    // That count is exact where both iterations stored both of their rows
    // (every store is then issued, and the face-factor stores of the TH
    // kernels are absent); elsewhere the march waits for row L + 1 too
    // (vmcnt(kRowOps)), or for everything where row L + 1 was not requested.
    // Waiting for fewer outstanding operations than the exact count is
    // always safe; the exact count lets the stores of the last two
    // iterations drain while the next row is computed.
    if (!TH && L - 4 >= y0 && L <= y1)
      __builtin_amdgcn_s_waitcnt(sizeof(T) == 8 ? 0xCF73 : 0x8F7E);  // vmcnt(40 + kRowOps)
    else if (L + 1 <= y1 + 1)
      __builtin_amdgcn_s_waitcnt(sizeof(T) == 8 ? 0x0F7B : 0x0F76);  // vmcnt(kRowOps)
    else
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    static_assert(kRowOps == (sizeof(T) == 8 ? 11 : 6), "wait counts of the loop head");
    // row L + 2 goes into the buffer of row L - 1, whose values were read
    // into registers in the previous iteration
    __builtin_amdgcn_sched_barrier(0);
    if (L + 2 <= y1 + 1) issue(L + 2, b == 0 ? 2 : b - 1);
    __builtin_amdgcn_sched_barrier(0);
    const unsigned char* rb = ring + b * dma_row_bytes<T>();
    const T* rowv = (const T*)rb;
    const T* hrow = (const T*)(rb + 20 * 64 * (int)sizeof(T));
    C u[4], uk[4][4], hu[4], hk[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) u[c] = (C)rowv[c * 64 + lane];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) uk[k][c] = (C)rowv[(4 + 4 * k + c) * 64 + lane];
    // halo: lane 0 reads the west values (column x0 - 1, and x0 - 2 for rho
    // and m1), every other lane the east ones (only lane 63 uses them); halo
    // load lane h left its 16 bytes at h * kVpl values
    const int hbase = first ? 0 : 8;
    const int ein = first ? west1 : east0;   // the halo column's element
    const int eout = first ? west2 : east1;  // the outer column's element
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      hu[c] = (C)hrow[(hbase + c) * kVpl + ein];
      hk[c] = (C)hrow[(hbase + 4 + c) * kVpl + ein];
    }
    const C orr = (C)hrow[hbase * kVpl + eout], om = (C)hrow[(hbase + 1) * kVpl + eout];

    // ---- row L: fluxes, the x-face i+1/2 and the y-face L - 1/2
    C f[4], g[4];
    fluxes(u, K.gm1, f, g);
    C hf[4], hg[4];
    fluxes(hu, K.gm1, hf, hg);
    C usx[4], dF[4], usy[4], dG[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const C d1 = maxw(0, u[c], f[c], g[c], K.w, K.r2a) - uk[0][c];
      const C d4 = maxw(3, u[c], f[c], g[c], K.w, K.r2a) - uk[3][c];
      const C uE = from_right_or(u[c], hu[c]);
      const C fE = from_right_or(f[c], hf[c]);
      const C u2E = from_right_or(uk[1][c], hk[c]);
      const C d2E = maxw(1, uE, fE, fE, K.w, K.r2a) - u2E;
      usx[c] = C(0.5) * (u[c] + uE) - (fE - f[c]) * K.r2k;
      dF[c] = K.ac * (d1 - d2E);
      const C pd3 = maxw(2, pu[c], pf[c], pg[c], K.w, K.r2a) - puk[2][c];
      usy[c] = C(0.5) * (pu[c] + u[c]) - (g[c] - pg[c]) * K.r2k;
      dG[c] = K.ac * (pd3 - d4);
    }

    // ---- row L - 1: the halo column's Maxwellians, the west edge face
    C hM[4], hd[4], usw[4], dFw[4], pd2[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const C hM1 = maxw(0, hpu[c], hpf[c], hpg[c], K.w, K.r2a);
      const C hM2 = maxw(1, hpu[c], hpf[c], hpg[c], K.w, K.r2a);
      hM[c] = first ? hM1 : hM2;
      hd[c] = hM[c] - hpk[c];
      pd2[c] = maxw(1, pu[c], pf[c], pg[c], K.w, K.r2a) - puk[1][c];
      usw[c] = C(0.5) * (hpu[c] + pu[c]) - (pf[c] - hpf[c]) * K.r2k;
      dFw[c] = K.ac * (hd[c] - pd2[c]);
    }

    // ---- row L - 1: density bounds (eq. (29)) of the own cell and of the
    // halo cell (edge lanes)
    const C rW = from_left_or(pusx[0], usw[0]);
    C mu1 = pu[0], nu1 = pu[0];
    mu1 = vmin(mu1, rW);
    nu1 = vmax(nu1, rW);
    mu1 = vmin(mu1, pusx[0]);
    nu1 = vmax(nu1, pusx[0]);
    mu1 = vmin(mu1, pusy[0]);
    nu1 = vmax(nu1, pusy[0]);
    mu1 = vmin(mu1, usy[0]);
    nu1 = vmax(nu1, usy[0]);
    const C xin = first ? usw[0] : pusx[0];
    const C rwo = first ? opr : hpu[0], rwe = first ? hpu[0] : opr;
    const C mwo = first ? opm : hpu[1], mwe = first ? hpu[1] : opm;
    const C xout = C(0.5) * (rwo + rwe) - (mwe - mwo) * K.r2k;
    const C hy = C(0.5) * (hpu[0] + hu[0]) - (hu[2] - hpu[2]) * K.r2k;
    C hmu = hpu[0], hnu = hpu[0];
    hmu = vmin(hmu, first ? xout : xin);
    hnu = vmax(hnu, first ? xout : xin);
    hmu = vmin(hmu, first ? xin : xout);
    hnu = vmax(hnu, first ? xin : xout);
    hmu = vmin(hmu, hpy);
    hnu = vmax(hnu, hpy);
    hmu = vmin(hmu, hy);
    hnu = vmax(hnu, hy);

    // ---- theta of the x-face i+1/2 and the west edge face of row L - 1,
    // and of the y-face L - 3/2
    const C muE = from_right_or(mu1, hmu);
    const C nuE = from_right_or(nu1, hnu);
    int gx, gy, gw;
    double thx = face_theta<LIMS>(sc, pusx, pdF, K.kappa, mu1, nu1, muE, nuE, gx);
    double thy = face_theta<LIMS>(sc, pusy, pdG, K.kappa, pmu, pnu, mu1, nu1, gy);
    double th_edge = face_theta<LIMS>(sc, usw, dFw, K.kappa, hmu, hnu, mu1, nu1, gw);
    if (sponge) {
      if (in_sponge(sc, gi, L - 1, nx, ny) || in_sponge(sc, gi + 1, L - 1, nx, ny)) thx = 0.0;
      if (in_sponge(sc, gi, L - 2, nx, ny) || in_sponge(sc, gi, L - 1, nx, ny)) thy = 0.0;
      if (in_sponge(sc, x0 - 1, L - 1, nx, ny) || in_sponge(sc, x0, L - 1, nx, ny)) th_edge = 0.0;
    }
    const bool row1 = L - 1 >= y0 && L - 1 < y1;
    const bool row2 = L - 2 >= y0 && L - 2 < y1;
    if (row1 && !last) {
      n_guard += gx;
      n_lim += (thx < 1.0);
    }
    if (row1) {
      n_guard += gy;
      n_lim += (thy < 1.0);
    }
    if (row1 && first) {
      n_guard += gw;
      n_lim += (th_edge < 1.0);
    }
    if (TH || (LIMS == 0 && A.theta_x)) {
      if (row1 && first) A.theta_x[(long long)(L - 1) * (nx + 1) + x0] = th_edge;
      if (row1) A.theta_x[(long long)(L - 1) * (nx + 1) + gi + 1] = thx;
      if ((row1 || row2) && L - 1 >= 0 && L - 1 <= ny) A.theta_y[(long long)(L - 1) * nx + gi] = thy;
    }

    // ---- rows L - 1 and L - 2: streaming and the moment slot (eqs. (25), (27))
    const C tR = (C)thx;
    const C tL = from_left_or(tR, (C)th_edge);
    const C tB = (C)thy;
    C fin[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const C pM1 = maxw(0, pu[c], pf[c], pg[c], K.w, K.r2a);
      const C pM3 = maxw(2, pu[c], pf[c], pg[c], K.w, K.r2a);
      const C pM4 = maxw(3, pu[c], pf[c], pg[c], K.w, K.r2a);
      const C pd1 = pM1 - puk[0][c];
      const C pd4 = pM4 - puk[3][c];
      const C u1n = from_left_or(pM1 + tR * pd1, hM[c] + tL * hd[c]);
      const C M2E = from_right_or(maxw(1, pu[c], pf[c], pg[c], K.w, K.r2a), hM[c]);
      const C d2E = from_right_or(pd2[c], hd[c]);
      const C u2n = M2E + tR * d2E;
      const C u3n = qM3[c] + tB * qd3[c];
      C s = K.alpha * pu[c];
      s = s + (u1n - tL * pd2[c]);
      s = s + (u2n - tR * pd1);
      s = s + (u3n - tB * pd4);
      const C u4n = pM4 + tB * pd4;
      fin[c] = qP[c] + (u4n - tB * qd3[c]);
      if (row1) {
        put(out_at(4 + c, L - 1), (T)u1n);
        put(out_at(8 + c, L - 1), (T)u2n);
        put(out_at(12 + c, L - 1), (T)u3n);
      }
      if (row2) {
        put(out_at(c, L - 2), (T)fin[c]);
        put(out_at(16 + c, L - 2), (T)u4n);
      }
      qP[c] = s;
      qM3[c] = pM3;
      qd3[c] = pM3 - puk[2][c];
    }
    if (row2) {
      const double l = cell_wavespeed((double)(T)fin[0], (double)(T)fin[1], (double)(T)fin[2],
                                      (double)(T)fin[3], sc.gamma);
      if (l < 0.0) {
        n_bad += 1;
        n_cls += bad_class((double)(T)fin[0], (double)(T)fin[1], (double)(T)fin[2], (double)(T)fin[3],
                           sc.gamma);
      } else {
        lmax = vmax(lmax, l);
      }
      const double r = (double)(T)fin[0], lo = (double)pmu, hi = (double)pnu;
      n_lmp += (r < lo - kLmpTol<T> * fabs(lo)) || (r > hi + kLmpTol<T> * fabs(hi));
    }
    pmu = mu1;
    pnu = nu1;
    hpy = hy;
    opr = orr;
    opm = om;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      pu[c] = u[c];
      pf[c] = f[c];
      pg[c] = g[c];
      pusx[c] = usx[c];
      pdF[c] = dF[c];
      pusy[c] = usy[c];
      pdG[c] = dG[c];
      hpu[c] = hu[c];
      hpk[c] = hk[c];
      hpf[c] = hf[c];
      hpg[c] = hg[c];
#pragma unroll
      for (int k = 0; k < 4; ++k) puk[k][c] = uk[k][c];
    }
    b = b == 2 ? 0 : b + 1;
  }

#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lmax = vmax(lmax, __shfl_xor(lmax, off, 64));
    n_lmp += __shfl_xor(n_lmp, off, 64);
    n_bad += __shfl_xor(n_bad, off, 64);
    n_guard += __shfl_xor(n_guard, off, 64);
    n_lim += __shfl_xor(n_lim, off, 64);
  }
  unsigned n_nf, n_rho;
  reduce_classes(n_cls, n_nf, n_rho);
  if (lane == 0) publish(sl, (A.slot + 1) % 3, lmax, n_bad, n_guard, n_lim, n_lmp, n_nf, n_rho);
}

// ------------------------------------------ short march, LDS-staged

// The march of march_short with the state rows brought in by direct loads
// into LDS two rows ahead, as in march_lmp_dma (the same ring, halo loads and
// waits): same arithmetic, evaluation order and results.  It serves the
// blocked state of a context (single instance, width a multiple of 64, no
// boundary descriptions), where a strip row is one contiguous range; planar
// states take march_short.
template <class T, class C, int LIMS, bool TH, bool BLK>
__device__ __forceinline__ void march_short_dma(const StepArgs& A, const Inst& in, Slots* sl, int xs,
                                                int ys, int lane, int wave) {
  const Scheme& sc = A.sc;
  const int nx = in.nx, ny = in.ny;
  const int x0 = xs * 64;
  const int gi = x0 + lane;
  const bool first = lane == 0, last = lane == 63;
  const int y0 = ys * in.strip_h;
  const int y1 = min(y0 + in.strip_h, ny);
  const bool sponge = LIMS == 0 && sc.sponge > 0;

  const double lam = __longlong_as_double((long long)sl->lam[A.slot]);
  const StepConst<T, C> K = step_const<T, C>(sc, lam);

  if (xs == 0 && ys == 0 && lane == 0) {
    sl->lam[(A.slot + 2) % 3] = 0ull;
    sl->t[(A.slot + 1) % 3] = sl->t[A.slot] + in.dx / K.a;
    if (sc.a_mode == 1 && K.a < 2.0 * lam / (1.0 - sc.alpha)) atomicOr(&sl->cnt[CNT_BOUCHUT], 1ull);
  }

  // the instance's first value: planar, cell (0, 0) of plane 0; blocked,
  // its whole state follows the instances before it
  const T* __restrict__ sbase = (const T*)A.src + in.off * (BLK ? 20 : 1);
  T* __restrict__ dbase = (T*)A.dst + in.off * (BLK ? 20 : 1);
  const long long P = A.plane;
  const unsigned unx = (unsigned)nx;
  auto out_at = [&](int q, int R) -> T* {
    if constexpr (BLK)
      return dbase + ((long long)R * nx + x0) * 20 + q * 64 + lane;
    else
      return &(dbase + q * P)[(unsigned)R * unx + (unsigned)gi];
  };

  extern __shared__ __align__(16) unsigned char dma_lds[];
  unsigned char* ring = dma_lds + wave * kDmaRing * dma_row_bytes<T>();
  constexpr int kPpl = 1024 / (64 * (int)sizeof(T));
  constexpr int kLanesPerPlane = 64 / kPpl;
  const long long lane_elem = BLK ? (long long)lane * (16 / (int)sizeof(T))
                                  : (long long)(lane / kLanesPerPlane) * P + (lane % kLanesPerPlane) * (16 / (int)sizeof(T));
  constexpr int kVpl = 16 / (int)sizeof(T);
  const bool hlane = lane < 16;
  int wstart, west1, estart, east0;
  {
    const int a2 = map_index(x0 - 2, nx, sc.bc_x), a1 = map_index(x0 - 1, nx, sc.bc_x);
    wstart = min(a2, a1) / kVpl * kVpl;
    west1 = a1 - wstart;
    const int b0 = map_index(x0 + 64, nx, sc.bc_x), b1 = map_index(x0 + 65, nx, sc.bc_x);
    estart = min(b0, b1) / kVpl * kVpl;
    east0 = b0 - estart;
  }
  const int hq = lane < 8 ? lane : (lane < 12 ? lane - 8 : lane - 4);
  const int hcol = lane < 8 ? wstart : estart;
  const long long halo_elem = BLK ? (long long)(hcol >> 6) * 1280 + hq * 64 + (hcol & 63) : (long long)hq * P + hcol;
  auto issue = [&](int R, int b) {
    const long long ro = (long long)map_index(R, ny, sc.bc_y) * nx * (BLK ? 20 : 1);
    unsigned char* dst = ring + b * dma_row_bytes<T>();
#pragma unroll
    for (int q = 0; q < 20; q += kPpl) {
      const T* g = BLK ? sbase + ro + (long long)xs * 1280 + q * 64 + lane_elem
                       : sbase + (long long)q * P + ro + x0 + lane_elem;
      __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)(dst + q * 64 * (int)sizeof(T)), 16, 0, 0);
    }
    if (hlane) {
      const T* g = sbase + halo_elem + ro;
      __builtin_amdgcn_global_load_lds((const void*)g, (lds_void*)(dst + 20 * 64 * (int)sizeof(T)), 16, 0, 0);
    }
  };
  constexpr int kRowOps = 20 / kPpl + 1;

  C pu[4] = {}, pg[4] = {}, pM3[4] = {}, pd3[4] = {}, pP[4] = {};
  double lmax = 0.0;
  unsigned n_bad = 0, n_guard = 0, n_lim = 0, n_cls = 0;

  issue(y0 - 1, 0);
  issue(y0, 1);
  int b = 0;
  for (int L = y0 - 1; L <= y1; ++L) {
    // the waits of march_lmp_dma: row L was requested at the top of
    // iteration L - 2; newer are that iteration's 20 stores, row L + 1's
    // loads and the 20 stores of iteration L - 1, exact where both
    // iterations stored both of their rows
    if (!TH && L - 3 >= y0 && L + 1 <= y1)
      __builtin_amdgcn_s_waitcnt(sizeof(T) == 8 ? 0xCF73 : 0x8F7E);  // vmcnt(40 + kRowOps)
    else if (L + 1 <= y1)
      __builtin_amdgcn_s_waitcnt(sizeof(T) == 8 ? 0x0F7B : 0x0F76);  // vmcnt(kRowOps)
    else
      __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    static_assert(kRowOps == (sizeof(T) == 8 ? 11 : 6), "wait counts of the loop head");
    __builtin_amdgcn_sched_barrier(0);
    if (L + 2 <= y1) issue(L + 2, b == 0 ? 2 : b - 1);
    __builtin_amdgcn_sched_barrier(0);
    const unsigned char* rb = ring + b * dma_row_bytes<T>();
    const T* rowv = (const T*)rb;
    const T* hrow = (const T*)(rb + 20 * 64 * (int)sizeof(T));
    C u[4], uk[4][4], hu[4], hk[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) u[c] = (C)rowv[c * 64 + lane];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int c = 0; c < 4; ++c) uk[k][c] = (C)rowv[(4 + 4 * k + c) * 64 + lane];
    const int hbase = first ? 0 : 8;
    const int ein = first ? west1 : east0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      hu[c] = (C)hrow[(hbase + c) * kVpl + ein];
      hk[c] = (C)hrow[(hbase + 4 + c) * kVpl + ein];
    }

    C f[4], g[4], hf[4], hg[4];
    fluxes(u, K.gm1, f, g);
    fluxes(hu, K.gm1, hf, hg);
    C M[4][4], d[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        M[k][c] = maxw(k, u[c], f[c], g[c], K.w, K.r2a);
        d[k][c] = M[k][c] - uk[k][c];
      }
    C usx[4], dF[4], M2E[4], d2E[4], usy[4], dG[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const C uE = from_right_or(u[c], hu[c]);
      const C fE = from_right_or(f[c], hf[c]);
      const C u2E = from_right_or(uk[1][c], hk[c]);
      M2E[c] = maxw(1, uE, fE, fE, K.w, K.r2a);
      d2E[c] = M2E[c] - u2E;
      usx[c] = C(0.5) * (u[c] + uE) - (fE - f[c]) * K.r2k;
      dF[c] = K.ac * (d[0][c] - d2E[c]);
      usy[c] = C(0.5) * (pu[c] + u[c]) - (g[c] - pg[c]) * K.r2k;
      dG[c] = K.ac * (pd3[c] - d[3][c]);
    }
    C usw[4], dFw[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const C hd1 = maxw(0, hu[c], hf[c], hg[c], K.w, K.r2a) - hk[c];
      usw[c] = C(0.5) * (hu[c] + u[c]) - (f[c] - hf[c]) * K.r2k;
      dFw[c] = K.ac * (hd1 - d[1][c]);
    }
    int gx, gy, gw;
    const C zero = C(0);
    double thx = face_theta<LIMS>(sc, usx, dF, K.kappa, zero, zero, zero, zero, gx);
    double thy = face_theta<LIMS>(sc, usy, dG, K.kappa, zero, zero, zero, zero, gy);
    double th_edge = face_theta<LIMS>(sc, usw, dFw, K.kappa, zero, zero, zero, zero, gw);
    if (sponge) {
      if (in_sponge(sc, gi, L, nx, ny) || in_sponge(sc, gi + 1, L, nx, ny)) thx = 0.0;
      if (in_sponge(sc, gi, L - 1, nx, ny) || in_sponge(sc, gi, L, nx, ny)) thy = 0.0;
      if (in_sponge(sc, x0 - 1, L, nx, ny) || in_sponge(sc, x0, L, nx, ny)) th_edge = 0.0;
    }
    const bool row0 = L >= y0 && L < y1;
    const bool row1 = L - 1 >= y0 && L - 1 < y1;
    if (row0 && !last) {
      n_guard += gx;
      n_lim += (thx < 1.0);
    }
    if (row0) {
      n_guard += gy;
      n_lim += (thy < 1.0);
    }
    if (row0 && first) {
      n_guard += gw;
      n_lim += (th_edge < 1.0);
    }
    if (TH || (LIMS == 0 && A.theta_x)) {
      if (row0 && first) A.theta_x[(long long)L * (nx + 1) + x0] = th_edge;
      if (row0) A.theta_x[(long long)L * (nx + 1) + gi + 1] = thx;
      if ((row0 || row1) && L >= 0 && L <= ny) A.theta_y[(long long)L * nx + gi] = thy;
    }

    const C tR = (C)thx;
    const C tL = from_left_or(tR, (C)th_edge);
    const C tB = (C)thy;
    C fin[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const C o1n = M[0][c] + tR * d[0][c];
      const C hM1 = maxw(0, hu[c], hf[c], hg[c], K.w, K.r2a);
      const C hd1 = hM1 - hk[c];
      const C u1n = from_left_or(o1n, hM1 + tL * hd1);
      const C u2n = M2E[c] + tR * d2E[c];
      const C u3n = pM3[c] + tB * pd3[c];
      C s = K.alpha * u[c];
      s = s + (u1n - tL * d[1][c]);
      s = s + (u2n - tR * d[0][c]);
      s = s + (u3n - tB * d[3][c]);
      const C u4n = M[3][c] + tB * d[3][c];
      fin[c] = pP[c] + (u4n - tB * pd3[c]);
      if (row0) {
        put(out_at(4 + c, L), (T)u1n);
        put(out_at(8 + c, L), (T)u2n);
        put(out_at(12 + c, L), (T)u3n);
      }
      if (row1) {
        put(out_at(c, L - 1), (T)fin[c]);
        put(out_at(16 + c, L - 1), (T)u4n);
      }
      pP[c] = s;
    }
    if (row1) {
      const double l = cell_wavespeed((double)(T)fin[0], (double)(T)fin[1], (double)(T)fin[2],
                                      (double)(T)fin[3], sc.gamma);
      if (l < 0.0) {
        n_bad += 1;
        n_cls += bad_class((double)(T)fin[0], (double)(T)fin[1], (double)(T)fin[2], (double)(T)fin[3],
                           sc.gamma);
      } else {
        lmax = vmax(lmax, l);
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      pu[c] = u[c];
      pg[c] = g[c];
      pM3[c] = M[2][c];
      pd3[c] = d[2][c];
    }
    b = b == 2 ? 0 : b + 1;
  }

#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lmax = vmax(lmax, __shfl_xor(lmax, off, 64));
    n_bad += __shfl_xor(n_bad, off, 64);
    n_guard += __shfl_xor(n_guard, off, 64);
    n_lim += __shfl_xor(n_lim, off, 64);
  }
  unsigned n_nf, n_rho;
  reduce_classes(n_cls, n_nf, n_rho);
  if (lane == 0) publish(sl, (A.slot + 1) % 3, lmax, n_bad, n_guard, n_lim, 0, n_nf, n_rho);
}

// The step kernel: T the state's storage type, C its arithmetic type, LMP the
// bounds-limited march, WPE the waves per SIMD the registers are sized for,
// LIMS a limiter set fixed at compile time (0: read from the scheme) and TH
// whether the face factors are written (with LIMS = 0 they are written
// whenever A.theta_x is set), BND whether boundary descriptions are read
// (only with LIMS = 0), DMA the LDS-staged marches, BLK the blocked state
// layout (with DMA only).
template <class T, class C, bool LMP, int WPE, int LIMS, bool TH, bool BND, bool DMA = false, bool BLK = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void step_kernel(StepArgs A) {
  const int lane = threadIdx.x & 63;
  // uniform across the wave: lets the compiler keep work-item data in SGPRs
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  int grp = blockIdx.x;
  if (A.xcd_remap && (A.groups & 7) == 0) {
    // groups are dispatched round-robin over the 8 XCDs: give each XCD one
    // contiguous range of strips so that neighbouring strips share its L2
    const int per = A.groups >> 3;
    grp = (grp & 7) * per + (grp >> 3);
  }
  const long long total = (long long)A.groups * A.waves_per_group;
  for (long long item = (long long)grp * A.waves_per_group + wave; item < A.n_items;
       item += total) {
    int ii = 0;
    Inst in;
    if (A.n_inst == 1) {
      in = A.inst0;
    } else {
      ii = A.item_inst[item];
      in = A.insts[ii];
    }
    const long long local = item - in.item0;
    const int xs = (int)(local % in.xs);
    const int ys = (int)(local / in.xs);
    if constexpr (LMP && DMA)
      march_lmp_dma<T, C, LIMS, TH, BLK>(A, in, A.slots + ii, xs, ys, lane, wave);
    else if constexpr (LMP)
      march_lmp<T, C, LIMS, TH, BND>(A, in, A.slots + ii, xs, ys, lane);
    else if constexpr (DMA)
      march_short_dma<T, C, LIMS, TH, BLK>(A, in, A.slots + ii, xs, ys, lane, wave);
    else
      march_short<T, C, LIMS, TH, BND>(A, in, A.slots + ii, xs, ys, lane);
  }
}

// ------------------------------------------------- per-cell blending (ablation)

// Per-cell blending, the first possibility of Section 3.1 (eq.
// (naive_blending)), which the paper sets aside in favour of the face
// blending above: every distribution leaving cell U is M_k(u_U) + theta_U
// d_k(U) and the rest population is blended with the cell's own factor, so
// the moment slot takes alpha u plus, face by face (W, E, S, N), the incoming
// distribution minus theta_C times the own distribution leaving through that
// face.  theta_U of a cell is the smallest factor of its four faces, read
// from the face fields the fused step kernel wrote for the same state (tx
// [ny][nx + 1], ty [ny + 1][nx]); a ghost cell takes the factor of the cell
// it copies.  One thread per cell, neighbours read from memory: a plain
// kernel for an ablation, not a tuned one.  It also does the step's
// bookkeeping (lambda slots, time, counters) in place of the fused kernel,
// whose slot record the launcher restores.
__device__ __forceinline__ double cell_factor(const double* tx, const double* ty, int i, int j, int nx) {
  double t = tx[(long long)j * (nx + 1) + i];
  t = vmin(t, tx[(long long)j * (nx + 1) + i + 1]);
  t = vmin(t, ty[(long long)j * nx + i]);
  t = vmin(t, ty[(long long)(j + 1) * nx + i]);
  return t;
}

template <class T>
__global__ __launch_bounds__(256) void percell_kernel(StepArgs A) {
  const Scheme& sc = A.sc;
  const Inst in = A.inst0;
  const int nx = in.nx, ny = in.ny;
  Slots* sl = A.slots;
  const double lam = __longlong_as_double((long long)sl->lam[A.slot]);
  const StepConst<T, T> K = step_const<T, T>(sc, lam);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sl->lam[(A.slot + 2) % 3] = 0ull;
    sl->t[(A.slot + 1) % 3] = sl->t[A.slot] + in.dx / K.a;
    if (sc.a_mode == 1 && K.a < 2.0 * lam / (1.0 - sc.alpha)) atomicOr(&sl->cnt[CNT_BOUCHUT], 1ull);
  }
  const T* __restrict__ S = (const T*)A.src;
  T* __restrict__ D = (T*)A.dst;
  const long long P = A.plane;
  const bool lmp = sc.order == 2 && (sc.limiters & 6) != 0;
  const bool faces = sc.order == 2 && sc.limiters != 0;
  double lmax = 0.0;
  unsigned n_bad = 0, n_guard = 0, n_lim = 0, n_lmp = 0, n_cls = 0;
  const long long ncell = (long long)nx * ny;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
       c += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(c / nx), i = (int)(c % nx);
    const int iw = map_index(i - 1, nx, sc.bc_x), ie = map_index(i + 1, nx, sc.bc_x);
    const int js = map_index(j - 1, ny, sc.bc_y), jn = map_index(j + 1, ny, sc.bc_y);
    const long long oc = c, ow = (long long)j * nx + iw, oe = (long long)j * nx + ie,
                    os = (long long)js * nx + i, on = (long long)jn * nx + i;
    const double thC = cell_factor(A.theta_x, A.theta_y, i, j, nx);
    const double thW = cell_factor(A.theta_x, A.theta_y, iw, j, nx);
    const double thE = cell_factor(A.theta_x, A.theta_y, ie, j, nx);
    const double thS = cell_factor(A.theta_x, A.theta_y, i, js, nx);
    const double thN = cell_factor(A.theta_x, A.theta_y, i, jn, nx);
    // the five cells' moments and fluxes
    T u[5][4], f[5][4], g[5][4];
    const long long o5[5] = {oc, ow, oe, os, on};
#pragma unroll
    for (int q = 0; q < 5; ++q) {
#pragma unroll
      for (int k = 0; k < 4; ++k) u[q][k] = S[k * P + o5[q]];
      fluxes(u[q], K.gm1, f[q], g[q]);
    }
    T fin[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      // d_k = M_k - u_k of the upwind cells and of the cell itself
      const T MW = maxw(0, u[1][k], f[1][k], g[1][k], K.w, K.r2a);
      const T ME = maxw(1, u[2][k], f[2][k], g[2][k], K.w, K.r2a);
      const T MS = maxw(2, u[3][k], f[3][k], g[3][k], K.w, K.r2a);
      const T MN = maxw(3, u[4][k], f[4][k], g[4][k], K.w, K.r2a);
      const T dW = MW - S[(4 + k) * P + ow];
      const T dE = ME - S[(8 + k) * P + oe];
      const T dS = MS - S[(12 + k) * P + os];
      const T dN = MN - S[(16 + k) * P + on];
      const T d1 = maxw(0, u[0][k], f[0][k], g[0][k], K.w, K.r2a) - S[(4 + k) * P + oc];
      const T d2 = maxw(1, u[0][k], f[0][k], g[0][k], K.w, K.r2a) - S[(8 + k) * P + oc];
      const T d3 = maxw(2, u[0][k], f[0][k], g[0][k], K.w, K.r2a) - S[(12 + k) * P + oc];
      const T d4 = maxw(3, u[0][k], f[0][k], g[0][k], K.w, K.r2a) - S[(16 + k) * P + oc];
      const T tC = (T)thC;
      const T u1n = MW + (T)thW * dW;
      const T u2n = ME + (T)thE * dE;
      const T u3n = MS + (T)thS * dS;
      const T u4n = MN + (T)thN * dN;
      T un = K.alpha * u[0][k];
      un = un + (u1n - tC * d2);
      un = un + (u2n - tC * d1);
      un = un + (u3n - tC * d4);
      un = un + (u4n - tC * d3);
      fin[k] = un;
      put(&D[k * P + oc], un);
      put(&D[(4 + k) * P + oc], u1n);
      put(&D[(8 + k) * P + oc], u2n);
      put(&D[(12 + k) * P + oc], u3n);
      put(&D[(16 + k) * P + oc], u4n);
    }
    n_lim += (thC < 1.0);
    // face states of the cell's four faces (eq. (12)): the guard of the west
    // and south faces (counted once per face, as in the fused kernel) and the
    // eq. (29) bounds of the LMP check
    {
      T rsx[2], rsy[2];
      for (int side = 0; side < 2; ++side) {
        const int L = side == 0 ? 1 : 0, R = side == 0 ? 0 : 2;  // W|C or C|E
        T us[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) us[k] = T(0.5) * (u[L][k] + u[R][k]) - (f[R][k] - f[L][k]) * K.r2k;
        rsx[side] = us[0];
        if (side == 0 && faces) {
          const double r0 = us[0], m1 = us[1], m2 = us[2], E = us[3];
          const double g0 = m1 * m1 + m2 * m2 - 2.0 * r0 * E;
          n_guard += (!(r0 > 0.0) || !(g0 < 0.0));
        }
      }
      for (int side = 0; side < 2; ++side) {
        const int L = side == 0 ? 3 : 0, R = side == 0 ? 0 : 4;  // S|C or C|N
        T us[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) us[k] = T(0.5) * (u[L][k] + u[R][k]) - (g[R][k] - g[L][k]) * K.r2k;
        rsy[side] = us[0];
        if (side == 0 && faces) {
          const double r0 = us[0], m1 = us[1], m2 = us[2], E = us[3];
          const double g0 = m1 * m1 + m2 * m2 - 2.0 * r0 * E;
          n_guard += (!(r0 > 0.0) || !(g0 < 0.0));
        }
      }
      if (lmp) {
        T lo = u[0][0], hi = u[0][0];
        lo = vmin(lo, rsx[0]);
        hi = vmax(hi, rsx[0]);
        lo = vmin(lo, rsx[1]);
        hi = vmax(hi, rsx[1]);
        lo = vmin(lo, rsy[0]);
        hi = vmax(hi, rsy[0]);
        lo = vmin(lo, rsy[1]);
        hi = vmax(hi, rsy[1]);
        const double r = (double)fin[0], dlo = (double)lo, dhi = (double)hi;
        n_lmp += (r < dlo - kLmpTol<T> * fabs(dlo)) || (r > dhi + kLmpTol<T> * fabs(dhi));
      }
    }
    const double l = cell_wavespeed((double)fin[0], (double)fin[1], (double)fin[2], (double)fin[3], sc.gamma);
    if (l < 0.0) {
      n_bad += 1;
      n_cls += bad_class((double)fin[0], (double)fin[1], (double)fin[2], (double)fin[3], sc.gamma);
    } else {
      lmax = vmax(lmax, l);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lmax = vmax(lmax, __shfl_xor(lmax, off, 64));
    n_bad += __shfl_xor(n_bad, off, 64);
    n_guard += __shfl_xor(n_guard, off, 64);
    n_lim += __shfl_xor(n_lim, off, 64);
    n_lmp += __shfl_xor(n_lmp, off, 64);
  }
  // unpacked per thread (below 2^16 each: see the launcher) before the
  // wave reduction
  unsigned n_nf = n_cls >> 16, n_rho = n_cls & 0xffffu;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    n_nf += __shfl_xor(n_nf, off, 64);
    n_rho += __shfl_xor(n_rho, off, 64);
  }
  if ((threadIdx.x & 63) == 0) publish(sl, (A.slot + 1) % 3, lmax, n_bad, n_guard, n_lim, n_lmp, n_nf, n_rho);
}

// ---------------------------------------------------------------- init etc.

// Wavespeed maximum of a moment field (4 planes of Src values, rounded to the
// storage type T first) into slots[slot]; counts non-admissible cells.
template <class Src, class T>
__global__ __launch_bounds__(256) void lambda_kernel(const Src* __restrict__ u, long long plane,
                                                     long long n, double gamma, Slots* sl,
                                                     int slot, int blocked) {
  double lmax = 0.0;
  unsigned bad = 0, nf = 0, nr = 0;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const double r = (double)(T)u[sidx(0, c, plane, blocked)], m1 = (double)(T)u[sidx(1, c, plane, blocked)],
                 m2 = (double)(T)u[sidx(2, c, plane, blocked)], E = (double)(T)u[sidx(3, c, plane, blocked)];
    const double l = cell_wavespeed(r, m1, m2, E, gamma);
    if (l < 0.0) {
      bad += 1;
      const unsigned k = bad_class(r, m1, m2, E, gamma);
      nf += k >> 16;
      nr += k & 0xffffu;
    } else {
      lmax = vmax(lmax, l);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    lmax = vmax(lmax, __shfl_xor(lmax, off, 64));
    bad += __shfl_xor(bad, off, 64);
    nf += __shfl_xor(nf, off, 64);
    nr += __shfl_xor(nr, off, 64);
  }
  // block reduction (every thread of the block reaches the barrier), then one
  // update per block
  __shared__ double wl[4];
  __shared__ unsigned wb[4][3];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    wl[w] = lmax;
    wb[w][0] = bad;
    wb[w][1] = nf;
    wb[w][2] = nr;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    lmax = vmax(vmax(wl[0], wl[1]), vmax(wl[2], wl[3]));
    bad = wb[0][0] + wb[1][0] + wb[2][0] + wb[3][0];
    nf = wb[0][1] + wb[1][1] + wb[2][1] + wb[3][1];
    nr = wb[0][2] + wb[1][2] + wb[2][2] + wb[3][2];
    raise_lambda(&sl->lam[slot], lmax);
    if (bad) atomicAdd(&sl->cnt[CNT_BAD], (unsigned long long)bad);
    if (nf) atomicAdd(&sl->cnt[CNT_NONFINITE], (unsigned long long)nf);
    if (nr) atomicAdd(&sl->cnt[CNT_RHO], (unsigned long long)nr);
  }
}

// Error-free sum of two doubles (Knuth's TwoSum; exact without contraction):
// s + e == a + b exactly.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bp = s - a;
  e = (a - (s - bp)) + (b - bp);
}
// (hi, lo) += (bh, bl) in double-double arithmetic.
__device__ __forceinline__ void dd_add(double& hi, double& lo, double bh, double bl) {
  double s, e;
  two_sum(hi, bh, s, e);
  e += lo + bl;
  hi = s + e;
  lo = e - (hi - s);
}

// Totals of the conserved moments (rho, m1, m2, E) over n cells of the
// moment slot, accumulated in double-double: one partial (hi, lo) per
// component and block, part[block][component][2].
template <class T>
__global__ __launch_bounds__(256) void totals_kernel(const T* __restrict__ S, long long plane,
                                                     long long n, double* __restrict__ part, int blocked) {
  double hi[4] = {0.0, 0.0, 0.0, 0.0}, lo[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int k = 0; k < 4; ++k) dd_add(hi[k], lo[k], (double)S[sidx(k, c, plane, blocked)], 0.0);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double oh = __shfl_xor(hi[k], off, 64), ol = __shfl_xor(lo[k], off, 64);
      dd_add(hi[k], lo[k], oh, ol);
    }
  // every thread of the block reaches the barrier
  __shared__ double wsum[4][4][2];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      wsum[w][k][0] = hi[k];
      wsum[w][k][1] = lo[k];
    }
  __syncthreads();
  if (threadIdx.x < 4) {
    const int k = threadIdx.x;
    double h = wsum[0][k][0], l = wsum[0][k][1];
    for (int q = 1; q < 4; ++q) dd_add(h, l, wsum[q][k][0], wsum[q][k][1]);
    part[((long long)blockIdx.x * 4 + k) * 2] = h;
    part[((long long)blockIdx.x * 4 + k) * 2 + 1] = l;
  }
}

// Minima of rho and of the internal energy density rho e = E - |m|^2 / (2 rho)
// over the cells of the moment slot whose four components are finite, one
// partial pair per block (+inf where a block has no such cell).
template <class T>
__global__ __launch_bounds__(256) void minima_kernel(const T* __restrict__ S, long long plane,
                                                     long long n, double* __restrict__ part, int blocked) {
  double mr = kHuge, me = kHuge;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    const double r = (double)S[sidx(0, c, plane, blocked)], m1 = (double)S[sidx(1, c, plane, blocked)],
                 m2 = (double)S[sidx(2, c, plane, blocked)], E = (double)S[sidx(3, c, plane, blocked)];
    if (!isfinite(r) || !isfinite(m1) || !isfinite(m2) || !isfinite(E)) continue;
    mr = vmin(mr, r);
    me = vmin(me, E - 0.5 * (m1 * m1 + m2 * m2) / r);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mr = vmin(mr, __shfl_xor(mr, off, 64));
    me = vmin(me, __shfl_xor(me, off, 64));
  }
  // every thread of the block reaches the barrier
  __shared__ double wm[4][2];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    wm[w][0] = mr;
    wm[w][1] = me;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * (long long)blockIdx.x] = vmin(vmin(wm[0][0], wm[1][0]), vmin(wm[2][0], wm[3][0]));
    part[2 * (long long)blockIdx.x + 1] = vmin(vmin(wm[0][1], wm[1][1]), vmin(wm[2][1], wm[3][1]));
  }
}

// u_k^0 = M_k(u0; a^0) (Section 4 preamble), moment slot = u0.
template <class T, class C>
__global__ __launch_bounds__(256) void init_kernel(const double* __restrict__ u0, long long n,
                                                   T* __restrict__ S, long long plane, Scheme sc,
                                                   const Slots* sl, int blocked) {
  const double lam = __longlong_as_double((long long)sl->lam[0]);
  const StepConst<T, C> K = step_const<T, C>(sc, lam);
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
    C u[4], f[4], g[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) u[k] = (C)(T)u0[k * n + c];
    fluxes(u, K.gm1, f, g);
#pragma unroll
    for (int k = 0; k < 4; ++k) S[sidx(k, c, plane, blocked)] = (T)u[k];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        S[sidx(4 + 4 * q + k, c, plane, blocked)] = (T)maxw(q, u[k], f[k], g[k], K.w, K.r2a);
  }
}

template <class T>
__global__ __launch_bounds__(256) void moments_kernel(const T* __restrict__ S, long long plane,
                                                      long long n, double* __restrict__ out, int blocked) {
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k * n + c] = (double)S[sidx(k, c, plane, blocked)];
  }
}

// One instance's state (n cells, a multiple of 64, first cell at offset off
// of every plane of `plane` cells) from one layout into the other:
// to_blocked = 1 planar -> blocked, 0 blocked -> planar.
template <class T>
__global__ __launch_bounds__(256) void relayout_kernel(const T* __restrict__ src, T* __restrict__ dst, long long n,
                                                       long long plane, long long off, int to_blocked) {
  const T* s = src + off * (to_blocked ? 1 : 20);
  T* d = dst + off * (to_blocked ? 20 : 1);
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n;
       c += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int q = 0; q < 20; ++q) d[sidx(q, c, plane, to_blocked)] = s[sidx(q, c, plane, !to_blocked)];
  }
}

__global__ void fill_u32_kernel(unsigned int* p, unsigned int v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void fill_f64_kernel(double* p, double v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

#ifndef VLBM_WPE_F64
#define VLBM_WPE_F64 1
#endif
#ifndef VLBM_WPE_F64_LMP
#define VLBM_WPE_F64_LMP 1
#endif
#ifndef VLBM_WPE_F32
#define VLBM_WPE_F32 2
#endif
#ifndef VLBM_WPE_F32_LMP
#define VLBM_WPE_F32_LMP 2
#endif

int grid_for(long long n, long long cap = 8192) {
  long long g = (n + 255) / 256;
  if (g > cap) g = cap;
  if (g < 1) g = 1;
  return (int)g;
}

// Reductions: a few blocks per CU, each thread striding over many cells, so
// that few block results meet at the slot.
int grid_for_reduce(long long n) { return grid_for(n, 1024); }

}  // namespace

namespace {
// Largest wavespeed of the Dirichlet boundary states of one instance, merged
// into slot `slot` (one workgroup striding over the four sides).
__global__ __launch_bounds__(256) void bnd_lambda_kernel(StepArgs A, int slot) {
  const Inst in = A.n_inst == 1 ? A.inst0 : A.insts[blockIdx.x];
  const BndDesc bd = bnd_desc(A, A.slots + blockIdx.x);
  double lmax = 0.0;
  for (int side = 0; side < 4; ++side) {
    const uint8_t* k = bd.kind[side];
    if (!k) continue;
    const int len = side < 2 ? in.ny : in.nx;
    const double* st = bd.state[side];
    for (int r = threadIdx.x; r < len; r += blockDim.x) {
      if (k[r] != BND_DIRICHLET) continue;
      const double l = cell_wavespeed(st[r], st[(long long)len + r], st[2LL * len + r],
                                      st[3LL * len + r], A.sc.gamma);
      lmax = vmax(lmax, l);
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) lmax = vmax(lmax, __shfl_xor(lmax, off, 64));
  if ((threadIdx.x & 63) == 0 && lmax > 0.0) raise_lambda(&A.slots[blockIdx.x].lam[slot], lmax);
}
}  // namespace

// Step launch.  The benchmarked limiter sets (PP + pressure; PP + LMP +
// pressure) of the second-order scheme without sponge layers run kernels
// with the set, and whether the face factors are written, fixed at compile
// time (same results; A/B on one box: 2% faster in float64 and on the
// ensembles, 4% on the LMP runs); all other configurations run the general
// kernels, and a grid with boundary descriptions the general kernels that
// read them.
// The LDS-staged bounds-limited march needs every strip full (width a
// multiple of 64), a single instance and no boundary descriptions; it runs
// for every limiter set with density bounds (fixed at compile time for the
// LMP and RLMP sets with PP and pressure).  Its LDS (three rows per wave) is
// dynamic, above the default limit in float64.
template <class T, bool LMP, int WPE, int LIMS, bool TH, bool BLK>
static void launch_dma(const StepArgs& a, dim3 grid, dim3 block, hipStream_t s) {
  const auto k = step_kernel<T, T, LMP, WPE, LIMS, TH, false, true, BLK>;
  // the limit is a property of the function on each device: raise it on the
  // first launch on every device (a failure leaves the error for the
  // launcher's hipGetLastError, and the launch itself then fails too)
  static std::atomic<unsigned long long> raised{0};
  int dev = -1;
  const bool known = hipGetDevice(&dev) == hipSuccess && dev >= 0 && dev < 64;
  const unsigned long long bit = known ? 1ull << dev : 0ull;
  if (!known || !(raised.load(std::memory_order_acquire) & bit)) {
    if (hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, dma_lds_bytes<T>(4)) ==
            hipSuccess &&
        known)
      raised.fetch_or(bit, std::memory_order_acq_rel);
  }
  hipLaunchKernelGGL(k, grid, block, (unsigned)dma_lds_bytes<T>((int)block.x / 64), s, a);
}

static bool dma_ok(const StepArgs& a) { return a.n_inst == 1 && a.inst0.nx % 64 == 0 && !a.bnd; }

template <class T, bool LMP, int WPE>
static void launch_step_as(const StepArgs& a, int lims, dim3 grid, dim3 block, hipStream_t s) {
  constexpr int kFixed = LMP ? (1 | 2 | 8) : (1 | 8);
  constexpr int kRelaxed = 1 | 4 | 8;  // (bounds-limited sets only)
  if (a.blocked) {
    // a context's blocked state: the LDS-staged marches (every instance's
    // width is a multiple of 64 and no instance has boundary descriptions)
    if (lims == kFixed && a.theta_x)
      launch_dma<T, LMP, WPE, kFixed, true, true>(a, grid, block, s);
    else if (lims == kFixed)
      launch_dma<T, LMP, WPE, kFixed, false, true>(a, grid, block, s);
    else if constexpr (LMP) {
      if (lims == kRelaxed && a.theta_x)
        launch_dma<T, LMP, WPE, kRelaxed, true, true>(a, grid, block, s);
      else if (lims == kRelaxed)
        launch_dma<T, LMP, WPE, kRelaxed, false, true>(a, grid, block, s);
      else
        launch_dma<T, LMP, WPE, 0, false, true>(a, grid, block, s);
    } else {
      launch_dma<T, LMP, WPE, 0, false, true>(a, grid, block, s);
    }
    return;
  }
  if constexpr (LMP) {
    if (dma_ok(a)) {
      // PP + LMP + pressure and PP + RLMP + pressure with the set fixed;
      // every other set, and sponge layers, with the set read at run time
      if (lims == kFixed && a.theta_x)
        launch_dma<T, LMP, WPE, kFixed, true, false>(a, grid, block, s);
      else if (lims == kFixed)
        launch_dma<T, LMP, WPE, kFixed, false, false>(a, grid, block, s);
      else if (lims == kRelaxed && a.theta_x)
        launch_dma<T, LMP, WPE, kRelaxed, true, false>(a, grid, block, s);
      else if (lims == kRelaxed)
        launch_dma<T, LMP, WPE, kRelaxed, false, false>(a, grid, block, s);
      else
        launch_dma<T, LMP, WPE, 0, false, false>(a, grid, block, s);
      return;
    }
  }
  if (a.bnd)
    hipLaunchKernelGGL((step_kernel<T, T, LMP, WPE, 0, false, true>), grid, block, 0, s, a);
  else if (lims == kFixed && a.theta_x)
    hipLaunchKernelGGL((step_kernel<T, T, LMP, WPE, kFixed, true, false>), grid, block, 0, s, a);
  else if (lims == kFixed)
    hipLaunchKernelGGL((step_kernel<T, T, LMP, WPE, kFixed, false, false>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((step_kernel<T, T, LMP, WPE, 0, false, false>), grid, block, 0, s, a);
}

hipError_t launch_bnd_lambda(const StepArgs& a, int slot, hipStream_t s) {
  hipLaunchKernelGGL(bnd_lambda_kernel, dim3((unsigned)a.n_inst), dim3(256), 0, s, a, slot);
  return hipGetLastError();
}

hipError_t launch_step(const StepArgs& a, int precision, hipStream_t s) {
  if (a.blocked && (a.bnd || (a.n_inst == 1 && a.inst0.nx % 64 != 0))) return hipErrorInvalidValue;
  const bool lmp = (a.sc.limiters & 6u) != 0 && a.sc.order == 2;
  const int lims = (a.sc.order == 2 && a.sc.sponge == 0 && a.sc.eps <= 1e-12) ? a.sc.limiters : 0;
  const dim3 block(64 * a.waves_per_group);
  const dim3 grid(a.groups);
  if (precision == 0) {
    if (lmp)
      launch_step_as<double, true, VLBM_WPE_F64_LMP>(a, lims, grid, block, s);
    else
      launch_step_as<double, false, VLBM_WPE_F64>(a, lims, grid, block, s);
  } else {
    if (lmp)
      launch_step_as<float, true, VLBM_WPE_F32_LMP>(a, lims, grid, block, s);
    else
      launch_step_as<float, false, VLBM_WPE_F32>(a, lims, grid, block, s);
  }
  return hipGetLastError();
}

hipError_t launch_init(const Scheme& sc, const Inst* insts, int n_inst, const Inst* /*dev*/,
                       long long plane, const double* u0, void* S, Slots* slots, int precision,
                       int blocked, hipStream_t s) {
  long long u0_off = 0;
  for (int i = 0; i < n_inst; ++i) {
    const Inst& in = insts[i];
    const long long n = (long long)in.nx * in.ny;
    const double* u = u0 + u0_off;
    if (precision == 0)
      hipLaunchKernelGGL((lambda_kernel<double, double>), dim3(grid_for_reduce(n)), dim3(256), 0, s, u,
                         n, n, sc.gamma, slots + i, 0, 0);
    else
      hipLaunchKernelGGL((lambda_kernel<double, float>), dim3(grid_for_reduce(n)), dim3(256), 0, s, u, n,
                         n, sc.gamma, slots + i, 0, 0);
    if (precision == 0)
      hipLaunchKernelGGL((init_kernel<double, double>), dim3(grid_for(n)), dim3(256), 0, s, u, n,
                         (double*)S + in.off * (blocked ? 20 : 1), plane, sc, (const Slots*)(slots + i), blocked);
    else
      hipLaunchKernelGGL((init_kernel<float, float>), dim3(grid_for(n)), dim3(256), 0, s, u, n,
                         (float*)S + in.off * (blocked ? 20 : 1), plane, sc, (const Slots*)(slots + i), blocked);
    u0_off += 4 * n;
  }
  return hipGetLastError();
}

hipError_t launch_lambda_state(const Scheme& sc, const Inst* insts, int n_inst, long long plane,
                               const void* S, Slots* slots, int slot, int precision, int blocked,
                               hipStream_t s) {
  for (int i = 0; i < n_inst; ++i) {
    const Inst& in = insts[i];
    const long long n = (long long)in.nx * in.ny;
    if (precision == 0)
      hipLaunchKernelGGL((lambda_kernel<double, double>), dim3(grid_for_reduce(n)), dim3(256), 0, s,
                         (const double*)S + in.off * (blocked ? 20 : 1), plane, n, sc.gamma, slots + i, slot, blocked);
    else
      hipLaunchKernelGGL((lambda_kernel<float, float>), dim3(grid_for_reduce(n)), dim3(256), 0, s,
                         (const float*)S + in.off * (blocked ? 20 : 1), plane, n, sc.gamma, slots + i, slot, blocked);
  }
  return hipGetLastError();
}

hipError_t launch_moments(const Inst& in, long long plane, const void* S, double* out,
                          int precision, int blocked, hipStream_t s) {
  const long long n = (long long)in.nx * in.ny;
  if (precision == 0)
    hipLaunchKernelGGL((moments_kernel<double>), dim3(grid_for(n)), dim3(256), 0, s,
                       (const double*)S + in.off * (blocked ? 20 : 1), plane, n, out, blocked);
  else
    hipLaunchKernelGGL((moments_kernel<float>), dim3(grid_for(n)), dim3(256), 0, s,
                       (const float*)S + in.off * (blocked ? 20 : 1), plane, n, out, blocked);
  return hipGetLastError();
}

hipError_t launch_relayout(const Inst* insts, int n_inst, long long plane, const void* src, void* dst,
                           int precision, int to_blocked, hipStream_t s) {
  for (int i = 0; i < n_inst; ++i) {
    const long long n = (long long)insts[i].nx * insts[i].ny;
    if (precision == 0)
      hipLaunchKernelGGL((relayout_kernel<double>), dim3(grid_for(n)), dim3(256), 0, s, (const double*)src,
                         (double*)dst, n, plane, insts[i].off, to_blocked);
    else
      hipLaunchKernelGGL((relayout_kernel<float>), dim3(grid_for(n)), dim3(256), 0, s, (const float*)src,
                         (float*)dst, n, plane, insts[i].off, to_blocked);
  }
  return hipGetLastError();
}

hipError_t launch_totals(const Inst& in, long long plane, const void* S, double* part,
                         int blocks, int precision, int blocked, hipStream_t s) {
  const long long n = (long long)in.nx * in.ny;
  if (precision == 0)
    hipLaunchKernelGGL((totals_kernel<double>), dim3(blocks), dim3(256), 0, s,
                       (const double*)S + in.off * (blocked ? 20 : 1), plane, n, part, blocked);
  else
    hipLaunchKernelGGL((totals_kernel<float>), dim3(blocks), dim3(256), 0, s,
                       (const float*)S + in.off * (blocked ? 20 : 1), plane, n, part, blocked);
  return hipGetLastError();
}

hipError_t launch_percell(const StepArgs& a, int precision, hipStream_t s) {
  const long long n = (long long)a.inst0.nx * a.inst0.ny;
  // 8192 blocks of 256 threads (or one thread per cell): a thread visits at
  // most 2^32 / 2^21 = 2048 cells, so its packed 16-bit class counts are exact
  const int blocks = grid_for(n);
  if (precision == 0)
    hipLaunchKernelGGL((percell_kernel<double>), dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((percell_kernel<float>), dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_minima(const Inst& in, long long plane, const void* S, double* part,
                         int blocks, int precision, int blocked, hipStream_t s) {
  const long long n = (long long)in.nx * in.ny;
  if (precision == 0)
    hipLaunchKernelGGL((minima_kernel<double>), dim3(blocks), dim3(256), 0, s,
                       (const double*)S + in.off * (blocked ? 20 : 1), plane, n, part, blocked);
  else
    hipLaunchKernelGGL((minima_kernel<float>), dim3(blocks), dim3(256), 0, s,
                       (const float*)S + in.off * (blocked ? 20 : 1), plane, n, part, blocked);
  return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned int* p, unsigned int v, long long n, hipStream_t s) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, double v, long long n, hipStream_t s) {
  hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace vlbm
