// Host side of the C ABI declared in include/vlbm.h.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "vlbm.h"
#include "vlbm_internal.h"

using vlbm::Inst;
using vlbm::Scheme;
using vlbm::Slots;

namespace {

constexpr int kMinStripRows = 4;  // bounds the work-item table in the workspace
constexpr int kMaxGridPerCu = 32;
constexpr int kTotalsBlocks = 1024;  // workgroups of the totals reduction
constexpr int kMaxStripRows = 4096;
constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

thread_local std::string g_init_error;

// Strips are 64 columns wide and aligned (every lane produces its column;
// the edge lanes read the halo columns themselves).
long long strips_x(int nx) { return (nx + 63) / 64; }

long long strips_y(int ny, int h) { return (ny + h - 1) / h; }

// Grid sizes the kernels address: cells of one instance are indexed with
// 32-bit row * nx + column offsets, the edge lanes step two columns past a
// strip, and a float32 row's size in bytes is a 32-bit buffer extent, so each
// side stays below 2^30 and an instance below 2^32 cells.
const char* check_shape(int32_t nx, int32_t ny) {
  if (nx < 1 || ny < 1) return "nx and ny must be >= 1";
  if (nx >= (1 << 30) || ny >= (1 << 30)) return "nx and ny must be < 2^30";
  if ((long long)nx * ny > 0xFFFFFFFFll) return "an instance must have fewer than 2^32 cells";
  return nullptr;
}

const char* check_params(const lbm_params* p) {
  if (!p) return "params is NULL";
  if (const char* m = check_shape(p->nx, p->ny)) return m;
  if (!(p->dx > 0.0) || !isfinite(p->dx)) return "dx must be > 0";
  if (!(p->gamma > 1.0)) return "gamma must be > 1";
  if (!(p->alpha >= 0.0 && p->alpha < 1.0)) return "alpha must lie in [0, 1)";
  if (!p->unsafe && p->alpha < 0.5) return "alpha < 1/2 breaks the convex decomposition (set unsafe)";
  if (p->order != 1 && p->order != 2) return "order must be 1 or 2";
  if (p->limiters & ~15u) return "unknown limiter bits";
  if (p->a_mode != LBM_A_DYNAMIC && p->a_mode != LBM_A_FIXED) return "unknown a_mode";
  if (p->a_mode == LBM_A_DYNAMIC) {
    if (!(p->a_beta > 0.0)) return "a_beta must be > 0";
    if (!p->unsafe && p->a_beta < 1.0) return "a_beta < 1 violates the Bouchut condition (set unsafe)";
  } else if (!(p->a_fixed > 0.0) || !isfinite(p->a_fixed)) {
    return "a_fixed must be > 0";
  }
  if (p->bc_x < 0 || p->bc_x > 1 || p->bc_y < 0 || p->bc_y > 1) return "unknown boundary condition";
  if (p->sponge < 0) return "sponge must be >= 0";
  if (p->precision != LBM_FP64 && p->precision != LBM_FP32_STATE) return "unknown precision";
  if (p->blend != LBM_BLEND_FACE && p->blend != LBM_BLEND_CELL) return "unknown blend";
  if (!(p->eps >= 0.0)) return "eps must be >= 0";
  if (!(p->rlmp_lo > 0.0 && p->rlmp_lo <= 1.0 && p->rlmp_hi >= 1.0)) return "bad RLMP factors";
  return nullptr;
}

Scheme make_scheme(const lbm_params* p) {
  Scheme s;
  s.gamma = p->gamma;
  s.alpha = p->alpha;
  s.beta = p->a_beta;
  s.a_fixed = p->a_fixed;
  s.eps = p->eps;
  s.rlmp_lo = p->rlmp_lo;
  s.rlmp_hi = p->rlmp_hi;
  s.a_mode = p->a_mode;
  s.order = p->order;
  s.limiters = (int)p->limiters;
  s.bc_x = p->bc_x;
  s.bc_y = p->bc_y;
  s.sponge = p->sponge;
  return s;
}

struct Layout {
  size_t slots, slots_save, red, insts, items, bndt, bufA, bufB, theta, total;
};

Layout layout(const lbm_params* p, int n, const int* nx, const int* ny) {
  const size_t elem = p->precision == LBM_FP64 ? 8 : 4;
  long long cells = 0, items = 0;
  for (int i = 0; i < n; ++i) {
    cells += (long long)nx[i] * ny[i];
    items += strips_x(nx[i]) * strips_y(ny[i], kMinStripRows);
  }
  Layout L;
  size_t o = 0;
  L.slots = o;
  o = align_up(o + sizeof(Slots) * (size_t)n);
  L.slots_save = o;  // the adjoint entry points park the slots here
  o = align_up(o + sizeof(Slots));
  L.red = o;  // block partials of lbm_totals
  o = align_up(o + sizeof(double) * 8 * (size_t)kTotalsBlocks);
  L.insts = o;
  o = align_up(o + sizeof(Inst) * (size_t)n);
  L.items = o;
  o = align_up(o + sizeof(int) * (size_t)(n > 1 ? items : 0));
  L.bndt = o;  // boundary descriptions of an ensemble's instances
  o = align_up(o + sizeof(vlbm::BndDesc) * (size_t)(n > 1 ? n : 0));
  L.bufA = o;
  o = align_up(o + (size_t)20 * cells * elem);
  L.bufB = o;
  o = align_up(o + (size_t)20 * cells * elem);
  L.theta = o;
  if (n == 1 && (p->precision == LBM_FP64 || p->blend == LBM_BLEND_CELL))  // face factors: adjoint, per-cell blending
    o = align_up(o + sizeof(double) * ((size_t)(nx[0] + 1) * ny[0] + (size_t)nx[0] * (ny[0] + 1)));
  L.total = o;
  return L;
}

}  // namespace

namespace vlbm {
const char* host_check_params(const lbm_params* p) { return check_params(p); }
Scheme host_make_scheme(const lbm_params* p) { return make_scheme(p); }
void host_set_error(const char* m) { g_init_error = m; }
}  // namespace vlbm

struct lbm_ctx {
  lbm_params p;
  Scheme sc;
  int n_inst = 0;
  std::vector<Inst> insts;
  std::vector<int> item_inst;
  long long plane = 0;
  long long n_items = 0;
  char* ws = nullptr;
  Layout lay;
  Slots* slots = nullptr;
  Inst* insts_dev = nullptr;
  int* items_dev = nullptr;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;  // private stream used only to record graphs
  long long step = 0;
  int strip_rows = 64;
  int strip_mode = 0;  // 0: every instance strip_rows; 1: matched to the instance's height
  int waves = 4;
  int xcd = 1;
  int grid_per_cu = 0;  // 0: one wave per strip; k > 0: persistent grid of k groups per CU
  int n_cu = 256;       // compute units of the context's device
  bool detached = false;  // the current state lives in a caller buffer (lbm_step_between)
  // the context's own state buffers hold the blocked layout (every width a
  // multiple of 64, face blending, no boundary descriptions):
  // a strip row of the state is one contiguous range for the LDS-staged
  // marches.  Caller buffers (lbm_get_state, lbm_set_state,
  // lbm_step_between, the adjoint) are planar; the library converts.
  int blocked = 0;
  // boundary descriptions per instance (caller-owned device arrays; copied
  // to the workspace table for ensembles); per instance and side: any
  // Dirichlet cell
  std::vector<vlbm::BndDesc> bnd;
  std::vector<std::array<bool, 4>> side_dirichlet;
  bool has_bnd = false, has_dirichlet = false;
  std::string err;
  std::map<std::tuple<int, int, int>, hipGraphExec_t> graphs;

  void* cur() const { return ws + ((step & 1) ? lay.bufB : lay.bufA); }
  void* other() const { return ws + ((step & 1) ? lay.bufA : lay.bufB); }
  size_t elem() const { return p.precision == LBM_FP64 ? 8 : 4; }
};

namespace {

lbm_status fail(lbm_ctx* c, lbm_status s, const std::string& m) {
  if (c)
    c->err = m;
  else
    g_init_error = m;
  return s;
}

lbm_status hip_fail(lbm_ctx* c, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(c, LBM_EDEVICE, m);
}

// Rows per strip of an instance of ny rows.  Mode 0: the context's strip
// height.  Mode 1 (ensembles of uneven sizes): the tallest power of two that
// neither exceeds the strip height nor a quarter of the instance's rows (at
// least kMinStripRows), so that small instances are cut into more, shorter
// strips while large ones keep tall strips and few re-read halo rows.
int inst_strip_rows(const lbm_ctx* c, int ny) {
  if (c->strip_mode == 0) return c->strip_rows;
  int h = kMinStripRows;
  while (h * 2 <= c->strip_rows && h * 2 <= ny / 4) h *= 2;
  return h;
}

// After lbm_step_between the context's own buffer no longer holds its
// current state: calls that read it fail until lbm_set_state.
lbm_status require_attached(lbm_ctx* c) {
  if (c->detached)
    return fail(c, LBM_EINVAL, "the current state is in a caller buffer (lbm_step_between); call lbm_set_state first");
  return LBM_OK;
}

// Rebuild the strip tables after a change of strip height.  Each instance's
// strips are consecutive work items; in mode 1 the instances with the tallest
// strips (and, among equal heights, the most rows) come first, so that the
// longest waves are dispatched first and the short ones fill the end of the
// launch.
void build_items(lbm_ctx* c) {
  std::vector<int> order(c->n_inst);
  for (int i = 0; i < c->n_inst; ++i) {
    order[i] = i;
    Inst& in = c->insts[i];
    in.strip_h = inst_strip_rows(c, in.ny);
    in.xs = (int)strips_x(in.nx);
    in.ys = (int)strips_y(in.ny, in.strip_h);
  }
  if (c->strip_mode == 1)
    std::stable_sort(order.begin(), order.end(), [c](int a, int b) {
      const Inst &x = c->insts[a], &y = c->insts[b];
      if (x.strip_h != y.strip_h) return x.strip_h > y.strip_h;
      return x.ny > y.ny;
    });
  c->n_items = 0;
  c->item_inst.clear();
  for (int i : order) {
    Inst& in = c->insts[i];
    in.item0 = c->n_items;
    const long long k = (long long)in.xs * in.ys;
    if (c->n_inst > 1)
      for (long long q = 0; q < k; ++q) c->item_inst.push_back(i);
    c->n_items += k;
  }
}

// Default strip height: the tallest of 64, 32, 16, 8, 4 rows that still
// yields one full round of strips (one wave each) over the chip's 1024 SIMDs
// at the step kernel's occupancy (1 wave per SIMD in float64, 2 with the
// float32 state), so that small grids are cut into enough waves while large
// ones keep the re-read halo rows per strip few.  lbm_autotune refines it.
int default_strip_rows(const lbm_ctx* c) {
  const long long want = c->p.precision == LBM_FP64 ? 1024 : 2048;
  int rows = 64;
  for (; rows > kMinStripRows; rows /= 2) {
    long long items = 0;
    for (const Inst& in : c->insts) items += strips_x(in.nx) * strips_y(in.ny, rows);
    if (items >= want) break;
  }
  return rows;
}

lbm_status upload_tables(lbm_ctx* c) {
  if (c->n_inst == 1) return LBM_OK;
  hipError_t e = hipMemcpyAsync(c->insts_dev, c->insts.data(), sizeof(Inst) * c->n_inst,
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->items_dev, c->item_inst.data(), sizeof(int) * c->item_inst.size(),
                       hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "uploading strip tables");
  return LBM_OK;
}

// New strip tables for the current strip height and mode; captured graphs,
// which hold the old launch, are dropped.
lbm_status rebuild_launch(lbm_ctx* c) {
  build_items(c);
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  return upload_tables(c);
}

// Workgroups of a step launch.  By default one wave per strip, for single
// instances and ensembles alike; with grid_per_cu = k > 0 a persistent grid
// of k workgroups per compute unit whose waves stride over the strips (the
// kernel loops over its work items either way).  On the 8192^2 blast and the
// 256-instance ensemble the persistent grid measured 1-4% slower; the
// autotuner times both.
int compute_groups(const lbm_ctx* c) {
  long long g = (c->n_items + c->waves - 1) / c->waves;
  if (c->grid_per_cu > 0) g = std::min(g, (long long)c->grid_per_cu * c->n_cu);
  if (c->xcd) g = (g + 7) / 8 * 8;
  return (int)g;
}

vlbm::StepArgs make_args(const lbm_ctx* c, const void* src, void* dst, int slot) {
  vlbm::StepArgs a;
  memset(&a, 0, sizeof(a));
  a.src = src;
  a.dst = dst;
  a.plane = c->plane;
  a.slots = c->slots;
  a.insts = c->insts_dev;
  a.item_inst = c->n_inst > 1 ? c->items_dev : nullptr;
  a.inst0 = c->insts[0];
  a.n_items = c->n_items;
  a.n_inst = c->n_inst;
  a.slot = slot;
  a.waves_per_group = c->waves;
  a.xcd_remap = c->xcd;
  a.groups = compute_groups(c);
  a.sc = c->sc;
  if (c->n_inst > 1)
    a.bnd_table = (const vlbm::BndDesc*)(c->ws + c->lay.bndt);
  else if (!c->bnd.empty())
    a.bnd1 = c->bnd[0];
  a.bnd = c->has_bnd ? 1 : 0;
  // a step of the context's own state, from its current buffer to the other
  a.blocked = (c->blocked && src == c->cur() && dst == c->other()) ? 1 : 0;
  return a;
}

// A step with Dirichlet boundary cells first raises lambda^n by their states
// (Bouchut's condition covers every state the stencil reads).  With the
// per-cell blending the fused kernel only supplies the face factors (into
// the caller's face buffers, else the workspace's): its slot record is parked
// around it and the per-cell kernel writes the state and does the step's
// bookkeeping.
hipError_t launch_step_with_bnd(const lbm_ctx* c, const vlbm::StepArgs& a) {
  if (c->has_dirichlet) {
    hipError_t e = vlbm::launch_bnd_lambda(a, a.slot, c->stream);
    if (e != hipSuccess) return e;
  }
  if (c->p.blend != LBM_BLEND_CELL) return vlbm::launch_step(a, c->p.precision, c->stream);
  vlbm::StepArgs f = a;
  if (!f.theta_x) {
    f.theta_x = (double*)(c->ws + c->lay.theta);
    f.theta_y = f.theta_x + (size_t)(c->insts[0].nx + 1) * c->insts[0].ny;
  }
  Slots* save = (Slots*)(c->ws + c->lay.slots_save);
  hipError_t e = hipMemcpyAsync(save, c->slots, sizeof(Slots), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = vlbm::launch_step(f, c->p.precision, c->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(c->slots, save, sizeof(Slots), hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess) e = vlbm::launch_percell(f, c->p.precision, c->stream);
  return e;
}

lbm_status launch_one(lbm_ctx* c) {
  if (lbm_status st = require_attached(c)) return st;
  vlbm::StepArgs a = make_args(c, c->cur(), c->other(), (int)(c->step % 3));
  hipError_t e = launch_step_with_bnd(c, a);
  if (e != hipSuccess) return hip_fail(c, e, "step launch");
  c->step += 1;
  return LBM_OK;
}

lbm_status read_slots(lbm_ctx* c, std::vector<Slots>& h) {
  h.resize(c->n_inst);
  hipError_t e = hipMemcpyAsync(h.data(), c->slots, sizeof(Slots) * c->n_inst,
                                hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "reading device slots");
  return LBM_OK;
}

lbm_status write_slots(lbm_ctx* c, const std::vector<Slots>& h) {
  hipError_t e = hipMemcpyAsync(c->slots, h.data(), sizeof(Slots) * c->n_inst,
                                hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "writing device slots");
  return LBM_OK;
}

double host_kinetic_speed(const lbm_ctx* c, double lam) {
  if (c->p.a_mode == LBM_A_FIXED) return c->p.a_fixed;
  return 2.0 * c->p.a_beta * lam / (1.0 - c->p.alpha);
}

double bits_to_double(unsigned long long b) {
  double d;
  memcpy(&d, &b, sizeof(d));
  return d;
}

lbm_status common_init(const lbm_params* p, int n, const int32_t* nx, const int32_t* ny,
                       const double* dx, const double* u0, void* ws, void* stream,
                       lbm_ctx** out) {
  if (!out) return fail(nullptr, LBM_EINVAL, "out is NULL");
  *out = nullptr;
  if (const char* m = check_params(p)) return fail(nullptr, LBM_EINVAL, m);
  if (n < 1 || !nx || !ny) return fail(nullptr, LBM_EINVAL, "need at least one instance");
  for (int i = 0; i < n; ++i)
    if (const char* m = check_shape(nx[i], ny[i])) return fail(nullptr, LBM_EINVAL, m);
  if (!u0 || !ws) return fail(nullptr, LBM_EINVAL, "u0 and workspace must be device pointers");
  if (((uintptr_t)ws) % kAlign) return fail(nullptr, LBM_EINVAL, "workspace must be 256-byte aligned");
  if (p->sponge > 0 && n > 1) return fail(nullptr, LBM_ENOTSUP, "sponge layers are single-instance only");
  if (p->blend == LBM_BLEND_CELL && n > 1)
    return fail(nullptr, LBM_ENOTSUP, "the per-cell blending is single-instance only");

  lbm_ctx* c = new lbm_ctx();
  c->p = *p;
  c->sc = make_scheme(p);
  c->n_inst = n;
  c->blocked = p->blend == LBM_BLEND_FACE ? 1 : 0;
  for (int i = 0; i < n; ++i) c->blocked &= nx[i] % 64 == 0 ? 1 : 0;
  c->stream = (hipStream_t)stream;
  c->lay = layout(p, n, nx, ny);
  c->ws = (char*)ws;
  c->slots = (Slots*)(c->ws + c->lay.slots);
  c->insts_dev = (Inst*)(c->ws + c->lay.insts);
  c->items_dev = (int*)(c->ws + c->lay.items);
  c->insts.resize(n);
  long long off = 0;
  for (int i = 0; i < n; ++i) {
    Inst& in = c->insts[i];
    in.off = off;
    in.nx = nx[i];
    in.ny = ny[i];
    in.dx = dx ? dx[i] : (n == 1 ? p->dx : 1.0 / nx[i]);
    if (!(in.dx > 0.0)) {
      delete c;
      return fail(nullptr, LBM_EINVAL, "dx must be > 0");
    }
    off += (long long)nx[i] * ny[i];
  }
  c->plane = off;
  {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
      c->n_cu = cus;
  }
  c->strip_rows = default_strip_rows(c);
  build_items(c);
  lbm_status st = upload_tables(c);
  if (st != LBM_OK) {
    g_init_error = c->err;
    delete c;
    return st;
  }
  hipError_t e = vlbm::launch_fill_u32((unsigned int*)c->slots, 0u,
                                       (long long)(sizeof(Slots) * n / 4), c->stream);
  if (e == hipSuccess)
    e = vlbm::launch_init(c->sc, c->insts.data(), n, c->insts_dev, c->plane, u0, c->cur(),
                          c->slots, p->precision, c->blocked, c->stream);
  if (e != hipSuccess) {
    std::string m = std::string("init launch: ") + hipGetErrorString(e);
    delete c;
    return fail(nullptr, LBM_EDEVICE, m);
  }
  std::vector<Slots> h;
  st = read_slots(c, h);
  if (st != LBM_OK) {
    g_init_error = c->err;
    delete c;
    return st;
  }
  for (int i = 0; i < n; ++i) {
    if (h[i].cnt[vlbm::CNT_BAD]) {
      const bool nf = h[i].cnt[vlbm::CNT_NONFINITE] != 0;
      char buf[200];
      snprintf(buf, sizeof(buf), "instance %d: %llu cells of u0 are not admissible (%llu non-finite, "
               "%llu with rho <= 0, the others with p <= 0)", i, h[i].cnt[vlbm::CNT_BAD],
               h[i].cnt[vlbm::CNT_NONFINITE], h[i].cnt[vlbm::CNT_RHO]);
      delete c;
      return fail(nullptr, nf ? LBM_ENONFINITE : LBM_EPOSITIVITY, buf);
    }
  }
  *out = c;
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_params* p) {
  if (check_params(p)) return 0;
  return layout(p, 1, &p->nx, &p->ny).total;
}

size_t lbm_batch_workspace_bytes(const lbm_params* p, int32_t n, const int32_t* nx,
                                 const int32_t* ny) {
  if (check_params(p) || n < 1 || !nx || !ny) return 0;
  for (int i = 0; i < n; ++i)
    if (check_shape(nx[i], ny[i])) return 0;
  return layout(p, n, nx, ny).total;
}

lbm_status lbm_init(const lbm_params* p, const double* u0_dev, void* workspace_dev, void* stream,
                    lbm_ctx** out) {
  if (!p) return fail(nullptr, LBM_EINVAL, "params is NULL");
  return common_init(p, 1, &p->nx, &p->ny, nullptr, u0_dev, workspace_dev, stream, out);
}

lbm_status lbm_init_batch(const lbm_params* p, int32_t n, const int32_t* nx, const int32_t* ny,
                          const double* dx_host, const double* u0_packed_dev, void* workspace_dev,
                          void* stream, lbm_ctx** out) {
  return common_init(p, n, nx, ny, dx_host, u0_packed_dev, workspace_dev, stream, out);
}

lbm_status lbm_step(lbm_ctx* c, int32_t nsteps) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (nsteps < 0) return fail(c, LBM_EINVAL, "nsteps must be >= 0");
  for (int32_t k = 0; k < nsteps; ++k) {
    lbm_status s = launch_one(c);
    if (s != LBM_OK) return s;
  }
  return LBM_OK;
}

}  // extern "C"

namespace {
// A graph holds at most kGraphChunk launches; longer runs replay it.  The
// chunk is a multiple of 6, the period of the (lambda slot, buffer) phase, so
// one graph serves every chunk of a run.  At most kMaxGraphs graphs are kept.
constexpr int32_t kGraphChunk = 1020;
constexpr size_t kMaxGraphs = 32;

lbm_status replay_graph(lbm_ctx* c, int32_t nsteps) {
  const auto key = std::make_tuple((int)nsteps, (int)(c->step % 3), (int)(c->step & 1));
  auto it = c->graphs.find(key);
  if (it == c->graphs.end()) {
    if (c->graphs.size() >= kMaxGraphs) {
      for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
      c->graphs.clear();
    }
    // record on a private stream (the legacy default stream cannot be
    // captured); the graph is then launched on the context's stream
    hipError_t e = hipSuccess;
    if (!c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamCreateWithFlags");
    e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamBeginCapture");
    const long long step0 = c->step;
    hipStream_t own = c->stream;
    c->stream = c->cap_stream;
    lbm_status st = LBM_OK;
    for (int32_t k = 0; k < nsteps && st == LBM_OK; ++k) st = launch_one(c);
    c->stream = own;
    c->step = step0;
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(c->cap_stream, &g);
    if (st != LBM_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
    it = c->graphs.emplace(key, x).first;
  }
  hipError_t e = hipGraphLaunch(it->second, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "hipGraphLaunch");
  c->step += nsteps;
  return LBM_OK;
}
}  // namespace

extern "C" {

lbm_status lbm_step_graph(lbm_ctx* c, int32_t nsteps) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (nsteps < 0) return fail(c, LBM_EINVAL, "nsteps must be >= 0");
  // a graph captured before lbm_step_between would step the context's own,
  // stale buffers
  if (lbm_status st = require_attached(c)) return st;
  while (nsteps > 0) {
    const int32_t k = nsteps > kGraphChunk ? kGraphChunk : nsteps;
    const lbm_status st = replay_graph(c, k);
    if (st != LBM_OK) return st;
    nsteps -= k;
  }
  return LBM_OK;
}

lbm_status lbm_step_theta(lbm_ctx* c, double* tx, double* ty) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (c->n_inst != 1) return fail(c, LBM_ENOTSUP, "face output is single-instance only");
  if (!tx || !ty) return fail(c, LBM_EINVAL, "theta buffers must be device pointers");
  if (lbm_status st = require_attached(c)) return st;
  vlbm::StepArgs a = make_args(c, c->cur(), c->other(), (int)(c->step % 3));
  a.theta_x = tx;
  a.theta_y = ty;
  hipError_t e = launch_step_with_bnd(c, a);
  if (e != hipSuccess) return hip_fail(c, e, "step launch");
  c->step += 1;
  return LBM_OK;
}

lbm_status lbm_moments(lbm_ctx* c, int32_t inst, double* out) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (inst < 0 || inst >= c->n_inst) return fail(c, LBM_EINVAL, "instance index out of range");
  if (!out) return fail(c, LBM_EINVAL, "output must be a device pointer");
  if (lbm_status st0 = require_attached(c)) return st0;
  hipError_t e = vlbm::launch_moments(c->insts[inst], c->plane, c->cur(), out, c->p.precision, c->blocked,
                                      c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "moments launch");
  std::vector<Slots> h;
  lbm_status st = read_slots(c, h);
  if (st != LBM_OK) return st;
  lbm_status res = LBM_OK;
  unsigned long long bad = 0, nonfinite = 0, guard = 0, bouchut = 0;
  for (int i = 0; i < c->n_inst; ++i) {
    bad += h[i].cnt[vlbm::CNT_BAD];
    nonfinite += h[i].cnt[vlbm::CNT_NONFINITE];
    guard += h[i].cnt[vlbm::CNT_GUARD];
    bouchut |= h[i].cnt[vlbm::CNT_BOUCHUT];
  }
  char buf[160];
  if (nonfinite) {
    snprintf(buf, sizeof(buf), "%llu cells with non-finite values were produced (%llu non-admissible in all)",
             nonfinite, bad);
    res = fail(c, LBM_ENONFINITE, buf);
  } else if (bad) {
    snprintf(buf, sizeof(buf), "%llu non-admissible cells were produced", bad);
    res = fail(c, LBM_EPOSITIVITY, buf);
  } else if (guard) {
    snprintf(buf, sizeof(buf), "%llu face states left the admissible set", guard);
    res = fail(c, LBM_EGUARD, buf);
  } else if (bouchut) {
    res = fail(c, LBM_EBOUCHUT, "the fixed kinetic speed fell below the Bouchut bound");
  }
  // every counter starts again from zero
  bool any = false;
  for (auto& s : h)
    for (int k = 0; k < vlbm::CNT_N; ++k) {
      any |= s.cnt[k] != 0;
      s.cnt[k] = 0;
    }
  if (any) {
    st = write_slots(c, h);
    if (st != LBM_OK) return st;
  }
  return res;
}

lbm_status lbm_diagnostics(lbm_ctx* c, int32_t inst, lbm_diag* d) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (inst < 0 || inst >= c->n_inst || !d) return fail(c, LBM_EINVAL, "bad instance or output");
  // minima of rho and rho e of the current state (block partials in the
  // workspace's reduction area, combined here); a detached context's state
  // is in a caller buffer, so its minima are not available
  const Inst& in = c->insts[inst];
  const long long n = (long long)in.nx * in.ny;
  const int blocks = (int)std::min<long long>((n + 255) / 256, kTotalsBlocks);
  std::vector<double> part;
  if (!c->detached) {
    double* dp = (double*)(c->ws + c->lay.red);
    hipError_t e = vlbm::launch_minima(in, c->plane, c->cur(), dp, blocks, c->p.precision, c->blocked,
                                       c->stream);
    part.resize((size_t)blocks * 2);
    if (e == hipSuccess)
      e = hipMemcpyAsync(part.data(), dp, sizeof(double) * part.size(), hipMemcpyDeviceToHost, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "minima");
  }
  std::vector<Slots> h;
  lbm_status st = read_slots(c, h);
  if (st != LBM_OK) return st;
  const Slots& s = h[inst];
  const int slot = (int)(c->step % 3);
  d->lambda = bits_to_double(s.lam[slot]);
  d->a = host_kinetic_speed(c, d->lambda);
  d->t = s.t[slot];
  d->step = c->step;
  d->n_guard = s.cnt[vlbm::CNT_GUARD];
  d->n_limited = s.cnt[vlbm::CNT_LIMITED];
  d->n_bad = s.cnt[vlbm::CNT_BAD];
  d->bouchut = (int32_t)s.cnt[vlbm::CNT_BOUCHUT];
  d->n_lmp = s.cnt[vlbm::CNT_LMP];
  d->n_nonfinite = s.cnt[vlbm::CNT_NONFINITE];
  d->n_rho = s.cnt[vlbm::CNT_RHO];
  d->n_rhoe = s.cnt[vlbm::CNT_BAD] - s.cnt[vlbm::CNT_NONFINITE] - s.cnt[vlbm::CNT_RHO];
  d->min_rho = NAN;
  d->min_rhoe = NAN;
  if (!part.empty()) {
    double mr = INFINITY, me = INFINITY;
    for (int b = 0; b < blocks; ++b) {
      mr = std::min(mr, part[2 * (size_t)b]);
      me = std::min(me, part[2 * (size_t)b + 1]);
    }
    d->min_rho = mr;
    d->min_rhoe = me;
  }
  return LBM_OK;
}

lbm_status lbm_totals(lbm_ctx* c, int32_t inst, double* out) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (inst < 0 || inst >= c->n_inst) return fail(c, LBM_EINVAL, "instance index out of range");
  if (!out) return fail(c, LBM_EINVAL, "output must be a host pointer to 4 doubles");
  if (lbm_status st0 = require_attached(c)) return st0;
  const Inst& in = c->insts[inst];
  const long long n = (long long)in.nx * in.ny;
  long long b = (n + 255) / 256;
  const int blocks = (int)(b < kTotalsBlocks ? b : kTotalsBlocks);
  double* part = (double*)(c->ws + c->lay.red);
  hipError_t e = vlbm::launch_totals(in, c->plane, c->cur(), part, blocks, c->p.precision, c->blocked,
                                     c->stream);
  std::vector<double> h((size_t)blocks * 8);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h.data(), part, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "totals");
  for (int k = 0; k < 4; ++k) {
    // combine the block partials in double-double (TwoSum, as on the device)
    double hi = 0.0, lo = 0.0;
    for (int q = 0; q < blocks; ++q) {
      const double bh = h[((size_t)q * 4 + k) * 2], bl = h[((size_t)q * 4 + k) * 2 + 1];
      const double s = hi + bh;
      const double bp = s - hi;
      double err = (hi - (s - bp)) + (bh - bp);
      err += lo + bl;
      const double nh = s + err;
      lo = err - (nh - s);
      hi = nh;
    }
    out[k] = hi + lo;
  }
  return LBM_OK;
}

size_t lbm_state_bytes(const lbm_ctx* c) {
  if (!c) return 0;
  return (size_t)20 * (size_t)c->plane * c->elem();
}

lbm_status lbm_get_state(lbm_ctx* c, void* dst) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (!dst) return fail(c, LBM_EINVAL, "destination must be a device pointer");
  if (lbm_status st = require_attached(c)) return st;
  hipError_t e = c->blocked ? vlbm::launch_relayout(c->insts.data(), c->n_inst, c->plane, c->cur(), dst,
                                                    c->p.precision, 0, c->stream)
                            : hipMemcpyAsync(dst, c->cur(), lbm_state_bytes(c), hipMemcpyDeviceToDevice,
                                             c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "get_state copy");
  return LBM_OK;
}

lbm_status lbm_set_state(lbm_ctx* c, const void* src) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (!src) return fail(c, LBM_EINVAL, "source must be a device pointer");
  if (src == c->cur() || src == c->other()) return fail(c, LBM_EINVAL, "src must be a caller buffer");
  hipError_t e = c->blocked ? vlbm::launch_relayout(c->insts.data(), c->n_inst, c->plane, src, c->cur(),
                                                    c->p.precision, 1, c->stream)
                            : hipMemcpyAsync(c->cur(), src, lbm_state_bytes(c), hipMemcpyDeviceToDevice,
                                             c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "set_state copy");
  const int slot = (int)(c->step % 3);
  for (int i = 0; i < c->n_inst && e == hipSuccess; ++i)
    e = vlbm::launch_fill_u32((unsigned int*)&c->slots[i].lam[slot], 0u, 2, c->stream);
  if (e == hipSuccess)
    e = vlbm::launch_lambda_state(c->sc, c->insts.data(), c->n_inst, c->plane, c->cur(),
                                  c->slots, slot, c->p.precision, c->blocked, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "set_state wavespeed");
  c->detached = false;
  return LBM_OK;
}

lbm_status lbm_step_between(lbm_ctx* c, const void* src, void* dst, double* tx, double* ty) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (c->n_inst != 1) return fail(c, LBM_ENOTSUP, "lbm_step_between is single-instance only");
  if (!src || !dst) return fail(c, LBM_EINVAL, "state buffers must be device pointers");
  if ((!tx) != (!ty)) return fail(c, LBM_EINVAL, "give both theta buffers or neither");
  const char* s0 = (const char*)src;
  const char* d0 = (const char*)dst;
  const size_t nb = lbm_state_bytes(c);
  if (s0 < d0 + nb && d0 < s0 + nb) return fail(c, LBM_EINVAL, "src and dst must not overlap");
  if (dst == c->cur()) return fail(c, LBM_EINVAL, "dst must not be the context's current state buffer");
  if (src == c->cur() || src == c->other() || dst == c->other())
    return fail(c, LBM_EINVAL, "src and dst must be caller buffers");
  vlbm::StepArgs a = make_args(c, src, dst, (int)(c->step % 3));
  a.theta_x = tx;
  a.theta_y = ty;
  hipError_t e = launch_step_with_bnd(c, a);
  if (e != hipSuccess) return hip_fail(c, e, "step launch");
  c->step += 1;
  c->detached = true;
  return LBM_OK;
}

lbm_status lbm_step_adjoint(lbm_ctx* c, const double* U, const double* Ub1, double* Ub0);
lbm_status lbm_init_adjoint(lbm_ctx* c, const double* u0, const double* Ub0, double* u0b);

lbm_status lbm_set_launch(lbm_ctx* c, int32_t rows, int32_t waves) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (rows != 0 && (rows < kMinStripRows || rows > kMaxStripRows))
    return fail(c, LBM_EINVAL, "strip rows must lie in [4, 4096]");
  if (waves != 0 && (waves < 1 || waves > 4)) return fail(c, LBM_EINVAL, "waves per group must lie in [1, 4]");
  if (rows) c->strip_rows = rows;
  if (waves) c->waves = waves;
  return rebuild_launch(c);
}

lbm_status lbm_set_strip_mode(lbm_ctx* c, int32_t mode) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (mode != 0 && mode != 1) return fail(c, LBM_EINVAL, "strip mode must be 0 or 1");
  c->strip_mode = mode;
  return rebuild_launch(c);
}

lbm_status lbm_set_instance_boundary(lbm_ctx* c, int32_t inst, int32_t side, const uint8_t* kind,
                                     const double* state) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (inst < 0 || inst >= c->n_inst) return fail(c, LBM_EINVAL, "instance index out of range");
  if (side < 0 || side > 3) return fail(c, LBM_EINVAL, "side must be 0 (west), 1 (east), 2 (south) or 3 (north)");
  if (c->p.blend == LBM_BLEND_CELL)
    return fail(c, LBM_ENOTSUP, "boundary descriptions are not supported with the per-cell blending");
  const int ax = side / 2;
  if ((ax == 0 ? c->p.bc_x : c->p.bc_y) != LBM_BC_OUTFLOW)
    return fail(c, LBM_EINVAL, "boundary descriptions need the side's axis to be non-periodic (LBM_BC_OUTFLOW)");
  const Inst& in = c->insts[inst];
  const int len = ax == 0 ? in.ny : in.nx, n = ax == 0 ? in.nx : in.ny;
  bool dirichlet = false;
  if (kind) {
    std::vector<uint8_t> h((size_t)len);
    hipError_t e = hipMemcpyAsync(h.data(), kind, (size_t)len, hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "reading boundary kinds");
    for (int r = 0; r < len; ++r) {
      if (h[r] > vlbm::BND_DIRICHLET) return fail(c, LBM_EINVAL, "unknown boundary kind");
      if (h[r] == vlbm::BND_WALL && n < 2) return fail(c, LBM_EINVAL, "a wall needs two cells along its axis");
      dirichlet |= h[r] == vlbm::BND_DIRICHLET;
    }
    if (dirichlet && !state) return fail(c, LBM_EINVAL, "Dirichlet cells need a state array");
    if (dirichlet) {
      // the Dirichlet states must be admissible (rho > 0, p > 0, finite)
      std::vector<double> st((size_t)4 * len);
      e = hipMemcpyAsync(st.data(), state, st.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) return hip_fail(c, e, "reading boundary states");
      const double gm1 = c->p.gamma - 1.0;
      for (int r = 0; r < len; ++r) {
        if (h[r] != vlbm::BND_DIRICHLET) continue;
        const double rho = st[r], m1 = st[(size_t)len + r], m2 = st[2 * (size_t)len + r],
                     E = st[3 * (size_t)len + r];
        const double p = gm1 * (E - 0.5 * (m1 * m1 + m2 * m2) / rho);
        if (!(rho > 0.0) || !(p > 0.0) || !std::isfinite(E) || !std::isfinite(m1) || !std::isfinite(m2))
          return fail(c, LBM_EINVAL, "a Dirichlet state is not admissible (rho > 0, p > 0, finite)");
      }
    }
  }
  if (c->bnd.size() != (size_t)c->n_inst) {
    c->bnd.assign(c->n_inst, vlbm::BndDesc{});
    c->side_dirichlet.assign(c->n_inst, {false, false, false, false});
  }
  c->bnd[inst].kind[side] = kind;
  c->bnd[inst].state[side] = kind ? state : nullptr;
  c->side_dirichlet[inst][side] = dirichlet;
  c->has_bnd = false;
  c->has_dirichlet = false;
  for (int i = 0; i < c->n_inst; ++i)
    for (int k = 0; k < 4; ++k) {
      c->has_bnd |= c->bnd[i].kind[k] != nullptr;
      c->has_dirichlet |= c->side_dirichlet[i][k];
    }
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  if (c->blocked && c->has_bnd) {
    // the kernels that read descriptions take the planar layout: convert the
    // current state once, through the other buffer (which the next step
    // overwrites anyway), and stay planar
    hipError_t e = vlbm::launch_relayout(c->insts.data(), c->n_inst, c->plane, c->cur(), c->other(),
                                         c->p.precision, 0, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->cur(), c->other(), lbm_state_bytes(c), hipMemcpyDeviceToDevice, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "state layout");
    c->blocked = 0;
  }
  if (c->n_inst > 1) {  // ensembles read the descriptions from the workspace table
    hipError_t e = hipMemcpyAsync(c->ws + c->lay.bndt, c->bnd.data(), sizeof(vlbm::BndDesc) * c->n_inst,
                                  hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "uploading boundary descriptions");
  }
  return LBM_OK;
}

lbm_status lbm_set_boundary(lbm_ctx* c, int32_t side, const uint8_t* kind, const double* state) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (c->n_inst != 1)
    return fail(c, LBM_ENOTSUP, "ensembles describe boundaries per instance (lbm_set_instance_boundary)");
  return lbm_set_instance_boundary(c, 0, side, kind, state);
}

lbm_status lbm_get_strip_mode(const lbm_ctx* c, int32_t* mode) {
  if (!c || !mode) return LBM_EINVAL;
  *mode = c->strip_mode;
  return LBM_OK;
}

lbm_status lbm_get_launch(const lbm_ctx* c, int32_t* rows, int32_t* waves) {
  if (!c || !rows || !waves) return LBM_EINVAL;
  *rows = c->strip_rows;
  *waves = c->waves;
  return LBM_OK;
}

lbm_status lbm_set_grid(lbm_ctx* c, int32_t groups_per_cu) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (groups_per_cu < 0 || groups_per_cu > kMaxGridPerCu)
    return fail(c, LBM_EINVAL, "groups per compute unit must lie in [0, 32]");
  c->grid_per_cu = groups_per_cu;
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  c->graphs.clear();
  return LBM_OK;
}

lbm_status lbm_get_grid(const lbm_ctx* c, int32_t* groups_per_cu, int32_t* groups) {
  if (!c || !groups_per_cu) return LBM_EINVAL;
  *groups_per_cu = c->grid_per_cu;
  if (groups) *groups = compute_groups(c);
  return LBM_OK;
}

lbm_status lbm_autotune(lbm_ctx* c, const char* path) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (lbm_status st0 = require_attached(c)) return st0;
  // cache key: everything that selects the kernel or shapes its work list —
  // instance count, first instance, total cells, precision, limiters, order,
  // boundary conditions, sponge, boundary descriptions, and a hash (FNV-1a)
  // of every instance's sides, so that ensembles with the same first
  // instance and cell count do not share an entry
  uint32_t h = 2166136261u;
  for (const Inst& in : c->insts)
    for (int v : {in.nx, in.ny})
      for (int b = 0; b < 4; ++b) h = (h ^ (uint32_t)((v >> (8 * b)) & 0xff)) * 16777619u;
  char key[200];
  long long cells = c->plane;
  snprintf(key, sizeof(key), "n%d_nx%d_ny%d_cells%lld_p%d_lim%u_o%d_bc%d%d_s%d_b%d_h%08x", c->n_inst,
           c->insts[0].nx, c->insts[0].ny, cells, c->p.precision, c->p.limiters, c->p.order, c->p.bc_x,
           c->p.bc_y, c->p.sponge, c->has_bnd ? 1 : 0, h);
  // cache lookup: a flat JSON object {"key": [rows, waves, groups per CU,
  // strip mode], ...} (missing trailing values are 0)
  std::string text;
  if (path) {
    FILE* f = fopen(path, "rb");
    if (f) {
      char b[4096];
      size_t r;
      while ((r = fread(b, 1, sizeof(b), f)) > 0) text.append(b, r);
      fclose(f);
      const std::string k = std::string("\"") + key + "\"";
      size_t pos = text.find(k);
      if (pos != std::string::npos) {
        int rows = 0, waves = 0, grid = 0, mode = 0;
        const int got = sscanf(text.c_str() + pos + k.size(), " : [ %d , %d , %d , %d ]", &rows, &waves,
                               &grid, &mode);
        if (got >= 2) {
          lbm_status st = lbm_set_launch(c, rows, waves);
          if (st == LBM_OK) st = lbm_set_grid(c, got >= 3 ? grid : 0);
          if (st == LBM_OK) st = lbm_set_strip_mode(c, got >= 4 ? mode : 0);
          return st;
        }
      }
    }
  }
  std::vector<Slots> saved;
  lbm_status st = read_slots(c, saved);
  if (st != LBM_OK) return st;
  const int rows_c[] = {4, 8, 16, 32, 64, 128, 256};
  const int waves_c[] = {1, 2, 4};
  const int grid_c[] = {0, 1, 2, 4};  // one wave per strip, or persistent grids
  const int n_modes = c->n_inst > 1 ? 2 : 1;  // matched strip heights: ensembles only
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return fail(c, LBM_EDEVICE, "hipEventCreate");
  float best = 1e30f;
  int best_r = c->strip_rows, best_w = c->waves, best_g = c->grid_per_cu, best_m = c->strip_mode;
  // average time of one launch of the shape (r, w, gpc, mode); launches all
  // read the current state and write the other buffer, so the state is not
  // advanced
  auto time_shape = [&](int r, int w, int gpc, int mode, float work_ms, float& ms) -> lbm_status {
    c->strip_mode = mode;
    lbm_status s2 = lbm_set_launch(c, r, w);
    if (s2 == LBM_OK) s2 = lbm_set_grid(c, gpc);
    if (s2 != LBM_OK) return s2;
    ms = -1.0f;
    // a persistent grid no smaller than one wave per strip is the same launch
    if (gpc > 0 && (long long)gpc * c->n_cu * w >= c->n_items) return LBM_OK;
    vlbm::StepArgs a = make_args(c, c->cur(), c->other(), (int)(c->step % 3));
    // one timed launch sizes the repetition count to about work_ms of work
    hipError_t e = vlbm::launch_step(a, c->p.precision, c->stream);
    if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
    if (e == hipSuccess) e = vlbm::launch_step(a, c->p.precision, c->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float t = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    int reps = t > 0.0f ? (int)(work_ms / t) : 64;
    reps = reps < 2 ? 2 : (reps > 256 ? 256 : reps);
    if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
    for (int k = 0; k < reps && e == hipSuccess; ++k) e = vlbm::launch_step(a, c->p.precision, c->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
    if (e != hipSuccess) return hip_fail(c, e, "autotune");
    ms = t / reps;
    return LBM_OK;
  };
  // first pass: every candidate with about 4 ms of launches; second pass: the
  // four fastest again, three times each with about 12 ms, interleaved, and
  // the median of the three (shapes within a few percent of each other are
  // told apart, and a single fast outlier does not decide)
  struct Cand {
    float ms;
    int r, w, g, m;
    float t[3];
  };
  std::vector<Cand> cands;
  auto bail = [&](lbm_status s2) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return s2;
  };
  int max_ny = 0;
  for (const Inst& in : c->insts) max_ny = std::max(max_ny, in.ny);
  for (int r : rows_c) {
    if (r > 2 * max_ny && r != 16) continue;
    for (int w : waves_c) {
      for (int gpc : grid_c) {
        for (int m = 0; m < n_modes; ++m) {
          float ms = -1.0f;
          st = time_shape(r, w, gpc, m, 4.0f, ms);
          if (st != LBM_OK) return bail(st);
          if (ms >= 0.0f) cands.push_back({ms, r, w, gpc, m, {0.0f, 0.0f, 0.0f}});
        }
      }
    }
  }
  std::sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
  if (cands.size() > 4) cands.resize(4);
  for (int round = 0; round < 3; ++round) {
    for (Cand& k : cands) {
      float ms = -1.0f;
      st = time_shape(k.r, k.w, k.g, k.m, 12.0f, ms);
      if (st != LBM_OK) return bail(st);
      k.t[round] = ms;
    }
  }
  for (Cand& k : cands) {
    std::sort(k.t, k.t + 3);
    k.ms = k.t[1];
  }
  for (const Cand& k : cands) {
    if (k.ms < best) {
      best = k.ms;
      best_r = k.r;
      best_w = k.w;
      best_g = k.g;
      best_m = k.m;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  st = write_slots(c, saved);
  if (st != LBM_OK) return st;
  c->strip_mode = best_m;
  st = lbm_set_launch(c, best_r, best_w);
  if (st == LBM_OK) st = lbm_set_grid(c, best_g);
  if (st != LBM_OK) return st;
  if (path) {
    // append the entry to the flat JSON object
    std::string body = text;
    size_t end = body.rfind('}');
    char entry[256];
    snprintf(entry, sizeof(entry), "\"%s\": [%d, %d, %d, %d]", key, best_r, best_w, best_g, best_m);
    if (end == std::string::npos) {
      body = std::string("{\n  ") + entry + "\n}\n";
    } else {
      std::string head = body.substr(0, end);
      bool empty = head.find('"') == std::string::npos;
      while (!head.empty() && (head.back() == '\n' || head.back() == ' ')) head.pop_back();
      body = head + (empty ? "\n  " : ",\n  ") + entry + "\n}\n";
    }
    FILE* f = fopen(path, "wb");
    if (!f) return fail(c, LBM_EINVAL, "cannot write the autotune cache file");
    fwrite(body.data(), 1, body.size(), f);
    fclose(f);
  }
  return LBM_OK;
}

const char* lbm_status_string(lbm_status s) {
  switch (s) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOTSUP: return "not supported";
    case LBM_EDEVICE: return "device error";
    case LBM_EPOSITIVITY: return "non-admissible state";
    case LBM_ENONFINITE: return "non-finite value";
    case LBM_EBOUCHUT: return "Bouchut condition violated";
    case LBM_EGUARD: return "face state outside the admissible set";
  }
  return "unknown status";
}

const char* lbm_last_error(const lbm_ctx* c) {
  if (!c) return g_init_error.c_str();
  return c->err.c_str();
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  delete c;
}

}  // extern "C"

// ------------------------------------------------------------- adjoint entry points
namespace {
lbm_status adjoint_checks(lbm_ctx* c, const double* U, const double* Ub1, const double* Ub0) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (c->n_inst != 1 || c->p.precision != LBM_FP64)
    return fail(c, LBM_ENOTSUP, "the adjoint is single-instance float64 only");
  if (c->p.blend != LBM_BLEND_FACE) return fail(c, LBM_ENOTSUP, "the adjoint covers the face blending only");
  if (!U || !Ub1 || !Ub0) return fail(c, LBM_EINVAL, "adjoint buffers must be device pointers");
  if (U == Ub0 || Ub1 == Ub0) return fail(c, LBM_EINVAL, "Ubar_n must not alias the inputs");
  if ((const void*)U == c->other() || (const void*)U == c->cur())
    return fail(c, LBM_EINVAL, "U_n must not be one of the context's own state buffers");
  if (c->insts[0].ny > 65535) return fail(c, LBM_ENOTSUP, "the adjoint supports ny <= 65535");
  return LBM_OK;
}
vlbm::BndKinds bnd_kinds(const lbm_ctx* c) {
  vlbm::BndKinds k;
  for (int s = 0; s < 4; ++s) k.k[s] = c->bnd.empty() ? nullptr : c->bnd[0].kind[s];
  return k;
}
}  // namespace

extern "C" lbm_status lbm_step_adjoint_theta(lbm_ctx* c, const double* U, const double* tx,
                                             const double* ty, const double* Ub1, double* Ub0) {
  lbm_status st = adjoint_checks(c, U, Ub1, Ub0);
  if (st != LBM_OK) return st;
  if (!tx || !ty) return fail(c, LBM_EINVAL, "theta buffers must be device pointers");
  if ((const double*)Ub0 == tx || (const double*)Ub0 == ty)
    return fail(c, LBM_EINVAL, "Ubar_n must not alias the theta fields");
  // a^n: fixed, or from lambda^n of U_n in the slot the next forward step
  // clears before it reads it (no other slot is touched)
  const int scratch = (int)((c->step + 2) % 3);
  hipError_t e = hipSuccess;
  if (c->p.a_mode != LBM_A_FIXED) {
    e = vlbm::launch_fill_u32((unsigned int*)&c->slots[0].lam[scratch], 0u, 2, c->stream);
    if (e == hipSuccess)
      e = vlbm::launch_lambda_state(c->sc, c->insts.data(), 1, c->plane, U, c->slots, scratch,
                                    LBM_FP64, 0, c->stream);
    // the forward step's lambda^n also covers the Dirichlet states
    if (e == hipSuccess && c->has_dirichlet)
      e = vlbm::launch_bnd_lambda(make_args(c, U, nullptr, scratch), scratch, c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint wavespeed");
  }
  e = vlbm::launch_adjoint_step(c->sc, c->insts[0], c->plane, U, Ub1, Ub0, tx, ty, c->slots,
                                scratch, bnd_kinds(c), c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "adjoint launch");
  return LBM_OK;
}

extern "C" lbm_status lbm_step_adjoint(lbm_ctx* c, const double* U, const double* Ub1,
                                       double* Ub0) {
  lbm_status st0 = adjoint_checks(c, U, Ub1, Ub0);
  if (st0 != LBM_OK) return st0;
  const Inst& in = c->insts[0];
  double* tx = (double*)(c->ws + c->lay.theta);
  double* ty = tx + (size_t)(in.nx + 1) * in.ny;
  // lambda^n of U (scratch slot: a second Slots record is not available, so
  // use the slot that the next forward step would clear)
  const int scratch = (int)((c->step + 2) % 3);
  hipError_t e = vlbm::launch_fill_u32((unsigned int*)&c->slots[0].lam[scratch], 0u, 2, c->stream);
  if (e == hipSuccess)
    e = vlbm::launch_lambda_state(c->sc, c->insts.data(), 1, c->plane, U, c->slots, scratch,
                                  LBM_FP64, 0, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "adjoint wavespeed");
  // theta^n of U with the forward kernel (its state output goes to the
  // context's other buffer, which the next forward step overwrites anyway;
  // the slots it touches are parked and restored on the stream, no host
  // round trip)
  Slots* save = (Slots*)(c->ws + c->lay.slots_save);
  e = hipMemcpyAsync(save, c->slots, sizeof(Slots), hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "adjoint slot save");
  vlbm::StepArgs a = make_args(c, U, c->other(), scratch);
  a.theta_x = tx;
  a.theta_y = ty;
  // (lambda^n raised by the Dirichlet states first, as in the forward step)
  e = launch_step_with_bnd(c, a);
  if (e != hipSuccess) return hip_fail(c, e, "adjoint theta");
  e = vlbm::launch_adjoint_step(c->sc, in, c->plane, U, Ub1, Ub0, tx, ty, c->slots, scratch,
                                bnd_kinds(c), c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "adjoint launch");
  // restore the scalar slots (lambda, t, counters) of the forward run
  e = hipMemcpyAsync(c->slots, save, sizeof(Slots), hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "adjoint slot restore");
  return LBM_OK;
}

extern "C" lbm_status lbm_init_adjoint(lbm_ctx* c, const double* u0, const double* Ub0,
                                       double* u0b) {
  if (!c) return fail(nullptr, LBM_EINVAL, "ctx is NULL");
  if (c->n_inst != 1 || c->p.precision != LBM_FP64)
    return fail(c, LBM_ENOTSUP, "the adjoint is single-instance float64 only");
  if (c->p.blend != LBM_BLEND_FACE) return fail(c, LBM_ENOTSUP, "the adjoint covers the face blending only");
  if (!u0 || !Ub0 || !u0b) return fail(c, LBM_EINVAL, "adjoint buffers must be device pointers");
  Slots* save = (Slots*)(c->ws + c->lay.slots_save);
  hipError_t e = hipMemcpyAsync(save, c->slots, sizeof(Slots), hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "init adjoint slot save");
  // lambda^0 of u0 into a scratch slot
  const int scratch = (int)((c->step + 2) % 3);
  e = vlbm::launch_fill_u32((unsigned int*)&c->slots[0].lam[scratch], 0u, 2, c->stream);
  if (e == hipSuccess)
    e = vlbm::launch_lambda_state(c->sc, c->insts.data(), 1, (long long)c->insts[0].nx * c->insts[0].ny,
                                  u0, c->slots, scratch, LBM_FP64, 0, c->stream);
  if (e == hipSuccess)
    e = vlbm::launch_adjoint_init(c->sc, c->insts[0], u0, Ub0, u0b, c->slots, scratch, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "init adjoint launch");
  e = hipMemcpyAsync(c->slots, save, sizeof(Slots), hipMemcpyDeviceToDevice, c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "init adjoint slot restore");
  return LBM_OK;
}
