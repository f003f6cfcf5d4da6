// The allocation-free step entry point (lbm_step_noalloc): one time step of
// a single instance from a caller state into another caller state, with no
// context and no workspace.  The per-step scalars the kernels need (the
// lambda slots, the time slots and the event counters) live in a file-scope
// device array instead of a workspace, so a call allocates nothing, host or
// device, and launches only kernels (three fills and reductions, one step).
//
// The array exists once per device.  Its device address is looked up once
// per device, with that device current, and kept in a table; host code uses
// only that address (the array's own name denotes a host-side stand-in).

#include <math.h>
#include <string.h>

#include <mutex>

#include "vlbm.h"
#include "vlbm_internal.h"

using vlbm::Slots;

namespace {

// One 128-byte record of per-step scalars (vlbm::Slots) at the start; the
// rest is padding to the stated size.
constexpr size_t kScratchBytes = LBM_NOALLOC_SCRATCH_BYTES;
static_assert(sizeof(Slots) <= kScratchBytes, "the scalar record fits the scratch array");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the scratch array on the current device (looked up on
// the first call for that device).
lbm_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    vlbm::host_set_error("lbm_step_noalloc: hipGetDevice failed");
    return LBM_EDEVICE;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    vlbm::host_set_error("lbm_step_noalloc: device index beyond the scratch table (64 devices)");
    return LBM_ENOTSUP;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      vlbm::host_set_error("lbm_step_noalloc: hipGetSymbolAddress of the scratch array failed");
      return LBM_EDEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LBM_OK;
}

lbm_status fail(lbm_status s, const char* m) {
  vlbm::host_set_error(m);
  return s;
}

// Rows per strip: the tallest of 64, 32, 16, 8, 4 that still gives one wave
// per SIMD of the chip (1024 SIMDs; 2 waves per SIMD with the float32 state),
// the default of a new context.
int strip_rows(int nx, int ny, int precision) {
  const long long want = precision == LBM_FP64 ? 1024 : 2048;
  int rows = 64;
  for (; rows > 4; rows /= 2)
    if ((long long)((nx + 63) / 64) * ((ny + rows - 1) / rows) >= want) break;
  return rows;
}

}  // namespace

extern "C" lbm_status lbm_step_noalloc(const lbm_params* p, const void* src_dev, void* dst_dev,
                                       void* stream, lbm_diag* diag_host) {
  if (const char* m = vlbm::host_check_params(p)) return fail(LBM_EINVAL, m);
  if (p->blend != LBM_BLEND_FACE) return fail(LBM_ENOTSUP, "lbm_step_noalloc: face blending only");
  if (!src_dev || !dst_dev) return fail(LBM_EINVAL, "lbm_step_noalloc: state buffers must be device pointers");
  const long long cells = (long long)p->nx * p->ny;
  const size_t bytes = (size_t)20 * (size_t)cells * (p->precision == LBM_FP64 ? 8 : 4);
  const char* s0 = (const char*)src_dev;
  const char* d0 = (const char*)dst_dev;
  if (s0 < d0 + bytes && d0 < s0 + bytes) return fail(LBM_EINVAL, "lbm_step_noalloc: src and dst must not overlap");
  void* base = nullptr;
  if (lbm_status st = scratch_address(&base)) return st;
  Slots* sl = (Slots*)base;
  hipStream_t s = (hipStream_t)stream;

  const vlbm::Scheme sc = vlbm::host_make_scheme(p);
  vlbm::Inst in{};
  in.off = 0;
  in.item0 = 0;
  in.dx = p->dx;
  in.nx = p->nx;
  in.ny = p->ny;
  in.strip_h = strip_rows(p->nx, p->ny, p->precision);
  in.xs = (p->nx + 63) / 64;
  in.ys = (p->ny + in.strip_h - 1) / in.strip_h;

  // zero the record, lambda^n of src into slot 0, then clear the counters
  // that the reduction raised for non-admissible cells of src (they count
  // the step's output cells only, as in a context)
  hipError_t e = vlbm::launch_fill_u32((unsigned int*)sl, 0u, (long long)(sizeof(Slots) / 4), s);
  if (e == hipSuccess) e = vlbm::launch_lambda_state(sc, &in, 1, cells, src_dev, sl, 0, p->precision, 0, s);
  if (e == hipSuccess)
    e = vlbm::launch_fill_u32((unsigned int*)((char*)base + offsetof(Slots, cnt)), 0u,
                              (long long)(sizeof(sl->cnt) / 4), s);
  if (e != hipSuccess) return fail(LBM_EDEVICE, "lbm_step_noalloc: wavespeed launch failed");

  vlbm::StepArgs a;
  memset(&a, 0, sizeof(a));
  a.src = src_dev;
  a.dst = dst_dev;
  a.plane = cells;
  a.slots = sl;
  a.insts = nullptr;
  a.item_inst = nullptr;
  a.inst0 = in;
  a.n_items = (long long)in.xs * in.ys;
  a.n_inst = 1;
  a.slot = 0;
  a.waves_per_group = 4;
  a.xcd_remap = 1;
  a.groups = (int)(((a.n_items + 3) / 4 + 7) / 8 * 8);
  a.sc = sc;
  a.bnd = 0;
  e = vlbm::launch_step(a, p->precision, s);
  if (e != hipSuccess) return fail(LBM_EDEVICE, "lbm_step_noalloc: step launch failed");
  if (!diag_host) return LBM_OK;

  Slots h;
  e = hipMemcpyAsync(&h, base, sizeof(Slots), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return fail(LBM_EDEVICE, "lbm_step_noalloc: reading the step's scalars failed");
  double lam;
  memcpy(&lam, &h.lam[0], sizeof(lam));
  diag_host->lambda = lam;
  diag_host->a = p->a_mode == LBM_A_FIXED ? p->a_fixed : 2.0 * p->a_beta * lam / (1.0 - p->alpha);
  diag_host->t = h.t[1];
  diag_host->step = 1;
  diag_host->n_guard = (int64_t)h.cnt[vlbm::CNT_GUARD];
  diag_host->n_limited = (int64_t)h.cnt[vlbm::CNT_LIMITED];
  diag_host->n_bad = (int64_t)h.cnt[vlbm::CNT_BAD];
  diag_host->bouchut = (int32_t)h.cnt[vlbm::CNT_BOUCHUT];
  diag_host->n_lmp = (int64_t)h.cnt[vlbm::CNT_LMP];
  diag_host->n_nonfinite = (int64_t)h.cnt[vlbm::CNT_NONFINITE];
  diag_host->n_rho = (int64_t)h.cnt[vlbm::CNT_RHO];
  diag_host->n_rhoe = diag_host->n_bad - diag_host->n_nonfinite - diag_host->n_rho;
  diag_host->min_rho = NAN;
  diag_host->min_rhoe = NAN;
  if (diag_host->n_nonfinite) return fail(LBM_ENONFINITE, "lbm_step_noalloc: non-finite cells were produced");
  if (diag_host->n_bad) return fail(LBM_EPOSITIVITY, "lbm_step_noalloc: non-admissible cells were produced");
  if (diag_host->n_guard) return fail(LBM_EGUARD, "lbm_step_noalloc: face states left the admissible set");
  if (diag_host->bouchut) return fail(LBM_EBOUCHUT, "lbm_step_noalloc: the fixed kinetic speed fell below the Bouchut bound");
  return LBM_OK;
}
