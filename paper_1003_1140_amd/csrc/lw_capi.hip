// lw_capi.hip -- host runtime behind the C ABI of include/lw.h.
//
// Owns the per-context device state (direction and frequency grids, the FP64
// accumulator S, the device error record), validates arguments on the host,
// picks launch shapes and enqueues the kernels on the context's stream.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "lw_internal.h"
#include "lw_mfma.h"



namespace {

const unsigned long long kNoError = ~0ull;

lw_status fail(lw_ctx* c, lw_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

lw_status hip_fail(lw_ctx* c, hipError_t e, const char* what) {
  return fail(c, LW_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define LW_HIP(call, what)                        \
  do {                                            \
    hipError_t e_ = (call);                       \
    if (e_ != hipSuccess) return hip_fail(c, e_, what); \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

void free_dev(void* p) {
  if (p) (void)hipFree(p);
}

// S [ns][nd][nw], and in coherent synthesis the summed amplitudes A [ns][nd][nw][4]; both zeroed.
lw_status alloc_accumulator(lw_ctx* c) {
  c->epoch += 1;
  free_dev(c->d_S);
  free_dev(c->d_A);
  c->d_S = nullptr;
  c->d_A = nullptr;
  if (c->nd <= 0 || c->nw <= 0) return LW_OK;
  size_t n = (size_t)c->ns * c->nd * c->nw;
  LW_HIP(hipMalloc(&c->d_S, n * sizeof(double)), "hipMalloc(S)");
  LW_HIP(lw::launch_fill_f64(c->d_S, (int64_t)n, 0.0, c->stream), "zero S");
  if (c->coherent) {
    LW_HIP(hipMalloc(&c->d_A, 4 * n * sizeof(double)), "hipMalloc(A)");
    LW_HIP(lw::launch_fill_f64(c->d_A, (int64_t)(4 * n), 0.0, c->stream), "zero A");
  }
  return LW_OK;
}

// Accumulator the FP32 kernel's partial rows are reduced into.
double* direct_target(lw_ctx* c) { return c->coherent ? c->d_A : c->d_S; }

// Orthonormal e1, e2 perpendicular to the unit vector n, (e1, e2, n) right-handed.
void basis(const double n[3], double e1[3], double e2[3]) {
  // pick the axis least aligned with n
  double a[3] = {0, 0, 0};
  int m = 0;
  for (int i = 1; i < 3; ++i)
    if (fabs(n[i]) < fabs(n[m])) m = i;
  a[m] = 1.0;
  // e1 = normalise(a - (a.n) n)
  double an = a[0] * n[0] + a[1] * n[1] + a[2] * n[2];
  for (int i = 0; i < 3; ++i) e1[i] = a[i] - an * n[i];
  double l = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  for (int i = 0; i < 3; ++i) e1[i] /= l;
  // e2 = n x e1
  e2[0] = n[1] * e1[2] - n[2] * e1[1];
  e2[1] = n[2] * e1[0] - n[0] * e1[2];
  e2[2] = n[0] * e1[1] - n[1] * e1[0];
}

lw_status check_batch(lw_ctx* c, const lw_batch* b) {
  if (!b) return fail(c, LW_EINVAL, "batch is NULL");
  if (b->n_particles < 0) return fail(c, LW_EINVAL, "n_particles < 0");
  if (b->n_particles == 0) return LW_OK;
  const void* need[] = {b->offsets, b->x, b->y, b->z, b->bx, b->by, b->bz, b->ax, b->ay, b->az,
                        b->t0, b->dt, b->charge, b->weight};
  const char* names[] = {"offsets", "x", "y", "z", "bx", "by", "bz", "ax", "ay", "az",
                         "t0", "dt", "charge", "weight"};
  for (int i = 0; i < 14; ++i)
    if (!need[i]) return fail(c, LW_EINVAL, "batch.%s is NULL", names[i]);
  if (b->flags & ~LW_BATCH_F64_ACCEL) return fail(c, LW_EINVAL, "unknown batch flags 0x%x", b->flags);
  return LW_OK;
}

lw_status check_grids(lw_ctx* c) {
  if (c->nd <= 0) return fail(c, LW_ESTATE, "directions not set");
  if (c->nw <= 0) return fail(c, LW_ESTATE, "frequencies not set");
  return LW_OK;
}

using lw::DirectShape;
using lw::direct_shape;

// Partial sums of lw_accumulate_noalloc: a file-scope device array, one copy per GPU the
// library runs on, held until the process ends.  In host code `scratch` only names the
// symbol; its device address on each GPU comes from hipGetSymbolAddress (scratch_on).
constexpr size_t kNoallocScratchBytes = (size_t)LW_NOALLOC_SCRATCH_MB << 20;
static __device__ __attribute__((aligned(256))) unsigned char scratch[kNoallocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array, looked up once per device with that device
// current (lw_create calls it, so the no-allocation entry point finds it ready).
lw_status scratch_on(lw_ctx* c, void** out) {
  if (c->device < 0 || c->device >= kMaxDevices) return fail(c, LW_EUNSUPPORTED, "device index %d too large", c->device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[c->device]) {
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) return fail(c, LW_EDEVICE, "hipGetDevice failed");
    if (prev != c->device && hipSetDevice(c->device) != hipSuccess) return fail(c, LW_EDEVICE, "hipSetDevice failed");
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != c->device) (void)hipSetDevice(prev);
    if (e != hipSuccess || !p) return fail(c, LW_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[c->device] = p;
  }
  *out = g_scratch_ptr[c->device];
  return LW_OK;
}

// Wait for the stream, then turn the device's records into a status: a batch that outgrew
// the matrix-core plan first (its result is incomplete), then bad data.
lw_status read_device_errors(lw_ctx* c) {
  unsigned long long e[2] = {kNoError, kNoError};
  LW_HIP(hipMemcpyAsync(e, c->d_err, sizeof(e), hipMemcpyDeviceToHost, c->stream), "copy error records");
  LW_HIP(hipStreamSynchronize(c->stream), "sync");
  if (e[1] != kNoError)
    return fail(c, LW_ESTATE,
                "particle %llu: retarded-time span outgrew the matrix-core plan (plan the batch again with "
                "lw_workspace_size or lw_plan_batch and redo the accumulation)", e[1]);
  if (e[0] != kNoError)
    return fail(c, LW_ERANGE, "particle %llu has |beta| >= 1, a non-finite sample or decreasing offsets", e[0]);
  return LW_OK;
}

// LW_PATH_AUTO: the matrix-core FP16 path where it measured faster (long frequency lists) and
// can serve the call (no per-particle output), else the FP32 path.
lw_path resolve_path(const lw_ctx* c, lw_path path, bool per_particle) {
  if (path != LW_PATH_AUTO) return path;
  return (!per_particle && c->nw >= LW_AUTO_MIN_FREQUENCIES) ? LW_PATH_MFMA_F16 : LW_PATH_FP32;
}

size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

}  // namespace

namespace lw {

static hipError_t next_event(lw_ctx* c, hipEvent_t* e) {
  if (c->ev_used == c->ev_pool.size()) {
    hipEvent_t n;
    hipError_t err = hipEventCreate(&n);
    if (err != hipSuccess) return err;
    c->ev_pool.push_back(n);
  }
  *e = c->ev_pool[c->ev_used++];
  return hipSuccess;
}

hipError_t prof_begin(lw_ctx* c, int kind) {
  if (!c->prof) return hipSuccess;
  hipEvent_t a, b;
  hipError_t e = next_event(c, &a);
  if (e == hipSuccess) e = next_event(c, &b);
  if (e != hipSuccess) return e;
  c->ev_marks.push_back({kind, {a, b}});
  return hipEventRecord(a, c->stream);
}

hipError_t prof_end(lw_ctx* c) {
  if (!c->prof || c->ev_marks.empty()) return hipSuccess;
  return hipEventRecord(c->ev_marks.back().second.second, c->stream);
}

}  // namespace lw

extern "C" {

lw_status lw_create(lw_ctx** out, int device, void* stream) {
  if (!out) return LW_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return LW_EDEVICE;
  if (device < 0 || device >= n) return LW_EINVAL;
  lw_ctx* c = new lw_ctx();
  c->device = device;
  c->stream = (hipStream_t)stream;
  DeviceGuard g(device);
  if (hipMalloc(&c->d_err, 2 * sizeof(unsigned long long)) != hipSuccess) {
    delete c;
    return LW_ENOMEM;
  }
  c->d_overflow = c->d_err + 1;  // one allocation: both records are cleared and read together
  if (lw::launch_fill_u64(c->d_err, 2, kNoError, c->stream) != hipSuccess) {
    (void)hipFree(c->d_err);
    delete c;
    return LW_EDEVICE;
  }
  c->mfma = lw::mfma_cache_create();
  void* sp = nullptr;
  const lw_status sst = scratch_on(c, &sp);
  if (sst != LW_OK) {
    lw_destroy(c);
    return sst;
  }
  *out = c;
  return LW_OK;
}

void lw_destroy(lw_ctx* c) {
  if (!c) return;
  DeviceGuard g(c->device);
  (void)hipStreamSynchronize(c->stream);
  lw::mfma_cache_destroy(c->mfma);
  free_dev(c->plan.d_perm);
  free_dev(c->plan.d_order);
  free_dev(c->d_ticket);
  free_dev(c->d_wgtime);
  free_dev(c->d_flag);
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  free_dev(c->d_flops);
  free_dev(c->d_dirs);
  free_dev(c->d_wturn);
  free_dev(c->d_omega);
  free_dev(c->d_S);
  free_dev(c->d_A);
  free_dev(c->d_diag);
  free_dev(c->d_err);
  delete c;
}

const char* lw_last_error(const lw_ctx* c) { return c ? c->err.c_str() : "null context"; }

lw_status lw_set_stream(lw_ctx* c, void* stream) {
  if (!c) return LW_EINVAL;
  c->stream = (hipStream_t)stream;
  return LW_OK;
}

lw_status lw_set_directions(lw_ctx* c, const double* n_xyz, int32_t nd) {
  if (!c) return LW_EINVAL;
  if (!n_xyz || nd <= 0) return fail(c, LW_EINVAL, "need nd > 0 directions");
  std::vector<double> h((size_t)nd * lw::kDirStride);
  for (int32_t d = 0; d < nd; ++d) {
    const double* v = n_xyz + 3 * d;
    double l = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    if (!(l > 0.0) || !isfinite(l)) return fail(c, LW_EINVAL, "direction %d is zero or not finite", d);
    double n[3] = {v[0] / l, v[1] / l, v[2] / l}, e1[3], e2[3];
    basis(n, e1, e2);
    for (int i = 0; i < 3; ++i) {
      h[(size_t)d * 9 + i] = n[i];
      h[(size_t)d * 9 + 3 + i] = e1[i];
      h[(size_t)d * 9 + 6 + i] = e2[i];
    }
  }
  DeviceGuard g(c->device);
  LW_HIP(hipStreamSynchronize(c->stream), "sync");
  free_dev(c->d_dirs);
  c->d_dirs = nullptr;
  LW_HIP(hipMalloc(&c->d_dirs, h.size() * sizeof(double)), "hipMalloc(dirs)");
  LW_HIP(hipMemcpy(c->d_dirs, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice),
         "copy dirs");
  c->h_dirs = h;
  c->nd = nd;
  lw::mfma_cache_invalidate(c->mfma);
  return alloc_accumulator(c);
}

lw_status lw_set_frequencies(lw_ctx* c, const double* omega, int32_t nw) {
  if (!c) return LW_EINVAL;
  if (!omega || nw <= 0) return fail(c, LW_EINVAL, "need nw > 0 frequencies");
  std::vector<double> w(omega, omega + nw), wt(nw);
  for (int32_t j = 0; j < nw; ++j) {
    if (!(w[j] > 0.0) || !isfinite(w[j])) return fail(c, LW_EINVAL, "frequency %d is not finite and > 0", j);
    wt[j] = w[j] / (2.0 * M_PI);
  }
  DeviceGuard g(c->device);
  LW_HIP(hipStreamSynchronize(c->stream), "sync");
  free_dev(c->d_wturn);
  free_dev(c->d_omega);
  c->d_wturn = c->d_omega = nullptr;
  LW_HIP(hipMalloc(&c->d_wturn, nw * sizeof(double)), "hipMalloc(omega)");
  LW_HIP(hipMalloc(&c->d_omega, nw * sizeof(double)), "hipMalloc(omega)");
  LW_HIP(hipMemcpy(c->d_wturn, wt.data(), nw * sizeof(double), hipMemcpyHostToDevice), "copy omega");
  LW_HIP(hipMemcpy(c->d_omega, w.data(), nw * sizeof(double), hipMemcpyHostToDevice), "copy omega");
  c->h_omega = w;
  c->nw = nw;
  lw::mfma_cache_invalidate(c->mfma);
  return alloc_accumulator(c);
}

lw_status lw_set_log_frequencies(lw_ctx* c, double wmin, double wmax, int32_t nw) {
  if (!c) return LW_EINVAL;
  if (!(wmin > 0.0) || !(wmax >= wmin) || !isfinite(wmax) || nw <= 0)
    return fail(c, LW_EINVAL, "need 0 < wmin <= wmax and nw > 0");
  std::vector<double> w(nw);
  for (int32_t j = 0; j < nw; ++j)
    w[j] = nw == 1 ? wmin : wmin * pow(wmax / wmin, (double)j / (double)(nw - 1));
  w[0] = wmin;
  if (nw > 1) w[nw - 1] = wmax;
  return lw_set_frequencies(c, w.data(), nw);
}

lw_status lw_get_frequencies(const lw_ctx* c, double* out) {
  if (!c || !out) return LW_EINVAL;
  memcpy(out, c->h_omega.data(), c->h_omega.size() * sizeof(double));
  return LW_OK;
}

lw_status lw_set_species(lw_ctx* c, int32_t ns) {
  if (!c) return LW_EINVAL;
  if (ns < 1 || ns > lw::kMaxSpecies)
    return fail(c, LW_EINVAL, "n_species must be in [1, %d]", lw::kMaxSpecies);
  DeviceGuard g(c->device);
  LW_HIP(hipStreamSynchronize(c->stream), "sync");
  c->ns = ns;
  return alloc_accumulator(c);
}

lw_status lw_workspace_size(lw_ctx* c, const lw_batch* b, lw_path path, size_t* bytes) {
  if (!c || !bytes) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  path = resolve_path(c, path, false);
  if (!b || b->n_particles < 0) return fail(c, LW_EINVAL, "bad batch");
  *bytes = 0;
  if (path == LW_PATH_FP32) {
    DirectShape s = direct_shape(c, b->n_particles);
    *bytes = align256((size_t)s.n_blocks * c->ns * c->nd * c->nw * lw::direct_ncomp(c) *
                      sizeof(double));
    return LW_OK;
  }
  if (path == LW_PATH_MFMA_F16 || path == LW_PATH_MFMA_BF16) {
    DeviceGuard g(c->device);
    return lw::mfma_workspace_size(c, b, path, bytes);
  }
  return fail(c, LW_EINVAL, "unknown path %d", (int)path);
}

lw_status lw_accumulate(lw_ctx* c, const lw_batch* b, lw_path path, void* ws, size_t ws_bytes,
                        float* per_particle) {
  if (!c) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  st = check_batch(c, b);
  if (st != LW_OK) return st;
  if (b->n_particles == 0) return LW_OK;
  path = resolve_path(c, path, per_particle != nullptr);
  size_t need = 0;
  if (path == LW_PATH_MFMA_F16 || path == LW_PATH_MFMA_BF16) {
    DeviceGuard g0(c->device);
    st = lw::mfma_workspace_need(c, b, path, &need);  // no synchronisation for a planned batch
  } else {
    st = lw_workspace_size(c, b, path, &need);
  }
  if (st != LW_OK) return st;
  if (need > 0 && (!ws || ws_bytes < need))
    return fail(c, LW_ENOMEM, "workspace too small: need %zu bytes, got %zu", need, ws_bytes);
  if (((uintptr_t)ws & 255) != 0) return fail(c, LW_EINVAL, "workspace must be 256-byte aligned");
  DeviceGuard g(c->device);
  if (path == LW_PATH_FP32) {
    DirectShape s = direct_shape(c, b->n_particles);
    lw::DirectArgs a;
    a.b = lw::view_of(b);
    a.dirs = c->d_dirs;
    a.wturn = c->d_wturn;
    a.nd = c->nd;
    a.nw = c->nw;
    a.ns = c->ns;
    a.ncomp = lw::direct_ncomp(c);
    a.pb = s.pb;
    a.n_blocks = s.n_blocks;
    a.n_tiles = s.n_tiles;
    a.partial = (double*)ws;
    a.per_particle = per_particle;
    a.amp = nullptr;
    a.err = c->d_err;
    a.perm = nullptr;
    a.order = nullptr;
    a.ticket = nullptr;
    a.n_items = 0;
    const auto& pl = c->plan;
    const bool persistent = c->tune_persistent && pl.valid && pl.offsets == (const void*)b->offsets &&
                            pl.n == b->n_particles && pl.nd == c->nd && pl.nw == c->nw &&
                            pl.ns == c->ns && pl.ncomp == a.ncomp && pl.wpt == s.wpt &&
                            pl.pb == s.pb;
    LW_HIP(lw::prof_begin(c, lw::kProfDirect), "profile");
    if (persistent) {
      a.perm = pl.d_perm;
      a.order = pl.d_order;
      a.ticket = c->d_ticket;
      a.n_items = pl.n_items;
      if (c->prof && !c->capturing) {
        if (c->wgtime_cap < pl.workgroups) {
          free_dev(c->d_wgtime);
          c->wgtime_cap = 0;
          LW_HIP(hipMalloc(&c->d_wgtime, 3 * sizeof(unsigned long long) * (size_t)pl.workgroups),
                 "hipMalloc(work-group timing)");
          c->wgtime_cap = pl.workgroups;
        }
        a.wg_time = c->d_wgtime;
        c->wgtime_n = pl.workgroups;
      }
      LW_HIP(lw::launch_fill_u32(c->d_ticket, 1, 0u, c->stream), "reset ticket");
      LW_HIP(lw::launch_direct_f32_persistent(a, s.wpt, pl.workgroups, c->stream),
             "launch lw_direct_f32 (persistent)");
    } else {
      LW_HIP(lw::launch_direct_f32(a, s.wpt, c->stream), "launch lw_direct_f32");
    }
    LW_HIP(lw::prof_end(c), "profile");
    LW_HIP(lw::launch_reduce_partials(a.partial, s.n_blocks,
                                      (int64_t)c->ns * c->nd * c->nw * a.ncomp, direct_target(c),
                                      c->stream),
           "launch lw_reduce_partials");
  } else if (path == LW_PATH_MFMA_F16 || path == LW_PATH_MFMA_BF16) {
    st = lw::mfma_accumulate(c, b, path, ws, ws_bytes, per_particle);
    if (st != LW_OK) return st;
  } else {
    return fail(c, LW_EINVAL, "unknown path %d", (int)path);
  }
  c->calls += 1;
  return LW_OK;
}

lw_status lw_accumulate_noalloc(lw_ctx* c, const lw_batch* b) {
  if (!c) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  st = check_batch(c, b);
  if (st != LW_OK) return st;
  if (b->n_particles == 0) return LW_OK;
  const DirectShape s = direct_shape(c, b->n_particles);
  const int ncomp = lw::direct_ncomp(c);
  const size_t need = (size_t)s.n_blocks * c->ns * c->nd * c->nw * ncomp * sizeof(double);
  if (need > kNoallocScratchBytes)
    return fail(c, LW_ENOMEM,
                "the batch needs %zu bytes of partial sums, more than the %zu-byte static scratch of "
                "lw_accumulate_noalloc: split the batch or use lw_accumulate with a workspace",
                need, kNoallocScratchBytes);
  void* sp = nullptr;
  st = scratch_on(c, &sp);  // found by lw_create: a lookup, no allocation
  if (st != LW_OK) return st;
  DeviceGuard g(c->device);
  lw::DirectArgs a;
  a.b = lw::view_of(b);
  a.dirs = c->d_dirs;
  a.wturn = c->d_wturn;
  a.nd = c->nd;
  a.nw = c->nw;
  a.ns = c->ns;
  a.ncomp = ncomp;
  a.pb = s.pb;
  a.n_blocks = s.n_blocks;
  a.n_tiles = s.n_tiles;
  a.partial = (double*)sp;  // every row is written by its item before the reduction reads it
  a.per_particle = nullptr;
  a.amp = nullptr;
  a.err = c->d_err;
  a.perm = nullptr;
  a.order = nullptr;
  a.ticket = nullptr;
  a.n_items = 0;
  LW_HIP(lw::launch_direct_f32(a, s.wpt, c->stream), "launch lw_direct_f32 (no allocation)");
  LW_HIP(lw::launch_reduce_partials(a.partial, s.n_blocks, (int64_t)c->ns * c->nd * c->nw * ncomp,
                                    direct_target(c), c->stream),
         "launch lw_reduce_partials");
  c->calls += 1;
  return LW_OK;
}

lw_status lw_read_spectra(lw_ctx* c, double* out) {
  if (!c || !out) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  DeviceGuard g(c->device);
  size_t n = (size_t)c->ns * c->nd * c->nw;
  if (c->coherent)
    LW_HIP(lw::launch_coherent_power(c->d_A, (int64_t)n, c->d_S, c->stream), "launch coherent power");
  LW_HIP(hipMemcpyAsync(out, c->d_S, n * sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy S");
  return read_device_errors(c);
}

lw_status lw_reset(lw_ctx* c) {
  if (!c) return LW_EINVAL;
  DeviceGuard g(c->device);
  if (c->d_S)
    LW_HIP(lw::launch_fill_f64(c->d_S, (int64_t)c->ns * c->nd * c->nw, 0.0, c->stream), "zero S");
  if (c->d_A)
    LW_HIP(lw::launch_fill_f64(c->d_A, (int64_t)4 * c->ns * c->nd * c->nw, 0.0, c->stream), "zero A");
  LW_HIP(lw::launch_fill_u64(c->d_err, 2, kNoError, c->stream), "reset error records");
  return LW_OK;
}

lw_status lw_load_accumulator(lw_ctx* c, const double* in) {
  if (!c || !in) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  if (c->coherent)
    return fail(c, LW_ESTATE, "coherent synthesis keeps amplitudes: use lw_load_amplitudes");
  DeviceGuard g(c->device);
  size_t n = (size_t)c->ns * c->nd * c->nw;
  LW_HIP(hipMemcpyAsync(c->d_S, in, n * sizeof(double), hipMemcpyHostToDevice, c->stream), "load S");
  LW_HIP(hipStreamSynchronize(c->stream), "sync");
  return LW_OK;
}

lw_status lw_save_accumulator(lw_ctx* c, const char* path) {
  if (!c || !path) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  DeviceGuard g(c->device);
  const size_t n = (size_t)c->ns * c->nd * c->nw * (c->coherent ? 4 : 1);
  std::vector<double> acc(n);
  LW_HIP(hipMemcpyAsync(acc.data(), c->coherent ? c->d_A : c->d_S, n * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream),
         "copy accumulator");
  LW_HIP(hipStreamSynchronize(c->stream), "sync");
  lw::Bytes b;
  for (int d = 0; d < c->nd; ++d) b.put(&c->h_dirs[(size_t)lw::kDirStride * d], 3 * sizeof(double));
  b.put(c->h_omega.data(), c->nw * sizeof(double));
  b.put(acc.data(), n * sizeof(double));
  const int64_t f[5] = {c->ns, c->nd, c->nw, c->coherent ? 1 : 0, 0};
  if (!lw::write_lw_file(path, "LWACC001", f, b)) return fail(c, LW_EINVAL, "cannot write %s", path);
  return LW_OK;
}

lw_status lw_load_accumulator_file(lw_ctx* c, const char* path) {
  if (!c || !path) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  lw::FileHeader h;
  lw::Bytes b;
  std::string why;
  if (!lw::read_lw_file(path, "LWACC001", &h, &b, &why)) return fail(c, LW_EINVAL, "%s: %s", path, why.c_str());
  if (h.f[0] != c->ns || h.f[1] != c->nd || h.f[2] != c->nw || h.f[3] != (c->coherent ? 1 : 0))
    return fail(c, LW_EINVAL, "%s holds %lld species x %lld directions x %lld frequencies (%s), the context "
                "%d x %d x %d (%s)", path, (long long)h.f[0], (long long)h.f[1], (long long)h.f[2],
                h.f[3] ? "coherent" : "incoherent", c->ns, c->nd, c->nw, c->coherent ? "coherent" : "incoherent");
  const size_t n = (size_t)c->ns * c->nd * c->nw * (c->coherent ? 4 : 1);
  if (b.v.size() != (3 * (size_t)c->nd + c->nw + n) * sizeof(double))
    return fail(c, LW_EINVAL, "%s: payload length does not match its header", path);
  for (int d = 0; d < c->nd; ++d) {
    double nv[3];
    b.get(nv, sizeof(nv));
    if (memcmp(nv, &c->h_dirs[(size_t)lw::kDirStride * d], sizeof(nv)) != 0)
      return fail(c, LW_EINVAL, "%s: direction %d differs from the context's", path, d);
  }
  std::vector<double> om(c->nw);
  b.get(om.data(), c->nw * sizeof(double));
  if (memcmp(om.data(), c->h_omega.data(), c->nw * sizeof(double)) != 0)
    return fail(c, LW_EINVAL, "%s: frequencies differ from the context's", path);
  std::vector<double> acc(n);
  b.get(acc.data(), n * sizeof(double));
  DeviceGuard g(c->device);
  LW_HIP(hipMemcpyAsync(c->coherent ? c->d_A : c->d_S, acc.data(), n * sizeof(double), hipMemcpyHostToDevice,
                        c->stream),
         "load accumulator");
  LW_HIP(hipStreamSynchronize(c->stream), "sync");
  return LW_OK;
}

lw_status lw_set_mfma_options(lw_ctx* c, int32_t bands, int32_t products_f16,
                              int32_t products_bf16) {
  if (!c) return LW_EINVAL;
  return lw::mfma_set_options(c, bands, products_f16, products_bf16);
}

lw_status lw_set_mfma_chunk_bytes(lw_ctx* c, int64_t bytes) {
  if (!c) return LW_EINVAL;
  return lw::mfma_set_chunk_bytes(c, bytes);
}

lw_status lw_mfma_plan_info(lw_ctx* c, const lw_batch* b, lw_path path, int64_t* host_out) {
  if (!c || !host_out) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  st = check_batch(c, b);
  if (st != LW_OK) return st;
  path = resolve_path(c, path, false);
  if (path != LW_PATH_MFMA_F16 && path != LW_PATH_MFMA_BF16)
    return fail(c, LW_EINVAL, "plan information is for the matrix-core paths");
  DeviceGuard g(c->device);
  return lw::mfma_plan_info(c, b, path, host_out);
}

lw_status lw_set_profiling(lw_ctx* c, int32_t enable) {
  if (!c) return LW_EINVAL;
  DeviceGuard g(c->device);
  if (enable && !c->d_flops) {
    LW_HIP(hipMalloc(&c->d_flops, sizeof(unsigned long long)), "hipMalloc(flops)");
    LW_HIP(lw::launch_fill_u64(c->d_flops, 1, 0ull, c->stream), "zero flops");
  }
  c->prof = enable != 0;
  return LW_OK;
}

lw_status lw_profile_read(lw_ctx* c, double* out) {
  if (!c || !out) return LW_EINVAL;
  DeviceGuard g(c->device);
  LW_HIP(hipStreamSynchronize(c->stream), "sync");
  double ms[lw::kProfKinds] = {0, 0, 0};
  double n[lw::kProfKinds] = {0, 0, 0};
  for (auto& m : c->ev_marks) {
    float t = 0.f;
    LW_HIP(hipEventElapsedTime(&t, m.second.first, m.second.second), "event time");
    ms[m.first] += t;
    n[m.first] += 1;
  }
  unsigned long long fl = 0;
  if (c->d_flops) {
    LW_HIP(hipMemcpy(&fl, c->d_flops, sizeof(fl), hipMemcpyDeviceToHost), "copy flops");
    LW_HIP(lw::launch_fill_u64(c->d_flops, 1, 0ull, c->stream), "zero flops");
    LW_HIP(hipStreamSynchronize(c->stream), "sync");
  }
  out[0] = ms[lw::kProfDirect];
  out[1] = ms[lw::kProfSpread];
  out[2] = ms[lw::kProfGemm];
  out[3] = (double)fl * c->flop_mult;
  out[4] = n[lw::kProfDirect];
  out[5] = n[lw::kProfGemm];
  out[6] = n[lw::kProfSpread];
  c->ev_marks.clear();
  c->ev_used = 0;
  return LW_OK;
}

lw_status lw_profile_cu_busy(lw_ctx* c, double* out) {
  if (!c || !out) return LW_EINVAL;
  if (c->wgtime_n <= 0 || !c->d_wgtime)
    return fail(c, LW_ESTATE, "no persistent FP32 launch was made with profiling on");
  DeviceGuard g(c->device);
  std::vector<unsigned long long> h(3 * (size_t)c->wgtime_n);
  LW_HIP(hipStreamSynchronize(c->stream), "sync");
  LW_HIP(hipMemcpy(h.data(), c->d_wgtime, h.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost),
         "copy work-group timing");
  int khz = 0;
  LW_HIP(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, c->device), "wall clock rate");
  if (khz <= 0) return fail(c, LW_EDEVICE, "device reports no wall clock rate");
  std::vector<double> busy(1u << 12, 0.0);
  std::vector<char> seen(1u << 12, 0);
  for (int w = 0; w < c->wgtime_n; ++w) {
    const unsigned key = (unsigned)(h[3 * w] & 0xfffu);
    const unsigned long long t0 = h[3 * w + 1], t1 = h[3 * w + 2];
    busy[key] += t1 > t0 ? (double)(t1 - t0) : 0.0;
    seen[key] = 1;
  }
  double n = 0, lo = 0, hi = 0, sum = 0;
  for (size_t k = 0; k < busy.size(); ++k) {
    if (!seen[k]) continue;
    const double ms = busy[k] / (double)khz;
    lo = n == 0 ? ms : std::min(lo, ms);
    hi = n == 0 ? ms : std::max(hi, ms);
    sum += ms;
    n += 1;
  }
  out[0] = n;
  out[1] = lo;
  out[2] = n > 0 ? sum / n : 0.0;
  out[3] = hi;
  return LW_OK;
}

lw_status lw_plan_batch(lw_ctx* c, const lw_batch* b, lw_path path) {
  if (!c) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  st = check_batch(c, b);
  if (st != LW_OK) return st;
  DeviceGuard g(c->device);
  path = resolve_path(c, path, false);
  if (path == LW_PATH_MFMA_F16 || path == LW_PATH_MFMA_BF16) {
    size_t bytes = 0;
    return lw::mfma_workspace_size(c, b, path, &bytes);  // sizes the grids and phase tables
  }
  if (path != LW_PATH_FP32) return fail(c, LW_EINVAL, "unknown path %d", (int)path);
  auto& pl = c->plan;
  pl.valid = false;
  c->epoch += 1;  // the plan's buffers are refilled (and may move)
  const int64_t P = b->n_particles;
  if (P == 0) return LW_OK;
  std::vector<int64_t> off(P + 1);
  LW_HIP(hipMemcpyAsync(off.data(), b->offsets, (P + 1) * sizeof(int64_t), hipMemcpyDeviceToHost,
                        c->stream),
         "copy offsets");
  LW_HIP(hipStreamSynchronize(c->stream), "sync");
  std::vector<int64_t> perm(P);
  for (int64_t p = 0; p < P; ++p) {
    if (off[p + 1] < off[p]) return fail(c, LW_EINVAL, "offsets decrease at particle %lld", (long long)p);
    perm[p] = p;
  }
  // longest trajectories first; equal lengths keep index order
  std::stable_sort(perm.begin(), perm.end(), [&](int64_t x, int64_t y) {
    return off[x + 1] - off[x] > off[y + 1] - off[y];
  });
  const DirectShape s = direct_shape(c, P);
  std::vector<int64_t> cost(s.n_blocks, 0);
  for (int64_t i = 0; i < P; ++i) cost[i / s.pb] += off[perm[i] + 1] - off[perm[i]] + 1;
  const int64_t n_items = s.n_blocks * (int64_t)c->nd * s.n_tiles;
  std::vector<int64_t> order(n_items);
  for (int64_t i = 0; i < n_items; ++i) order[i] = i;
  // item id = (block * nd + d) * n_tiles + tile; heaviest blocks first
  const int64_t per_block = (int64_t)c->nd * s.n_tiles;
  std::stable_sort(order.begin(), order.end(),
                   [&](int64_t x, int64_t y) { return cost[x / per_block] > cost[y / per_block]; });
  if (pl.perm_cap < (size_t)P) {
    free_dev(pl.d_perm);
    pl.d_perm = nullptr;
    pl.perm_cap = 0;
    LW_HIP(hipMalloc(&pl.d_perm, P * sizeof(int64_t)), "hipMalloc(perm)");
    pl.perm_cap = P;
  }
  if (pl.order_cap < (size_t)n_items) {
    free_dev(pl.d_order);
    pl.d_order = nullptr;
    pl.order_cap = 0;
    LW_HIP(hipMalloc(&pl.d_order, n_items * sizeof(int64_t)), "hipMalloc(order)");
    pl.order_cap = n_items;
  }
  if (!c->d_ticket) LW_HIP(hipMalloc(&c->d_ticket, sizeof(unsigned)), "hipMalloc(ticket)");
  LW_HIP(hipMemcpy(pl.d_perm, perm.data(), P * sizeof(int64_t), hipMemcpyHostToDevice), "copy perm");
  LW_HIP(hipMemcpy(pl.d_order, order.data(), n_items * sizeof(int64_t), hipMemcpyHostToDevice),
         "copy order");
  hipDeviceProp_t prop;
  LW_HIP(hipGetDeviceProperties(&prop, c->device), "device properties");
  const size_t shmem = lw::direct_lds(c->ns, lw::direct_ncomp(c), s.wpt);
  const int per_cu = lw::direct_persistent_occupancy(s.wpt, shmem);
  pl.workgroups = (int)std::min<int64_t>((int64_t)prop.multiProcessorCount * per_cu, n_items);
  pl.offsets = (const void*)b->offsets;
  pl.n = P;
  pl.nd = c->nd;
  pl.nw = c->nw;
  pl.ns = c->ns;
  pl.ncomp = lw::direct_ncomp(c);
  pl.wpt = s.wpt;
  pl.pb = s.pb;
  pl.n_tiles = s.n_tiles;
  pl.n_blocks = s.n_blocks;
  pl.n_items = n_items;
  pl.valid = true;
  return LW_OK;
}

// ------------------------------------------------------------------ particle subsets as batches
namespace {

constexpr int kScanThreads = 1024;

// dst[0] = 0 and dst[i + 1] = the summed lengths of particles idx[0] .. idx[i]: one work-group
// walks the list in runs of 1024, an inclusive scan per wave by shuffles and one lane adding
// the sixteen wave totals in order.  An index outside [0, P), or a particle with a negative
// length, counts as empty and sets *bad.
__global__ __launch_bounds__(kScanThreads) void subset_offsets_kernel(const int64_t* offsets, int64_t P,
                                                                      const int64_t* idx, int64_t n,
                                                                      int64_t* dst, unsigned* bad) {
  __shared__ int64_t s_wave[kScanThreads / 64];
  __shared__ int64_t s_carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) {
    s_carry = 0;
    dst[0] = 0;
  }
  __syncthreads();
  for (int64_t base = 0; base < n; base += kScanThreads) {
    const int64_t i = base + tid;
    int64_t len = 0;
    if (i < n) {
      const int64_t p = idx[i];
      if (p >= 0 && p < P) len = offsets[p + 1] - offsets[p];
      if (p < 0 || p >= P || len < 0) {
        len = 0;
        atomicOr(bad, 1u);
      }
    }
    int64_t v = len;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t u = __shfl_up(v, off);
      if (lane >= off) v += u;
    }
    if (lane == 63) s_wave[wave] = v;
    __syncthreads();
    if (tid == 0) {
      int64_t run = s_carry;
      for (int w = 0; w < kScanThreads / 64; ++w) {
        const int64_t t = s_wave[w];
        s_wave[w] = run;
        run += t;
      }
      s_carry = run;
    }
    __syncthreads();
    if (i < n) dst[i + 1] = s_wave[wave] + v;
    __syncthreads();  // the next run rewrites s_wave
  }
}

struct GatherArgs {
  lw::BatchView src;
  const int64_t* idx;
  const int64_t* dst_offsets;
  double *x, *y, *z, *bx, *by, *bz;
  float *ax, *ay, *az;      // FP32 d(beta)/dt, or null
  double *adx, *ady, *adz;  // FP64 d(beta)/dt, or null
  double *t0, *dt;
  float *charge, *weight;
  int32_t* species;         // null when the destination has none
};

// One work-group per listed particle copies its samples (the shorter of its length in the
// source and its slot in the destination, so that both stay in bounds) and its per-particle
// values; an index outside the source is skipped.
__global__ __launch_bounds__(256) void gather_particles_kernel(GatherArgs a) {
  const int64_t i = blockIdx.x;
  const int64_t p = a.idx[i];
  if (p < 0 || p >= a.src.n_particles) return;
  const int64_t so = a.src.offsets[p], d0 = a.dst_offsets[i];
  const int64_t len = min(a.src.offsets[p + 1] - so, a.dst_offsets[i + 1] - d0);
  for (int64_t k = threadIdx.x; k < len; k += blockDim.x) {
    a.x[d0 + k] = a.src.x[so + k];
    a.y[d0 + k] = a.src.y[so + k];
    a.z[d0 + k] = a.src.z[so + k];
    a.bx[d0 + k] = a.src.bx[so + k];
    a.by[d0 + k] = a.src.by[so + k];
    a.bz[d0 + k] = a.src.bz[so + k];
    if (a.adx) {
      a.adx[d0 + k] = a.src.adx[so + k];
      a.ady[d0 + k] = a.src.ady[so + k];
      a.adz[d0 + k] = a.src.adz[so + k];
    } else {
      a.ax[d0 + k] = a.src.ax[so + k];
      a.ay[d0 + k] = a.src.ay[so + k];
      a.az[d0 + k] = a.src.az[so + k];
    }
  }
  if (threadIdx.x == 0) {
    a.t0[i] = a.src.t0[p];
    a.dt[i] = a.src.dt[p];
    a.charge[i] = a.src.charge[p];
    a.weight[i] = a.src.weight[p];
    if (a.species) a.species[i] = a.src.species ? a.src.species[p] : 0;
  }
}

}  // namespace

lw_status lw_subset_offsets(lw_ctx* c, const lw_batch* b, const int64_t* indices, int64_t n,
                            int64_t* dst_offsets, int64_t* host_total) {
  if (!c) return LW_EINVAL;
  lw_status st = check_batch(c, b);
  if (st != LW_OK) return st;
  if (n < 0 || (n > 0 && !indices) || !dst_offsets || !host_total) return fail(c, LW_EINVAL, "bad index list");
  if (c->capturing) return fail(c, LW_ESTATE, "lw_subset_offsets synchronises: not inside graph capture");
  DeviceGuard g(c->device);
  if (!c->d_flag) LW_HIP(hipMalloc(&c->d_flag, sizeof(unsigned)), "hipMalloc(flag)");
  LW_HIP(lw::launch_fill_u32(c->d_flag, 1, 0u, c->stream), "clear flag");
  hipLaunchKernelGGL(subset_offsets_kernel, dim3(1), dim3(kScanThreads), 0, c->stream, b->offsets,
                     b->n_particles, indices, n, dst_offsets, c->d_flag);
  LW_HIP(hipGetLastError(), "launch subset_offsets");
  int64_t total = 0;
  unsigned bad = 0;
  LW_HIP(hipMemcpyAsync(&total, dst_offsets + n, sizeof(int64_t), hipMemcpyDeviceToHost, c->stream), "read total");
  LW_HIP(hipMemcpyAsync(&bad, c->d_flag, sizeof(unsigned), hipMemcpyDeviceToHost, c->stream), "read flag");
  LW_HIP(hipStreamSynchronize(c->stream), "synchronise");
  if (bad) return fail(c, LW_EINVAL, "index outside the batch, or a particle of negative length");
  *host_total = total;
  return LW_OK;
}

lw_status lw_gather_particles(lw_ctx* c, const lw_batch* b, const int64_t* indices, int64_t n,
                              const lw_batch* dst) {
  if (!c) return LW_EINVAL;
  lw_status st = check_batch(c, b);
  if (st != LW_OK) return st;
  if (n < 0 || (n > 0 && !indices) || !dst) return fail(c, LW_EINVAL, "bad index list or destination");
  if (n == 0) return LW_OK;
  if (dst->n_particles != n) return fail(c, LW_EINVAL, "destination holds %lld particles, not %lld",
                                         (long long)dst->n_particles, (long long)n);
  st = check_batch(c, dst);
  if (st != LW_OK) return st;
  if ((dst->flags & LW_BATCH_F64_ACCEL) != (b->flags & LW_BATCH_F64_ACCEL))
    return fail(c, LW_EINVAL, "source and destination differ in the precision of d(beta)/dt");
  if (n > 0x7fffffffLL) return fail(c, LW_EINVAL, "at most 2^31 - 1 particles per gather");
  DeviceGuard g(c->device);
  GatherArgs a;
  a.src = lw::view_of(b);
  a.idx = indices;
  a.dst_offsets = dst->offsets;
  // the destination's arrays are the caller's, written here (lw_batch declares them const
  // for the calls that only read)
  a.x = const_cast<double*>(dst->x);
  a.y = const_cast<double*>(dst->y);
  a.z = const_cast<double*>(dst->z);
  a.bx = const_cast<double*>(dst->bx);
  a.by = const_cast<double*>(dst->by);
  a.bz = const_cast<double*>(dst->bz);
  const lw::BatchView dv = lw::view_of(dst);
  a.ax = const_cast<float*>(dv.ax);
  a.ay = const_cast<float*>(dv.ay);
  a.az = const_cast<float*>(dv.az);
  a.adx = const_cast<double*>(dv.adx);
  a.ady = const_cast<double*>(dv.ady);
  a.adz = const_cast<double*>(dv.adz);
  a.t0 = const_cast<double*>(dst->t0);
  a.dt = const_cast<double*>(dst->dt);
  a.charge = const_cast<float*>(dst->charge);
  a.weight = const_cast<float*>(dst->weight);
  a.species = const_cast<int32_t*>(dst->species);
  hipLaunchKernelGGL(gather_particles_kernel, dim3((unsigned)n), dim3(256), 0, c->stream, a);
  LW_HIP(hipGetLastError(), "launch gather_particles");
  return LW_OK;
}

lw_status lw_accumulate_subset(lw_ctx* c, const lw_batch* b, const int64_t* indices, int64_t n_idx,
                               void* ws, size_t ws_bytes, float* per_particle) {
  if (!c) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  st = check_batch(c, b);
  if (st != LW_OK) return st;
  if (n_idx < 0 || (n_idx > 0 && !indices)) return fail(c, LW_EINVAL, "bad index list");
  if (n_idx == 0) return LW_OK;
  const DirectShape s = direct_shape(c, n_idx);
  const int ncomp = lw::direct_ncomp(c);
  const size_t need =
      align256((size_t)s.n_blocks * c->ns * c->nd * c->nw * ncomp * sizeof(double));
  if (!ws || ws_bytes < need)
    return fail(c, LW_ENOMEM, "workspace too small: need %zu bytes, got %zu", need, ws_bytes);
  DeviceGuard g(c->device);
  lw::DirectArgs a;
  // the kernel walks n_idx positions and maps each through the index list
  a.b = lw::view_of(b);
  a.b.n_particles = n_idx;
  a.dirs = c->d_dirs;
  a.wturn = c->d_wturn;
  a.nd = c->nd;
  a.nw = c->nw;
  a.ns = c->ns;
  a.ncomp = ncomp;
  a.pb = s.pb;
  a.n_blocks = s.n_blocks;
  a.n_tiles = s.n_tiles;
  a.partial = (double*)ws;
  a.per_particle = per_particle;
  a.amp = nullptr;
  a.err = c->d_err;
  a.perm = indices;
  a.order = nullptr;
  a.ticket = nullptr;
  a.n_items = 0;
  LW_HIP(lw::prof_begin(c, lw::kProfDirect), "profile");
  LW_HIP(lw::launch_direct_f32(a, s.wpt, c->stream), "launch lw_direct_f32 (subset)");
  LW_HIP(lw::prof_end(c), "profile");
  LW_HIP(lw::launch_reduce_partials(a.partial, s.n_blocks, (int64_t)c->ns * c->nd * c->nw * ncomp,
                                    direct_target(c), c->stream),
         "launch lw_reduce_partials");
  c->calls += 1;
  return LW_OK;
}

lw_status lw_set_tuning(lw_ctx* c, int32_t wpt, int32_t pb, int32_t persistent, int32_t bands,
                        int32_t tile) {
  if (!c) return LW_EINVAL;
  if (wpt != 0 && wpt != 1 && wpt != 2 && wpt != 4 && wpt != 8)
    return fail(c, LW_EINVAL, "frequencies per thread must be 0 (automatic), 1, 2, 4 or 8");
  if (pb < 0 || pb > 4096) return fail(c, LW_EINVAL, "particles per item must be in [0, 4096]");
  if (tile < 0 || tile > 4)
    return fail(c, LW_EINVAL,
                "contraction tile must be 0 (keep), 1 (128x128), 2 (256x128), 3 (128x256) or 4 (256x256)");
  c->tune_wpt = wpt;
  c->tune_pb = pb;
  c->tune_persistent = persistent ? 1 : 0;
  lw_status st = LW_OK;
  if (bands > 0) st = lw::mfma_set_bands(c, bands);
  if (st == LW_OK && tile > 0) st = lw::mfma_set_tile(c, tile);
  return st;
}

lw_status lw_graph_capture(lw_ctx* c, const lw_batch* b, lw_path path, void* ws, size_t ws_bytes,
                           lw_graph** out) {
  if (!c || !out) return LW_EINVAL;
  *out = nullptr;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  st = check_batch(c, b);
  if (st != LW_OK) return st;
  DeviceGuard g(c->device);
  path = resolve_path(c, path, false);
  if (path == LW_PATH_MFMA_F16 || path == LW_PATH_MFMA_BF16) {
    size_t bytes = 0;
    st = lw::mfma_workspace_size(c, b, path, &bytes);  // plan the grids outside the capture
    if (st != LW_OK) return st;
  }
  hipStream_t cs = nullptr;
  LW_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "create capture stream");
  hipStream_t saved = c->stream;
  const bool prof = c->prof;
  c->stream = cs;
  c->prof = false;
  c->capturing = true;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    st = lw_accumulate(c, b, path, ws, ws_bytes, nullptr);
    hipError_t e2 = hipStreamEndCapture(cs, &graph);
    if (e2 != hipSuccess && st == LW_OK) st = hip_fail(c, e2, "end capture");
  } else {
    st = hip_fail(c, e, "begin capture");
  }
  c->capturing = false;
  c->prof = prof;
  c->stream = saved;
  (void)hipStreamDestroy(cs);
  if (st != LW_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  lw_graph* gr = new lw_graph();
  gr->ctx = c;
  gr->graph = graph;
  gr->epoch = c->epoch;
  gr->mfma_epoch = lw::mfma_epoch(c->mfma);
  e = hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(graph);
    delete gr;
    return hip_fail(c, e, "instantiate graph");
  }
  *out = gr;
  return LW_OK;
}

lw_status lw_graph_launch(lw_graph* gr) {
  if (!gr || !gr->ctx) return LW_EINVAL;
  lw_ctx* c = gr->ctx;
  if (gr->epoch != c->epoch || gr->mfma_epoch != lw::mfma_epoch(c->mfma))
    return fail(c, LW_ESTATE,
                "the context's accumulators, grids, tables or plan changed since this graph was "
                "captured: capture it again");
  DeviceGuard g(c->device);
  LW_HIP(hipGraphLaunch(gr->exec, c->stream), "launch graph");
  c->calls += 1;
  return LW_OK;
}

void lw_graph_destroy(lw_graph* gr) {
  if (!gr) return;
  if (gr->ctx) {
    DeviceGuard g(gr->ctx->device);
    (void)hipStreamSynchronize(gr->ctx->stream);
  }
  if (gr->exec) (void)hipGraphExecDestroy(gr->exec);
  if (gr->graph) (void)hipGraphDestroy(gr->graph);
  delete gr;
}

lw_status lw_set_coherent(lw_ctx* c, int32_t coherent) {
  if (!c) return LW_EINVAL;
  DeviceGuard g(c->device);
  LW_HIP(hipStreamSynchronize(c->stream), "sync");
  c->coherent = coherent != 0;
  return alloc_accumulator(c);
}

lw_status lw_get_basis(const lw_ctx* c, double* out) {
  if (!c || !out) return LW_EINVAL;
  if (c->nd <= 0) return LW_ESTATE;
  memcpy(out, c->h_dirs.data(), c->h_dirs.size() * sizeof(double));
  return LW_OK;
}

lw_status lw_read_amplitudes(lw_ctx* c, double* out) {
  if (!c || !out) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  if (!c->coherent) return fail(c, LW_ESTATE, "amplitudes are kept in coherent synthesis only");
  DeviceGuard g(c->device);
  size_t n = (size_t)4 * c->ns * c->nd * c->nw;
  LW_HIP(hipMemcpyAsync(out, c->d_A, n * sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy A");
  return read_device_errors(c);
}

lw_status lw_load_amplitudes(lw_ctx* c, const double* in) {
  if (!c || !in) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  if (!c->coherent) return fail(c, LW_ESTATE, "amplitudes are kept in coherent synthesis only");
  DeviceGuard g(c->device);
  size_t n = (size_t)4 * c->ns * c->nd * c->nw;
  LW_HIP(hipMemcpyAsync(c->d_A, in, n * sizeof(double), hipMemcpyHostToDevice, c->stream), "load A");
  LW_HIP(hipStreamSynchronize(c->stream), "sync");
  return LW_OK;
}

lw_status lw_accumulate_amplitudes(lw_ctx* c, const lw_batch* b, lw_path path, void* ws,
                                   size_t ws_bytes, double* amp) {
  if (!c) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  st = check_batch(c, b);
  if (st != LW_OK) return st;
  if (b->n_particles == 0) return LW_OK;
  if (!amp) return fail(c, LW_EINVAL, "amplitude state is NULL");
  if (((uintptr_t)amp & 15) != 0) return fail(c, LW_EINVAL, "amplitude state must be 16-byte aligned");
  DeviceGuard g(c->device);
  path = resolve_path(c, path, false);
  if (path == LW_PATH_MFMA_F16 || path == LW_PATH_MFMA_BF16) {
    size_t need = 0;
    st = lw::mfma_workspace_need(c, b, path, &need);  // no synchronisation for a planned batch
    if (st != LW_OK) return st;
    if (!ws || ws_bytes < need)
      return fail(c, LW_ENOMEM, "workspace too small: need %zu bytes, got %zu", need, ws_bytes);
    if (((uintptr_t)ws & 255) != 0) return fail(c, LW_EINVAL, "workspace must be 256-byte aligned");
    st = lw::mfma_accumulate(c, b, path, ws, ws_bytes, nullptr, amp);
    if (st != LW_OK) return st;
    c->calls += 1;
    return LW_OK;
  }
  if (path != LW_PATH_FP32) return fail(c, LW_EINVAL, "unknown path %d", (int)path);
  const DirectShape s = direct_shape(c, b->n_particles);
  lw::DirectArgs a;
  a.b = lw::view_of(b);
  a.dirs = c->d_dirs;
  a.wturn = c->d_wturn;
  a.nd = c->nd;
  a.nw = c->nw;
  a.ns = c->ns;
  a.ncomp = 4;
  a.pb = s.pb;
  a.n_blocks = s.n_blocks;
  a.n_tiles = s.n_tiles;
  a.partial = nullptr;
  a.per_particle = nullptr;
  a.amp = amp;
  a.err = c->d_err;
  a.perm = nullptr;
  a.order = nullptr;
  a.ticket = nullptr;
  a.n_items = 0;
  LW_HIP(lw::prof_begin(c, lw::kProfDirect), "profile");
  LW_HIP(lw::launch_direct_f32(a, s.wpt, c->stream), "launch lw_direct_f32 (amplitude state)");
  LW_HIP(lw::prof_end(c), "profile");
  c->calls += 1;
  return LW_OK;
}

lw_status lw_amplitude_workspace_size(lw_ctx* c, int64_t n_particles, size_t* bytes) {
  if (!c || !bytes) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  if (n_particles < 0) return fail(c, LW_EINVAL, "n_particles < 0");
  const int64_t n_blocks = (n_particles + lw::kAmpRows - 1) / lw::kAmpRows;
  *bytes = align256((size_t)n_blocks * c->ns * c->nd * c->nw * lw::direct_ncomp(c) * sizeof(double));
  return LW_OK;
}

lw_status lw_spectrum_from_amplitudes(lw_ctx* c, const lw_batch* b, const double* amp, void* ws,
                                      size_t ws_bytes) {
  if (!c) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  if (!b || b->n_particles < 0) return fail(c, LW_EINVAL, "bad batch");
  if (b->n_particles == 0) return LW_OK;
  if (!b->charge || !b->weight) return fail(c, LW_EINVAL, "batch.charge and batch.weight are needed");
  if (!amp) return fail(c, LW_EINVAL, "amplitude state is NULL");
  if (((uintptr_t)amp & 15) != 0) return fail(c, LW_EINVAL, "amplitude state must be 16-byte aligned");
  size_t need = 0;
  st = lw_amplitude_workspace_size(c, b->n_particles, &need);
  if (st != LW_OK) return st;
  if (!ws || ws_bytes < need)
    return fail(c, LW_ENOMEM, "workspace too small: need %zu bytes, got %zu", need, ws_bytes);
  if (((uintptr_t)ws & 255) != 0) return fail(c, LW_EINVAL, "workspace must be 256-byte aligned");
  DeviceGuard g(c->device);
  const int ncomp = lw::direct_ncomp(c);
  const int64_t cols = (int64_t)c->nd * c->nw;
  const int64_t n_blocks = (b->n_particles + lw::kAmpRows - 1) / lw::kAmpRows;
  LW_HIP(lw::launch_amp_reduce(amp, b->n_particles, cols, b->charge, b->weight, b->species, c->ns,
                               ncomp, (double*)ws, c->d_err, c->stream),
         "launch lw_amp_reduce");
  LW_HIP(lw::launch_reduce_partials((const double*)ws, n_blocks, (int64_t)c->ns * cols * ncomp,
                                    direct_target(c), c->stream),
         "launch lw_reduce_partials");
  return LW_OK;
}

lw_status lw_spectral_diagnostics(lw_ctx* c, const double* S, const double* weights,
                                  const double* ranges, double* avg_out, double* diag_out) {
  if (!c || !diag_out) return LW_EINVAL;
  lw_status st = check_grids(c);
  if (st != LW_OK) return st;
  const int nd = c->nd, nw = c->nw, ns = c->ns;
  std::vector<double> a(nd, 1.0);
  if (weights) a.assign(weights, weights + nd);
  double a_sum = 0.0;
  for (int d = 0; d < nd; ++d) {
    if (!(a[d] >= 0.0) || !isfinite(a[d])) return fail(c, LW_EINVAL, "weight %d is negative or not finite", d);
    a_sum += a[d];
  }
  if (!(a_sum > 0.0)) return fail(c, LW_EINVAL, "observer weights sum to zero");
  double r[4] = {1e-2, 0.3, 3.0, 30.0};
  if (ranges) memcpy(r, ranges, sizeof(r));
  for (int i = 0; i < 4; i += 2)
    if (!(r[i] > 0.0) || !(r[i + 1] >= r[i]) || !isfinite(r[i + 1]))
      return fail(c, LW_EINVAL, "slope window %d must satisfy 0 < lo <= hi", i / 2);
  DeviceGuard g(c->device);
  const size_t n_avg = (size_t)ns * nw, n_out = (size_t)ns * (nd + 1) * lw::kDiagFields;
  const size_t need = (size_t)nd + n_avg + n_out;
  if (c->diag_cap < need) {
    LW_HIP(hipStreamSynchronize(c->stream), "sync");
    free_dev(c->d_diag);
    c->d_diag = nullptr;
    c->diag_cap = 0;
    LW_HIP(hipMalloc(&c->d_diag, need * sizeof(double)), "hipMalloc(diagnostics)");
    c->diag_cap = need;
  }
  double* d_a = c->d_diag;
  double* d_avg = d_a + nd;
  double* d_out = d_avg + n_avg;
  if (!S) {
    if (c->coherent)
      LW_HIP(lw::launch_coherent_power(c->d_A, (int64_t)ns * nd * nw, c->d_S, c->stream),
             "launch coherent power");
    S = c->d_S;
  }
  LW_HIP(hipMemcpyAsync(d_a, a.data(), nd * sizeof(double), hipMemcpyHostToDevice, c->stream), "copy weights");
  LW_HIP(lw::launch_spectral_diagnostics(S, d_a, a_sum, ns, nd, nw, c->d_omega, r, d_avg, d_out, c->stream),
         "launch diagnostics");
  if (avg_out)
    LW_HIP(hipMemcpyAsync(avg_out, d_avg, n_avg * sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy avg");
  LW_HIP(hipMemcpyAsync(diag_out, d_out, n_out * sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy diag");
  LW_HIP(hipStreamSynchronize(c->stream), "sync");
  return LW_OK;
}

lw_status lw_pitch_cones(lw_ctx* c, int64_t n, const double* ux, const double* uy, const double* uz,
                         const double* axis, const double* theta_c, int32_t n_cones, double dtheta,
                         const double* edges, int32_t n_bins, int64_t* counts_out, double* dev_out,
                         int32_t* member) {
  if (!c) return LW_EINVAL;
  if (n < 0 || (n > 0 && (!ux || !uy || !uz))) return fail(c, LW_EINVAL, "bad momentum arrays");
  if (!axis || !theta_c || !edges || !counts_out || !dev_out) return fail(c, LW_EINVAL, "NULL argument");
  if (n_cones < 1 || n_cones > lw::kMaxCones) return fail(c, LW_EINVAL, "1 to %d cones", lw::kMaxCones);
  if (n_bins < 1 || n_bins > lw::kMaxPitchBins) return fail(c, LW_EINVAL, "1 to %d bins", lw::kMaxPitchBins);
  if (!(dtheta > 0.0) || !isfinite(dtheta)) return fail(c, LW_EINVAL, "dtheta must be > 0");
  for (int i = 0; i < n_bins; ++i)
    if (!(edges[i] < edges[i + 1]) || !isfinite(edges[i + 1])) return fail(c, LW_EINVAL, "edges must increase");
  const double an = sqrt(axis[0] * axis[0] + axis[1] * axis[1] + axis[2] * axis[2]);
  if (!(an > 0.0) || !isfinite(an)) return fail(c, LW_EINVAL, "axis is zero or not finite");
  const double a[3] = {axis[0] / an, axis[1] / an, axis[2] / an};
  std::vector<double> host(2 * (size_t)n_cones + n_bins + 1);
  for (int m = 0; m < n_cones; ++m) {
    if (!isfinite(theta_c[m])) return fail(c, LW_EINVAL, "cone %d is not finite", m);
    const double lo = std::max(0.0, theta_c[m] - dtheta), hi = std::min(0.5 * M_PI, theta_c[m] + dtheta);
    host[2 * m] = cos(hi);
    host[2 * m + 1] = cos(lo);
  }
  std::copy(edges, edges + n_bins + 1, host.begin() + 2 * n_cones);
  DeviceGuard g(c->device);
  const size_t rows = (size_t)(n_cones + 1) * n_bins;
  const size_t need = host.size() * sizeof(double) + rows * (sizeof(unsigned long long) + sizeof(double));
  if (c->diag_cap * sizeof(double) < need) {
    LW_HIP(hipStreamSynchronize(c->stream), "sync");
    free_dev(c->d_diag);
    c->d_diag = nullptr;
    c->diag_cap = 0;
    const size_t words = (need + sizeof(double) - 1) / sizeof(double);
    LW_HIP(hipMalloc(&c->d_diag, words * sizeof(double)), "hipMalloc(pitch)");
    c->diag_cap = words;
  }
  double* d_bounds = c->d_diag;
  double* d_edges = d_bounds + 2 * n_cones;
  unsigned long long* d_counts = (unsigned long long*)(d_edges + n_bins + 1);
  double* d_dev = (double*)(d_counts + rows);
  LW_HIP(hipMemcpyAsync(d_bounds, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice, c->stream),
         "copy cones");
  LW_HIP(lw::launch_fill_u64(d_counts, (int64_t)rows, 0ull, c->stream), "zero counts");
  LW_HIP(lw::launch_pitch_cones(n, ux, uy, uz, a, d_bounds, n_cones, d_edges, n_bins, d_counts, d_dev,
                                member, c->stream),
         "launch pitch cones");
  LW_HIP(hipMemcpyAsync(counts_out, d_counts, rows * sizeof(int64_t), hipMemcpyDeviceToHost, c->stream),
         "copy counts");
  LW_HIP(hipMemcpyAsync(dev_out, d_dev, (size_t)n_cones * n_bins * sizeof(double), hipMemcpyDeviceToHost,
                        c->stream),
         "copy deviation");
  LW_HIP(hipStreamSynchronize(c->stream), "sync");
  return LW_OK;
}

lw_status lw_stats(const lw_ctx* c, int64_t* calls) {
  if (!c || !calls) return LW_EINVAL;
  *calls = c->calls;
  return LW_OK;
}

}  // extern "C"
