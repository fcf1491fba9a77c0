// lw_direct.hip -- FP32 accumulation of the discretised Lienard-Wiechert
// spectral integral on gfx950 (paper, Section 2.2).
//
// One work-group (256 threads, 4 wave64) owns an item = (block of `pb`
// particles, one observer direction, one tile of 256*WPT frequencies); each
// thread owns WPT frequencies (strided by 256 so stores coalesce).
//
// Per particle, samples are processed in chunks of 256:
//   1. prepass (FP64, one sample per thread): kappa = 1 - n.beta, the two
//      components of g = n x ((n-beta) x betadot) / kappa^2 on (e1, e2),
//      pre-multiplied by dt, and the retarded time tau = t - n.r; staged in
//      LDS as {tau: f64, g1: f32, g2: f32} (16 B, one ds_read_b128 per sample
//      for the whole wave: every lane reads the same address);
//   2. accumulate: for each staged sample and each owned frequency, the phase
//      w*tau/(2 pi) is formed and reduced to a turn fraction in FP64, the
//      phase factor comes from the hardware sin/cos (which take turns), and
//      four FP32 FMAs add g1, g2 times (cos, sin) into the running sums.  The
//      FP32 sums are folded into FP64 every 16 samples.
// At the end of a particle, w q^2 |A|^2 / (4 pi^2) is added (FP64) to an LDS
// accumulator of the particle's species (incoherent synthesis); in coherent
// synthesis the four amplitude components times w q are added instead, so the
// particles of a species interfere before the square is taken.  At the end of
// the item the accumulators are written to the item's own rows of the partial
// buffer, and lw_reduce_partials sums the rows in a fixed order, so results are
// bitwise reproducible.  With a per-particle amplitude state (in-situ
// recording over time windows) the raw amplitude A_p of the window is added to
// the particle's own state row; that pass needs no LDS accumulator.
#include <hip/hip_runtime.h>
#include <math.h>

#include "lw_internal.h"

namespace lw {

struct __attribute__((aligned(16))) Staged {
  double tau;
  float g1, g2;
};

__device__ __forceinline__ void record_error(unsigned long long* err, int64_t p) {
  atomicMin(err, (unsigned long long)p);
}

// FP64 prepass of one sample; returns false (and zero contribution) on bad data.
__device__ __forceinline__ Staged prepass(const BatchView& b, int64_t idx, double t, double dtp,
                                          const double n[3], const double e1[3],
                                          const double e2[3], bool* bad) {
  const double bx = b.bx[idx], by = b.by[idx], bz = b.bz[idx];
  double ax, ay, az;
  load_accel(b, idx, ax, ay, az);
  const double rx = b.x[idx], ry = b.y[idx], rz = b.z[idx];
  const double b2 = bx * bx + by * by + bz * bz;
  const double kappa = 1.0 - (n[0] * bx + n[1] * by + n[2] * bz);
  // n x ((n - beta) x a) = (n - beta)(n.a) - a kappa ; its e-components use n.e = 0
  const double na = n[0] * ax + n[1] * ay + n[2] * az;
  const double be1 = e1[0] * bx + e1[1] * by + e1[2] * bz;
  const double be2 = e2[0] * bx + e2[1] * by + e2[2] * bz;
  const double ae1 = e1[0] * ax + e1[1] * ay + e1[2] * az;
  const double ae2 = e2[0] * ax + e2[1] * ay + e2[2] * az;
  const double scale = dtp / (kappa * kappa);
  const double g1 = -(na * be1 + kappa * ae1) * scale;
  const double g2 = -(na * be2 + kappa * ae2) * scale;
  const double tau = t - (n[0] * rx + n[1] * ry + n[2] * rz);
  Staged s;
  const bool ok = (b2 < 1.0) && isfinite(tau) && isfinite(g1) && isfinite(g2);
  *bad = !ok;
  s.tau = ok ? tau : 0.0;
  s.g1 = ok ? (float)g1 : 0.0f;
  s.g2 = ok ? (float)g2 : 0.0f;
  return s;
}

// One work item: (block of pb particles, direction, frequency tile).
template <int WPT>
__device__ __forceinline__ void direct_item(const DirectArgs& a, int64_t item, Staged* stage,
                                            double* sacc) {
  const int tid = threadIdx.x;
  const int tile = (int)(item % a.n_tiles);
  item /= a.n_tiles;
  const int d = (int)(item % a.nd);
  const int64_t blk = item / a.nd;

  double wt[WPT];
  int jw[WPT];
#pragma unroll
  for (int i = 0; i < WPT; ++i) {
    jw[i] = tile * kThreads * WPT + i * kThreads + tid;
    wt[i] = jw[i] < a.nw ? a.wturn[jw[i]] : 0.0;
  }
  double n[3], e1[3], e2[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    n[c] = a.dirs[kDirStride * d + c];
    e1[c] = a.dirs[kDirStride * d + 3 + c];
    e2[c] = a.dirs[kDirStride * d + 6 + c];
  }
  const int nrow = a.partial ? a.ns * a.ncomp : 0;  // LDS accumulator rows of WPT x kThreads
  for (int r = 0; r < nrow; ++r)
#pragma unroll
    for (int i = 0; i < WPT; ++i) sacc[(r * WPT + i) * kThreads + tid] = 0.0;

  const int64_t p0 = blk * a.pb;
  const int64_t p1 = min(p0 + (int64_t)a.pb, a.b.n_particles);
  for (int64_t pi = p0; pi < p1; ++pi) {
    const int64_t p = a.perm ? a.perm[pi] : pi;
    const int64_t base = a.b.offsets[p];
    const int64_t len = a.b.offsets[p + 1] - base;
    if (len < 0) {  // decreasing offsets: reported, contributes nothing
      if (tid == 0) record_error(a.err, p);
      continue;
    }
    const double t0 = a.b.t0[p], dtp = a.b.dt[p];

    double acc[WPT][4];
#pragma unroll
    for (int i = 0; i < WPT; ++i) acc[i][0] = acc[i][1] = acc[i][2] = acc[i][3] = 0.0;

    for (int64_t c0 = 0; c0 < len; c0 += kThreads) {
      Staged sm = {0.0, 0.0f, 0.0f};
      const int64_t k = c0 + tid;
      if (k < len) {
        bool bad = false;
        sm = prepass(a.b, base + k, t0 + (double)k * dtp, dtp, n, e1, e2, &bad);
        if (bad) record_error(a.err, p);
      }
      __syncthreads();  // the previous chunk has been consumed
      stage[tid] = sm;
      __syncthreads();
      const int cnt = (int)min((int64_t)kThreads, len - c0);
      for (int sb = 0; sb < cnt; sb += kFlush) {
        const int se = min(sb + kFlush, cnt);
        float f32[WPT][4];
#pragma unroll
        for (int i = 0; i < WPT; ++i) f32[i][0] = f32[i][1] = f32[i][2] = f32[i][3] = 0.0f;
#pragma unroll 4
        for (int kk = sb; kk < se; ++kk) {
          const Staged s = stage[kk];
#pragma unroll
          for (int i = 0; i < WPT; ++i) {
            const double x = wt[i] * s.tau;       // phase in turns
            const float fr = (float)(x - rint(x));  // turn fraction in [-1/2, 1/2]
            const float sn = __builtin_amdgcn_sinf(fr);  // sin(2 pi fr)
            const float cs = __builtin_amdgcn_cosf(fr);  // cos(2 pi fr)
            f32[i][0] = fmaf(s.g1, cs, f32[i][0]);
            f32[i][1] = fmaf(s.g1, sn, f32[i][1]);
            f32[i][2] = fmaf(s.g2, cs, f32[i][2]);
            f32[i][3] = fmaf(s.g2, sn, f32[i][3]);
          }
        }
#pragma unroll
        for (int i = 0; i < WPT; ++i)
#pragma unroll
          for (int c = 0; c < 4; ++c) acc[i][c] += (double)f32[i][c];
      }
    }
    if (a.amp) {  // this thread alone owns rows (p, d, jw[i]) of the state
#pragma unroll
      for (int i = 0; i < WPT; ++i) {
        if (jw[i] < a.nw) {
          double* o = a.amp + (((size_t)p * a.nd + d) * a.nw + jw[i]) * 4;
#pragma unroll
          for (int c = 0; c < 4; ++c) o[c] += acc[i][c];
        }
      }
    }
    if (!a.partial) continue;
    int sp = a.b.species ? a.b.species[p] : 0;
    if (sp < 0 || sp >= a.ns) {  // out-of-range species: reported, contributes nothing
      if (tid == 0) record_error(a.err, p);
      continue;
    }
    const double q = (double)a.b.charge[p];
    const double wq = (double)a.b.weight[p] * q;
    const double fac = wq * q * (1.0 / (4.0 * M_PI * M_PI));
    if (a.ncomp == 4) {
#pragma unroll
      for (int i = 0; i < WPT; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) sacc[((sp * 4 + c) * WPT + i) * kThreads + tid] += wq * acc[i][c];
    }
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      const double s2 = fac * (acc[i][0] * acc[i][0] + acc[i][1] * acc[i][1] +
                               acc[i][2] * acc[i][2] + acc[i][3] * acc[i][3]);
      if (a.ncomp == 1) sacc[(sp * WPT + i) * kThreads + tid] += s2;
      if (a.per_particle && jw[i] < a.nw)
        a.per_particle[((size_t)p * a.nd + d) * a.nw + jw[i]] = (float)s2;
    }
  }
  if (!a.partial) return;
  for (int s = 0; s < a.ns; ++s) {
#pragma unroll
    for (int i = 0; i < WPT; ++i) {
      if (jw[i] >= a.nw) continue;
      const size_t row = (((size_t)blk * a.ns + s) * a.nd + d) * a.nw + jw[i];
      for (int c = 0; c < a.ncomp; ++c)
        a.partial[row * a.ncomp + c] = sacc[((s * a.ncomp + c) * WPT + i) * kThreads + tid];
    }
  }
}

template <int WPT>
__global__ __launch_bounds__(kThreads) void lw_direct_f32_kernel(DirectArgs a) {
  __shared__ Staged stage[kThreads];
  extern __shared__ double sacc[];  // [ns][ncomp][WPT][kThreads]
  direct_item<WPT>(a, blockIdx.x, stage, sacc);
}

// Persistent form: a fixed set of work-groups pulls items, longest first, from a ticket.
template <int WPT>
__global__ __launch_bounds__(kThreads) void lw_direct_f32_persistent_kernel(DirectArgs a) {
  __shared__ Staged stage[kThreads];
  __shared__ int64_t s_item;
  extern __shared__ double sacc[];  // [ns][ncomp][WPT][kThreads]
  const unsigned long long t_start = a.wg_time ? __builtin_amdgcn_s_memrealtime() : 0ull;
  for (;;) {
    __syncthreads();  // the previous item's LDS use is over
    if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(a.ticket, 1u);
    __syncthreads();
    const int64_t i = s_item;
    if (i >= a.n_items) break;
    direct_item<WPT>(a, a.order ? a.order[i] : i, stage, sacc);
  }
  if (a.wg_time && threadIdx.x == 0) {
    // compute unit of this work-group: XCC id, then HW_ID bits 8..15 (CU, shader array, engine)
    const unsigned hw = __builtin_amdgcn_s_getreg((31 << 11) | 4);    // HW_REG_HW_ID, 32 bits
    const unsigned xcc = __builtin_amdgcn_s_getreg((31 << 11) | 20);  // HW_REG_XCC_ID, 32 bits
    unsigned long long* r = a.wg_time + 3 * (size_t)blockIdx.x;
    r[0] = ((unsigned long long)(xcc & 0xfu) << 8) | ((hw >> 8) & 0xffu);
    r[1] = t_start;
    r[2] = __builtin_amdgcn_s_memrealtime();
  }
}

__global__ void lw_reduce_partials_kernel(const double* __restrict__ partial, int64_t n_blocks,
                                          int64_t rows, double* __restrict__ S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  double acc = 0.0;
  for (int64_t b = 0; b < n_blocks; ++b) acc += partial[b * rows + i];
  S[i] += acc;
}

__global__ void fill_f64_kernel(double* p, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void fill_u64_kernel(unsigned long long* p, int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_direct_f32(const DirectArgs& a, int wpt, hipStream_t stream) {
  const int64_t items = a.n_blocks * (int64_t)a.nd * a.n_tiles;
  if (items <= 0) return hipSuccess;
  const size_t shmem = a.partial ? direct_lds(a.ns, a.ncomp, wpt) : 0;
  if (shmem > kMaxDirectLds) return hipErrorInvalidValue;
  dim3 grid((unsigned)items), block(kThreads);
  const void* fn = nullptr;
  switch (wpt) {
    case 1: fn = (const void*)lw_direct_f32_kernel<1>; break;
    case 2: fn = (const void*)lw_direct_f32_kernel<2>; break;
    case 4: fn = (const void*)lw_direct_f32_kernel<4>; break;
    case 8: fn = (const void*)lw_direct_f32_kernel<8>; break;
    default: return hipErrorInvalidValue;
  }
  if (shmem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
  }
  switch (wpt) {
    case 1: hipLaunchKernelGGL(lw_direct_f32_kernel<1>, grid, block, shmem, stream, a); break;
    case 2: hipLaunchKernelGGL(lw_direct_f32_kernel<2>, grid, block, shmem, stream, a); break;
    case 4: hipLaunchKernelGGL(lw_direct_f32_kernel<4>, grid, block, shmem, stream, a); break;
    default: hipLaunchKernelGGL(lw_direct_f32_kernel<8>, grid, block, shmem, stream, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_direct_f32_persistent(const DirectArgs& a, int wpt, int workgroups,
                                        hipStream_t stream) {
  if (a.n_items <= 0) return hipSuccess;
  const size_t shmem = a.partial ? direct_lds(a.ns, a.ncomp, wpt) : 0;
  if (shmem > kMaxDirectLds) return hipErrorInvalidValue;
  const void* fn = nullptr;
  switch (wpt) {
    case 1: fn = (const void*)lw_direct_f32_persistent_kernel<1>; break;
    case 2: fn = (const void*)lw_direct_f32_persistent_kernel<2>; break;
    case 4: fn = (const void*)lw_direct_f32_persistent_kernel<4>; break;
    case 8: fn = (const void*)lw_direct_f32_persistent_kernel<8>; break;
    default: return hipErrorInvalidValue;
  }
  if (shmem > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shmem);
    if (e != hipSuccess) return e;
  }
  dim3 grid((unsigned)workgroups), block(kThreads);
  switch (wpt) {
    case 1: hipLaunchKernelGGL(lw_direct_f32_persistent_kernel<1>, grid, block, shmem, stream, a); break;
    case 2: hipLaunchKernelGGL(lw_direct_f32_persistent_kernel<2>, grid, block, shmem, stream, a); break;
    case 4: hipLaunchKernelGGL(lw_direct_f32_persistent_kernel<4>, grid, block, shmem, stream, a); break;
    default: hipLaunchKernelGGL(lw_direct_f32_persistent_kernel<8>, grid, block, shmem, stream, a); break;
  }
  return hipGetLastError();
}

int direct_persistent_occupancy(int wpt, size_t shmem) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (wpt) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, lw_direct_f32_persistent_kernel<1>, kThreads, shmem); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, lw_direct_f32_persistent_kernel<2>, kThreads, shmem); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, lw_direct_f32_persistent_kernel<4>, kThreads, shmem); break;
    case 8: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, lw_direct_f32_persistent_kernel<8>, kThreads, shmem); break;
    default: break;
  }
  return (e == hipSuccess && n > 0) ? n : 1;
}

__global__ void fill_u32_kernel(unsigned* p, int64_t n, unsigned v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u32(unsigned* p, int64_t n, unsigned v, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  hipLaunchKernelGGL(fill_u32_kernel, grid, block, 0, stream, p, n, v);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(const double* partial, int64_t n_blocks, int64_t rows, double* S,
                                  hipStream_t stream) {
  if (rows <= 0) return hipSuccess;
  dim3 grid((unsigned)((rows + 255) / 256)), block(256);
  hipLaunchKernelGGL(lw_reduce_partials_kernel, grid, block, 0, stream, partial, n_blocks, rows, S);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  hipLaunchKernelGGL(fill_f64_kernel, grid, block, 0, stream, p, n, v);
  return hipGetLastError();
}

hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v,
                           hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  hipLaunchKernelGGL(fill_u64_kernel, grid, block, 0, stream, p, n, v);
  return hipGetLastError();
}

}  // namespace lw
