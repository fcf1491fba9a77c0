// lw_amplitude.hip -- spectra from amplitude state (paper, Section 2.2 recording scheme).
//
// In-situ recording integrates the retarded-field amplitude of each particle
// from the start of the run up to the current step and squares it only when a
// spectrum is wanted, so a spectrum taken between two steps is the difference
// of two such squares.  Incoherent synthesis therefore keeps one complex
// amplitude per (particle, direction, frequency) across time windows; coherent
// synthesis keeps one per (species, direction, frequency).  These kernels turn
// the per-particle state into either form:
//   incoherent: S[s][d][j] += sum_{p in s} w_p q_p^2 |a_p[d][j]|^2 / (4 pi^2)
//   coherent:   A[s][d][j] += sum_{p in s} w_p q_p a_p[d][j]
// State rows hold four FP64 numbers: (Re, Im) of the component on e1, then on e2.
//
// The reduction is HBM-bound (32 B of state per particle and column, read
// once): a work-group owns 256 consecutive columns (d, j) of kAmpRows
// particles, so each particle row is one contiguous 8 KiB read per work-group,
// and sums in registers per species in particle order; lw_reduce_partials then
// adds the blocks' rows in block order, so results are reproducible.
#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

#include "lw_internal.h"

namespace lw {

constexpr int kUnroll = 4;

template <int NCOMP>
__global__ __launch_bounds__(256) void lw_amp_reduce_kernel(
    const double* __restrict__ amp, int64_t P, int64_t cols, const float* __restrict__ charge,
    const float* __restrict__ weight, const int32_t* __restrict__ species, int ns,
    int64_t n_blocks, double* __restrict__ partial, unsigned long long* err) {
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = col < cols;
  for (int64_t blk = blockIdx.y; blk < n_blocks; blk += gridDim.y) {
    double acc[kMaxSpecies][NCOMP];
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s)
#pragma unroll
      for (int c = 0; c < NCOMP; ++c) acc[s][c] = 0.0;
    const int64_t p0 = blk * kAmpRows;
    const int64_t p1 = min(p0 + (int64_t)kAmpRows, P);
    // kUnroll rows are loaded before any is summed (more bytes in flight per wave); the
    // sums still take the rows in particle order
    for (int64_t pb = p0; pb < p1; pb += kUnroll) {
      double v[kUnroll][4];
      int sp[kUnroll];
      double wq[kUnroll], q[kUnroll];
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        const int64_t p = pb + u;
        const bool in = p < p1;
        sp[u] = in ? (species ? species[p] : 0) : -1;
        q[u] = in ? (double)charge[p] : 0.0;
        wq[u] = in ? (double)weight[p] * q[u] : 0.0;
        v[u][0] = v[u][1] = v[u][2] = v[u][3] = 0.0;
        if (in && live) {
          const double2* src = reinterpret_cast<const double2*>(amp + ((size_t)p * cols + col) * 4);
          const double2 lo = src[0], hi = src[1];
          v[u][0] = lo.x;
          v[u][1] = lo.y;
          v[u][2] = hi.x;
          v[u][3] = hi.y;
        }
      }
#pragma unroll
      for (int u = 0; u < kUnroll; ++u) {
        // rows past the block end carry sp = -1 and are skipped silently
        if (pb + u < p1 && (sp[u] < 0 || sp[u] >= ns)) {  // reported once, contributes nothing
          if (blockIdx.x == 0 && threadIdx.x == 0) atomicMin(err, (unsigned long long)(pb + u));
        }
        if (NCOMP == 4) {
#pragma unroll
          for (int s = 0; s < kMaxSpecies; ++s)
#pragma unroll
            for (int c = 0; c < NCOMP; ++c) acc[s][c] += (s == sp[u]) ? wq[u] * v[u][c] : 0.0;
        } else {
          const double fac = wq[u] * q[u] * (1.0 / (4.0 * M_PI * M_PI));
          const double s2 =
              fac * (v[u][0] * v[u][0] + v[u][1] * v[u][1] + v[u][2] * v[u][2] + v[u][3] * v[u][3]);
#pragma unroll
          for (int s = 0; s < kMaxSpecies; ++s) acc[s][0] += (s == sp[u]) ? s2 : 0.0;
        }
      }
    }
    if (!live) continue;
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) {
      if (s < ns) {
        double* dst = partial + (((size_t)blk * ns + s) * cols + col) * NCOMP;
#pragma unroll
        for (int c = 0; c < NCOMP; ++c) dst[c] = acc[s][c];
      }
    }
  }
}

__global__ void lw_coherent_power_kernel(const double* __restrict__ A, int64_t n,
                                         double* __restrict__ S) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double2* a = reinterpret_cast<const double2*>(A + 4 * i);
  const double2 lo = a[0], hi = a[1];
  S[i] = (lo.x * lo.x + lo.y * lo.y + hi.x * hi.x + hi.y * hi.y) * (1.0 / (4.0 * M_PI * M_PI));
}

hipError_t launch_amp_reduce(const double* amp, int64_t P, int64_t cols, const float* charge,
                             const float* weight, const int32_t* species, int ns, int ncomp,
                             double* partial, unsigned long long* err, hipStream_t stream) {
  if (P <= 0 || cols <= 0) return hipSuccess;
  if (ns < 1 || ns > kMaxSpecies || (ncomp != 1 && ncomp != 4)) return hipErrorInvalidValue;
  const int64_t n_blocks = (P + kAmpRows - 1) / kAmpRows;
  const int64_t col_tiles = (cols + 255) / 256;
  if (col_tiles > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid((unsigned)col_tiles, (unsigned)std::min<int64_t>(n_blocks, 65535)), block(256);
  if (ncomp == 4)
    hipLaunchKernelGGL(lw_amp_reduce_kernel<4>, grid, block, 0, stream, amp, P, cols, charge, weight,
                       species, ns, n_blocks, partial, err);
  else
    hipLaunchKernelGGL(lw_amp_reduce_kernel<1>, grid, block, 0, stream, amp, P, cols, charge, weight,
                       species, ns, n_blocks, partial, err);
  return hipGetLastError();
}

hipError_t launch_coherent_power(const double* A, int64_t n, double* S, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  hipLaunchKernelGGL(lw_coherent_power_kernel, grid, block, 0, stream, A, n, S);
  return hipGetLastError();
}

}  // namespace lw
