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

__global__ __launch_bounds__(256) void lw_amp_reduce_kernel(
    const double* __restrict__ amp, int64_t P, int64_t cols, const float* __restrict__ charge,
    const float* __restrict__ weight, const int32_t* __restrict__ species, int ns, int ncomp,
    int64_t n_blocks, double* __restrict__ partial, unsigned long long* err) {
  const int64_t col = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = col < cols;
  for (int64_t blk = blockIdx.y; blk < n_blocks; blk += gridDim.y) {
    double acc[kMaxSpecies][4];
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) acc[s][0] = acc[s][1] = acc[s][2] = acc[s][3] = 0.0;
    const int64_t p0 = blk * kAmpRows;
    const int64_t p1 = min(p0 + (int64_t)kAmpRows, P);
    for (int64_t p = p0; p < p1; ++p) {
      const int sp = species ? species[p] : 0;
      if (sp < 0 || sp >= ns) {  // reported once, contributes nothing
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicMin(err, (unsigned long long)p);
        continue;
      }
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      if (live) {
        const double2* src = reinterpret_cast<const double2*>(amp + ((size_t)p * cols + col) * 4);
        const double2 lo = src[0], hi = src[1];
        v[0] = lo.x;
        v[1] = lo.y;
        v[2] = hi.x;
        v[3] = hi.y;
      }
      const double q = (double)charge[p];
      const double wq = (double)weight[p] * q;
      if (ncomp == 4) {
#pragma unroll
        for (int s = 0; s < kMaxSpecies; ++s)
          if (s == sp)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[s][c] += wq * v[c];
      } else {
        const double fac = wq * q * (1.0 / (4.0 * M_PI * M_PI));
        const double s2 = fac * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2] + v[3] * v[3]);
#pragma unroll
        for (int s = 0; s < kMaxSpecies; ++s)
          if (s == sp) acc[s][0] += s2;
      }
    }
    if (!live) continue;
#pragma unroll
    for (int s = 0; s < kMaxSpecies; ++s) {
      if (s >= ns) break;
      double* dst = partial + (((size_t)blk * ns + s) * cols + col) * ncomp;
      for (int c = 0; c < ncomp; ++c) dst[c] = acc[s][c];
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
  hipLaunchKernelGGL(lw_amp_reduce_kernel, grid, block, 0, stream, amp, P, cols, charge, weight,
                     species, ns, ncomp, n_blocks, partial, err);
  return hipGetLastError();
}

hipError_t launch_coherent_power(const double* A, int64_t n, double* S, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  hipLaunchKernelGGL(lw_coherent_power_kernel, grid, block, 0, stream, A, n, S);
  return hipGetLastError();
}

}  // namespace lw
