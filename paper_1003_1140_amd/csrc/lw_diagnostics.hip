// lw_diagnostics.hip -- spectral diagnostics of an accumulated spectrum (paper, Section 3.3).
//
// The results characterise each observer's spectrum by its peak frequency and
// by power-law indices below (alpha) and above (beta) the peak, and show a
// spectrum averaged over the observers (placed as in Section 2.2).  Here:
//   observer average  S_avg[s][j] = sum_d a_d S[s][d][j] / sum_d a_d;
//   peak              k = first index of max_j S, refined to the vertex of the
//                     parabola through (ln w, ln S) at k-1, k, k+1 when it
//                     opens downwards (clamped to [ln w_{k-1}, ln w_{k+1}]);
//   slopes            least squares of ln S on ln w over the bins with S > 0
//                     and lo w_k <= w <= hi w_k, one window below the peak
//                     (alpha) and one above (beta); NaN with fewer than 2 bins.
// Output row: [k, w_k, w_peak, S_k, alpha, n_alpha, beta, n_beta].
//
// One work-group per (species, row), rows 0..nd-1 the observers and row nd
// their average; reductions go through LDS in a fixed tree, so results are
// reproducible.  The work is a few kilobytes per row: launch-latency bound.
#include <hip/hip_runtime.h>
#include <math.h>

#include "lw_internal.h"

namespace lw {

constexpr int kDiagThreads = 256;

__global__ void lw_observer_average_kernel(const double* __restrict__ S, const double* __restrict__ a,
                                           double a_sum, int ns, int nd, int nw,
                                           double* __restrict__ avg) {
  // products and sums rounded separately and observers taken in order, so that the
  // average (and the peak picked from it) does not depend on how the compiler fuses them
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)ns * nw) return;
  const int s = (int)(i / nw), j = (int)(i % nw);
  double acc = 0.0;
  for (int d = 0; d < nd; ++d) acc += a[d] * S[((size_t)s * nd + d) * nw + j];
  avg[i] = acc / a_sum;
}

template <int N>
__device__ __forceinline__ void block_sum(double (*buf)[kDiagThreads], double v[N]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < N; ++q) buf[q][t] = v[q];
  __syncthreads();
  for (int h = kDiagThreads / 2; h > 0; h >>= 1) {
    if (t < h)
#pragma unroll
      for (int q = 0; q < N; ++q) buf[q][t] += buf[q][t + h];
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < N; ++q) v[q] = buf[q][0];
  __syncthreads();
}

__global__ __launch_bounds__(kDiagThreads) void lw_row_diagnostics_kernel(
    const double* __restrict__ S, const double* __restrict__ avg, const double* __restrict__ w,
    int nd, int nw, double alo, double ahi, double blo, double bhi, double* __restrict__ out) {
  __shared__ double buf[6][kDiagThreads];
  __shared__ int ibuf[kDiagThreads];
  const int t = threadIdx.x;
  const int s = blockIdx.x / (nd + 1), d = blockIdx.x % (nd + 1);
  const double* row = d < nd ? S + ((size_t)s * nd + d) * nw : avg + (size_t)s * nw;

  // first index of the largest value
  double best = -INFINITY;
  int bi = nw;
  for (int j = t; j < nw; j += kDiagThreads)
    if (row[j] > best || bi == nw) {
      best = row[j];
      bi = j;
    }
  buf[0][t] = best;
  ibuf[t] = bi;
  __syncthreads();
  for (int h = kDiagThreads / 2; h > 0; h >>= 1) {
    if (t < h) {
      const double vo = buf[0][t + h];
      const int io = ibuf[t + h];
      if (io < nw && (ibuf[t] == nw || vo > buf[0][t] || (vo == buf[0][t] && io < ibuf[t]))) {
        buf[0][t] = vo;
        ibuf[t] = io;
      }
    }
    __syncthreads();
  }
  const int k = ibuf[0];
  const double sk = row[k], wk = w[k];
  __syncthreads();

  // slope windows: first the counts and means, then the centred sums
  double m[6] = {0, 0, 0, 0, 0, 0};  // n_a, sx_a, sy_a, n_b, sx_b, sy_b
  const double a0 = alo * wk, a1 = ahi * wk, b0 = blo * wk, b1 = bhi * wk;
  for (int j = t; j < nw; j += kDiagThreads) {
    const double v = row[j], wj = w[j];
    if (!(v > 0.0)) continue;
    const double x = log(wj), y = log(v);
    if (wj >= a0 && wj <= a1) {
      m[0] += 1.0;
      m[1] += x;
      m[2] += y;
    }
    if (wj >= b0 && wj <= b1) {
      m[3] += 1.0;
      m[4] += x;
      m[5] += y;
    }
  }
  block_sum<6>(buf, m);
  const double xa = m[0] > 0 ? m[1] / m[0] : 0.0, ya = m[0] > 0 ? m[2] / m[0] : 0.0;
  const double xb = m[3] > 0 ? m[4] / m[3] : 0.0, yb = m[3] > 0 ? m[5] / m[3] : 0.0;
  double c[4] = {0, 0, 0, 0};  // sxy_a, sxx_a, sxy_b, sxx_b
  for (int j = t; j < nw; j += kDiagThreads) {
    const double v = row[j], wj = w[j];
    if (!(v > 0.0)) continue;
    const double x = log(wj), y = log(v);
    if (wj >= a0 && wj <= a1) {
      c[0] += (x - xa) * (y - ya);
      c[1] += (x - xa) * (x - xa);
    }
    if (wj >= b0 && wj <= b1) {
      c[2] += (x - xb) * (y - yb);
      c[3] += (x - xb) * (x - xb);
    }
  }
  block_sum<4>(buf, c);
  if (t != 0) return;
  double wpeak = wk;
  if (k > 0 && k < nw - 1 && row[k - 1] > 0.0 && row[k + 1] > 0.0 && sk > 0.0) {
    const double x0 = log(w[k - 1]), x1 = log(wk), x2 = log(w[k + 1]);
    const double y0 = log(row[k - 1]), y1 = log(sk), y2 = log(row[k + 1]);
    const double den = (x0 - x1) * (x0 - x2) * (x1 - x2);
    const double A = (x2 * (y1 - y0) + x1 * (y0 - y2) + x0 * (y2 - y1)) / den;
    const double B = (x2 * x2 * (y0 - y1) + x1 * x1 * (y2 - y0) + x0 * x0 * (y1 - y2)) / den;
    if (A < 0.0) wpeak = exp(fmin(fmax(-B / (2.0 * A), x0), x2));
  }
  double* o = out + (size_t)blockIdx.x * 8;
  o[0] = (double)k;
  o[1] = wk;
  o[2] = wpeak;
  o[3] = sk;
  o[4] = (m[0] >= 2.0 && c[1] > 0.0) ? c[0] / c[1] : NAN;
  o[5] = m[0];
  o[6] = (m[3] >= 2.0 && c[3] > 0.0) ? c[2] / c[3] : NAN;
  o[7] = m[3];
}

hipError_t launch_spectral_diagnostics(const double* S, const double* a, double a_sum, int ns, int nd,
                                       int nw, const double* omega, const double ranges[4],
                                       double* avg, double* out, hipStream_t stream) {
  if (ns <= 0 || nd <= 0 || nw <= 0) return hipSuccess;
  const int64_t n = (int64_t)ns * nw;
  hipLaunchKernelGGL(lw_observer_average_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream,
                     S, a, a_sum, ns, nd, nw, avg);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lw_row_diagnostics_kernel, dim3((unsigned)(ns * (nd + 1))), dim3(kDiagThreads), 0,
                     stream, S, avg, omega, nd, nw, ranges[0], ranges[1], ranges[2], ranges[3], out);
  return hipGetLastError();
}

}  // namespace lw
