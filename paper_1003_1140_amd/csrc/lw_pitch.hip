// lw_pitch.hip -- pitch-cone selection of the ensemble in momentum space (paper, Section 3.2).
//
// The paper compares the particles whose momenta lie in narrow cones about inclinations
// theta_m from the streaming direction with the whole ensemble, as gamma^2 histograms,
// and reports each cone's relative deviation from isotropy.  One thread per particle:
// cos theta = |u . a| / |u| (the pitch angle folded to [0, pi/2], so both beams count),
// membership by comparing cos theta with each cone's bounds, gamma^2 = 1 + |u|^2 binned by
// binary search over the edges, counts in an LDS histogram added to the output with
// integer atomics (exact and order-independent).  Products and sums are rounded
// separately, as written, so every decision is reproducible.
#include <hip/hip_runtime.h>
#include <math.h>

#include "lw_internal.h"

namespace lw {

__global__ void lw_pitch_kernel(int64_t n, const double* __restrict__ ux, const double* __restrict__ uy,
                                const double* __restrict__ uz, double a0, double a1, double a2,
                                const double* __restrict__ bounds, int nc, const double* __restrict__ edges,
                                int nb, unsigned long long* counts, int32_t* member) {
#pragma clang fp contract(off)
  extern __shared__ unsigned int hist[];  // [nc + 1][nb]
  const int rows = (nc + 1) * nb;
  for (int r = threadIdx.x; r < rows; r += blockDim.x) hist[r] = 0u;
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double x = ux[i], y = uy[i], z = uz[i];
    const double u2 = x * x + y * y + z * z;
    const double upar = fabs(x * a0 + y * a1 + z * a2);
    const double c = u2 > 0.0 ? upar / sqrt(u2) : 1.0;  // a particle at rest counts as on-axis
    const double g2 = 1.0 + u2;
    int lo = 0, hi = nb + 1;  // number of edges <= g2
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (edges[mid] <= g2) lo = mid + 1; else hi = mid;
    }
    const int b = lo - 1;
    const bool inside = b >= 0 && b < nb;
    if (inside) atomicAdd(&hist[nc * nb + b], 1u);
    int first = -1;
    for (int m = 0; m < nc; ++m) {
      if (c >= bounds[2 * m] && c <= bounds[2 * m + 1]) {
        if (first < 0) first = m;
        if (inside) atomicAdd(&hist[m * nb + b], 1u);
      }
    }
    if (member) member[i] = first;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < rows; r += blockDim.x)
    if (hist[r]) atomicAdd(&counts[r], (unsigned long long)hist[r]);
}

// deviation[m][b] = (counts[m][b] / counts[nc][b]) / (bounds_lo - bounds_hi); NaN for an empty bin
__global__ void lw_pitch_deviation_kernel(const unsigned long long* counts, const double* bounds, int nc,
                                          int nb, double* dev) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc * nb) return;
  const int m = i / nb, b = i % nb;
  const unsigned long long all = counts[nc * nb + b];
  const double frac = bounds[2 * m + 1] - bounds[2 * m];
  dev[i] = all ? ((double)counts[i] / (double)all) / frac : NAN;
}

hipError_t launch_pitch_cones(int64_t n, const double* ux, const double* uy, const double* uz,
                              const double axis[3], const double* bounds, int nc, const double* edges,
                              int nb, unsigned long long* counts, double* dev, int32_t* member,
                              hipStream_t stream) {
  const size_t shmem = sizeof(unsigned int) * (size_t)(nc + 1) * nb;
  if (n > 0) {
    const int64_t blocks = (n + 255) / 256;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lw_pitch_kernel, dim3((unsigned)blocks), dim3(256), shmem, stream, n, ux, uy, uz,
                       axis[0], axis[1], axis[2], bounds, nc, edges, nb, counts, member);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(lw_pitch_deviation_kernel, dim3((unsigned)((nc * nb + 255) / 256)), dim3(256), 0,
                     stream, counts, bounds, nc, nb, dev);
  return hipGetLastError();
}

}  // namespace lw
