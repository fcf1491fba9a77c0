// lw_internal.h -- structures shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lw.h"

namespace lw {

constexpr int kMaxSpecies = 8;
constexpr int kThreads = 256;  // work-group size of the accumulation kernels
constexpr int kFlush = 16;     // FP32 partial sums are folded into FP64 every kFlush samples

// Per direction, on the device: unit n, then two unit vectors e1, e2 with
// (e1, e2, n) right-handed and orthonormal.  The integrand is perpendicular
// to n, so its two components on e1, e2 carry all of |A|^2.
constexpr int kDirStride = 9;

struct BatchView {
  int64_t n_particles;
  const int64_t* offsets;
  const double *x, *y, *z, *bx, *by, *bz;
  const float *ax, *ay, *az;
  const double *t0, *dt;
  const float *charge, *weight;
  const int32_t* species;
};

struct DirectArgs {
  BatchView b;
  const double* dirs;    // [nd][kDirStride]
  const double* wturn;   // [nw] omega / (2 pi): frequency in turns per unit time
  int32_t nd, nw, ns;
  int32_t pb;            // particles per work item
  int64_t n_blocks;      // ceil(P / pb)
  int32_t n_tiles;       // frequency tiles of kThreads * WPT
  double* partial;       // [n_blocks][ns][nd][nw]
  float* per_particle;   // [P][nd][nw] or null
  unsigned long long* err;  // lowest offending particle index (atomic min)
};

// Launchers (lw_direct.hip).
hipError_t launch_direct_f32(const DirectArgs& a, int wpt, hipStream_t stream);
hipError_t launch_reduce_partials(const double* partial, int64_t n_blocks, int64_t rows, double* S,
                                  hipStream_t stream);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t stream);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v,
                           hipStream_t stream);

struct MfmaPlanCache;

}  // namespace lw

// Context state (opaque behind the C ABI).
struct lw_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int32_t nd = 0, nw = 0, ns = 1;
  std::vector<double> h_dirs;    // [nd][9]: n, e1, e2
  std::vector<double> h_omega;   // [nw]
  double* d_dirs = nullptr;
  double* d_wturn = nullptr;     // omega / (2 pi)
  double* d_omega = nullptr;
  double* d_S = nullptr;         // [ns][nd][nw]
  unsigned long long* d_err = nullptr;
  std::string err;
  int64_t calls = 0;
  lw::MfmaPlanCache* mfma = nullptr;
  // kernel timing with HIP events (lw_set_profiling)
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_marks;  // (kind, (start, stop))
  unsigned long long* d_flops = nullptr;  // useful matrix-core FLOPs counted on the device
  int flop_mult = 1;                     // products of the last matrix-core launch
};

namespace lw {
enum ProfKind { kProfDirect = 0, kProfSpread = 1, kProfGemm = 2, kProfKinds = 3 };
// Record an event pair around a launch when profiling is on (no-op otherwise).
hipError_t prof_begin(lw_ctx* c, int kind);
hipError_t prof_end(lw_ctx* c);
}  // namespace lw
