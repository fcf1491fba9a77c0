// lw_internal.h -- structures shared by the host runtime and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

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
  const float *ax, *ay, *az;      // FP32 d(beta)/dt, or null when adx.. are set
  const double *t0, *dt;
  const float *charge, *weight;
  const int32_t* species;
  const double *adx, *ady, *adz;  // FP64 d(beta)/dt (LW_BATCH_F64_ACCEL), or null
};

// The device view of a caller's batch.
inline BatchView view_of(const lw_batch* b) {
  const bool f64 = (b->flags & LW_BATCH_F64_ACCEL) != 0;
  BatchView v{b->n_particles, b->offsets, b->x,  b->y,  b->z,      b->bx,     b->by,     b->bz,
              b->ax,          b->ay,      b->az, b->t0, b->dt,     b->charge, b->weight, b->species,
              nullptr,        nullptr,    nullptr};
  if (f64) {
    v.adx = (const double*)(const void*)b->ax;
    v.ady = (const double*)(const void*)b->ay;
    v.adz = (const double*)(const void*)b->az;
    v.ax = v.ay = v.az = nullptr;
  }
  return v;
}

// d(beta)/dt of sample i in FP64, whatever the batch stores.
__device__ __forceinline__ void load_accel(const BatchView& b, int64_t i, double& ax, double& ay, double& az) {
  if (b.adx) {
    ax = b.adx[i];
    ay = b.ady[i];
    az = b.adz[i];
  } else {
    ax = (double)b.ax[i];
    ay = (double)b.ay[i];
    az = (double)b.az[i];
  }
}

struct DirectArgs {
  BatchView b;
  const double* dirs;    // [nd][kDirStride]
  const double* wturn;   // [nw] omega / (2 pi): frequency in turns per unit time
  int32_t nd, nw, ns;
  int32_t ncomp;         // rows per (species, direction, frequency): 1 = power, 4 = amplitude
  int32_t pb;            // particles per work item
  int64_t n_blocks;      // ceil(P / pb)
  int32_t n_tiles;       // frequency tiles of kThreads * WPT
  double* partial;       // [n_blocks][ns][nd][nw][ncomp], or null (amplitude state only)
  float* per_particle;   // [P][nd][nw] or null
  double* amp;           // per-particle amplitude state [P][nd][nw][4] (added into), or null
  unsigned long long* err;  // lowest offending particle index (atomic min)
  // persistent launch (all null/0 for the plain grid)
  const int64_t* perm;   // particle order (blocks take consecutive entries), or null
  const int64_t* order;  // item order for the ticket queue, or null
  unsigned* ticket;      // queue head, zeroed before the launch
  int64_t n_items;
  // persistent launch with profiling: per work-group {compute-unit key, start, end} of the
  // real-time counter, [workgroups][3], or null
  unsigned long long* wg_time = nullptr;
};

// Launchers (lw_direct.hip).
hipError_t launch_direct_f32(const DirectArgs& a, int wpt, hipStream_t stream);
// Persistent variant: `workgroups` work-groups take items from a.ticket until a.n_items.
hipError_t launch_direct_f32_persistent(const DirectArgs& a, int wpt, int workgroups,
                                        hipStream_t stream);
hipError_t launch_fill_u32(unsigned* p, int64_t n, unsigned v, hipStream_t stream);
hipError_t launch_reduce_partials(const double* partial, int64_t n_blocks, int64_t rows, double* S,
                                  hipStream_t stream);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t stream);
hipError_t launch_fill_u64(unsigned long long* p, int64_t n, unsigned long long v,
                           hipStream_t stream);

// Amplitude state (lw_amplitude.hip).  Particles per row block of the state reduction.
constexpr int kAmpRows = 256;
// partial[blk][ns][cols][ncomp] from amp[P][cols][4]: w q^2 |a|^2 / (4 pi^2) (ncomp 1) or
// w q a (ncomp 4), summed over the block's particles by species.
hipError_t launch_amp_reduce(const double* amp, int64_t P, int64_t cols, const float* charge,
                             const float* weight, const int32_t* species, int ns, int ncomp,
                             double* partial, unsigned long long* err, hipStream_t stream);
// S[i] = |A_i|^2 / (4 pi^2) for the n four-component amplitudes A.
hipError_t launch_coherent_power(const double* A, int64_t n, double* S, hipStream_t stream);

// Spectral diagnostics (lw_diagnostics.hip): observer average avg [ns][nw] with weights a [nd]
// (sum a_sum), then per (species, row) [k, w_k, w_peak, S_k, alpha, n_alpha, beta, n_beta]
// into out [ns][nd + 1][8]; ranges = alpha_lo, alpha_hi, beta_lo, beta_hi.
constexpr int kDiagFields = 8;
// Pitch cones (lw_pitch.hip): counts [nc + 1][nb] (zeroed by the caller), deviation
// [nc][nb], member [n] or null; bounds [nc][2] = (cos theta_hi, cos theta_lo); axis unit.
constexpr int kMaxCones = 16, kMaxPitchBins = 256;
hipError_t launch_pitch_cones(int64_t n, const double* ux, const double* uy, const double* uz,
                              const double axis[3], const double* bounds, int nc, const double* edges,
                              int nb, unsigned long long* counts, double* dev, int32_t* member,
                              hipStream_t stream);
hipError_t launch_spectral_diagnostics(const double* S, const double* a, double a_sum, int ns, int nd,
                                       int nw, const double* omega, const double ranges[4],
                                       double* avg, double* out, hipStream_t stream);

struct MfmaPlanCache;

// ---- the library's binary files (accumulator and network snapshots) ----
// 64-byte header: 8-byte magic, five int64 fields, payload length, FNV-1a 64 checksum of the
// payload; then the payload.  Host byte order (little-endian on every supported host).
struct FileHeader {
  char magic[8];
  int64_t f[5];
  uint64_t payload;
  uint64_t sum;
};
static_assert(sizeof(FileHeader) == 64, "file header is 64 bytes");

inline uint64_t fnv1a64(const void* data, size_t n) {
  const unsigned char* p = (const unsigned char*)data;
  uint64_t h = 0xcbf29ce484222325ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 0x100000001b3ull;
  }
  return h;
}

// Byte buffer with typed appends and reads (the payload of a file).
struct Bytes {
  std::vector<char> v;
  size_t at = 0;
  void put(const void* p, size_t n) { v.insert(v.end(), (const char*)p, (const char*)p + n); }
  bool get(void* p, size_t n) {
    if (at + n > v.size()) return false;
    memcpy(p, v.data() + at, n);
    at += n;
    return true;
  }
};

inline bool write_lw_file(const char* path, const char magic[8], const int64_t f[5], const Bytes& b) {
  FileHeader h;
  memcpy(h.magic, magic, 8);
  for (int i = 0; i < 5; ++i) h.f[i] = f[i];
  h.payload = b.v.size();
  h.sum = fnv1a64(b.v.data(), b.v.size());
  FILE* fp = fopen(path, "wb");
  if (!fp) return false;
  bool ok = fwrite(&h, sizeof(h), 1, fp) == 1 && (b.v.empty() || fwrite(b.v.data(), b.v.size(), 1, fp) == 1);
  ok = (fclose(fp) == 0) && ok;
  return ok;
}

// Reads the whole file; false with a reason on a missing, short, foreign or corrupted file.
inline bool read_lw_file(const char* path, const char magic[8], FileHeader* h, Bytes* b, std::string* why) {
  FILE* fp = fopen(path, "rb");
  if (!fp) {
    *why = "cannot open the file";
    return false;
  }
  bool ok = fread(h, sizeof(*h), 1, fp) == 1;
  if (!ok) *why = "file shorter than its header";
  if (ok && memcmp(h->magic, magic, 8) != 0) {
    ok = false;
    *why = "not a file of this kind (magic)";
  }
  if (ok && h->payload > ((uint64_t)1 << 40)) {
    ok = false;
    *why = "implausible payload length";
  }
  if (ok) {
    b->v.resize(h->payload);
    b->at = 0;
    if (h->payload && fread(b->v.data(), h->payload, 1, fp) != 1) {
      ok = false;
      *why = "file shorter than its payload";
    }
  }
  fclose(fp);
  if (ok && fnv1a64(b->v.data(), b->v.size()) != h->sum) {
    ok = false;
    *why = "checksum mismatch";
  }
  return ok;
}

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
  // coherent synthesis: summed amplitudes [ns][nd][nw][4] = (Re, Im) on e1, then on e2
  bool coherent = false;
  double* d_A = nullptr;
  // diagnostics scratch: weights [nd], average [ns][nw], rows [ns][nd + 1][8]
  double* d_diag = nullptr;
  size_t diag_cap = 0;
  unsigned long long* d_err = nullptr;
  // lowest particle index whose retarded-time span outgrew the matrix-core plan
  unsigned long long* d_overflow = nullptr;
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
  // FP32 launch shape overrides (0 = automatic); persistent launch when a plan matches
  int tune_wpt = 0, tune_pb = 0, tune_persistent = 1;
  struct Plan {
    bool valid = false;
    const void* offsets = nullptr;  // batch identity the plan was made for
    int64_t n = -1;
    int32_t nd = 0, nw = 0, ns = 0, ncomp = 0, wpt = 0, pb = 0, n_tiles = 0;
    int64_t n_blocks = 0, n_items = 0;
    int workgroups = 0;
    int64_t* d_perm = nullptr;
    size_t perm_cap = 0;
    int64_t* d_order = nullptr;
    size_t order_cap = 0;
  } plan;
  unsigned* d_ticket = nullptr;
  // per work-group timing of the last persistent FP32 launch made with profiling on
  unsigned long long* d_wgtime = nullptr;
  int wgtime_cap = 0, wgtime_n = 0;
  unsigned* d_flag = nullptr;  // invalid-index flag of lw_subset_offsets
  bool capturing = false;  // inside lw_graph_capture: no synchronisation allowed
  // bumped whenever a device buffer that captured work refers to is freed, moved or refilled
  // for another batch (accumulators, grids, persistent plan); a graph records it at capture
  uint64_t epoch = 0;
};

struct lw_graph {
  lw_ctx* ctx = nullptr;
  uint64_t epoch = 0, mfma_epoch = 0;  // the context's buffers the graph was captured on
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace lw {
// FP32 kernel launch shape.
struct DirectShape {
  int wpt;
  int32_t n_tiles;
  int32_t pb;
  int64_t n_blocks;
};
inline int pick_wpt(int32_t nw) {
  if (nw <= kThreads) return 1;
  if (nw <= 2 * kThreads) return 2;
  if (nw <= 4 * kThreads) return 4;
  return 8;
}
// Rows per (species, direction, frequency) of the FP32 accumulator in this context's mode.
inline int direct_ncomp(const lw_ctx* c) { return c->coherent ? 4 : 1; }
// LDS of the per-species accumulator: ns * ncomp * WPT * kThreads doubles, kept within 160 KiB.
constexpr size_t kMaxDirectLds = 160 * 1024;
inline size_t direct_lds(int ns, int ncomp, int wpt) {
  return sizeof(double) * (size_t)ns * ncomp * kThreads * wpt;
}
inline DirectShape direct_shape(const lw_ctx* c, int64_t P) {
  DirectShape s;
  s.wpt = c->tune_wpt ? c->tune_wpt : pick_wpt(c->nw);
  while (s.wpt > 1 && direct_lds(c->ns, direct_ncomp(c), s.wpt) > kMaxDirectLds) s.wpt /= 2;
  s.n_tiles = (c->nw + kThreads * s.wpt - 1) / (kThreads * s.wpt);
  // aim at >= 8 work-groups per compute unit (256 CUs) before batching particles
  const int64_t per_particle_items = (int64_t)c->nd * s.n_tiles;
  int64_t pb = (P * per_particle_items) / (8 * 256);
  if (pb < 1) pb = 1;
  if (pb > 64) pb = 64;
  if (c->tune_pb) pb = c->tune_pb;
  s.pb = (int32_t)pb;
  s.n_blocks = (P + pb - 1) / pb;
  return s;
}
// Work-groups of the persistent FP32 kernel resident per compute unit.
int direct_persistent_occupancy(int wpt, size_t shmem);
}  // namespace lw

namespace lw {
enum ProfKind { kProfDirect = 0, kProfSpread = 1, kProfGemm = 2, kProfKinds = 3 };
// Record an event pair around a launch when profiling is on (no-op otherwise).
hipError_t prof_begin(lw_ctx* c, int kind);
hipError_t prof_end(lw_ctx* c);
}  // namespace lw
