// lw_mfma.hip -- matrix-core path of the spectral sum (paper, Section 2.2).
//
// The sum over samples A(w) = sum_k g_k e^{i w tau_k} is recast so that the
// phase factors form one dense table shared by all particles:
//
//  * The frequencies are split into bands b (contiguous runs of the frequency
//    list) with centre w_c and half-width D.  For each (particle, direction,
//    band) the samples are spread onto a uniform grid t_q = (q - W/2) h,
//    h = pi / (sigma D), of the retarded time measured from the particle's
//    first sample, after demodulation by e^{i w_c tau}:
//        F(q) = sum_k g_k e^{i w_c tau'_k} phi(q - u_k),  u_k = tau'_k / h + W/2,
//    with the "exponential of semicircle" kernel
//        phi(x) = exp(beta (sqrt(1 - (2x/W)^2) - 1)),  |x| < W/2
//    (Barnett, Magland & af Klinteberg 2019).  tau' = tau - tau_0 only shifts
//    the phase of A, which the incoherent |A|^2 does not see.
//  * Then, by the Poisson summation formula, for |w - w_c| <= D
//        A(w) e^{-i w tau_0} = sum_q F(q) e^{i (w - w_c) t_q} / Phi((w - w_c) h),
//    Phi the Fourier transform of phi, up to aliasing terms suppressed by the
//    kernel (~4e-7 of the signal at a band edge; W and sigma below).
//  * sum_q F(q) e^{i nu_j q h} is a complex matrix product C = E F with the
//    table E[j, q] = e^{i nu_j q h} (nu_j = w_j - w_c) shared by every particle
//    and direction.  Written as a real product it has rows (j, re|im), inner
//    index (q, re|im) and columns (particle, polarisation):
//        [C_re]   [E_re  -E_im] [F_re]
//        [C_im] = [E_im   E_re] [F_im]
//    and runs on v_mfma_f32_32x32x16_{f16,bf16} with FP32 accumulation.
//    Operands are rounded to FP16 (or BF16); optionally each is split into
//    hi + lo parts and three products are summed (hi*hi + hi*lo + lo*hi), or
//    (FP16) only F is split and two are summed (E_hi*F_hi + E_hi*F_lo).
//    The F columns are scaled by a power of two so |F| <= 1 before rounding.
//  * The epilogue squares the product, weights each column with
//    w_p q_p^2 / scale^2, sums over columns and writes per-row partial sums;
//    a fixed-order reduction adds re and im rows of each frequency, applies
//    1 / (4 pi^2 Phi^2) and accumulates into S.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <limits>
#include <type_traits>
#include <vector>

#include "lw_mfma.h"

namespace lw {

// Kernel width W, oversampling sigma and shape beta, chosen by the precision of the
// contraction.  The worst alias-to-signal ratio at a band edge, the sum over m != 0 of
// |Phi(xi + 2 pi m)| / Phi(xi) at xi = pi / sigma, is 8.5e-8 for (10, 1.6, 20.5) and 4.1e-7
// for (8, 2, 18.4).  The first makes the contraction's inner dimension a fifth shorter for
// a quarter more spreading taps, but its deconvolution 1 / Phi grows 10x from the band
// centre to the edge (against 2.8x): harmless when the operands are split into hi + lo
// parts (rounding ~2^-22), not when a single FP16 or BF16 product carries ~2^-11.
struct KernelShape {
  int w;
  double sigma, beta;
};
constexpr KernelShape kShapeSplit = {10, 1.6, 20.5};   // hi/lo operands, three products
constexpr KernelShape kShapeSingle = {8, 2.0, 18.4};   // a table rounded once: one or two products
constexpr int kWMax = 10;
constexpr int kMaxBands = 16;
constexpr int kTileM = 128;        // GEMM rows per work-group
constexpr int kTileN = 128;        // GEMM columns per work-group (64 particles x 2 polarisations)
constexpr int kTileK = 32;         // inner-dimension step staged in LDS
constexpr int kPad = 8;            // LDS row padding (halves)
constexpr int kSpreadWin = 256;    // grid points per spreading window (one per thread)
constexpr int kTapCoef = 9;        // tap weight polynomials: degree 8 in z = 2 frac(u) - 1

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct Band {
  int j0, nj;        // frequency index range
  double wc, h;      // centre frequency, grid spacing
  double wc_turn;    // wc / (2 pi)
  int qmax;          // grid points allotted per (particle, direction)
  int m;             // GEMM rows (2 nj rounded up to kTileM)
  int kp;            // inner dimension stride (2 qmax rounded up to kTileK)
  int row_off;       // first row of this band in the stacked row space
  int64_t e_off;     // offset of this band's table (elements)
  int64_t f_off;     // offset of this band's F block (floats) inside one chunk
};

struct MfmaPlanCache {
  bool valid = false;
  int bands_req = 1;
  int products_f16 = 3, products_bf16 = 3;
  int tile = 4;  // contraction tile: 1 = 128 x 128, 2 = 256 x 128, 3 = 128 x 256, 4 = 256 x 256
  int64_t chunk_bytes = 24LL << 30;  // cap on F (all directions and bands) per chunk of particles
  KernelShape shape = kShapeSplit;  // spreading kernel the tables were built for
  uint64_t epoch = 0;               // bumped when the tables are freed
  int nb = 0;
  Band band[kMaxBands];
  double span = 0.0;     // span the tables were sized for
  int dtype = -1;        // 0: f16, 1: bf16 (table element type)
  int rows = 0;          // sum of band rows
  int64_t e_elems = 0;
  void* e_hi = nullptr;
  void* e_lo = nullptr;
  double* rowfac = nullptr;  // [nw] 1 / (4 pi^2 Phi(nu h)^2)
  double* rowc = nullptr;    // [nw][2] e^{-i nu W h / 2} / Phi(nu h): amplitude factor of a row pair
  int32_t* row_of_j = nullptr;  // [nw] stacked row of (j, re)
  double* d_span = nullptr;  // device scratch for the span reduction
  // the last batch whose span was measured against these tables (lw_workspace_size,
  // lw_plan_batch, or an accumulation that planned): later calls on it need no measurement,
  // the spreading kernel reports a particle that outgrew the plan instead
  const void* planned_offsets = nullptr;
  int64_t planned_n = -1;
  uint64_t planned_epoch = ~0ull;
};

struct SpreadArgs {
  BatchView b;
  int64_t p_begin;
  int32_t n_local;       // particles in this chunk
  const double* dirs;    // [nd][kDirStride]
  int32_t nd;
  Band band[kMaxBands];
  int nb;
  int64_t f_dir;         // floats of F per direction
  float* F;              // chunk F blocks, [d][band][2 n_local][kp]
  unsigned* colmax;      // [nd][nb][2 * n_local] float bits of max |F|
  int32_t* colq;         // [nd][nb][n_local] grid points of each particle
  int32_t n_ftile;       // column tiles per band
  int32_t ns;            // species count (a species outside [0, ns) is a data error)
  unsigned long long* err;
  unsigned long long* overflow;  // lowest particle whose span needs more grid points than planned
  unsigned long long* flops;  // null, or useful FLOPs of one product of the contraction
  // phi(i - W/2 + 1 - f) = sum_k tapc[i][k] z^k, z = 2 f - 1: the W tap weights of a sample
  // (mirror-symmetric: tapc[W - 1 - i][k] = (-1)^k tapc[i][k])
  // with fractional grid coordinate f (Chebyshev interpolants, within 2e-8 of phi)
  float tapc[kWMax][kTapCoef];
};

struct GemmArgs {
  BatchView b;
  int64_t p_begin;
  int32_t n_local;
  int32_t n_ftile;
  Band band[kMaxBands];
  int nb;
  int32_t nd;
  int64_t f_dir;         // floats of F per direction
  int order[kMaxBands];             // bands in launch order (heaviest first)
  int tiles_before[kMaxBands + 1];  // prefix count of work-groups per band, per direction
  const void* e_hi;
  const void* e_lo;
  const float* F;
  const unsigned* colmax;
  const int32_t* colq;
  const int32_t* perm;   // [nd][nb][n_local] particles of each (direction, band) by decreasing q
  double* partial;       // [nd][n_ftile][ns][rows], or [nd][n_ftile][ns][rows][2] when coherent
  int32_t ns, rows;
  // coherent synthesis: columns keep their phase e^{i w tau_0} and add w q A per species
  int32_t coherent;
  const double* dirs;    // [nd][kDirStride]
  const double* wturn;   // [nw] omega / (2 pi)
  // amplitude state: each column's amplitude is added to amp[p][d][j][2 pol + (re, im)]
  // (no partial sums); rowc [nw][2] is the row factor the reduction applies otherwise
  double* amp;
  const double* rowc;
  int32_t wturn_n;       // nw
};

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ double dot3(const double a[3], double x, double y, double z) {
  return a[0] * x + a[1] * y + a[2] * z;
}

__device__ __forceinline__ double retarded_time(const BatchView& b, int64_t idx, double t,
                                                const double n[3]) {
  return t - dot3(n, b.x[idx], b.y[idx], b.z[idx]);
}


// ------------------------------------------------------------------ span of every (particle, direction)
__global__ void lw_span_kernel(BatchView b, const double* dirs, int nd, double* out_max) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double s = 0.0;
  if (i < b.n_particles * (int64_t)nd) {
    const int64_t p = i / nd;
    const int d = (int)(i % nd);
    const int64_t o = b.offsets[p], len = b.offsets[p + 1] - o;
    if (len > 1) {
      const double n[3] = {dirs[kDirStride * d], dirs[kDirStride * d + 1], dirs[kDirStride * d + 2]};
      const double ta = retarded_time(b, o, b.t0[p], n);
      const double tb = retarded_time(b, o + len - 1, b.t0[p] + (double)(len - 1) * b.dt[p], n);
      s = tb - ta;
      if (!(s >= 0.0) || !isfinite(s)) s = 0.0;  // bad data is flagged by the spread kernel
    }
  }
  // wave max, then one atomic per wave (positive doubles order like their bit patterns)
  for (int off = 32; off > 0; off >>= 1) s = fmax(s, __shfl_xor(s, off));
  if ((threadIdx.x & 63) == 0 && s > 0.0)
    atomicMax((unsigned long long*)out_max, (unsigned long long)__double_as_longlong(s));
}

// ------------------------------------------------------------------ phase table
template <typename T>
__global__ void lw_etable_kernel(T* hi, T* lo, const double* omega, Band bd) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = (int64_t)bd.m * bd.kp;
  if (i >= total) return;
  const int row = (int)(i / bd.kp), kk = (int)(i % bd.kp);
  const int jl = row >> 1, a = row & 1;  // a: 0 = re row, 1 = im row
  const int q = kk >> 1, c = kk & 1;     // c: 0 = multiplies F_re, 1 = multiplies F_im
  double v = 0.0;
  if (jl < bd.nj && q < bd.qmax) {
    const double nu = omega[bd.j0 + jl] - bd.wc;
    // turn fraction of nu q h / (2 pi) in FP64, then FP64 sin/cos
    const double x = nu * (double)q * bd.h * (0.5 / M_PI);
    const double f = x - rint(x);
    const double cs = cos(2.0 * M_PI * f), sn = sin(2.0 * M_PI * f);
    // rows: re = [cos, -sin], im = [sin, cos]
    v = (a == 0) ? (c == 0 ? cs : -sn) : (c == 0 ? sn : cs);
  }
  const T h = (T)v;
  hi[bd.e_off + i] = h;
  lo[bd.e_off + i] = (T)(v - (double)h);
}

// ------------------------------------------------------------------ spreading
// One work-group per (particle of the chunk, direction, group of up to two bands).
// Samples are sorted in tau because dtau/dt = kappa > 0, so each sample's W taps (W even)
// cover grid points lo_s .. lo_s + W - 1 with lo_s = floor(u_s) - W/2 + 1 nondecreasing in
// s, in every band.  The trajectory is walked in chunks of 256 samples, each loaded once:
//   1. one thread per sample: the prepass (retarded time, integrand) shared by the bands,
//      and each band's grid coordinate;
//   2. per band in turn: the demodulated integrand and the W tap weights
//      phi(lo_s + i - u_s) go to LDS, and first[x] = the first sample of the chunk whose
//      taps reach grid point base + x (built by the samples themselves, no search); the
//      samples reaching q are then exactly first[x] .. first[x + W] - 1;
//   3. per band, one lane (or S lanes taking every S-th sample, summed across lanes) per
//      pair of adjacent grid points adds w g over the samples reaching either point;
//   4. a point below the next chunk's first tap is final and is written to F (FP32); the
//      points at or above it (fewer than W: the next chunk starts with the sample whose
//      taps reach that tap) are carried to the next chunk in a small LDS buffer; the
//      chunk's points that no sample reached are written as zeros.
// A chunk takes the samples whose taps stay within kWin points of the oldest unwritten
// point in every band; the next chunk starts with the first sample it did not take.
// kWin = 512 covers a 256-sample chunk up to two grid points per sample; the work-group
// keeps 19 KB of LDS, and with at most 80 VGPRs (the launch bound below asks for six waves
// per SIMD) six work-groups share a CU.
constexpr int kWin = 512;
constexpr int kSpreadWavesPerSimd = 6;
constexpr int kBandGroup = 2;  // bands per work-group

template <int kW>
struct SpreadStage {
  static_assert(kW % 2 == 0 && kW <= kWMax, "even widths: the tap window must not depend on frac(u)");
  float4 g[kSpreadWin];           // demodulated integrand (re1, im1, re2, im2) of the band
  // tap i of sample s at w[i + 1][s]; rows 0 and kW + 1 stay zero, so that a pair of
  // adjacent grid points reads taps i and i + 1 of any sample reaching either of them
  float w[kW + 2][kSpreadWin];
  int lo[kSpreadWin];             // first grid point of each sample's taps
  short first[kWin + kW + 1];     // first sample reaching grid point base + x
  // grid sums still open at a chunk boundary, per band, read and written in turn
  float4 carry[kBandGroup][2][kW];
};

// One sample's trajectory data, loaded a chunk ahead of its use.
struct RawSample {
  double x, y, z, bx, by, bz;
  float ax, ay, az;
};

__device__ __forceinline__ void load_raw(const BatchView& b, int64_t o, int64_t len, int64_t kc,
                                         RawSample& r) {
  const int64_t k = kc + threadIdx.x;
  if (k >= len) return;
  const int64_t idx = o + k;
  r.x = b.x[idx];
  r.y = b.y[idx];
  r.z = b.z[idx];
  r.bx = b.bx[idx];
  r.by = b.by[idx];
  r.bz = b.bz[idx];
  if (b.adx) {
    r.ax = (float)b.adx[idx];
    r.ay = (float)b.ady[idx];
    r.az = (float)b.adz[idx];
  } else {
    r.ax = b.ax[idx];
    r.ay = b.ay[idx];
    r.az = b.az[idx];
  }
}

__device__ __forceinline__ float dot3f(const float a[3], float x, float y, float z) {
  return fmaf(a[0], x, fmaf(a[1], y, a[2] * z));
}

// The band-independent part of a sample: retarded time from the first sample (FP64) and
// the integrand's two polarisation components (FP32); invalid samples are reported.
struct Prepass {
  double taup;
  float g1, g2;
  bool ok;
};

__device__ __forceinline__ Prepass prepass(const SpreadArgs& a, const RawSample& r, const double* n,
                                           const float* frame, int64_t p, int64_t k, double t0, double dtp,
                                           double tau0) {
  const float* nf = frame;
  const float* e1f = frame + 3;
  const float* e2f = frame + 6;
  const double bx = r.bx, by = r.by, bz = r.bz;
  // kappa = 1 - n.beta cancels as |beta| -> 1 and stays FP64; the integrand is used in FP32
  // and is formed in FP32 from it (e.(n x ((n - beta) x a)) = -(e.beta)(n.a) - kappa (e.a))
  const double kap = 1.0 - dot3(n, bx, by, bz);
  const float kf = (float)kap, bxf = (float)bx, byf = (float)by, bzf = (float)bz;
  const float na = dot3f(nf, r.ax, r.ay, r.az);
  const float sc = (float)dtp * __builtin_amdgcn_rcpf(kf * kf);
  Prepass q;
  q.g1 = -(na * dot3f(e1f, bxf, byf, bzf) + kf * dot3f(e1f, r.ax, r.ay, r.az)) * sc;
  q.g2 = -(na * dot3f(e2f, bxf, byf, bzf) + kf * dot3f(e2f, r.ax, r.ay, r.az)) * sc;
  q.taup = (t0 + (double)k * dtp - dot3(n, r.x, r.y, r.z)) - tau0;
  q.ok = (bx * bx + by * by + bz * bz < 1.0) && isfinite(q.taup) && isfinite(q.g1) && isfinite(q.g2);
  if (!q.ok) atomicMin(a.err, (unsigned long long)p);
  return q;
}

// Grid coordinate of a sample in one band, kept within the grid even for invalid samples
// (those add nothing): the first tap's grid point and the fraction of u.
template <int kW>
__device__ __forceinline__ void grid_coord(const Prepass& q, double inv_h, double umax, int& lo, float& fu) {
  double u = q.taup * inv_h + 0.5 * kW;
  u = q.ok ? fmin(fmax(u, 0.5 * kW), umax) : 0.5 * kW;
  const double iu = floor(u);
  fu = (float)(u - iu);
  lo = (int)iu - (kW / 2 - 1);
}

// One band's stage of a sample: demodulated integrand and the W tap weights.
template <int kW>
__device__ __forceinline__ void stage_band(SpreadStage<kW>& st, const Prepass& q, double wc_turn, int lo,
                                           float fu, const float (*tap)[kTapCoef]) {
  const int tid = threadIdx.x;
  const double x = wc_turn * q.taup;
  const float fr = (float)(x - rint(x));
  const float cs = __builtin_amdgcn_cosf(fr), sn = __builtin_amdgcn_sinf(fr);
  st.lo[tid] = lo;
  const float z = 2.0f * fu - 1.0f, z2 = z * z;
  // phi(q - u) for q = lo + i: tap i is E(z^2) + z O(z^2) and tap W - 1 - i is E - z O, with
  // E and O the even and odd parts of tap i's polynomial, each by Horner in z^2
  static_assert(kTapCoef % 2 == 1, "the highest power is even");
#pragma unroll
  for (int i = 0; i < kW / 2; ++i) {
    float e = tap[i][kTapCoef - 1], o = tap[i][kTapCoef - 2];
#pragma unroll
    for (int c = kTapCoef - 3; c >= 0; c -= 2) e = fmaf(e, z2, tap[i][c]);
#pragma unroll
    for (int c = kTapCoef - 4; c >= 1; c -= 2) o = fmaf(o, z2, tap[i][c]);
    st.w[i + 1][tid] = fmaf(z, o, e);
    st.w[kW - i][tid] = fmaf(-z, o, e);
  }
  const float G1 = q.ok ? q.g1 : 0.f, G2 = q.ok ? q.g2 : 0.f;
  st.g[tid] = make_float4(G1 * cs, G1 * sn, G2 * cs, G2 * sn);
}

// Work-groups go to the eight XCDs in turn (block b to XCD b mod 8).  This numbering gives
// each XCD a contiguous run of n items instead, so that neighbouring items -- every (direction,
// band group) of one particle -- run on one XCD and read the particle's trajectory through
// one L2.  XCD x holds blocks x, x + 8, ...: m + (x < r) of them with n = 8 m + r, numbered
// from x m + min(x, r); the map is a bijection of [0, n).
__device__ __forceinline__ int xcd_contiguous(int b, int n) {
  const int m = n / 8, r = n % 8, x = b % 8, j = b / 8;
  return x * m + min(x, r) + j;
}

// Sum N values over each aligned group of S consecutive lanes (S a power of two up to 64),
// leaving the sum in every lane of the group.  Within a row of 16 lanes the partners come
// from DPP lane permutations (after the xor-1 and xor-2 steps all lanes of a quad agree, so
// the half-row and row mirrors pair equal-valued groups); wider groups use shuffles.
template <int kCtrl>
__device__ __forceinline__ float dpp_partner(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), kCtrl, 0xF, 0xF, false));
}

template <int N>
__device__ __forceinline__ void group_sum(float* v, int S) {
  constexpr int kXor1 = 0xB1, kXor2 = 0x4E, kHalfMirror = 0x141, kMirror = 0x140;
#pragma unroll
  for (int j = 0; j < N; ++j) v[j] += dpp_partner<kXor1>(v[j]);
  if (S >= 4) {
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] += dpp_partner<kXor2>(v[j]);
  }
  if (S >= 8) {
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] += dpp_partner<kHalfMirror>(v[j]);
  }
  if (S >= 16) {
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] += dpp_partner<kMirror>(v[j]);
  }
  for (int off = 16; off < S; off <<= 1) {
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] += __shfl_xor(v[j], off);
  }
}

// Sum over each half-wave (lanes 0-31 and 32-63) without LDS traffic: the four in-row DPP
// steps of group_sum leave every lane of a row of 16 with its row's sum, and the row
// broadcast (lane 15 of a row to the next row, rows 1 and 3 written) adds row 0's sum into
// row 1 and row 2's into row 3, so lanes 31 and 63 hold their half-wave's sum.
__device__ __forceinline__ float half_wave_sum(float v) {
  constexpr int kRowBcast15 = 0x142;
  float t[1] = {v};
  group_sum<1>(t, 16);
  return t[0] + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(t[0]), kRowBcast15, 0xA, 0xF, false));
}

// A band's walk along the trajectory, shared by the work-group in LDS.
struct BandWalk {
  int Q;      // grid points of the column
  int qdone;  // grid points [0, qdone) are written
  int cbase;  // first grid point of the open sums carried in from the previous chunk
  int par;    // carry buffer read by this chunk
};

// Gather of one band over the staged chunk: pairs of grid points, final points to the
// band's two F columns (byte pointers c0, c1), the open ones to the carry buffer.  Every
// thread reads the walk state before the first barrier here; thread 0 writes it back after,
// to be read after the next chunk's first barrier.  Returns the band's new qdone.
template <int kW>
__device__ __forceinline__ int gather_band(SpreadStage<kW>& st, BandWalk& bws, int k, int take, int cnt,
                                           bool last, char* c0, char* c1, float& wmax) {
  const int tid = threadIdx.x;
  const BandWalk bw = bws;
  const int base = st.lo[0];
  const int top = st.lo[take - 1] + kW - 1;  // highest grid point touched
  const int G = min(top - base + 1, kWin);
  // grid points below the next chunk's first tap are final after this chunk
  int qfin = bw.Q;
  if (!last) qfin = min(bw.Q, take < cnt ? st.lo[take] : top + 1);
  // first sample reaching each grid point of the chunk
  if (tid < take) {
    const int prev = tid == 0 ? base - 1 : st.lo[tid - 1] + kW - 1;
    const int mine = st.lo[tid] + kW - 1;
    for (int x = max(prev + 1, base) - base; x <= min(mine - base, G - 1); ++x) st.first[x] = (short)tid;
  }
  if (tid <= kW) st.first[max(G, 0) + tid] = (short)take;  // past the last point: no sample
  float4* const cin = st.carry[k][bw.par];
  float4* const cout = st.carry[k][bw.par ^ 1];
  __syncthreads();
  const int G2 = (G + 1) >> 1;
  int S = 1;
  while (S < 64 && 2 * S * G2 <= kSpreadWin) S *= 2;
  const int per_pass = kSpreadWin / S;
  for (int yb = 0; yb < G2; yb += per_pass) {
    const int y = yb + tid / S, sl = tid % S;
    const bool live = y < G2;
    const int x0 = live ? 2 * y : 0;
    // (clamped, and the tap index too: on invalid, unsorted data an entry may be stale);
    // lanes past the last pair get an empty range
    const int s_begin = min(max((int)st.first[x0], 0), take);
    const int s_end = live ? min(max((int)st.first[x0 + 1 + kW], s_begin), take) : s_begin;
    float acc[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[j] = 0.f;
    const int q0 = base + x0;
#pragma unroll 1
    for (int s = s_begin + sl; s < s_end; s += S) {
      const int r = min(max(q0 - st.lo[s], -1), kW - 1) + 1;  // row of tap x0 - lo
      const float w0 = st.w[r][s], w1 = st.w[r + 1][s];
      const float4 gv = st.g[s];
      acc[0] = fmaf(w0, gv.x, acc[0]);
      acc[1] = fmaf(w0, gv.y, acc[1]);
      acc[2] = fmaf(w0, gv.z, acc[2]);
      acc[3] = fmaf(w0, gv.w, acc[3]);
      acc[4] = fmaf(w1, gv.x, acc[4]);
      acc[5] = fmaf(w1, gv.y, acc[5]);
      acc[6] = fmaf(w1, gv.z, acc[6]);
      acc[7] = fmaf(w1, gv.w, acc[7]);
    }
    if (S > 1) group_sum<8>(acc, S);
    if (live && sl == 0) {
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int x = x0 + j;
        if (x < G) {
          const int q = base + x;
          float4 v = make_float4(acc[4 * j], acc[4 * j + 1], acc[4 * j + 2], acc[4 * j + 3]);
          // sums opened by the previous chunk (its last W points at most; the carry window
          // is checked, so that stale entries of invalid data stay unread)
          const unsigned ci = (unsigned)(q - bw.cbase);
          if (ci < (unsigned)kW) {
            const float4 c = cin[ci];
            v.x += c.x;
            v.y += c.y;
            v.z += c.z;
            v.w += c.w;
          }
          // q >= qdone on valid data (the chunk starts at or after the oldest pending point);
          // on invalid data, which is reported, a point may be rewritten, still within [1, Q)
          if (q < qfin) {
            const uint32_t off = (uint32_t)q * 8u;  // byte offset of point q (q < Q <= 4e6)
            *(float2*)(c0 + off) = make_float2(v.x, v.y);
            *(float2*)(c1 + off) = make_float2(v.z, v.w);
            wmax = fmaxf(fmaxf(fmaxf(fmaxf(wmax, fabsf(v.x)), fabsf(v.y)), fabsf(v.z)), fabsf(v.w));
          } else {
            const unsigned co = (unsigned)(q - qfin);  // < W on valid data
            if (co < (unsigned)kW) cout[co] = v;
          }
        }
      }
    }
  }
  // final points outside [base, base + G) were reached by no sample: below the first
  // chunk's first tap, in a gap between two samples wider than the kernel, or past the
  // last tap of the trajectory
  for (int q = bw.qdone + tid; q < min(base, qfin); q += kSpreadWin) {
    *(float2*)(c0 + (uint32_t)q * 8u) = make_float2(0.f, 0.f);
    *(float2*)(c1 + (uint32_t)q * 8u) = make_float2(0.f, 0.f);
  }
  for (int q = max(base + G, bw.qdone) + tid; q < qfin; q += kSpreadWin) {
    *(float2*)(c0 + (uint32_t)q * 8u) = make_float2(0.f, 0.f);
    *(float2*)(c1 + (uint32_t)q * 8u) = make_float2(0.f, 0.f);
  }
  if (tid == 0) bws = BandWalk{bw.Q, max(bw.qdone, qfin), qfin, bw.par ^ 1};
  return max(bw.qdone, qfin);
}

// The particle's two F columns of band bi for direction d, as byte pointers.
__device__ __forceinline__ void band_columns(const SpreadArgs& a, int bi, int d, int pl, char*& c0, char*& c1) {
  const Band& bd = a.band[bi];
  float* Fb = a.F + (size_t)d * a.f_dir + bd.f_off;
  c0 = (char*)(Fb + (size_t)(2 * pl) * bd.kp);
  c1 = (char*)(Fb + (size_t)(2 * pl + 1) * bd.kp);
}

template <int kW>
__global__ __launch_bounds__(kSpreadWin, kSpreadWavesPerSimd) void lw_spread_kernel(SpreadArgs a) {
  __shared__ SpreadStage<kW> st;
  __shared__ BandWalk s_walk[kBandGroup];
  __shared__ float s_wmax[kBandGroup][kSpreadWin / 64];
  // the first W/2 tap polynomials, read at one address by all lanes (held as kernel
  // arguments they would crowd the scalar registers)
  __shared__ float s_tap[kW / 2][kTapCoef];
  // the direction and its polarisation axes in FP32 (read at one address by all lanes)
  __shared__ float s_frame[9];
  __shared__ double s_n[3];

  const int tid = threadIdx.x;
  // block -> item -> (particle, direction, band group); groups fastest so one particle's
  // work is adjacent, and each XCD takes a contiguous run of items
  const int ng = (a.nb + kBandGroup - 1) / kBandGroup;
  const int item = xcd_contiguous((int)blockIdx.x, (int)gridDim.x);
  const int gi = item % ng;
  const int d = (item / ng) % a.nd;
  const int pl = item / (ng * a.nd);
  const int b0 = gi * kBandGroup;
  const int nbg = min(kBandGroup, a.nb - b0);  // bands of this group (1 or 2)
  const int64_t p = a.p_begin + pl;
  const int64_t o = a.b.offsets[p], len = a.b.offsets[p + 1] - o;
  const double t0 = a.b.t0[p], dtp = a.b.dt[p];
  const int ncol = 2 * a.n_local;
  double n[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) n[c] = a.dirs[kDirStride * d + c];
  if (tid < 9) s_frame[tid] = (float)a.dirs[kDirStride * d + tid];
  if (tid < 3) s_n[tid] = a.dirs[kDirStride * d + tid];

  if (tid == 0 && gi == 0 && d == 0 && a.b.species) {
    const int sp = a.b.species[p];
    if (sp < 0 || sp >= a.ns) atomicMin(a.err, (unsigned long long)p);
  }
  if (tid == 0 && gi == 0 && d == 0 && len < 0) atomicMin(a.err, (unsigned long long)p);
  double tau0 = 0.0;
  if (len > 0) tau0 = retarded_time(a.b, o, t0, n);
  if (tid < nbg) {
    const Band& bd = a.band[b0 + tid];
    int Q = 0;
    if (len > 0) {
      const double taul = retarded_time(a.b, o + len - 1, t0 + (double)(len - 1) * dtp, n);
      double span = taul - tau0;
      if (!(span >= 0.0) || !isfinite(span)) span = 0.0;
      const double qneed = ceil(span / bd.h) + kW + 1;
      // a batch that outgrew the plan is reported, not silently clipped
      if (qneed > (double)bd.qmax) atomicMin(a.overflow, (unsigned long long)p);
      Q = (int)fmin(qneed, (double)bd.qmax);
    }
    s_walk[tid] = BandWalk{Q, 0, 0, 0};
  }
  st.w[0][tid] = 0.f;
  st.w[kW + 1][tid] = 0.f;
  if (tid < kBandGroup * 2 * kW) (&st.carry[0][0][0])[tid] = make_float4(0.f, 0.f, 0.f, 0.f);
  if (tid < (kW / 2) * kTapCoef) s_tap[tid / kTapCoef][tid % kTapCoef] = a.tapc[tid / kTapCoef][tid % kTapCoef];
  __syncthreads();
  float wmax0 = 0.0f, wmax1 = 0.0f;  // this thread's largest |F| written, per band
  // each thread's copy of the bands' qdone, for the chunk's fit test (which precedes the
  // chunk's first barrier, so it cannot read the shared walk state)
  int qd0 = 0, qd1 = 0;
  int64_t kc = 0;
  // the chunk after this one usually starts one sample before this one ends: its data
  // is requested while this chunk is processed
  RawSample raw, next;
  int64_t k_next = 0;
  load_raw(a.b, o, len, 0, next);
  while (kc < len) {
    if (k_next != kc) load_raw(a.b, o, len, kc, next);  // the guess missed: load now
    raw = next;
    const int cnt = (int)min((int64_t)kSpreadWin, len - kc);
    k_next = kc + (kc + cnt < len ? cnt - 1 : cnt);
    Prepass pq = {0.0, 0.f, 0.f, false};
    if (tid < cnt) pq = prepass(a, raw, s_n, s_frame, p, kc + tid, t0, dtp, tau0);
    if (k_next < len) load_raw(a.b, o, len, k_next, next);  // after the prepass: raw is dead
    // each band's grid coordinate; a chunk takes the samples whose taps stay within kWin
    // of the oldest unwritten point in every band; its last sample waits for the next
    // chunk unless it ends the trajectory, so that the next chunk's first tap is known here
    // (the count also orders the previous chunk's reads of the stage before this chunk's
    // writes)
    int lo0, lo1 = 0;
    float fu0, fu1 = 0.f;
    {
      const Band& bd = a.band[b0];
      grid_coord<kW>(pq, 1.0 / bd.h, (double)bd.qmax + 0.5 * kW, lo0, fu0);
    }
    bool fit = tid < cnt && lo0 - qd0 <= kWin - kW;
    if (nbg > 1) {
      const Band& bd = a.band[b0 + 1];
      grid_coord<kW>(pq, 1.0 / bd.h, (double)bd.qmax + 0.5 * kW, lo1, fu1);
      fit = fit && lo1 - qd1 <= kWin - kW;
    }
    const bool more = kc + cnt < len;
    const int fits = __syncthreads_count(fit);
    int take = min(fits, more ? cnt - 1 : cnt);
    take = max(take, 1);
    const bool last = kc + take >= len;
#pragma unroll 1
    for (int k = 0; k < nbg; ++k) {
      if (k > 0) __syncthreads();  // the previous band's gather no longer reads the stage
      const Band& bd = a.band[b0 + k];
      if (tid < cnt) stage_band<kW>(st, pq, bd.wc_turn, k ? lo1 : lo0, k ? fu1 : fu0, s_tap);
      if (tid < kW) st.carry[k][s_walk[k].par ^ 1][tid] = make_float4(0.f, 0.f, 0.f, 0.f);
      __syncthreads();
      char *c0, *c1;
      band_columns(a, b0 + k, d, pl, c0, c1);
      float wm = k ? wmax1 : wmax0;
      const int qd = gather_band<kW>(st, s_walk[k], k, take, cnt, last, c0, c1, wm);
      if (k) {
        wmax1 = wm;
        qd1 = qd;
      } else {
        wmax0 = wm;
        qd0 = qd;
      }
    }
    kc += take;
  }
  // column maximum (one value for both polarisation columns keeps them on one scale)
  for (int off = 32; off > 0; off >>= 1) {
    wmax0 = fmaxf(wmax0, __shfl_xor(wmax0, off));
    wmax1 = fmaxf(wmax1, __shfl_xor(wmax1, off));
  }
  if ((tid & 63) == 0) {
    s_wmax[0][tid >> 6] = wmax0;
    s_wmax[1][tid >> 6] = wmax1;
  }
  __syncthreads();
#pragma unroll 1
  for (int k = 0; k < nbg; ++k) {
    const int Q = s_walk[k].Q;
    char *c0, *c1;
    band_columns(a, b0 + k, d, pl, c0, c1);
    // The inner dimension is read in groups of eight floats: clear the rest of the
    // column's last group (at most three grid points, within kp), so that the contraction
    // loads whole groups and needs no mask.
    if (tid < ((2 * Q + 7) / 8 * 8 - 2 * Q) / 2) {
      *(float2*)(c0 + (uint32_t)(Q + tid) * 8u) = make_float2(0.f, 0.f);
      *(float2*)(c1 + (uint32_t)(Q + tid) * 8u) = make_float2(0.f, 0.f);
    }
    if (tid == 0) {
      const int bi = b0 + k, db = d * a.nb + bi;
      float m = 0.f;
      for (int w = 0; w < kSpreadWin / 64; ++w) m = fmaxf(m, s_wmax[k][w]);
      a.colmax[db * ncol + 2 * pl] = __float_as_uint(m);
      a.colmax[db * ncol + 2 * pl + 1] = __float_as_uint(m);
      a.colq[db * a.n_local + pl] = Q;
      // rows (2 nj) x columns (2 polarisations) x inner (2 Q) multiply-adds of one product
      if (a.flops) atomicAdd(a.flops, 2ull * (2ull * a.band[bi].nj) * 2ull * (2ull * Q));
    }
  }
}

// ------------------------------------------------------------------ column order
// One work-group per (direction, band, block of up to kSortBlock particles): the block's
// particles ordered by decreasing grid length q (ties by index), so that each contraction
// tile holds columns of similar inner length and stops where its longest column ends.  A
// tile (64 or 128 particles) never straddles two blocks; the contraction takes each tile's
// length as the maximum over its columns, so any order is correct and the sort only saves
// work.  Bitonic sort of 64-bit keys in LDS: deterministic.
constexpr int kSortBlock = 16384;

__global__ __launch_bounds__(1024) void lw_sort_columns_kernel(const int32_t* colq, int n_local,
                                                               int32_t* perm) {
  __shared__ unsigned long long key[kSortBlock];
  const int nblk = (n_local + kSortBlock - 1) / kSortBlock;
  const int seg = blockIdx.x / nblk;
  const int i0 = (blockIdx.x % nblk) * kSortBlock;
  const int n = min(kSortBlock, n_local - i0);
  const int32_t* q = colq + (size_t)seg * n_local;
  int n2 = 1;
  while (n2 < n) n2 <<= 1;
  for (int i = threadIdx.x; i < n2; i += blockDim.x)
    key[i] = i < n ? ((unsigned long long)(0x7fffffffu - (unsigned)q[i0 + i]) << 32) | (unsigned)(i0 + i)
                   : ~0ull;
  __syncthreads();
  for (int k = 2; k <= n2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < n2; i += blockDim.x) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const unsigned long long x = key[i], y = key[l];
          if ((x > y) == up) {
            key[i] = y;
            key[l] = x;
          }
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    perm[(size_t)seg * n_local + i0 + i] = (int32_t)(key[i] & 0xffffffffull);
}

// ------------------------------------------------------------------ DFT contraction on MFMA
template <typename T>
struct MfmaOp;
template <>
struct MfmaOp<_Float16> {
  typedef half8 vec;
  static __device__ __forceinline__ f32x16 mma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};
template <>
struct MfmaOp<__bf16> {
  typedef bf16x8 vec;
  static __device__ __forceinline__ f32x16 mma(vec a, vec b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};

// Global loads of one inner step into registers (A: 8-element vectors of the phase
// table; B: float4 of F).  The loads are unconditional (columns past the chunk read
// column 0) so that nothing waits on them before they are stored; the store step
// zeroes what lies past each column's length.
template <typename T, int NP, int A_VEC, int B_VEC, int NT>
__device__ __forceinline__ void gemm_load_step(u32x4 (&ra0)[A_VEC], u32x4 (&ra1)[A_VEC],
                                               f32x4 (&rb)[B_VEC], const T* E_hi, const T* E_lo,
                                               const float* Fb, const int* s_q2, const int* s_fcol,
                                               int tid, int row0, int kp, int k0) {
#pragma unroll
  for (int v = 0; v < A_VEC; ++v) {
    const int c = tid + v * NT;
    const int r = c / (kTileK / 8), kc = (c % (kTileK / 8)) * 8;
    const size_t g = (size_t)(row0 + r) * kp + k0 + kc;
    ra0[v] = *(const u32x4*)(E_hi + g);
    if (NP > 1) ra1[v] = *(const u32x4*)(E_lo + g);
  }
#pragma unroll
  for (int v = 0; v < B_VEC; ++v) {
    const int c = tid + v * NT;
    const int col = c / (kTileK / 4), kc = (c % (kTileK / 4)) * 4;
    const int fc = max(s_fcol[col], 0);
    rb[v] = *(const f32x4*)(Fb + (size_t)fc * kp + k0 + kc);
  }
}

// Registers -> LDS: A as loaded; B scaled to |F| <= 1 and rounded (hi, and lo = rest),
// zero past each column's length.
template <typename T, int NP, int A_VEC, int B_VEC, int NT, int LD>
__device__ __forceinline__ void gemm_store_step(const u32x4 (&ra0)[A_VEC], const u32x4 (&ra1)[A_VEC],
                                                const f32x4 (&rb)[B_VEC], T* sA0, T* sA1, T* sB0,
                                                T* sB1, const float* s_scale, const int* s_q2,
                                                const int* s_fcol, int tid, int k0) {
#pragma unroll
  for (int v = 0; v < A_VEC; ++v) {
    const int c = tid + v * NT;
    const int r = c / (kTileK / 8), kc = (c % (kTileK / 8)) * 8;
    *(u32x4*)&sA0[r * LD + kc] = ra0[v];
    if (NP > 1) *(u32x4*)&sA1[r * LD + kc] = ra1[v];
  }
#pragma unroll
  for (int v = 0; v < B_VEC; ++v) {
    const int c = tid + v * NT;
    const int col = c / (kTileK / 4), kc = (c % (kTileK / 4)) * 4;
    const int lim = s_fcol[col] >= 0 ? s_q2[col] - (k0 + kc) : 0;  // valid elements of the float4
    const float sc = s_scale[col];
    const float x0 = lim > 0 ? rb[v].x * sc : 0.f, x1 = lim > 1 ? rb[v].y * sc : 0.f;
    const float x2 = lim > 2 ? rb[v].z * sc : 0.f, x3 = lim > 3 ? rb[v].w * sc : 0.f;
    typedef T t4 __attribute__((ext_vector_type(4)));
    const t4 hv = {(T)x0, (T)x1, (T)x2, (T)x3};
    *(t4*)&sB0[col * LD + kc] = hv;
    if (NP > 1) {
      const t4 lv = {(T)(x0 - (float)hv[0]), (T)(x1 - (float)hv[1]), (T)(x2 - (float)hv[2]),
                     (T)(x3 - (float)hv[3])};
      *(t4*)&sB1[col * LD + kc] = lv;
    }
  }
}

// Work-group tile TM x 128 with 8 waves arranged WM x WN (TM = 64 WM), each wave owning
// 64 rows x (128 / WN) columns as 2 x NB MFMA blocks of 32 x 32.  The inner dimension
// advances in steps of 32 through two LDS buffers: while the MFMAs of step k read one
// buffer, the operands of step k+1 travel from global memory to registers and then to
// the other buffer, with one barrier per step.
// MFMA 32x32x16 operand layout: lane l holds A[m = l%32][k = 8(l/32) .. +7] and
// B[k = 8(l/32) .. +7][n = l%32]; result register r of lane l is row
// 8(r/4) + 4(l/32) + r%4, column l%32.
template <typename T, int PRODUCTS, int WM>
__global__ __launch_bounds__(512) void lw_dft_mfma_kernel(GemmArgs a) {
  typedef typename MfmaOp<T>::vec vec;
  constexpr int NT = 512;
  constexpr int NW = NT / 64;
  constexpr int WN = NW / WM;
  constexpr int TM = 64 * WM;
  constexpr int NB = kTileN / (32 * WN);
  constexpr int LD = kTileK + kPad;
  static_assert(PRODUCTS == 1 || PRODUCTS == 3, "one or three products");
  constexpr int NP = PRODUCTS > 1 ? 2 : 1;
  constexpr int A_VEC = TM * kTileK / 8 / NT;       // 8-element vectors of A per thread
  constexpr int B_VEC = kTileN * kTileK / 4 / NT;   // float4 of F per thread
  static_assert(A_VEC >= 1 && B_VEC >= 1, "tile too small for the work-group");
  __shared__ __attribute__((aligned(16))) T sA[2][NP][TM * LD];
  __shared__ __attribute__((aligned(16))) T sB[2][NP][kTileN * LD];
  __shared__ float s_scale[kTileN];
  __shared__ int s_q2[kTileN];
  __shared__ int s_fcol[kTileN];  // F column of each tile column (-1 past the chunk)
  __shared__ int s_kmax;
  __shared__ float s_colw[kMaxSpecies][kTileN];
  __shared__ double s_rows[NW][64];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // block -> (band in heaviest-first order, column group, row tile).  Work-groups are
  // dispatched round-robin over the 8 XCDs; the mapping gives each XCD whole column
  // groups with all their row tiles in sequence, so a column group's F tile is read
  // from HBM once and reused from that XCD's L2 by the other row tiles.
  int oi = 0;
  while (oi + 1 < a.nb && (int)blockIdx.x >= a.tiles_before[oi + 1]) ++oi;
  const int bi = a.order[oi];
  const Band bd = a.band[bi];
  const int local = blockIdx.x - a.tiles_before[oi];
  const int mtiles = bd.m / TM;
  const int ngroups = a.nd * a.n_ftile;     // (direction, column tile) pairs
  const int xcd = local % 8, seq = local / 8;
  const int grp = (seq / mtiles) * 8 + xcd;
  if (grp >= ngroups) return;               // padding of the XCD-aware numbering
  const int mt = seq % mtiles;
  const int nt = grp % a.n_ftile;
  const int d = grp / a.n_ftile;
  const int ncol = 2 * a.n_local;
  const int db = d * a.nb + bi;
  const int col0 = nt * kTileN;
  const int row0 = mt * TM;
  const T* E_hi = (const T*)a.e_hi + bd.e_off;
  const T* E_lo = (const T*)a.e_lo + bd.e_off;
  const float* Fb = a.F + (size_t)d * a.f_dir + bd.f_off;

  if (tid == 0) s_kmax = 0;
  __syncthreads();
  if (tid < kTileN) {
    const int c = col0 + tid;
    float sc = 1.0f;
    int q2 = 0, fc = -1;
    for (int s = 0; s < a.ns; ++s) s_colw[s][tid] = 0.0f;
    if (c < ncol) {
      const int pl = a.perm[db * a.n_local + c / 2];  // columns in decreasing-length order
      fc = 2 * pl + (c & 1);
      const float m = __uint_as_float(a.colmax[db * ncol + fc]);
      if (m > 0.0f) {
        int e;
        frexpf(m, &e);  // m = f 2^e, f in [0.5, 1)
        sc = ldexpf(1.0f, -e);
      }
      q2 = 2 * a.colq[db * a.n_local + pl];
      atomicMax(&s_kmax, q2);
      const int64_t p = a.p_begin + pl;
      const int sp = a.b.species ? a.b.species[p] : 0;
      if (sp >= 0 && sp < a.ns) {
        const float qq = a.b.charge[p];
        s_colw[sp][tid] = a.b.weight[p] * qq * qq / (sc * sc);
      }
    }
    s_scale[tid] = sc;
    s_q2[tid] = q2;
    s_fcol[tid] = fc;
  }
  __syncthreads();
  const int kend = min(((s_kmax + kTileK - 1) / kTileK) * kTileK, bd.kp);

  u32x4 ra0[A_VEC], ra1[A_VEC];
  f32x4 rb[B_VEC];
  f32x16 acc[2][NB];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  const int wr = wave / WN, wc = wave % WN;
  if (kend > 0) {
    gemm_load_step<T, NP, A_VEC, B_VEC, NT>(ra0, ra1, rb, E_hi, E_lo, Fb, s_q2, s_fcol, tid, row0,
                                            bd.kp, 0);
    gemm_store_step<T, NP, A_VEC, B_VEC, NT, LD>(ra0, ra1, rb, sA[0][0], sA[0][NP - 1], sB[0][0],
                                                 sB[0][NP - 1], s_scale, s_q2, s_fcol, tid, 0);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = 0; k0 < kend; k0 += kTileK) {
    const bool more = k0 + kTileK < kend;
    if (more)
      gemm_load_step<T, NP, A_VEC, B_VEC, NT>(ra0, ra1, rb, E_hi, E_lo, Fb, s_q2, s_fcol, tid, row0,
                                              bd.kp, k0 + kTileK);
    const T* A0 = sA[buf][0];
    const T* A1 = sA[buf][NP - 1];
    const T* B0 = sB[buf][0];
    const T* B1 = sB[buf][NP - 1];
#pragma unroll
    for (int ks = 0; ks < kTileK; ks += 16) {
      const int kk = ks + 8 * (lane >> 5);
      vec fa[NP][2], fb[NP][NB];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int r = wr * 64 + i * 32 + (lane & 31);
        fa[0][i] = *(const vec*)&A0[r * LD + kk];
        if (NP > 1) fa[NP - 1][i] = *(const vec*)&A1[r * LD + kk];
      }
#pragma unroll
      for (int j = 0; j < NB; ++j) {
        const int cc = wc * (32 * NB) + j * 32 + (lane & 31);
        fb[0][j] = *(const vec*)&B0[cc * LD + kk];
        if (NP > 1) fb[NP - 1][j] = *(const vec*)&B1[cc * LD + kk];
      }
      // products outermost: consecutive MFMAs write different accumulators
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = MfmaOp<T>::mma(fa[0][i], fb[0][j], acc[i][j]);
      if (PRODUCTS > 1) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) acc[i][j] = MfmaOp<T>::mma(fa[0][i], fb[NP - 1][j], acc[i][j]);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < NB; ++j) acc[i][j] = MfmaOp<T>::mma(fa[NP - 1][i], fb[0][j], acc[i][j]);
      }
    }
    if (more)
      gemm_store_step<T, NP, A_VEC, B_VEC, NT, LD>(ra0, ra1, rb, sA[buf ^ 1][0], sA[buf ^ 1][NP - 1],
                                                   sB[buf ^ 1][0], sB[buf ^ 1][NP - 1], s_scale, s_q2,
                                                   s_fcol, tid, k0 + kTileK);
    __syncthreads();
    buf ^= 1;
  }

  // epilogue: per species, sum_c colw[c] * C[r][c]^2 over this tile's columns
  for (int s = 0; s < a.ns; ++s) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        float v = 0.0f;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
          const int cc = wc * (32 * NB) + j * 32 + (lane & 31);
          const float c = acc[i][j][r];
          v = fmaf(c * c, s_colw[s][cc], v);
        }
        // sum over the 32 columns held by lanes with the same lane / 32
        v = half_wave_sum(v);
        if ((lane & 31) == 31) s_rows[wave][i * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4)] = (double)v;
      }
    __syncthreads();
    if (tid < TM) {
      // row tid of the tile: the WN waves of row group tid / 64 hold its column sums
      const int g = tid / 64, rr = tid % 64;
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < WN; ++w) v += s_rows[g * WN + w][rr];
      a.partial[(((size_t)d * a.n_ftile + nt) * a.ns + s) * a.rows + bd.row_off + row0 + tid] = v;
    }
  }
}

// ------------------------------------------------------------------ swizzled variants
// (64 MI) x (32 NJ WN) tiles: 2 x WN waves, each (32 MI) x (32 NJ) as MI x NJ MFMA blocks.
// WN = 2, MI = 2 gives 128 x 128 tiles of four waves (two work-groups share a CU); WN = 4
// gives tiles of eight waves 256 columns wide, which halve the phase-table bytes per
// product: the table tiles are re-read by every column group.  MI = 4 (256 x 256) halves the
// F bytes per product as well (F tiles are re-read by every row tile) and issues 0.5
// fragment reads per MFMA instead of 0.67; it needs every band's row count to be a multiple
// of 256 and all 256 VGPRs that two waves per SIMD leave each wave.  (Four waves of 128 x
// 128, NJ = 4, one wave per SIMD with the accumulators in AGPRs, measured 15 % slower: no
// second wave covers the fragment-read latency.)  The launches use NJ = 2.
// LDS rows hold 32 halves (four 16-byte chunks) without padding; chunk c of row r is stored
// at slot c ^ ((r >> 2) & 3).  A 16-byte access is served sixteen lanes at a time over 64
// four-byte banks (256 bytes), so each group of sixteen lanes must touch sixteen distinct
// 16-byte slots modulo 256 bytes: the fragment reads (sixteen consecutive rows, one chunk)
// and the staging writes (four rows, four chunks) both do.
__device__ __forceinline__ int swz(int r, int c) { return r * 32 + ((c ^ ((r >> 2) & 3)) << 3); }

// A group of eight zeros: the source of every F group that lies wholly past its column's end.
__device__ __attribute__((aligned(16))) float lw_zero_group[8];

// Amplitude-state epilogue (waves of 32 MI rows and 32 NJ columns): each (column,
// frequency) amplitude C e^{i w_j tau_0p} rowc_j / scale is added to the particle's own
// state row.  A state row belongs to one column pair of one tile, so the adds do not race.
// A lane's accumulators hold one column (one polarisation of one particle) at 8 of every
// 16 frequencies, while a particle's state runs along frequency with both polarisations
// side by side.  Each wave therefore passes its values through its own 2 KB of LDS, 16
// particles x 8 frequencies at a time, and then adds them lane by frequency: 8 consecutive
// lanes update 256 contiguous bytes of one particle's state.
template <int MI, int NJ>
__device__ __forceinline__ void amplitude_epilogue(const GemmArgs& a, const f32x16 (&acc)[MI][NJ],
                                                   const int* s_fcol, const float* s_scale,
                                                   const double* s_tau0, float* s_x, const Band& bd,
                                                   int d, int row0, int wr, int wc, int lane) {
  // s_x: [16 particles][8 frequencies][2 polarisations][re, im] floats
  const int h = lane >> 5, cl = lane & 31;
#pragma unroll
  for (int i = 0; i < MI; ++i) {
    const int jbase = (row0 + wr * 32 * MI + i * 32) >> 1;  // first frequency of the block
#pragma unroll
    for (int jb = 0; jb < NJ; ++jb) {
      const int c0 = wc * 32 * NJ + jb * 32;  // the wave's first column in this block
      const double tau0 = s_tau0[c0 + cl];
      const float inv = 1.0f / s_scale[c0 + cl];
#pragma unroll
      for (int hq = 0; hq < 2; ++hq) {
        // register 4 q + 2 e (re) and + 1 (im) of block i is frequency 4 q + 2 h + e
#pragma unroll
        for (int qq = 0; qq < 2; ++qq)
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const int r = 4 * (2 * hq + qq) + 2 * e, jh = 4 * qq + 2 * h + e;
            const int jl = max(min(jbase + 8 * hq + jh, bd.nj - 1), 0);  // rows past the band are dropped below
            const double x = a.wturn[bd.j0 + jl] * tau0;
            const float fr = (float)(x - rint(x));
            const float cs = __builtin_amdgcn_cosf(fr), sn = __builtin_amdgcn_sinf(fr);
            const float zr = acc[i][jb][r], zi = acc[i][jb][r + 1];
            *(float2*)&s_x[(((cl >> 1) * 8 + jh) * 2 + (cl & 1)) * 2] =
                make_float2((zr * cs - zi * sn) * inv, (zr * sn + zi * cs) * inv);
          }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int t = lane + 64 * k, pp = t >> 3, jh = t & 7;
          const int jl = jbase + 8 * hq + jh;
          const int fc = s_fcol[c0 + 2 * pp];  // polarisation 0; polarisation 1 is fc + 1
          const f32x4 v = *(const f32x4*)&s_x[(pp * 8 + jh) * 4];
          if (fc >= 0 && jl < bd.nj) {
            const int j = bd.j0 + jl;
            const double fr_c = a.rowc[2 * j], fi_c = a.rowc[2 * j + 1];
            double* o = a.amp + (((size_t)(a.p_begin + (fc >> 1)) * a.nd + d) * (size_t)a.wturn_n + j) * 4;
#pragma unroll
            for (int pol = 0; pol < 2; ++pol) {
              const double ur = (double)v[2 * pol], ui = (double)v[2 * pol + 1];
              o[2 * pol] += ur * fr_c - ui * fi_c;
              o[2 * pol + 1] += ur * fi_c + ui * fr_c;
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");  // reads done before the next writes
        __builtin_amdgcn_wave_barrier();
      }
    }
  }
}

// Coherent epilogue (waves of 32 MI rows, two rows of waves per tile).  A lane holds, for one
// column (particle p, polarisation = column parity), the real and imaginary rows of a frequency
// in adjacent accumulator registers.  The column's amplitude up to the row factor applied by
// the reduction is C e^{i w_j tau_0p} (phase reduced to a turn fraction in FP64, hardware
// sin/cos in turns); w_p q_p / scale times it is summed over the tile's columns of each species
// and polarisation and written as partial[...][row][polarisation], the real part on the row of
// (j, re) and the imaginary part on the row of (j, im).
template <int WN, int MI, int NJ>
__device__ __forceinline__ void coherent_epilogue(const GemmArgs& a, const f32x16 (&acc)[MI][NJ],
                                                  const float (*s_colw)[32 * NJ * WN],
                                                  const double* s_tau0, double (*s_rows)[64 * MI],
                                                  const Band& bd, int d, int nt, int row0, int wr,
                                                  int wc, int lane, int wave, int tid) {
  constexpr int TM = 64 * MI, WR = 32 * MI;  // tile rows, rows per wave
  for (int s = 0; s < a.ns; ++s) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int rp = 0; rp < 8; ++rp) {
        const int r = 4 * (rp >> 1) + 2 * (rp & 1);                     // the (j, re) register
        const int rl = i * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);  // row within the wave
        const int jl = (row0 + wr * WR + rl) >> 1;
        float vr = 0.0f, vi = 0.0f;
        if (jl < bd.nj) {
          const double wt = a.wturn[bd.j0 + jl];
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            const int cc = wc * 32 * NJ + j * 32 + (lane & 31);
            const float wq = s_colw[s][cc];
            const double x = wt * s_tau0[cc];
            const float fr = (float)(x - rint(x));
            const float cs = __builtin_amdgcn_cosf(fr), sn = __builtin_amdgcn_sinf(fr);
            const float zr = acc[i][j][r], zi = acc[i][j][r + 1];
            vr = fmaf(wq, zr * cs - zi * sn, vr);
            vi = fmaf(wq, zr * sn + zi * cs, vi);
          }
        }
        // sum the columns of equal polarisation (lanes of equal parity in each half-wave)
        for (int off = 16; off > 1; off >>= 1) {
          vr += __shfl_xor(vr, off);
          vi += __shfl_xor(vi, off);
        }
        if ((lane & 31) < 2) {
          const int pol = lane & 1;
          s_rows[wave][2 * rl + pol] = (double)vr;
          s_rows[wave][2 * (rl + 1) + pol] = (double)vi;
        }
      }
    __syncthreads();
    for (int t = tid; t < 2 * TM; t += 2 * 64 * WN) {
      const int row = t >> 1, pol = t & 1;
      const int g = row / WR, rr = row % WR;
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < WN; ++w) v += s_rows[g * WN + w][2 * rr + pol];
      a.partial[((((size_t)d * a.n_ftile + nt) * a.ns + s) * a.rows + bd.row_off + row0 + row) * 2 + pol] = v;
    }
  }
}

template <typename T, int PRODUCTS, int WN, int MI, int NJ>
__global__ __launch_bounds__(128 * WN, WN == 2 && MI == 2 ? 2 : 1) void lw_dft_mfma_r128_kernel(GemmArgs a) {
  typedef typename MfmaOp<T>::vec vec;
  constexpr int NT = 128 * WN, NW = 2 * WN, TN = 32 * NJ * WN;
  // operand parts: the table is split into hi + lo for three products, F for two or three
  constexpr int NPA = PRODUCTS == 3 ? 2 : 1, NPB = PRODUCTS > 1 ? 2 : 1;
  static_assert(PRODUCTS >= 1 && PRODUCTS <= 3, "one, two or three products");
  constexpr int TM = 64 * MI, WR = 32 * MI;  // tile rows, rows per wave
  typedef T t8 __attribute__((ext_vector_type(8)));
  typedef float f32x8 __attribute__((ext_vector_type(8)));
  constexpr int AV = TM * 4 / NT;  // 16-byte table chunks per thread and stage
  constexpr int BV = TN * 4 / NT;  // 8-float F chunks per thread and stage
  static_assert(kTileK == 32, "four 16-byte chunks per LDS row");
  static_assert(AV >= 1 && BV >= 1, "staging layout");
  __shared__ __attribute__((aligned(16))) T sA[2][NPA][TM * 32];
  __shared__ __attribute__((aligned(16))) T sB[2][NPB][TN * 32];
  __shared__ float s_scale[TN];
  __shared__ int s_q2[TN];
  __shared__ int s_fcol[TN];
  __shared__ float s_colw[kMaxSpecies][TN];  // w q^2 / scale^2 (w q / scale when coherent)
  __shared__ double s_tau0[TN];              // first retarded time of each column (coherent)
  __shared__ int s_kmax;
  // the epilogue's row sums reuse the table buffers (after a barrier that ends the loop)
  static_assert(sizeof(sA) >= sizeof(double) * NW * 64 * MI, "row sums fit the table buffers");
  double(*s_rows)[64 * MI] = reinterpret_cast<double(*)[64 * MI]>(&sA[0][0][0]);

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int oi = 0;
  while (oi + 1 < a.nb && (int)blockIdx.x >= a.tiles_before[oi + 1]) ++oi;
  const int bi = a.order[oi];
  const Band bd = a.band[bi];
  const int local = blockIdx.x - a.tiles_before[oi];
  const int mtiles = bd.m / TM;
  const int ngroups = a.nd * a.n_ftile;
  const int xcd = local % 8, seq = local / 8;
  const int grp = (seq / mtiles) * 8 + xcd;
  if (grp >= ngroups) return;
  const int mt = seq % mtiles;
  const int nt = grp % a.n_ftile;
  const int d = grp / a.n_ftile;
  const int ncol = 2 * a.n_local;
  const int db = d * a.nb + bi;
  const int col0 = nt * TN;
  const int row0 = mt * TM;
  const T* E_hi = (const T*)a.e_hi + bd.e_off;
  const T* E_lo = (const T*)a.e_lo + bd.e_off;
  const float* Fb = a.F + (size_t)d * a.f_dir + bd.f_off;

  if (tid == 0) s_kmax = 0;
  __syncthreads();
  if (tid < TN) {
    const int c = col0 + tid;
    float sc = 1.0f;
    int q2 = 0, fc = -1;
    double tau0 = 0.0;
    for (int s = 0; s < a.ns; ++s) s_colw[s][tid] = 0.0f;
    if (c < ncol) {
      const int pl = a.perm[db * a.n_local + c / 2];
      fc = 2 * pl + (c & 1);
      const float m = __uint_as_float(a.colmax[db * ncol + fc]);
      if (m > 0.0f) {
        int e;
        frexpf(m, &e);
        sc = ldexpf(1.0f, -e);
      }
      q2 = 2 * a.colq[db * a.n_local + pl];
      atomicMax(&s_kmax, q2);
      const int64_t p = a.p_begin + pl;
      const int sp = a.b.species ? a.b.species[p] : 0;
      if (sp >= 0 && sp < a.ns) {
        const float qq = a.b.charge[p];
        s_colw[sp][tid] = a.coherent ? a.b.weight[p] * qq / sc : a.b.weight[p] * qq * qq / (sc * sc);
      }
      if (a.coherent || a.amp) {  // as the spreading kernel measures tau' from it
        const int64_t o = a.b.offsets[p];
        if (a.b.offsets[p + 1] > o) {
          const double* n = a.dirs + kDirStride * d;
          tau0 = a.b.t0[p] - (n[0] * a.b.x[o] + n[1] * a.b.y[o] + n[2] * a.b.z[o]);
        }
      }
    }
    s_scale[tid] = sc;
    s_q2[tid] = q2;
    s_fcol[tid] = fc;
    s_tau0[tid] = tau0;
  }
  __syncthreads();
  const int kend = min(((s_kmax + kTileK - 1) / kTileK) * kTileK, bd.kp);

  // staging: thread t moves chunk t % 4 of rows (columns) t / 4 + (NT / 4) v, through two
  // register sets (one filled while the other waits to be stored).
  const int sr = tid >> 2, sc4 = tid & 3;
  // stage s of the inner dimension covers [32 s, 32 s + 32); LDS buffer s % 2
  const int nst = kend / kTileK;
  const int last = max(nst - 1, 0) * kTileK;
  typedef u32x4 RegA[AV][NPA];
  typedef f32x4 RegB[BV][2];
  // the thread's BV columns: F offset (column 0 stands in past the chunk, with length 0),
  // length and scale stay fixed over the inner loop
  size_t fofs[BV];
  int q2v[BV];
  float sclv[BV];
#pragma unroll
  for (int v = 0; v < BV; ++v) {
    const int col = sr + (NT / 4) * v;
    fofs[v] = (size_t)max(s_fcol[col], 0) * bd.kp + sc4 * 8;
    q2v[v] = s_fcol[col] >= 0 ? s_q2[col] : 0;
    sclv[v] = s_scale[col];
  }
  // stage k0 (past the end: the table re-reads the last stage, F reads zeros)
  auto load = [&](RegA& ra, RegB& rb, int k0) {
    const int ke = min(k0, last);
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const size_t g = (size_t)(row0 + sr + (NT / 4) * v) * bd.kp + ke + sc4 * 8;
      ra[v][0] = *(const u32x4*)(E_hi + g);
      if (NPA > 1) ra[v][NPA - 1] = *(const u32x4*)(E_lo + g);
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      // groups past the column's end read zeros; the group that holds the end was cleared
      // past it by the spreading kernel
      const float* src = k0 + sc4 * 8 < q2v[v] ? Fb + fofs[v] + k0 : lw_zero_group;
      rb[v][0] = *(const f32x4*)src;
      rb[v][1] = *(const f32x4*)(src + 4);
    }
  };
  auto store = [&](const RegA& ra, const RegB& rb, int buf) {
#pragma unroll
    for (int v = 0; v < AV; ++v) {
      const int r = sr + (NT / 4) * v;
      *(u32x4*)&sA[buf][0][swz(r, sc4)] = ra[v][0];
      if (NPA > 1) *(u32x4*)&sA[buf][NPA - 1][swz(r, sc4)] = ra[v][NPA - 1];
    }
#pragma unroll
    for (int v = 0; v < BV; ++v) {
      const int r = sr + (NT / 4) * v;
      const float scl = sclv[v];
      if constexpr (std::is_same<T, _Float16>::value || MI == 4) {
        const f32x8 x = __builtin_shufflevector(rb[v][0], rb[v][1], 0, 1, 2, 3, 4, 5, 6, 7) * scl;
        // split x = hi + lo, both rounded to T, converting pairs of lanes at once
        const t8 hv = __builtin_convertvector(x, t8);
        *(t8*)&sB[buf][0][swz(r, sc4)] = hv;
        if (NPB > 1)
          *(t8*)&sB[buf][NPB - 1][swz(r, sc4)] = __builtin_convertvector(x - __builtin_convertvector(hv, f32x8), t8);
      } else {  // BF16 in 128-row tiles: lane by lane schedules better (measured); in 256-row
                // tiles it needs more than the 256 VGPRs available
        t8 hv, lv;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const float x = (e < 4 ? rb[v][0][e] : rb[v][1][e - 4]) * scl;
          hv[e] = (T)x;
          if (NPB > 1) lv[e] = (T)(x - (float)hv[e]);
        }
        *(t8*)&sB[buf][0][swz(r, sc4)] = hv;
        if (NPB > 1) *(t8*)&sB[buf][NPB - 1][swz(r, sc4)] = lv;
      }
    }
  };

  f32x16 acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.0f;

  const int wr = wave / WN, wc = wave % WN;
  auto compute = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      const int ch = 2 * ks + (lane >> 5);
      vec fa[NPA][MI], fb[NPB][NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const int r = wr * WR + i * 32 + (lane & 31);
        fa[0][i] = *(const vec*)&sA[buf][0][swz(r, ch)];
        if (NPA > 1) fa[NPA - 1][i] = *(const vec*)&sA[buf][NPA - 1][swz(r, ch)];
      }
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int cc = wc * 32 * NJ + j * 32 + (lane & 31);
        fb[0][j] = *(const vec*)&sB[buf][0][swz(cc, ch)];
        if (NPB > 1) fb[NPB - 1][j] = *(const vec*)&sB[buf][NPB - 1][swz(cc, ch)];
      }
      // products outermost: consecutive MFMAs write different accumulators
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = MfmaOp<T>::mma(fa[0][i], fb[0][j], acc[i][j]);
      if (PRODUCTS > 1) {  // table hi x F lo
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j) acc[i][j] = MfmaOp<T>::mma(fa[0][i], fb[NPB - 1][j], acc[i][j]);
      }
      if (PRODUCTS > 2) {  // table lo x F hi
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int j = 0; j < NJ; ++j) acc[i][j] = MfmaOp<T>::mma(fa[NPA - 1][i], fb[0][j], acc[i][j]);
      }
    }
  };

  RegA ra0, ra1;
  RegB rb0, rb1;
  if (nst > 0) {
    load(ra0, rb0, 0);
    load(ra1, rb1, kTileK);
    store(ra0, rb0, 0);
  }
  __syncthreads();
  // Loads and stores run unconditionally (stages past the end re-read the table's last
  // stage, read zeros for F and fill a buffer nobody reads), so the loop body has no
  // branches around memory operations.  A stage's loads are waited for when that stage is
  // stored; the compiler issues them at the end of the phase before (their registers are
  // not free earlier), so they have one compute phase to arrive.
  // Stages go in pairs with no exit in between (an exit there makes the compiler copy the
  // accumulators every iteration): with an odd count the last pair's second stage lies
  // past every column's end, so its F operand is zero and it adds nothing.
  for (int st = 0; st < nst; st += 2) {
    // buffer 0 holds stage st, register set 1 stage st + 1
    load(ra0, rb0, (st + 2) * kTileK);
    compute(0);
    store(ra1, rb1, 1);
    __syncthreads();
    load(ra1, rb1, (st + 3) * kTileK);
    compute(1);
    store(ra0, rb0, 0);
    __syncthreads();
  }

  if (a.amp) {
    static_assert(sizeof(sA) >= NW * 512 * sizeof(float), "2 KB of the table buffers per wave");
    amplitude_epilogue<MI, NJ>(a, acc, s_fcol, s_scale, s_tau0, reinterpret_cast<float*>(&sA[0][0][0]) + wave * 512,
                               bd, d, row0, wr, wc, lane);
    return;
  }
  if (a.coherent) {
    coherent_epilogue<WN, MI, NJ>(a, acc, s_colw, s_tau0, s_rows, bd, d, nt, row0, wr, wc, lane, wave, tid);
    return;
  }
  for (int s = 0; s < a.ns; ++s) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        float v = 0.0f;
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          const int cc = wc * 32 * NJ + j * 32 + (lane & 31);
          const float c = acc[i][j][r];
          v = fmaf(c * c, s_colw[s][cc], v);
        }
        v = half_wave_sum(v);
        if ((lane & 31) == 31) s_rows[wave][i * 32 + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4)] = (double)v;
      }
    __syncthreads();
    for (int t = tid; t < TM; t += NT) {
      const int g = t / WR, rr = t % WR;
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < WN; ++w) v += s_rows[g * WN + w][rr];
      a.partial[(((size_t)d * a.n_ftile + nt) * a.ns + s) * a.rows + bd.row_off + row0 + t] = v;
    }
  }
}

// S[s][d][j] += rowfac[j] * sum over column tiles of (re row + im row)
__global__ void lw_mfma_reduce_kernel(const double* partial, int n_ftile, int ns, int rows,
                                      const int32_t* row_of_j, const double* rowfac, int nw,
                                      int nd, double* S) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nd * ns * nw) return;
  const int j = i % nw;
  const int s = (i / nw) % ns;
  const int d = i / (nw * ns);
  const int r = row_of_j[j];
  double acc = 0.0;
  for (int t = 0; t < n_ftile; ++t) {
    const double* pr = partial + (((size_t)d * n_ftile + t) * ns + s) * rows;
    acc += pr[r] + pr[r + 1];
  }
  S[((size_t)s * nd + d) * nw + j] += acc * rowfac[j];
}

// A[s][d][j][2 pol + (re, im)] += rowc[j] * sum over column tiles of the row pair (j, re), (j, im)
__global__ void lw_mfma_reduce_coherent_kernel(const double* partial, int n_ftile, int ns, int rows,
                                               const int32_t* row_of_j, const double* rowc, int nw,
                                               int nd, double* A) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nd * ns * nw) return;
  const int j = i % nw;
  const int s = (i / nw) % ns;
  const int d = i / (nw * ns);
  const int r = row_of_j[j];
  double re[2] = {0.0, 0.0}, im[2] = {0.0, 0.0};
  for (int t = 0; t < n_ftile; ++t) {
    const double* pr = partial + (((size_t)d * n_ftile + t) * ns + s) * rows * 2;
#pragma unroll
    for (int pol = 0; pol < 2; ++pol) {
      re[pol] += pr[2 * r + pol];
      im[pol] += pr[2 * (r + 1) + pol];
    }
  }
  const double fr = rowc[2 * j], fi = rowc[2 * j + 1];
  double* out = A + (((size_t)s * nd + d) * nw + j) * 4;
#pragma unroll
  for (int pol = 0; pol < 2; ++pol) {
    out[2 * pol] += re[pol] * fr - im[pol] * fi;
    out[2 * pol + 1] += re[pol] * fi + im[pol] * fr;
  }
}

// ------------------------------------------------------------------ host side
namespace {

double es_phi_host(double x, const KernelShape& k) {
  const double y = 2.0 * x / k.w;
  const double r = 1.0 - y * y;
  return r > 0.0 ? exp(k.beta * (sqrt(r) - 1.0)) : 0.0;
}

// Tap weight polynomials of the spreading kernel: for tap i and z = 2 f - 1 in [-1, 1],
// g_i(z) = phi(i - W/2 + 1 - (z + 1) / 2) interpolated at the kTapCoef Chebyshev points of
// the first kind, then rewritten in powers of z for Horner evaluation.  The sqrt edge of
// phi limits the interpolant to ~1.6e-8 of phi's peak; the coefficients sum to ~1.25 in
// absolute value, so FP32 evaluation adds < 1e-7.  phi is even, so g_{W-1-i}(z) = g_i(-z):
// the last W/2 taps are stored as the mirror images of the first (odd powers change sign),
// and the device evaluates each mirrored pair from one even and one odd part.
void tap_polynomials(float out[kWMax][kTapCoef], const KernelShape& ks) {
  constexpr int N = kTapCoef;
  double T[N][N] = {};  // T[j] = power coefficients of the Chebyshev polynomial T_j
  T[0][0] = 1.0;
  T[1][1] = 1.0;
  for (int j = 2; j < N; ++j)
    for (int k = 0; k < N; ++k) T[j][k] = (k > 0 ? 2.0 * T[j - 1][k - 1] : 0.0) - T[j - 2][k];
  for (int i = 0; i < kWMax; ++i)
    for (int k = 0; k < N; ++k) out[i][k] = 0.0f;
  for (int i = 0; i < ks.w / 2; ++i) {  // taps W - 1 - i are the mirror images
    double g[N], zk[N];
    for (int k = 0; k < N; ++k) {
      zk[k] = cos((2 * k + 1) * M_PI / (2.0 * N));
      g[k] = es_phi_host((double)(i - (ks.w / 2 - 1)) - 0.5 * (zk[k] + 1.0), ks);
    }
    double mono[N] = {};
    for (int j = 0; j < N; ++j) {
      double cj = 0.0;
      for (int k = 0; k < N; ++k) cj += g[k] * cos(j * (2 * k + 1) * M_PI / (2.0 * N));
      cj *= (j == 0 ? 1.0 : 2.0) / N;
      for (int k = 0; k < N; ++k) mono[k] += cj * T[j][k];
    }
    for (int k = 0; k < N; ++k) {
      out[i][k] = (float)mono[k];
      out[ks.w - 1 - i][k] = (k % 2 ? -1.0f : 1.0f) * out[i][k];
    }
  }
}

// The kernel as the spreading applies it: at x = i - W/2 + 1 - f (f in [0, 1)) the
// polynomial of tap i at z = 2 f - 1, from the same FP32 coefficients.
double applied_phi_host(double x, const KernelShape& k, const float (*tapc)[kTapCoef]) {
  const double t = x + (double)(k.w / 2 - 1);
  const double i = ceil(t);
  if (i < 0.0 || i > (double)(k.w - 1)) return 0.0;
  const double z = 2.0 * (i - t) - 1.0;
  const float* c = tapc[(int)i];
  double v = c[kTapCoef - 1];
  for (int m = kTapCoef - 2; m >= 0; --m) v = v * z + (double)c[m];
  return v;
}

// Fourier transform of the applied kernel, Phi(xi) = int phi(x) cos(xi x) dx, by 8-point
// Gauss-Legendre on every unit interval between tap breakpoints (a polynomial on each), so
// that the deconvolution divides out exactly what the spreading put in.
double es_ft_host(double xi, const KernelShape& k) {
  static const double gx[8] = {-0.9602898564975363, -0.7966664774136267, -0.5255324099163290,
                               -0.1834346424956498, 0.1834346424956498,  0.5255324099163290,
                               0.7966664774136267,  0.9602898564975363};
  static const double gw[8] = {0.1012285362903763, 0.2223810344533745, 0.3137066458778873,
                               0.3626837833783620, 0.3626837833783620, 0.3137066458778873,
                               0.2223810344533745, 0.1012285362903763};
  float tapc[kWMax][kTapCoef];
  tap_polynomials(tapc, k);
  double s = 0.0;
  for (int p = 0; p < k.w; ++p) {  // unit panels [-W/2 + p, -W/2 + p + 1]
    const double c = -0.5 * k.w + p + 0.5;
    for (int i = 0; i < 8; ++i) {
      const double x = c + 0.5 * gx[i];
      s += 0.5 * gw[i] * applied_phi_host(x, k, tapc) * cos(xi * x);
    }
  }
  return s;
}

lw_status set_err(lw_ctx* c, lw_status st, const char* msg) {
  c->err = msg;
  return st;
}

#define MF_HIP(call, what)                                                      \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess) {                                                     \
      c->err = std::string(what) + ": " + hipGetErrorString(e_);                \
      return LW_EDEVICE;                                                        \
    }                                                                           \
  } while (0)

int chunk_particles(const MfmaPlanCache* pc, int nd, int64_t P) {
  // particles per chunk bounded so that F (all directions) stays near 24 GiB: fewer, larger
  // launches.  With two bands on 1e5 particles, 12 GiB (7 chunks) made the spreading kernel
  // 8 % faster than 6 GiB (13); 24 GiB (4) saved 1.6 % more of the step, and 48 or 96 GiB
  // no more (the contraction slows as the spread gains)
  int64_t per = 0;
  for (int b = 0; b < pc->nb; ++b) per += 2 * (int64_t)pc->band[b].kp * sizeof(float);
  per *= nd;
  int64_t n = per > 0 ? pc->chunk_bytes / per : 8192;
  // column indices (direction, band, 2 x particle) stay within int32
  n = std::min<int64_t>(n, ((int64_t)1 << 30) / ((int64_t)nd * pc->nb));
  n = std::max<int64_t>(64, n);  // at least one tile of columns, whatever the cap
  n = (n / 64) * 64;
  return (int)std::min<int64_t>(n, ((P + 63) / 64) * 64);
}

struct WsLayout {
  size_t f, colmax, colq, perm, partial, total;
  int chunk, n_ftile;
  int64_t f_dir;  // floats of F per direction
};

size_t al(size_t n) { return (n + 255) & ~(size_t)255; }

WsLayout ws_layout(const lw_ctx* c, const MfmaPlanCache* pc, int64_t P) {
  WsLayout w;
  const int nd = c->nd, nb = pc->nb;
  w.chunk = chunk_particles(pc, nd, P);
  w.n_ftile = (2 * w.chunk + kTileN - 1) / kTileN;
  int64_t fl = 0;
  for (int b = 0; b < nb; ++b) fl += (int64_t)2 * w.chunk * pc->band[b].kp;
  w.f_dir = fl;
  size_t off = 0;
  w.f = off;
  off += al((size_t)fl * nd * sizeof(float));
  w.colmax = off;
  off += al((size_t)nd * nb * 2 * w.chunk * sizeof(unsigned));
  w.colq = off;
  off += al((size_t)nd * nb * w.chunk * sizeof(int32_t));
  w.perm = off;
  off += al((size_t)nd * nb * w.chunk * sizeof(int32_t));
  w.partial = off;
  off += al((size_t)nd * w.n_ftile * c->ns * pc->rows * (c->coherent ? 2 : 1) * sizeof(double));
  w.total = off;
  return w;
}

void free_tables(MfmaPlanCache* pc) {
  pc->epoch += 1;
  if (pc->e_hi) (void)hipFree(pc->e_hi);
  if (pc->e_lo) (void)hipFree(pc->e_lo);
  if (pc->rowfac) (void)hipFree(pc->rowfac);
  if (pc->rowc) (void)hipFree(pc->rowc);
  if (pc->row_of_j) (void)hipFree(pc->row_of_j);
  pc->e_hi = pc->e_lo = nullptr;
  pc->rowfac = nullptr;
  pc->rowc = nullptr;
  pc->row_of_j = nullptr;
  pc->valid = false;
}

// Largest retarded-time span over the batch and directions (synchronous).
lw_status batch_span(lw_ctx* c, const lw_batch* b, double* span) {
  MfmaPlanCache* pc = c->mfma;
  if (!pc->d_span) MF_HIP(hipMalloc(&pc->d_span, sizeof(double)), "hipMalloc(span)");
  MF_HIP(launch_fill_f64(pc->d_span, 1, 0.0, c->stream), "fill span");
  const int64_t n = b->n_particles * (int64_t)c->nd;
  if (n > 0) {
    dim3 grid((unsigned)((n + 255) / 256)), block(256);
    hipLaunchKernelGGL(lw_span_kernel, grid, block, 0, c->stream, view_of(b), c->d_dirs, c->nd,
                       pc->d_span);
    MF_HIP(hipGetLastError(), "launch span");
  }
  double h = 0.0;
  MF_HIP(hipMemcpyAsync(&h, pc->d_span, sizeof(double), hipMemcpyDeviceToHost, c->stream), "copy span");
  MF_HIP(hipStreamSynchronize(c->stream), "sync");
  *span = h;
  return LW_OK;
}

// Band boundaries (frequency indices jb[0] = 0 < ... < jb[nb] = nw) that minimise the
// contraction's work, the sum over bands of rows x grid points: 2 nj rounded up to a row
// tile, times span / h + W + 1 with h = pi / (sigma D) and D the band's half-width.  The
// spread costs the same for any split (every band spreads every sample).  On a log grid
// the upper band keeps a wide D however it is cut, so it should hold few frequencies.
// Boundaries fall on multiples of 128 frequencies when there are enough (so that every
// band's row count suits 256-row tiles), on a coarser step when the grid is long (at most
// 256 candidate positions), and anywhere on short grids.
std::vector<int> band_bounds(const std::vector<double>& w, int nb, double span, const KernelShape& ks) {
  const int nw = (int)w.size();
  std::vector<int> jb(nb + 1);
  for (int b = 0; b <= nb; ++b) jb[b] = (int)((int64_t)nw * b / nb);  // equal counts
  if (nb < 2) return jb;
  int g = nw >= 128 * nb ? 128 : 1;
  while (nw / g > 256) g *= 2;
  std::vector<int> pos;
  for (int j = 0; j < nw; j += g) pos.push_back(j);
  pos.push_back(nw);
  const int np = (int)pos.size();
  if (np - 1 < nb) return jb;
  // cost of one band over [pos[k], pos[l])
  std::vector<double> cost((size_t)np * np, 0.0);
  for (int k = 0; k + 1 < np; ++k) {
    double lo = w[pos[k]], hi = w[pos[k]];
    for (int l = k + 1; l < np; ++l) {
      for (int j = pos[l - 1]; j < pos[l]; ++j) {
        lo = std::min(lo, w[j]);
        hi = std::max(hi, w[j]);
      }
      const double wc = 0.5 * (lo + hi);
      const double D = std::max(0.5 * (hi - lo), 1e-6 * std::max(wc, 1e-300));
      const double rows = (double)(((2 * (pos[l] - pos[k]) + kTileM - 1) / kTileM) * kTileM);
      cost[(size_t)k * np + l] = rows * (span * ks.sigma * D / M_PI + ks.w + 1);
    }
  }
  // best[b][l]: least cost of b bands covering [0, pos[l]); from[b][l]: start of the last one
  const double inf = std::numeric_limits<double>::infinity();
  std::vector<double> best((size_t)(nb + 1) * np, inf);
  std::vector<int> from((size_t)(nb + 1) * np, -1);
  best[0] = 0.0;
  for (int b = 1; b <= nb; ++b)
    for (int l = b; l < np; ++l)
      for (int k = b - 1; k < l; ++k) {
        const double v = best[(size_t)(b - 1) * np + k] + cost[(size_t)k * np + l];
        if (v < best[(size_t)b * np + l]) {
          best[(size_t)b * np + l] = v;
          from[(size_t)b * np + l] = k;
        }
      }
  if (!(best[(size_t)nb * np + np - 1] < inf)) return jb;
  int l = np - 1;
  for (int b = nb; b >= 1; --b) {
    jb[b] = pos[l];
    l = from[(size_t)b * np + l];
  }
  jb[0] = 0;
  return jb;
}

lw_status build_plan(lw_ctx* c, double span, int dtype, const KernelShape& ks) {
  MfmaPlanCache* pc = c->mfma;
  free_tables(pc);
  pc->shape = ks;
  const int nb = std::max(1, std::min(pc->bands_req, std::min(kMaxBands, c->nw)));
  pc->nb = nb;
  pc->span = span;
  pc->dtype = dtype;
  const std::vector<double>& w = c->h_omega;
  const std::vector<int> jb = band_bounds(w, nb, span, ks);
  int row = 0;
  int64_t eoff = 0, foff = 0;
  for (int b = 0; b < nb; ++b) {
    Band& bd = pc->band[b];
    bd.j0 = jb[b];
    const int j1 = jb[b + 1];
    bd.nj = j1 - bd.j0;
    double lo = w[bd.j0], hi = w[bd.j0];
    for (int j = bd.j0; j < j1; ++j) {
      lo = std::min(lo, w[j]);
      hi = std::max(hi, w[j]);
    }
    bd.wc = 0.5 * (lo + hi);
    double D = 0.5 * (hi - lo);
    D = std::max(D, 1e-6 * std::max(bd.wc, 1e-300));
    bd.h = M_PI / (ks.sigma * D);
    bd.wc_turn = bd.wc / (2.0 * M_PI);
    const double qd = ceil(span / bd.h) + ks.w + 1;
    if (qd > 4.0e6) return set_err(c, LW_EUNSUPPORTED, "retarded-time span too long for the matrix-core grid");
    bd.qmax = (int)qd;
    bd.m = ((2 * bd.nj + kTileM - 1) / kTileM) * kTileM;
    bd.kp = ((2 * bd.qmax + kTileK - 1) / kTileK) * kTileK;
    bd.row_off = row;
    bd.e_off = eoff;
    bd.f_off = foff;  // in units of (columns x kp); scaled by chunk at launch
    row += bd.m;
    eoff += (int64_t)bd.m * bd.kp;
    foff += bd.kp;
  }
  pc->rows = row;
  pc->e_elems = eoff;
  const size_t esz = 2;  // f16 and bf16 are both 2 bytes
  MF_HIP(hipMalloc(&pc->e_hi, (size_t)eoff * esz), "hipMalloc(E)");
  MF_HIP(hipMalloc(&pc->e_lo, (size_t)eoff * esz), "hipMalloc(E)");
  for (int b = 0; b < nb; ++b) {
    const Band& bd = pc->band[b];
    const int64_t tot = (int64_t)bd.m * bd.kp;
    dim3 grid((unsigned)((tot + 255) / 256)), block(256);
    if (dtype == 0)
      hipLaunchKernelGGL(lw_etable_kernel<_Float16>, grid, block, 0, c->stream,
                         (_Float16*)pc->e_hi, (_Float16*)pc->e_lo, c->d_omega, bd);
    else
      hipLaunchKernelGGL(lw_etable_kernel<__bf16>, grid, block, 0, c->stream, (__bf16*)pc->e_hi,
                         (__bf16*)pc->e_lo, c->d_omega, bd);
    MF_HIP(hipGetLastError(), "launch etable");
  }
  std::vector<double> rf(c->nw), rcx(2 * (size_t)c->nw);
  std::vector<int32_t> rj(c->nw);
  for (int b = 0; b < nb; ++b) {
    const Band& bd = pc->band[b];
    for (int jl = 0; jl < bd.nj; ++jl) {
      const int j = bd.j0 + jl;
      const double nu = w[j] - bd.wc;
      const double ph = es_ft_host(nu * bd.h, ks);
      rf[j] = 1.0 / (4.0 * M_PI * M_PI * ph * ph);
      rj[j] = bd.row_off + 2 * jl;
      // grid point q sits at retarded time (q - W/2) h after the first sample
      rcx[2 * j] = cos(-nu * 0.5 * ks.w * bd.h) / ph;
      rcx[2 * j + 1] = sin(-nu * 0.5 * ks.w * bd.h) / ph;
    }
  }
  MF_HIP(hipMalloc(&pc->rowc, 2 * (size_t)c->nw * sizeof(double)), "hipMalloc(rowc)");
  MF_HIP(hipMemcpy(pc->rowc, rcx.data(), 2 * (size_t)c->nw * sizeof(double), hipMemcpyHostToDevice),
         "copy rowc");
  MF_HIP(hipMalloc(&pc->rowfac, c->nw * sizeof(double)), "hipMalloc(rowfac)");
  MF_HIP(hipMalloc(&pc->row_of_j, c->nw * sizeof(int32_t)), "hipMalloc(rows)");
  MF_HIP(hipMemcpy(pc->rowfac, rf.data(), c->nw * sizeof(double), hipMemcpyHostToDevice), "copy rowfac");
  MF_HIP(hipMemcpy(pc->row_of_j, rj.data(), c->nw * sizeof(int32_t), hipMemcpyHostToDevice), "copy rows");
  MF_HIP(hipStreamSynchronize(c->stream), "sync");
  pc->valid = true;
  return LW_OK;
}

// Make sure the tables cover the batch; grows the span with headroom.  With measure = false a
// planned batch (same offsets pointer and particle count, tables unchanged since) is taken as
// covered without a synchronisation: the spreading kernel records any particle that needs
// more grid points than planned, and the next read reports it.  Inside a graph capture
// nothing may synchronise: the plan made before the capture is used as is.
lw_status ensure_plan(lw_ctx* c, const lw_batch* b, lw_path path, bool measure) {
  MfmaPlanCache* pc = c->mfma;
  const int dtype = path == LW_PATH_MFMA_BF16 ? 1 : 0;
  const int products = dtype ? pc->products_bf16 : pc->products_f16;
  const KernelShape& ks = products == 3 ? kShapeSplit : kShapeSingle;
  const bool same = pc->valid && pc->dtype == dtype && pc->shape.w == ks.w;
  if (c->capturing) {
    if (same) return LW_OK;
    return set_err(c, LW_ESTATE, "matrix-core tables must be planned before graph capture");
  }
  if (!measure && same && pc->planned_offsets == (const void*)b->offsets &&
      pc->planned_n == b->n_particles && pc->planned_epoch == pc->epoch)
    return LW_OK;
  double span = 0.0;
  lw_status st = batch_span(c, b, &span);
  if (st != LW_OK) return st;
  if (!(same && span <= pc->span)) {
    const double want = std::max(span * 1.25, same ? pc->span : 0.0);
    st = build_plan(c, want, dtype, ks);
    if (st != LW_OK) return st;
  }
  pc->planned_offsets = (const void*)b->offsets;
  pc->planned_n = b->n_particles;
  pc->planned_epoch = pc->epoch;
  return LW_OK;
}

}  // namespace

MfmaPlanCache* mfma_cache_create() { return new MfmaPlanCache(); }

void mfma_cache_destroy(MfmaPlanCache* pc) {
  if (!pc) return;
  free_tables(pc);
  if (pc->d_span) (void)hipFree(pc->d_span);
  delete pc;
}

uint64_t mfma_epoch(const MfmaPlanCache* pc) { return pc ? pc->epoch : 0; }

void mfma_cache_invalidate(MfmaPlanCache* pc) {
  if (pc) free_tables(pc);
}

lw_status mfma_set_options(lw_ctx* c, int bands, int products_f16, int products_bf16) {
  MfmaPlanCache* pc = c->mfma;
  if (bands < 1 || bands > kMaxBands) return set_err(c, LW_EINVAL, "bands must be in [1, 16]");
  if (products_f16 < 1 || products_f16 > 3 || (products_bf16 != 1 && products_bf16 != 3))
    return set_err(c, LW_EINVAL, "products must be 1, 2 or 3 for FP16 and 1 or 3 for BF16");
  if (bands != pc->bands_req) free_tables(pc);
  pc->bands_req = bands;
  pc->products_f16 = products_f16;
  pc->products_bf16 = products_bf16;
  return LW_OK;
}

lw_status mfma_set_bands(lw_ctx* c, int bands) {
  MfmaPlanCache* pc = c->mfma;
  return mfma_set_options(c, bands, pc->products_f16, pc->products_bf16);
}

lw_status mfma_set_tile(lw_ctx* c, int tile) {
  if (tile < 1 || tile > 4) return set_err(c, LW_EINVAL, "tile shape must be 1, 2, 3 or 4");
  c->mfma->tile = tile;
  return LW_OK;
}

lw_status mfma_set_chunk_bytes(lw_ctx* c, int64_t bytes) {
  if (bytes < 0) return set_err(c, LW_EINVAL, "chunk cap must be >= 0 bytes (0: the default)");
  c->mfma->chunk_bytes = bytes ? bytes : (24LL << 30);
  return LW_OK;
}

lw_status mfma_plan_info(lw_ctx* c, const lw_batch* b, lw_path path, int64_t* out) {
  size_t bytes = 0;
  lw_status st = mfma_workspace_size(c, b, path, &bytes);  // plans the batch
  if (st != LW_OK) return st;
  const MfmaPlanCache* pc = c->mfma;
  const int64_t P = b->n_particles;
  const WsLayout L = ws_layout(c, pc, std::max<int64_t>(P, 1));
  out[0] = P > 0 ? L.chunk : 0;
  out[1] = P > 0 ? (P + L.chunk - 1) / L.chunk : 0;
  out[2] = pc->nb;
  out[3] = (int64_t)bytes;
  return LW_OK;
}

lw_status mfma_workspace_size(lw_ctx* c, const lw_batch* b, lw_path path, size_t* bytes) {
  if (!b || b->n_particles < 0) return set_err(c, LW_EINVAL, "bad batch");
  if (b->n_particles == 0) {
    *bytes = 0;
    return LW_OK;
  }
  lw_status st = ensure_plan(c, b, path, true);
  if (st != LW_OK) return st;
  *bytes = ws_layout(c, c->mfma, b->n_particles).total;
  return LW_OK;
}

lw_status mfma_workspace_need(lw_ctx* c, const lw_batch* b, lw_path path, size_t* bytes) {
  if (!b || b->n_particles < 0) return set_err(c, LW_EINVAL, "bad batch");
  if (b->n_particles == 0) {
    *bytes = 0;
    return LW_OK;
  }
  lw_status st = ensure_plan(c, b, path, false);
  if (st != LW_OK) return st;
  *bytes = ws_layout(c, c->mfma, b->n_particles).total;
  return LW_OK;
}

lw_status mfma_accumulate(lw_ctx* c, const lw_batch* b, lw_path path, void* ws, size_t ws_bytes,
                          float* per_particle, double* amp) {
  if (per_particle)
    return set_err(c, LW_EUNSUPPORTED, "per-particle output is available on the FP32 path only");
  lw_status st = ensure_plan(c, b, path, false);
  if (st != LW_OK) return st;
  MfmaPlanCache* pc = c->mfma;
  const WsLayout L = ws_layout(c, pc, b->n_particles);
  if (ws_bytes < L.total) return set_err(c, LW_ENOMEM, "workspace too small for the matrix-core plan");
  char* base = (char*)ws;
  float* F = (float*)(base + L.f);
  unsigned* colmax = (unsigned*)(base + L.colmax);
  int32_t* colq = (int32_t*)(base + L.colq);
  int32_t* perm = (int32_t*)(base + L.perm);
  double* partial = (double*)(base + L.partial);
  const int products = path == LW_PATH_MFMA_BF16 ? pc->products_bf16 : pc->products_f16;

  SpreadArgs sa;
  GemmArgs ga;
  sa.b = ga.b = view_of(b);
  sa.nb = ga.nb = pc->nb;
  sa.nd = ga.nd = c->nd;
  sa.dirs = c->d_dirs;
  sa.f_dir = ga.f_dir = L.f_dir;
  for (int i = 0; i < pc->nb; ++i) {
    Band bd = pc->band[i];
    bd.f_off = pc->band[i].f_off * 2 * L.chunk;
    sa.band[i] = ga.band[i] = bd;
  }
  sa.F = F;
  ga.F = F;
  sa.colmax = colmax;
  ga.colmax = colmax;
  sa.colq = colq;
  ga.colq = colq;
  ga.perm = perm;
  sa.err = c->d_err;
  sa.overflow = c->d_overflow;
  sa.ns = c->ns;
  sa.flops = c->prof ? c->d_flops : nullptr;
  tap_polynomials(sa.tapc, pc->shape);
  c->flop_mult = products;
  ga.e_hi = pc->e_hi;
  ga.e_lo = pc->e_lo;
  ga.partial = partial;
  ga.ns = c->ns;
  ga.rows = pc->rows;
  ga.coherent = c->coherent && !amp ? 1 : 0;
  ga.dirs = c->d_dirs;
  ga.wturn = c->d_wturn;
  ga.wturn_n = c->nw;
  ga.amp = amp;
  ga.rowc = pc->rowc;
  // bands by decreasing work (grid points per particle), so the long tiles start first
  for (int i = 0; i < pc->nb; ++i) ga.order[i] = i;
  std::sort(ga.order, ga.order + pc->nb,
            [&](int x, int y) { return pc->band[x].qmax * pc->band[x].m > pc->band[y].qmax * pc->band[y].m; });
  int tile = pc->tile;  // 256-row tiles need every band's rows to be a multiple of 256
  for (int i = 0; i < pc->nb; ++i)
    if (pc->band[i].m % 256 != 0) tile = tile == 2 ? 1 : tile == 4 ? 3 : tile;
  if (tile == 2 && (c->coherent || amp)) tile = 3;  // that kernel has no such epilogues
  if (tile == 2 && products == 2) tile = 1;          // nor two products
  const int tm = tile == 2 || tile == 4 ? 256 : 128;
  const int tn = tile >= 3 ? 256 : 128;
  const bool bf = path == LW_PATH_MFMA_BF16;

  const int ngroups = (pc->nb + kBandGroup - 1) / kBandGroup;  // spreading work-groups per column
  for (int64_t p0 = 0; p0 < b->n_particles; p0 += L.chunk) {
    const int nl = (int)std::min<int64_t>(L.chunk, b->n_particles - p0);
    const int nft = (2 * nl + tn - 1) / tn;
    sa.p_begin = ga.p_begin = p0;
    sa.n_local = ga.n_local = nl;
    sa.n_ftile = ga.n_ftile = nft;
    MF_HIP(prof_begin(c, kProfSpread), "profile");
    if (pc->shape.w == kShapeSplit.w)
      hipLaunchKernelGGL(lw_spread_kernel<kShapeSplit.w>, dim3((unsigned)((int64_t)nl * c->nd * ngroups)),
                         dim3(kSpreadWin), 0, c->stream, sa);
    else
      hipLaunchKernelGGL(lw_spread_kernel<kShapeSingle.w>, dim3((unsigned)((int64_t)nl * c->nd * ngroups)),
                         dim3(kSpreadWin), 0, c->stream, sa);
    MF_HIP(hipGetLastError(), "launch spread");
    MF_HIP(prof_end(c), "profile");
    hipLaunchKernelGGL(lw_sort_columns_kernel,
                       dim3((unsigned)(c->nd * pc->nb * ((nl + kSortBlock - 1) / kSortBlock))), dim3(1024), 0,
                       c->stream, colq, nl, perm);
    MF_HIP(hipGetLastError(), "launch column sort");
    int tiles = 0;
    for (int oi = 0; oi < pc->nb; ++oi) {
      ga.tiles_before[oi] = tiles;
      const int groups = c->nd * nft;
      tiles += (pc->band[ga.order[oi]].m / tm) * ((groups + 7) / 8) * 8;
    }
    ga.tiles_before[pc->nb] = tiles;
    MF_HIP(prof_begin(c, kProfGemm), "profile");
#define LW_GEMM_R128(T, P)                                                                       \
  do {                                                                                           \
    if (tile == 4)                                                                               \
      hipLaunchKernelGGL((lw_dft_mfma_r128_kernel<T, P, 4, 4, 2>), dim3(tiles), dim3(512), 0, c->stream, ga); \
    else if (tile == 3)                                                                          \
      hipLaunchKernelGGL((lw_dft_mfma_r128_kernel<T, P, 4, 2, 2>), dim3(tiles), dim3(512), 0, c->stream, ga); \
    else                                                                                         \
      hipLaunchKernelGGL((lw_dft_mfma_r128_kernel<T, P, 2, 2, 2>), dim3(tiles), dim3(256), 0, c->stream, ga); \
  } while (0)
#define LW_GEMM(T, P)                                                                            \
  do {                                                                                           \
    if (tile == 2)                                                                               \
      hipLaunchKernelGGL((lw_dft_mfma_kernel<T, P, 4>), dim3(tiles), dim3(512), 0, c->stream, ga); \
    else                                                                                         \
      LW_GEMM_R128(T, P);                                                                        \
  } while (0)
    if (!bf && products == 1) LW_GEMM(_Float16, 1);
    else if (!bf && products == 2) LW_GEMM_R128(_Float16, 2);
    else if (!bf) LW_GEMM(_Float16, 3);
    else if (products == 1) LW_GEMM(__bf16, 1);
    else LW_GEMM(__bf16, 3);
#undef LW_GEMM
#undef LW_GEMM_R128
    MF_HIP(hipGetLastError(), "launch dft_mfma");
    MF_HIP(prof_end(c), "profile");
    if (!amp) {
      const int n = c->nd * c->ns * c->nw;
      dim3 grid((unsigned)((n + 255) / 256)), block(256);
      if (c->coherent)
        hipLaunchKernelGGL(lw_mfma_reduce_coherent_kernel, grid, block, 0, c->stream, partial, nft,
                           c->ns, pc->rows, pc->row_of_j, pc->rowc, c->nw, c->nd, c->d_A);
      else
        hipLaunchKernelGGL(lw_mfma_reduce_kernel, grid, block, 0, c->stream, partial, nft, c->ns,
                           pc->rows, pc->row_of_j, pc->rowfac, c->nw, c->nd, c->d_S);
      MF_HIP(hipGetLastError(), "launch mfma reduce");
    }
  }
  return LW_OK;
}

}  // namespace lw
