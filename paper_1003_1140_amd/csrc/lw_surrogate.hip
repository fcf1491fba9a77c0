// lw_surrogate.hip -- learned spectrum surrogate: trajectory features and a small MLP
// trained and evaluated with BF16 matrix-core kernels (FP32 accumulation).
//
// The surrogate maps 16 features of one (particle, direction) pair to the
// normalised log spectrum on a fixed frequency grid; the exact accumulation
// kernels produce its training targets, judge a held-out fraction and take over
// for the pairs its error head flags.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <type_traits>
#include <vector>

#include "lw_internal.h"

namespace lw {

constexpr int kFeat = 16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16v __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ features
// One work-group per (particle, group of up to kDirGroup directions): the
// trajectory is read twice (moments, then deflections from the mean velocity)
// and the direction-dependent sums of the group ride along with the first pass.
// Sums in FP64, reduced across the wave by DPP.
constexpr int kDirGroup = 4;

constexpr int kFeatThreads = 64;  // one wave per (particle, direction group)

// Wave reductions of FP64 values without LDS traffic: DPP lane permutations of the two
// 32-bit halves.  The four in-row steps give every lane of a row of 16 its row's value; the
// row broadcasts then fold row 0 into row 1 (and row 2 into row 3), and rows 0-1 into row 3,
// so lane 63 holds the result, which is read out to every lane.  Lanes a row mask leaves out
// keep their own value (so a sum holds partial garbage there, in rows never read).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp64(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = (int)u, hi = (int)(u >> 32);
  const int plo = __builtin_amdgcn_update_dpp(lo, lo, kCtrl, kRowMask, 0xF, false);
  const int phi = __builtin_amdgcn_update_dpp(hi, hi, kCtrl, kRowMask, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)phi << 32) | (unsigned)plo));
}

template <typename Op>
__device__ __forceinline__ double wave_reduce(double v, Op op) {
  constexpr int kXor1 = 0xB1, kXor2 = 0x4E, kHalfMirror = 0x141, kMirror = 0x140;
  constexpr int kRowBcast15 = 0x142, kRowBcast31 = 0x143;
  v = op(v, dpp64<kXor1, 0xF>(v));
  v = op(v, dpp64<kXor2, 0xF>(v));
  v = op(v, dpp64<kHalfMirror, 0xF>(v));
  v = op(v, dpp64<kMirror, 0xF>(v));
  v = op(v, dpp64<kRowBcast15, 0xA>(v));
  v = op(v, dpp64<kRowBcast31, 0xC>(v));
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)u, 63), hi = __builtin_amdgcn_readlane((int)(u >> 32), 63);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

struct OpSum {
  __device__ double operator()(double a, double b) const { return a + b; }
};
struct OpMin {
  __device__ double operator()(double a, double b) const { return fmin(a, b); }
};
struct OpMax {
  __device__ double operator()(double a, double b) const { return fmax(a, b); }
};

__global__ __launch_bounds__(kFeatThreads) void lw_features_kernel(BatchView b, const double* dirs, int nd,
                                                          float* feats, unsigned long long* err) {
  // direction-independent sums 0..9, then per direction g: kappa sum, kappa min, cone count,
  // radiated energy sum |n x ((n - beta) x betadot)|^2 / kappa^5
  constexpr int NI = 10, NQ = NI + 4 * kDirGroup;
  __shared__ double s_tot[NQ];
  const int tid = threadIdx.x;
  const int n_groups = (nd + kDirGroup - 1) / kDirGroup;
  const int64_t p = blockIdx.x / n_groups;
  const int d0 = (int)(blockIdx.x % n_groups) * kDirGroup;
  const int ng = min(kDirGroup, nd - d0);
  double n[kDirGroup][3];
  #pragma unroll
  for (int g = 0; g < kDirGroup; ++g)
    for (int c = 0; c < 3; ++c) n[g][c] = g < ng ? dirs[kDirStride * (d0 + g) + c] : 0.0;
  // the two polarisation axes e1, e2 normal to each direction, read at one address by all
  // lanes
  __shared__ double s_e[kDirGroup][6];
  if (tid < kDirGroup * 6) {
    const int g = tid / 6;
    s_e[g][tid % 6] = g < ng ? dirs[kDirStride * (d0 + g) + 3 + tid % 6] : 0.0;
  }
  __syncthreads();
  const int64_t o = b.offsets[p], len = b.offsets[p + 1] - o;
  double q[NQ];
  #pragma unroll
  for (int i = 0; i < NQ; ++i) q[i] = 0.0;
  #pragma unroll
  for (int g = 0; g < kDirGroup; ++g) q[NI + 4 * g + 1] = 1.0e300;
  // Precision: 1 - beta^2, kappa = 1 - n.beta, e.beta, the unit velocity and the cone test
  // are FP64 (they cancel as |beta| -> 1, or decide a count); gamma, |a_perp| and the
  // integrand's projections are FP32 values (relative error ~1e-7) summed in FP64.
  for (int64_t k = tid; k < len; k += kFeatThreads) {
    const int64_t i = o + k;
    const double bx = b.bx[i], by = b.by[i], bz = b.bz[i];
    double ax, ay, az;
    lw::load_accel(b, i, ax, ay, az);
    const double b2 = bx * bx + by * by + bz * bz;
    if (!(b2 < 1.0)) {
      atomicMin(err, (unsigned long long)p);
      continue;
    }
    const double y = 1.0 - b2;  // 1 / gamma^2
    const float gam = __builtin_amdgcn_rsqf((float)y);
    // 1 / |beta|: an FP32 reciprocal square root refined by one Newton step (relative
    // error ~1e-14); a particle at rest has u = 0
    double inv = 0.0;
    if (b2 > 0.0) {
      const double r0 = (double)__builtin_amdgcn_rsqf((float)b2);
      inv = r0 * (1.5 - 0.5 * b2 * r0 * r0);
    }
    const double ux = bx * inv, uy = by * inv, uz = bz * inv;
    const float axf = (float)ax, ayf = (float)ay, azf = (float)az;
    const float uxf = (float)ux, uyf = (float)uy, uzf = (float)uz;
    const float apar = axf * uxf + ayf * uyf + azf * uzf;
    const float px = axf - apar * uxf, py = ayf - apar * uyf, pz = azf - apar * uzf;
    const float ap2 = px * px + py * py + pz * pz;
    const float ap = __builtin_amdgcn_sqrtf(ap2);
    q[0] += (double)gam;
    q[1] += (double)gam * (double)gam;
    q[2] += (double)ap;
    q[3] += (double)ap2;
    q[4] += (double)ap2 * (double)ap2;
    if (k > 0) {
      double px0, py0, pz0;
      lw::load_accel(b, i - 1, px0, py0, pz0);
      const double dot = ax * px0 + ay * py0 + az * pz0;
      if (dot < 0.0) q[5] += 1.0;
    }
    q[6] = fmax(q[6], (double)ap);
    q[7] += ux;
    q[8] += uy;
    q[9] += uz;
    // inside the 1/gamma cone around the velocity: the angle to n is below 1/gamma
    // (<= 1 rad), i.e. the cosine u.n exceeds cos(1/gamma) = sum_k (-1)^k y^k / (2k)! with
    // y = 1/gamma^2 <= 1 (the series through y^9 is within 1/20! < 5e-19); a particle at
    // rest has angle 0 by convention
    double cos_cone = 0.0;
    #pragma unroll
    for (int m = 9; m >= 0; --m) {
      double f = 1.0;  // (2m)!
      for (int j = 2; j <= 2 * m; ++j) f *= (double)j;
      cos_cone = cos_cone * y + ((m & 1) ? -1.0 : 1.0) / f;
    }
    #pragma unroll
    for (int g = 0; g < kDirGroup; ++g) {
      const double* m = n[g];
      const double kap = 1.0 - (m[0] * bx + m[1] * by + m[2] * bz);
      q[NI + 4 * g] += kap;
      q[NI + 4 * g + 1] = fmin(q[NI + 4 * g + 1], kap);
      if (b2 == 0.0 || ux * m[0] + uy * m[1] + uz * m[2] > cos_cone) q[NI + 4 * g + 2] += 1.0;
      // |n x ((n - beta) x a)|^2 from its components on e1, e2 (normal to n):
      // e.(n x ((n - beta) x a)) = -(e.beta)(n.a) - kappa (e.a)
      const double* e1 = s_e[g];
      const double* e2 = s_e[g] + 3;
      const float na = (float)m[0] * axf + (float)m[1] * ayf + (float)m[2] * azf;
      const float e1b = (float)(e1[0] * bx + e1[1] * by + e1[2] * bz);
      const float e2b = (float)(e2[0] * bx + e2[1] * by + e2[2] * bz);
      const float e1a = (float)e1[0] * axf + (float)e1[1] * ayf + (float)e1[2] * azf;
      const float e2a = (float)e2[0] * axf + (float)e2[1] * ayf + (float)e2[2] * azf;
      const float kf = (float)kap;
      const float g1 = e1b * na + kf * e1a, g2 = e2b * na + kf * e2a;
      // 1 / kappa in FP64 (kappa^-5 leaves the FP32 range as gamma grows): FP32 reciprocal
      // and one Newton step
      const double r0 = (double)__builtin_amdgcn_rcpf(kf);
      const double ik = r0 * (2.0 - kap * r0), ik2 = ik * ik;
      q[NI + 4 * g + 3] += (double)(g1 * g1 + g2 * g2) * (ik2 * ik2 * ik);
    }
  }
  // index 6 is a maximum, the kappa minima of the directions are minima, the rest sums
  #pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const double v = i == 6 ? wave_reduce(q[i], OpMax()) :
                     (i >= NI && (i - NI) % 4 == 1 ? wave_reduce(q[i], OpMin()) : wave_reduce(q[i], OpSum()));
    if (tid == 0) s_tot[i] = v;
  }
  __syncthreads();
  const double N = (double)max(len, (int64_t)1);
  double ex = s_tot[7], ey = s_tot[8], ez = s_tot[9];
  const double el = sqrt(ex * ex + ey * ey + ez * ez);
  const double ie = el > 0.0 ? 1.0 / el : 0.0;
  ex *= ie;
  ey *= ie;
  ez *= ie;
  // pass 2: deflection of the unit velocity from the mean direction (FP32 angles, relative
  // error ~1e-7 against the angles' spread)
  const float exf = (float)ex, eyf = (float)ey, ezf = (float)ez;
  double th2 = 0.0;
  float thmax = 0.0f;
  for (int64_t k = tid; k < len; k += kFeatThreads) {
    const int64_t i = o + k;
    const float bx = (float)b.bx[i], by = (float)b.by[i], bz = (float)b.bz[i];
    const float bb = bx * bx + by * by + bz * bz;
    const float inv = bb > 0.0f ? __builtin_amdgcn_rsqf(bb) : 0.0f;
    const float ux = bx * inv, uy = by * inv, uz = bz * inv;
    const float cx = uy * ezf - uz * eyf, cy = uz * exf - ux * ezf, cz = ux * eyf - uy * exf;
    const float th = atan2f(__builtin_amdgcn_sqrtf(cx * cx + cy * cy + cz * cz), ux * exf + uy * eyf + uz * ezf);
    th2 += (double)th * (double)th;
    thmax = fmaxf(thmax, th);
  }
  const double t2 = wave_reduce(th2, OpSum());
  const double tm = wave_reduce((double)thmax, OpMax());
  if (tid < ng) {
    const int g = tid;
    const double eps = 1e-12;
    const double gm = s_tot[0] / N;
    const double gvar = fmax(s_tot[1] / N - gm * gm, 0.0);
    const double m2 = s_tot[3] / N;
    const double T = N * b.dt[p];
    const double rate = s_tot[5] / T;
    const double* m = n[g];
    const double cx = ey * m[2] - ez * m[1], cy = ez * m[0] - ex * m[2], cz = ex * m[1] - ey * m[0];
    const double ang_ne = atan2(sqrt(cx * cx + cy * cy + cz * cz), ex * m[0] + ey * m[1] + ez * m[2]);
    float* f = feats + ((size_t)p * nd + d0 + g) * kFeat;
    f[0] = (float)log(gm);
    f[1] = (float)(sqrt(gvar) / gm);
    f[2] = (float)log(s_tot[2] / N + eps);
    f[3] = (float)log(sqrt(m2) + eps);
    f[4] = (float)log(s_tot[6] + eps);
    f[5] = (float)(m2 > 0.0 ? (s_tot[4] / N) / (m2 * m2) : 0.0);
    f[6] = (float)(gm * sqrt(t2 / N));
    f[7] = (float)(gm * tm);
    f[8] = (float)rate;
    f[9] = (float)log(gm * gm * rate + 1e-6);
    f[10] = (float)log(T);
    f[11] = (float)log(s_tot[NI + 4 * g + 3] * b.dt[p] / (4.0 * M_PI) + 1e-30);
    f[12] = (float)(gm * ang_ne);
    f[13] = (float)log(s_tot[NI + 4 * g] / N);
    f[14] = (float)log(s_tot[NI + 4 * g + 1]);
    f[15] = (float)(s_tot[NI + 4 * g + 2] / N);
  }
}

// ------------------------------------------------------------------ BF16 MFMA GEMM
// C[i][j] = sum_k A(i,k) B(k,j), with A(i,k) = A[i*sai + k*sak] and B(k,j) = B[k*sbk + j*sbj].
// FP32 operands are rounded to BF16 as they are staged in LDS; products accumulate in FP32 on
// v_mfma_f32_32x32x16_bf16.  Epilogue (applied when the inner dimension is not split): add
// bias[j] and row_coeff * row_add[i*row_stride]; write C = v, and also H = GELU(v) when H is
// given (a layer's pre-activation and activation in one pass), or C = v GELU'(Z[i*ldc + j])
// when Z is given (the backward of the activation, fused into the product that feeds it).
struct GemmDesc {
  const float* A;
  int64_t sai, sak;
  const float* B;
  int64_t sbk, sbj;
  float* C;
  int64_t ldc;
  const float* bias;
  int64_t M, N, K;
  const float* row_add = nullptr;  // per-row term added to every column, or null
  int64_t row_stride = 0;
  float row_coeff = 0.0f;
  float* H = nullptr;              // GELU of the result, or null
  const float* Z = nullptr;        // multiply the result by GELU'(Z), or null
  float* part = nullptr;           // split inner dimension: partial products [splits][M][N]
  int splits = 1;
  int gelu_out = 0;                // 1: write C = GELU(v) instead (inference: no pre-activation kept)
};

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  const float cdf = 0.5f * (1.0f + erff(z * 0.70710678118654752f));
  const float pdf = 0.39894228040143268f * __expf(-0.5f * z * z);
  return cdf + z * pdf;
}

__device__ __forceinline__ float gemm_epilogue(const GemmDesc& g, int64_t ii, int64_t jj, float v) {
  if (g.bias) v += g.bias[jj];
  if (g.row_add) v += g.row_coeff * g.row_add[ii * g.row_stride];
  return v;
}

__device__ __forceinline__ void gemm_store(const GemmDesc& g, int64_t ii, int64_t jj, float v) {
  if (g.Z) v *= gelu_grad_f(g.Z[ii * g.ldc + jj]);
  g.C[ii * g.ldc + jj] = g.gelu_out ? gelu_f(v) : v;
  if (g.H) g.H[ii * g.ldc + jj] = gelu_f(v);
}

// General shapes and strides: 64 x 64 tile per work-group of 4 waves (2 x 2 blocks of 32 x 32),
// inner steps of 16, scalar loads.
__global__ __launch_bounds__(256) void lw_gemm_bf16_kernel(GemmDesc g) {
  constexpr int T = 64, KS = 16, LD = KS + 8;
  __shared__ __attribute__((aligned(16))) __bf16 sA[T * LD];
  __shared__ __attribute__((aligned(16))) __bf16 sB[T * LD];  // stored [j][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * T, j0 = (int64_t)blockIdx.y * T;
  const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
  f32x16v acc;
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  for (int64_t k0 = 0; k0 < g.K; k0 += KS) {
    for (int e = tid; e < T * KS; e += 256) {
      const int r = e / KS, kk = e % KS;
      const int64_t ii = i0 + r, k = k0 + kk;
      const float va = (ii < g.M && k < g.K) ? g.A[ii * g.sai + k * g.sak] : 0.0f;
      sA[r * LD + kk] = (__bf16)va;
      const int64_t jj = j0 + r;
      const float vb = (jj < g.N && k < g.K) ? g.B[k * g.sbk + jj * g.sbj] : 0.0f;
      sB[r * LD + kk] = (__bf16)vb;
    }
    __syncthreads();
    const int kk = 8 * (lane >> 5);
    const bf16x8 a = *(const bf16x8*)&sA[(wi + (lane & 31)) * LD + kk];
    const bf16x8 bb = *(const bf16x8*)&sB[(wj + (lane & 31)) * LD + kk];
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bb, acc, 0, 0, 0);
    __syncthreads();
  }
  for (int r = 0; r < 16; ++r) {
    const int64_t ii = i0 + wi + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
    const int64_t jj = j0 + wj + (lane & 31);
    if (ii < g.M && jj < g.N) gemm_store(g, ii, jj, gemm_epilogue(g, ii, jj, acc[r]));
  }
}

// Tiled form for operands with one unit stride each (A along k or along i, B along k or
// along j), dimensions that are multiples of 4 and 16-byte aligned rows: 128 x 128 tile per
// work-group of 4 waves (2 x 2, each 64 x 64 as 2 x 2 MFMA blocks), inner steps of 32 through
// two LDS buffers -- while the MFMAs of one step run, the next step's operands travel from
// memory to registers as float4 along the unit-stride index, and then to the other buffer.
// gridDim.z splits the inner dimension (partial tiles, added in a fixed order afterwards).
template <bool AK, bool BK>
__global__ __launch_bounds__(256) void lw_gemm_bf16_tiled_kernel(GemmDesc g) {
  constexpr int TM = 128, TN = 128, TK = 32, LD = TK + 8;
  __shared__ __attribute__((aligned(16))) __bf16 sA[2][TM * LD];  // [i][k]
  __shared__ __attribute__((aligned(16))) __bf16 sB[2][TN * LD];  // [j][k]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // tile of this work-group: blocks b, b + 8, ... share an XCD (work-groups are dealt to the 8
  // XCDs in turn); along that sequence the column tiles of one row tile come one after the
  // other, so the row tile of A is fetched once and reused from the XCD's L2
  const int ntn = (int)((g.N + TN - 1) / TN), ntm = (int)((g.M + TM - 1) / TM);
  const int xcd = (int)blockIdx.x % 8, seq = (int)blockIdx.x / 8;
  const int mt = (seq / ntn) * 8 + xcd, nt = seq % ntn;
  if (mt >= ntm) return;  // padding of the XCD-aware numbering
  const int64_t i0 = (int64_t)mt * TM, j0 = (int64_t)nt * TN;
  const int wi = (wave >> 1) * 64, wj = (wave & 1) * 64;
  // inner range of this split
  const int64_t kc = ((g.K + g.splits - 1) / g.splits + TK - 1) / TK * TK;
  const int64_t kb = (int64_t)blockIdx.z * kc, ke = min(g.K, kb + kc);

  f32x4 ra[4], rb[4];
  // float4 v of the thread: A (B) element block (row or column, k) of the tile
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int idx = tid + 256 * v;
      if (AK) {  // 128 rows x 8 float4 along k
        const int r = idx >> 3, kq = (idx & 7) * 4;
        const int64_t ii = i0 + r, k = k0 + kq;
        ra[v] = (ii < g.M && k < ke) ? *(const f32x4*)(g.A + ii * g.sai + k) : f32x4{0.f, 0.f, 0.f, 0.f};
      } else {   // 32 k x 32 float4 along i
        const int k = idx >> 5, rq = (idx & 31) * 4;
        const int64_t ii = i0 + rq, kk = k0 + k;
        ra[v] = (ii < g.M && kk < ke) ? *(const f32x4*)(g.A + ii + kk * g.sak) : f32x4{0.f, 0.f, 0.f, 0.f};
      }
      if (BK) {
        const int c = idx >> 3, kq = (idx & 7) * 4;
        const int64_t jj = j0 + c, k = k0 + kq;
        rb[v] = (jj < g.N && k < ke) ? *(const f32x4*)(g.B + jj * g.sbj + k) : f32x4{0.f, 0.f, 0.f, 0.f};
      } else {
        const int k = idx >> 5, cq = (idx & 31) * 4;
        const int64_t jj = j0 + cq, kk = k0 + k;
        rb[v] = (jj < g.N && kk < ke) ? *(const f32x4*)(g.B + jj + kk * g.sbk) : f32x4{0.f, 0.f, 0.f, 0.f};
      }
    }
  };
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  auto store = [&](int buf) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int idx = tid + 256 * v;
      if (AK) {
        const int r = idx >> 3, kq = (idx & 7) * 4;
        *(bf16x4*)&sA[buf][r * LD + kq] = bf16x4{(__bf16)ra[v][0], (__bf16)ra[v][1], (__bf16)ra[v][2], (__bf16)ra[v][3]};
      } else {
        const int k = idx >> 5, rq = (idx & 31) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) sA[buf][(rq + e) * LD + k] = (__bf16)ra[v][e];
      }
      if (BK) {
        const int c = idx >> 3, kq = (idx & 7) * 4;
        *(bf16x4*)&sB[buf][c * LD + kq] = bf16x4{(__bf16)rb[v][0], (__bf16)rb[v][1], (__bf16)rb[v][2], (__bf16)rb[v][3]};
      } else {
        const int k = idx >> 5, cq = (idx & 31) * 4;
#pragma unroll
        for (int e = 0; e < 4; ++e) sB[buf][(cq + e) * LD + k] = (__bf16)rb[v][e];
      }
    }
  };

  f32x16v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
  if (kb < ke) {
    load(kb);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = kb; k0 < ke; k0 += TK) {
    const bool more = k0 + TK < ke;
    if (more) load(k0 + TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 16) {
      const int kk = ks + 8 * (lane >> 5);
      bf16x8 fa[2], fb[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) fa[a] = *(const bf16x8*)&sA[buf][(wi + 32 * a + (lane & 31)) * LD + kk];
#pragma unroll
      for (int b = 0; b < 2; ++b) fb[b] = *(const bf16x8*)&sB[buf][(wj + 32 * b + (lane & 31)) * LD + kk];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[a], fb[b], acc[a][b], 0, 0, 0);
    }
    if (more) store(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t ii = i0 + wi + 32 * a + 8 * (r / 4) + 4 * (lane >> 5) + (r % 4);
        const int64_t jj = j0 + wj + 32 * b + (lane & 31);
        if (ii >= g.M || jj >= g.N) continue;
        if (g.splits > 1)
          g.part[((int64_t)blockIdx.z * g.M + ii) * g.N + jj] = acc[a][b][r];
        else
          gemm_store(g, ii, jj, gemm_epilogue(g, ii, jj, acc[a][b][r]));
      }
}

// Split inner dimension: C = sum over splits in order of the partial products, then the epilogue.
__global__ void lw_gemm_splitk_reduce_kernel(GemmDesc g) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.M * g.N) return;
  const int64_t ii = e / g.N, jj = e % g.N;
  float v = 0.0f;
  for (int z = 0; z < g.splits; ++z) v += g.part[(int64_t)z * g.M * g.N + e];
  gemm_store(g, ii, jj, gemm_epilogue(g, ii, jj, v));
}

// Inner-dimension splits of a product whose output alone gives too few tiles to fill the
// chip (weight gradients: 256 x 256 outputs over many rows).
constexpr int kMaxSplits = 64;
inline int gemm_splits(int64_t M, int64_t N, int64_t K) {
  const int64_t tiles = ((M + 127) / 128) * ((N + 127) / 128);
  int s = 1;
  while (s < kMaxSplits && tiles * s < 512 && K / (2 * s) >= 256) s *= 2;
  return s;
}

hipError_t gemm_bf16(const GemmDesc& g0, hipStream_t s) {
  if (g0.M <= 0 || g0.N <= 0) return hipSuccess;
  GemmDesc g = g0;
  const bool ak = g.sak == 1, ai = g.sai == 1, bk = g.sbk == 1, bj = g.sbj == 1;
  const auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  const bool tiled = (ak || ai) && (bk || bj) && g.M % 4 == 0 && g.N % 4 == 0 && g.K % 4 == 0 &&
                     al16(g.A) && al16(g.B) && (ak ? g.sai % 4 == 0 : g.sak % 4 == 0) &&
                     (bk ? g.sbj % 4 == 0 : g.sbk % 4 == 0);
  if (!tiled) {
    dim3 grid((unsigned)((g.M + 63) / 64), (unsigned)((g.N + 63) / 64)), block(256);
    hipLaunchKernelGGL(lw_gemm_bf16_kernel, grid, block, 0, s, g);
    return hipGetLastError();
  }
  g.splits = g.part ? gemm_splits(g.M, g.N, g.K) : 1;
  // row tiles rounded up to a multiple of 8 (one per XCD), times the column tiles
  const int64_t ntm = (g.M + 127) / 128, ntn = (g.N + 127) / 128;
  dim3 grid((unsigned)((ntm + 7) / 8 * 8 * ntn), 1, (unsigned)g.splits), block(256);
  if (ak && bk) hipLaunchKernelGGL((lw_gemm_bf16_tiled_kernel<true, true>), grid, block, 0, s, g);
  else if (ak) hipLaunchKernelGGL((lw_gemm_bf16_tiled_kernel<true, false>), grid, block, 0, s, g);
  else if (bk) hipLaunchKernelGGL((lw_gemm_bf16_tiled_kernel<false, true>), grid, block, 0, s, g);
  else hipLaunchKernelGGL((lw_gemm_bf16_tiled_kernel<false, false>), grid, block, 0, s, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g.splits == 1) return e;
  const int64_t n = g.M * g.N;
  hipLaunchKernelGGL(lw_gemm_splitk_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g);
  return hipGetLastError();
}

// ------------------------------------------------------------------ elementwise kernels

__global__ void lw_normalise_kernel(const float* x, int64_t n, int n_in, const float* norm, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const int k = (int)(i % n_in);
    out[i] = (x[i] - norm[k]) * norm[n_in + k];
  }
}

// dY = 2 (Y - T) / (rows * cols); per-block partial sums of (Y - T)^2
__global__ void lw_mse_kernel(const float* y, const float* t, float* dy, int64_t n, double scale,
                              double* partial) {
  __shared__ double s[4];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e2 = 0.0;
  if (i < n) {
    const double e = (double)y[i] - (double)t[i];
    e2 = e * e;
    dy[i] = (float)(2.0 * e * scale);
  }
  e2 = wave_reduce(e2, OpSum());
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = e2;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = s[0] + s[1] + s[2] + s[3];
}

// Weighted column sums in two fixed-order stages (deterministic):
// out[j] = sum_r w_r X[r][j], with X[r][cols] = 1 for j == cols (a bias column) and
// w_r = 1, or w_r = scale (e_r - t_r) when e is given.  Stage 1: work-group (j-block of
// 64, row block) sums its rows in four interleaved lanes; stage 2 adds the row blocks.
constexpr int kColsumRows = 128;  // rows per stage-1 work-group

__global__ __launch_bounds__(256) void lw_colsum_stage1_kernel(const float* x, int64_t rows, int cols,
                                                               int n_out, const float* e, const float* t,
                                                               double scale, double* partial) {
  __shared__ double sp[4][64];
  const int jl = threadIdx.x & 63, lane4 = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + jl;
  const int64_t r0 = (int64_t)blockIdx.y * kColsumRows, r1 = min(rows, r0 + kColsumRows);
  double s = 0.0;
  if (j < n_out)
    for (int64_t r = r0 + lane4; r < r1; r += 4) {
      const double w = e ? scale * ((double)e[r] - (double)t[r]) : 1.0;
      s += w * (j < cols ? (double)x[r * cols + j] : 1.0);
    }
  sp[lane4][jl] = s;
  __syncthreads();
  if (lane4 == 0 && j < n_out)
    partial[(size_t)blockIdx.y * n_out + j] = ((sp[0][jl] + sp[1][jl]) + sp[2][jl]) + sp[3][jl];
}

__global__ void lw_colsum_stage2_kernel(const double* partial, int blocks, int n_out, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n_out) return;
  double s = 0.0;
  for (int b = 0; b < blocks; ++b) s += partial[(size_t)b * n_out + j];
  out[j] = (float)s;
}

__global__ void lw_adamw_kernel(float* p, float* m, float* v, const float* g, int64_t n, float lr,
                                float wd, float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * ((mi / c1) / (sqrtf(vi / c2) + eps) + wd * p[i]);
}

// error head: e[r] = w . h[r] + b (FP32 dot products, one thread per row)
__global__ void lw_head_fwd_kernel(const float* h, int64_t rows, int hidden, const float* w, float* e) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  float s = w[hidden];
  for (int i = 0; i < hidden; ++i) s = fmaf(w[i], h[r * hidden + i], s);
  e[r] = s;
}


// flags[p] = 1 when any direction's predicted error exceeds the threshold
__global__ void lw_flag_kernel(const float* err, int64_t P, int nd, float threshold, int32_t* flags) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  int f = 0;
  if (err)
    for (int d = 0; d < nd; ++d) f |= !(err[p * nd + d] <= threshold);
  flags[p] = f;
}

// partial[slice][s][d][j] = sum over the slice's unflagged particles of
// w q^2 10^(ylog[p][d][j] + calib[d][j])
__global__ void lw_surrogate_sum_kernel(const float* ylog, const float* calib, const int32_t* flags,
                                        const int32_t* species,
                                        const float* charge, const float* weight, int64_t P, int nd,
                                        int nw, int ns, int64_t per_slice, double* partial) {
  const int64_t col = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;  // d * nw + j
  const int64_t slice = blockIdx.x;
  if (col >= (int64_t)nd * nw) return;
  double acc[kMaxSpecies];
  for (int s = 0; s < ns; ++s) acc[s] = 0.0;
  const int64_t p0 = slice * per_slice, p1 = min(P, p0 + per_slice);
  const double off = calib ? (double)calib[col] : 0.0;
  for (int64_t p = p0; p < p1; ++p) {
    if (flags[p]) continue;
    const int s = species ? species[p] : 0;
    if (s < 0 || s >= ns) continue;
    const double q = charge ? (double)charge[p] : 1.0;
    const double w = weight ? (double)weight[p] : 1.0;
    acc[s] += w * q * q * exp10((double)ylog[p * (int64_t)nd * nw + col] + off);
  }
  for (int s = 0; s < ns; ++s) partial[(slice * ns + s) * (int64_t)nd * nw + col] = acc[s];
}

// In-order list of the flagged particles (one work-group: per-thread counts over
// contiguous ranges, an exclusive scan in LDS, then the writes); count[0] = total.
__global__ __launch_bounds__(1024) void lw_compact_kernel(const int32_t* flags, int64_t P, int64_t* idx,
                                                          int64_t* count) {
  __shared__ int64_t s_scan[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (P + 1023) / 1024;
  const int64_t a = min(P, (int64_t)t * chunk), e = min(P, a + chunk);
  int64_t c = 0;
  for (int64_t p = a; p < e; ++p) c += flags[p] != 0;
  s_scan[t] = c;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // inclusive Hillis-Steele scan
    const int64_t v = t >= off ? s_scan[t - off] : 0;
    __syncthreads();
    s_scan[t] += v;
    __syncthreads();
  }
  int64_t w = s_scan[t] - c;
  for (int64_t p = a; p < e; ++p)
    if (flags[p]) idx[w++] = p;
  if (t == 1023) count[0] = s_scan[1023];
}

// out[p][d][j] = log10(pp[p][d][j] / (w_p q_p^2) + floor): training targets from the
// exact kernel's per-particle spectra
__global__ void lw_log_targets_kernel(const float* pp, const float* charge, const float* weight, int64_t P,
                                      int64_t cols, double floor_value, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P * cols) return;
  const int64_t p = i / cols;
  const double q = charge ? (double)charge[p] : 1.0;
  const double w = weight ? (double)weight[p] : 1.0;
  out[i] = (float)log10((double)pp[i] / (w * q * q) + floor_value);
}

// ------------------------------------------------------------------ fused inference forward
// The whole network for a tile of 128 rows in one work-group of eight waves, two per SIMD, so
// that one wave's activation arithmetic overlaps the other's products.  Wave (r, c) owns rows
// 32 r .. 32 r + 31 and output columns 128 c .. 128 c + 127: it keeps a layer's 32 x 128
// outputs transposed in MFMA accumulators (the weights are the products' first operand, so
// that a lane holds four consecutive units of one row) and writes the activation (GELU in
// FP32, rounded to BF16 as the layered products round their A operand) over its part of an
// LDS activation tile, 8 bytes per four units, which is the next layer's second operand; a
// layer's last barrier orders every wave's reads of the tile before the rewrite.  The weights come from a BF16 copy of the parameters (the rounding the
// layered products apply as they stage them) in slabs of 64 inner indices through two LDS
// buffers shared by the eight waves, the next slab read from memory while the current one is
// multiplied.  Each layer's arithmetic is the layered path's (bias, then the skip term; inner
// index ascending in steps of 16), except that GELU's erf is the Abramowitz-Stegun rational
// form 7.1.26 (absolute error below 1.5e-7, far under the BF16 rounding that follows) and the
// error head sums the hidden units in another order.  Rows are read once and written once.
constexpr int kFusedRows = 128;         // rows per work-group
constexpr int kFusedMaxWidth = 256;     // widest layer (input tile padded to whole slabs)
constexpr int kFusedLD = kFusedMaxWidth + 8;
constexpr int kFusedSlab = 64;          // inner indices per weight slab
constexpr int kFusedSlabLD = kFusedSlab + 8;
constexpr int kFusedMaxLayers = 9;
constexpr int kFusedThreads = 512;      // eight waves: four row blocks x two column halves

struct FusedMlp {
  const float* x;       // [rows][n_in] raw inputs
  const float* norm;    // [2][n_in] input shift and scale, or null
  const float* p;       // parameters, FP32 (biases)
  const __bf16* w;      // parameters rounded to BF16 (weights)
  int64_t w_off[kFusedMaxLayers], b_off[kFusedMaxLayers];
  int n_in, hidden, n_hidden, n_out;
  int64_t rows;
  float* y;             // [rows][n_out]
  const float* head;    // error head [hidden + 1], or null
  float* e;             // [rows] error head output, or null
  int skip_index;       // raw input added (times skip_coeff) to every output, or -1
  float skip_coeff;
};

__global__ void lw_round_bf16_kernel(const float* p, int64_t n, __bf16* w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = (__bf16)p[i];
}

// GELU(z) = z Phi(z) = max(z, 0) - |z| erfc(|z| / sqrt 2) / 2, with erfc(x) = P(t) exp(-x^2),
// t = 1 / (1 + p x), from Abramowitz & Stegun 7.1.26 (P's coefficients halved here, exactly)
__device__ __forceinline__ float gelu_as(float z) {
  const float az = fabsf(z);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, az, 1.0f));
  float q = fmaf(0.5f * 1.061405429f, t, 0.5f * -1.453152027f);
  q = fmaf(q, t, 0.5f * 1.421413741f);
  q = fmaf(q, t, 0.5f * -0.284496736f);
  q = fmaf(q, t, 0.5f * 0.254829592f);
  // exp(-z^2 / 2) = 2^(-z^2 log2(e) / 2)
  const float e = __builtin_amdgcn_exp2f(z * (z * -0.72134752044448170f));
  return fmaf(-az, q * t * e, fmaxf(z, 0.0f));
}

__global__ __launch_bounds__(kFusedThreads) void lw_mlp_fused_forward_kernel(FusedMlp f) {
  __shared__ __attribute__((aligned(16))) __bf16 sH[kFusedRows * kFusedLD];
  __shared__ __attribute__((aligned(16))) __bf16 sW[2][kFusedMaxWidth * kFusedSlabLD];  // [j][k]
  __shared__ float s_head[2][kFusedRows];  // error-head partial sums of the two column halves
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 3, wc = wave >> 2;  // row block, column half
  const int m = lane & 31, half = lane >> 5;
  const int64_t i0 = (int64_t)blockIdx.x * kFusedRows;
  __bf16* myH = sH + (size_t)(wr * 32) * kFusedLD;

  // input tile: normalised inputs rounded to BF16 (four at a time, several loads in flight),
  // zero-padded to whole slabs
  typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
  const int kin = (f.n_in + kFusedSlab - 1) / kFusedSlab * kFusedSlab;
  const int q4 = f.n_in / 4;
#pragma unroll 4
  for (int idx = tid; idx < kFusedRows * q4; idx += kFusedThreads) {
    const int r = idx / q4, c = 4 * (idx - r * q4);
    const int64_t ii = i0 + r;
    f32x4 v = ii < f.rows ? *(const f32x4*)(f.x + ii * f.n_in + c) : f32x4{0.f, 0.f, 0.f, 0.f};
    if (f.norm) v = (v - *(const f32x4*)(f.norm + c)) * *(const f32x4*)(f.norm + f.n_in + c);
    *(bf16x4*)&sH[r * kFusedLD + c] = bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
  }
  for (int idx = tid; idx < kFusedRows * (kin - f.n_in); idx += kFusedThreads) {
    const int r = idx / (kin - f.n_in);
    sH[r * kFusedLD + f.n_in + (idx - r * (kin - f.n_in))] = (__bf16)0.0f;
  }

  // weight slabs: thread t moves 16-byte pieces t + 512 v (column j = idx / 8, inner 8 (idx % 8))
  constexpr int kPieces = kFusedMaxWidth * kFusedSlab / 8 / kFusedThreads;
  // two register sets: a slab's loads are issued two slabs ahead of its products
  u32x4 rw[kPieces];
  auto load_slab = [&](const __bf16* W, int din, int dout, int k0) {
#pragma unroll
    for (int v = 0; v < kPieces; ++v) {
      const int idx = tid + kFusedThreads * v, j = idx >> 3, kq = (idx & 7) * 8;
      rw[v] = (j < dout && k0 + kq < din) ? *(const u32x4*)(W + (int64_t)j * din + k0 + kq) : u32x4{0u, 0u, 0u, 0u};
    }
  };
  auto store_slab = [&](int b) {
#pragma unroll
    for (int v = 0; v < kPieces; ++v) {
      const int idx = tid + kFusedThreads * v, j = idx >> 3, kq = (idx & 7) * 8;
      *(u32x4*)&sW[b][j * kFusedSlabLD + kq] = rw[v];
    }
  };

  f32x16v acc[4];
  const bool full = i0 + kFusedRows <= f.rows;  // a whole tile skips the per-row checks
  int buf = 0;
  for (int l = 0; l <= f.n_hidden; ++l) {
    const bool out_layer = l == f.n_hidden;
    const int din = l == 0 ? f.n_in : f.hidden;
    const int kdim = l == 0 ? kin : f.hidden;  // a multiple of the slab
    const int dout = out_layer ? f.n_out : f.hidden;
    const int nb = dout / 32;
    const __bf16* W = f.w + f.w_off[l];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[b][r] = 0.0f;
    // the buffer about to be filled was last read two barriers ago
    load_slab(W, din, dout, 0);
    store_slab(buf);
    __syncthreads();  // slab stored (and, before the first layer, the input tile)
    for (int k0 = 0; k0 < kdim; k0 += kFusedSlab) {
      const bool more = k0 + kFusedSlab < kdim;
      if (more) load_slab(W, din, dout, k0 + kFusedSlab);
#pragma unroll
      for (int q = 0; q < kFusedSlab; q += 32) {
        // both inner halves' fragments are read before the products, and all four column
        // blocks are multiplied, also past a narrower layer's width (its slab columns there
        // are zeros): a branch per block would make each product wait for its own read
        bf16x8 fa[2], fb[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          fa[h] = *(const bf16x8*)&myH[m * kFusedLD + k0 + q + 16 * h + 8 * half];
#pragma unroll
          for (int b = 0; b < 4; ++b)
            fb[h][b] = *(const bf16x8*)&sW[buf][(32 * (4 * wc + b) + m) * kFusedSlabLD + q + 16 * h + 8 * half];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fb[h][b], fa[h], acc[b], 0, 0, 0);
        // keep the 10 reads ahead of the 8 products (the scheduler otherwise reuses one
        // register for every weight fragment and waits for each read in turn)
        __builtin_amdgcn_sched_group_barrier(0x100, 10, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 8, 0);
      }
      if (more) store_slab(buf ^ 1);
      __syncthreads();
      buf ^= 1;
    }
    const float* bias = f.p + f.b_off[l];
    if (!out_layer) {
      // activations over this wave's rows and columns (every wave's reads of the tile ended
      // at the layer's last barrier); the error head dots the last hidden layer in FP32
      const bool head = f.head && l == f.n_hidden - 1;
      float hs = 0.0f;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        if (4 * wc + b < nb) {
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const int j = 32 * (4 * wc + b) + 8 * g + 4 * half;  // this lane's four units
            const f32x4 bj = *(const f32x4*)(bias + j);
            f32x4 h;
#pragma unroll
            for (int i = 0; i < 4; ++i) h[i] = gelu_as(acc[b][4 * g + i] + bj[i]);
            *(bf16x4*)&myH[m * kFusedLD + j] = bf16x4{(__bf16)h[0], (__bf16)h[1], (__bf16)h[2], (__bf16)h[3]};
            if (head) {
              const f32x4 hw = *(const f32x4*)(f.head + j);
#pragma unroll
              for (int i = 0; i < 4; ++i) hs = fmaf(hw[i], h[i], hs);
            }
          }
        }
        // one column block at a time: interleaving the blocks' activations would hold
        // their temporaries all at once
        __builtin_amdgcn_sched_barrier(0);
      }
      if (head) {
        // this column half's sum for the row, kept for the output layer's epilogue (after the
        // output layer's barriers) to add the two halves
        hs += __shfl_xor(hs, 32);
        if (half == 0) s_head[wc][wr * 32 + m] = hs;
      }
    }
  }
  // output layer epilogue, after the loop (inside it, the compiler would hoist the rows'
  // addresses out of the loop and hold them through every layer)
  {
    const int nb = f.n_out / 32;
    const float* bias = f.p + f.b_off[f.n_hidden];
    const int64_t ii = i0 + wr * 32 + m;  // this lane's row
    const bool ok = full || ii < f.rows;
    const float xs = f.skip_index >= 0 ? f.x[min(ii, f.rows - 1) * f.n_in + f.skip_index] : 0.0f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      if (4 * wc + b < nb) {
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int j = 32 * (4 * wc + b) + 8 * g + 4 * half;
          const f32x4 bj = *(const f32x4*)(bias + j);
          f32x4 v;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            v[i] = acc[b][4 * g + i] + bj[i];
            if (f.skip_index >= 0) v[i] += f.skip_coeff * xs;
          }
          if (ok) *(f32x4*)(f.y + ii * f.n_out + j) = v;
        }
      }
    }
    if (f.head && f.e && f.n_hidden >= 1 && wc == 0 && half == 0 && ok)
      f.e[ii] = s_head[0][wr * 32 + m] + s_head[1][wr * 32 + m] + f.head[f.hidden];
  }
}


// ------------------------------------------------------------------ calibration statistics
// Column statistics of x [rows][cols] with rows grouped by row index modulo `groups` (row
// r = p groups + g belongs to particle p and group g): over the kept particles of a slice of
// kStatSlice particles, the sum of v, of v^2 and the count, with v = x[r][j] + coeff
// row_add[r stride] (row_add optional) or 10 to that power.  A particle is kept when err is
// null or its largest err[p][g'] over the groups is <= threshold.  Stage 1: one work-group
// per (64 columns, slice, group), four row lanes summed in a fixed order; stage 2 adds the
// slices in order.
constexpr int kStatSlice = 256;

__global__ __launch_bounds__(256) void lw_column_stats_stage1_kernel(
    const float* x, int64_t P, int cols, int groups, const float* row_add, int64_t stride, double coeff,
    int exp10, const float* err, float threshold, double* partial) {
  __shared__ double s[3][4][64];
  const int jl = threadIdx.x & 63, rl = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + jl;
  const int64_t slice = blockIdx.y;
  const int g = blockIdx.z;
  const int64_t p0 = slice * kStatSlice, p1 = min(P, p0 + kStatSlice);
  double s1 = 0.0, s2 = 0.0, cnt = 0.0;
  for (int64_t p = p0 + rl; p < p1; p += 4) {
    bool keep = true;
    if (err)
      for (int h = 0; h < groups; ++h) keep = keep && err[p * groups + h] <= threshold;
    if (!keep || j >= cols) continue;
    const int64_t r = p * groups + g;
    double v = (double)x[r * cols + j];
    if (row_add) v += coeff * (double)row_add[r * stride];
    if (exp10) v = pow(10.0, v);
    s1 += v;
    s2 += v * v;
    cnt += 1.0;
  }
  s[0][rl][jl] = s1;
  s[1][rl][jl] = s2;
  s[2][rl][jl] = cnt;
  __syncthreads();
  if (rl == 0 && j < cols) {
    double* o = partial + ((slice * groups + g) * (int64_t)cols + j) * 3;
    for (int k = 0; k < 3; ++k) o[k] = s[k][0][jl] + s[k][1][jl] + s[k][2][jl] + s[k][3][jl];
  }
}

// out[g][j] = (mean, mean square) over the kept particles (zeros when none is kept)
__global__ void lw_column_stats_stage2_kernel(const double* partial, int64_t slices, int groups, int cols,
                                              double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)groups * cols) return;
  double s1 = 0.0, s2 = 0.0, cnt = 0.0;
  for (int64_t t = 0; t < slices; ++t) {
    const double* q = partial + (t * groups * (int64_t)cols + i) * 3;
    s1 += q[0];
    s2 += q[1];
    cnt += q[2];
  }
  out[2 * i] = cnt > 0.0 ? s1 / cnt : 0.0;
  out[2 * i + 1] = cnt > 0.0 ? s2 / cnt : 0.0;
}

// share[r] = log10(mean_j |10^pred[r][j] - 10^y[r][j]| / smean[r mod groups][j] + floor):
// one wave per row, lanes over the columns, a DPP sum.
__global__ __launch_bounds__(64) void lw_error_share_kernel(const float* pred, const float* y, int64_t rows,
                                                            int cols, int groups, const double* smean,
                                                            int64_t smean_stride, double floor_value,
                                                            float* share) {
  const int64_t r = blockIdx.x;
  if (r >= rows) return;
  const int g = (int)(r % groups);
  double acc = 0.0;
  for (int j = threadIdx.x; j < cols; j += 64) {
    const double d = fabs(pow(10.0, (double)pred[r * cols + j]) - pow(10.0, (double)y[r * cols + j]));
    acc += d / smean[((int64_t)g * cols + j) * smean_stride];
  }
  acc = wave_reduce(acc, OpSum());
  if (threadIdx.x == 0) share[r] = (float)log10(acc / cols + floor_value);
}

// Order-preserving 32-bit keys of the per-particle maxima max_g v[p][g] (NaN as the largest).
__device__ __forceinline__ uint32_t order_key(float f) {
  if (f != f) return 0xFFFFFFFFu;
  const uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float key_value(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k);
}

__global__ void lw_max_keys_kernel(const float* v, int64_t n, int groups, uint32_t* keys) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  uint32_t k = 0;
  for (int g = 0; g < groups; ++g) k = max(k, order_key(v[p * groups + g]));
  keys[p] = k;
}

// hist[b] += number of keys with (key & mask) == prefix and byte (key >> shift) & 255 == b
__global__ __launch_bounds__(256) void lw_radix_hist_kernel(const uint32_t* keys, int64_t n, uint32_t prefix,
                                                            uint32_t mask, int shift, unsigned* hist) {
  __shared__ unsigned h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t k = keys[i];
    if ((k & mask) == prefix) atomicAdd(&h[(k >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void lw_key_to_value_kernel(const uint32_t* key, double* out) { *out = (double)key_value(*key); }

// out[i] = log10(num[i s_num] / den[i s_den]) where both are positive, else 0
__global__ void lw_log_ratio_kernel(const double* num, int64_t s_num, const double* den, int64_t s_den,
                                    int64_t n, float* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double a = num[i * s_num], b = den[i * s_den];
  out[i] = (a > 0.0 && b > 0.0) ? (float)log10(a / b) : 0.0f;
}

}  // namespace lw

// ------------------------------------------------------------------ network object
struct lw_mlp {
  lw_ctx* c = nullptr;
  int n_in = 0, hidden = 0, n_hidden = 0, n_out = 0;
  int64_t n_params = 0;
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;  // main net (FP32 master)
  float *hp = nullptr, *hm = nullptr, *hv = nullptr, *hg = nullptr;  // error head [hidden + 1]
  int64_t step = 0, head_step = 0;
  int64_t rows_cap = 0;
  float* act = nullptr;  // z_l, h_l per hidden layer, y, dy, dh, dz, normalised x (rows_cap rows)
  float* norm = nullptr;  // device [2][n_in]: input shift and scale, or null (identity)
  int skip_index = -1;    // raw input added (times skip_coeff) to every output, or -1
  float skip_coeff = 0.0f;
  double* loss_part = nullptr;
  double* col_part = nullptr;  // stage-1 partial column sums [row blocks][max(n_out, hidden + 1)]
  float* err_buf = nullptr;
  float* splitk = nullptr;     // partial weight gradients [kMaxSplits][largest layer]
  __bf16* wbf = nullptr;       // parameters rounded to BF16 for the fused inference kernel
  std::vector<int64_t> w_off, b_off;
};

namespace {

lw_status mlp_fail(lw_mlp* n, lw_status st, const std::string& msg) {
  if (n && n->c) n->c->err = msg;
  return st;
}

#define MLP_HIP(call, what)                                                    \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) return mlp_fail(n, LW_EDEVICE, std::string(what) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Shapes the fused inference kernel takes: hidden width a multiple of 64 (whole weight slabs)
// and output width a multiple of 32, both up to 256; input width a multiple of 8 up to 256;
// 1 to 8 hidden layers; every layer's weights at a multiple of 8 parameters (16-byte BF16
// rows for the slab loads).
bool fused_shape(const lw_mlp* n) {
  if (n->hidden % lw::kFusedSlab != 0 || n->hidden > lw::kFusedMaxWidth || n->n_out % 32 != 0 ||
      n->n_out > lw::kFusedMaxWidth || n->n_in % 8 != 0 || n->n_in <= 0 || n->n_in > lw::kFusedMaxWidth ||
      n->n_hidden < 1 || n->n_hidden + 1 > lw::kFusedMaxLayers || !n->wbf)
    return false;
  for (int l = 0; l <= n->n_hidden; ++l)
    if (n->w_off[l] % 8 != 0) return false;
  return true;
}

int width(const lw_mlp* n, int l) {  // input width of layer l, l = 0..n_hidden (+1 = output)
  if (l == 0) return n->n_in;
  if (l <= n->n_hidden) return n->hidden;
  return n->n_out;
}

lw_status ensure_rows(lw_mlp* n, int64_t rows) {
  if (rows <= n->rows_cap) return LW_OK;
  if (n->act) (void)hipFree(n->act);
  if (n->loss_part) (void)hipFree(n->loss_part);
  if (n->err_buf) (void)hipFree(n->err_buf);
  if (n->col_part) (void)hipFree(n->col_part);
  n->act = nullptr;
  n->loss_part = nullptr;
  n->err_buf = nullptr;
  n->col_part = nullptr;
  const int64_t per_row = (int64_t)2 * n->n_hidden * n->hidden + 2 * n->n_out + 2 * n->hidden + n->n_in;
  MLP_HIP(hipMalloc(&n->act, (size_t)rows * per_row * sizeof(float)), "hipMalloc(activations)");
  const int64_t blocks = (rows * std::max(n->n_out, 1) + 255) / 256;
  MLP_HIP(hipMalloc(&n->loss_part, (size_t)blocks * sizeof(double)), "hipMalloc(loss)");
  MLP_HIP(hipMalloc(&n->err_buf, (size_t)rows * sizeof(float)), "hipMalloc(err)");
  const int64_t rblocks = (rows + lw::kColsumRows - 1) / lw::kColsumRows;
  const int64_t widest = std::max<int64_t>(std::max(n->n_out, n->hidden + 1), n->hidden);
  MLP_HIP(hipMalloc(&n->col_part, (size_t)rblocks * widest * sizeof(double)), "hipMalloc(column sums)");
  n->rows_cap = rows;
  return LW_OK;
}

// out[j] = sum_r w_r X[r][j] over j < n_out (see lw_colsum_stage1_kernel)
lw_status colsum(lw_mlp* n, const float* x, int64_t rows, int cols, int n_out, const float* e,
                 const float* t, double scale, float* out) {
  hipStream_t s = n->c->stream;
  const int rblocks = (int)((rows + lw::kColsumRows - 1) / lw::kColsumRows);
  hipLaunchKernelGGL(lw::lw_colsum_stage1_kernel, dim3((unsigned)((n_out + 63) / 64), (unsigned)rblocks),
                     dim3(256), 0, s, x, rows, cols, n_out, e, t, scale, n->col_part);
  MLP_HIP(hipGetLastError(), "column sums");
  hipLaunchKernelGGL(lw::lw_colsum_stage2_kernel, dim3((unsigned)((n_out + 255) / 256)), dim3(256), 0, s,
                     n->col_part, rblocks, n_out, out);
  MLP_HIP(hipGetLastError(), "column sums");
  return LW_OK;
}

float* z_of(lw_mlp* n, int l, int64_t rows) { return n->act + (size_t)(2 * l) * rows * n->hidden; }
float* h_of(lw_mlp* n, int l, int64_t rows) { return n->act + (size_t)(2 * l + 1) * rows * n->hidden; }
float* y_of(lw_mlp* n, int64_t rows) { return n->act + (size_t)(2 * n->n_hidden) * rows * n->hidden; }
float* dy_of(lw_mlp* n, int64_t rows) { return y_of(n, rows) + (size_t)rows * n->n_out; }
float* dh_of(lw_mlp* n, int64_t rows) { return dy_of(n, rows) + (size_t)rows * n->n_out; }
float* dz_of(lw_mlp* n, int64_t rows) { return dh_of(n, rows) + (size_t)rows * n->hidden; }
float* xn_of(lw_mlp* n, int64_t rows) { return dz_of(n, rows) + (size_t)rows * n->hidden; }

// the network's input: x itself, or (x - shift) * scale in FP32 when a normalisation is set
lw_status input_of(lw_mlp* n, const float* x, int64_t rows, const float** in) {
  *in = x;
  if (!n->norm) return LW_OK;
  float* xn = xn_of(n, rows);
  const int64_t cnt = rows * n->n_in;
  hipLaunchKernelGGL(lw::lw_normalise_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0,
                     n->c->stream, x, cnt, n->n_in, n->norm, xn);
  MLP_HIP(hipGetLastError(), "normalise");
  *in = xn;
  return LW_OK;
}

// forward: fills z_l, h_l and y (into `y` if given, else the workspace)
// keep_pre: also keep each hidden layer's pre-activation z (the backward needs it); inference
// writes the activations alone.
lw_status forward(lw_mlp* n, const float* raw, const float* x, int64_t rows, float* y, bool keep_pre = true) {
  hipStream_t s = n->c->stream;
  const float* in = x;
  for (int l = 0; l <= n->n_hidden; ++l) {
    const int din = width(n, l), dout = l < n->n_hidden ? n->hidden : n->n_out;
    float* out = l < n->n_hidden ? z_of(n, l, rows) : y;
    lw::GemmDesc g{in, din, 1, n->p + n->w_off[l], 1, din, out, dout, n->p + n->b_off[l], rows, dout, din};
    if (l == n->n_hidden && n->skip_index >= 0) {
      g.row_add = raw + n->skip_index;
      g.row_stride = n->n_in;
      g.row_coeff = n->skip_coeff;
    }
    if (l < n->n_hidden) {  // pre-activation and GELU in one pass
      if (keep_pre) {
        g.H = h_of(n, l, rows);
      } else {
        g.C = h_of(n, l, rows);
        g.gelu_out = 1;
      }
    }
    MLP_HIP(lw::gemm_bf16(g, s), "gemm forward");
    if (l < n->n_hidden) in = h_of(n, l, rows);
  }
  return LW_OK;
}

// backward from dy (already in the workspace) into n->g
lw_status backward(lw_mlp* n, const float* x, int64_t rows) {
  hipStream_t s = n->c->stream;
  const float* d = dy_of(n, rows);  // dLoss/d(pre-activation) of the current layer
  for (int l = n->n_hidden; l >= 0; --l) {
    const int din = width(n, l), dout = l < n->n_hidden ? n->hidden : n->n_out;
    const float* in = l == 0 ? x : h_of(n, l - 1, rows);
    // dW[o][i] = sum_r d[r][o] in[r][i]
    lw::GemmDesc gw{d, 1, dout, in, din, 1, n->g + n->w_off[l], din, nullptr, dout, din, rows};
    gw.part = n->splitk;  // many rows, few outputs: the rows are split over work-groups
    MLP_HIP(lw::gemm_bf16(gw, s), "gemm dW");
    lw_status cst = colsum(n, d, rows, dout, dout, nullptr, nullptr, 1.0, n->g + n->b_off[l]);
    if (cst != LW_OK) return cst;
    if (l > 0) {
      // dh[r][i] = sum_o d[r][o] W[o][i], then times gelu'(z)
      float* dh = (d == dz_of(n, rows)) ? dh_of(n, rows) : dz_of(n, rows);
      lw::GemmDesc gx{d, dout, 1, n->p + n->w_off[l], din, 1, dh, din, nullptr, rows, din, dout};
      gx.Z = z_of(n, l - 1, rows);  // times GELU'(z) of the layer below, in the same pass
      MLP_HIP(lw::gemm_bf16(gx, s), "gemm dX");
      d = dh;
    }
  }
  return LW_OK;
}

lw_status mse(lw_mlp* n, const float* y, const float* t, float* dy, int64_t count, double* loss) {
  hipStream_t s = n->c->stream;
  const int64_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(lw::lw_mse_kernel, dim3((unsigned)blocks), dim3(256), 0, s, y, t, dy, count,
                     1.0 / (double)count, n->loss_part);
  MLP_HIP(hipGetLastError(), "mse");
  if (loss) {
    std::vector<double> part(blocks);
    MLP_HIP(hipMemcpyAsync(part.data(), n->loss_part, blocks * sizeof(double), hipMemcpyDeviceToHost, s),
            "copy loss");
    MLP_HIP(hipStreamSynchronize(s), "sync");
    double sum = 0.0;
    for (double v : part) sum += v;
    *loss = sum / (double)count;
  }
  return LW_OK;
}

lw_status adamw(lw_mlp* n, float* p, float* m, float* v, const float* g, int64_t count, int64_t step,
                float lr, float wd) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(lw::lw_adamw_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                     n->c->stream, p, m, v, g, count, lr, wd, b1, b2, 1e-8f, c1, c2);
  MLP_HIP(hipGetLastError(), "adamw");
  return LW_OK;
}

}  // namespace

extern "C" {

lw_status lw_features(lw_ctx* c, const lw_batch* b, float* feats) {
  if (!c || !b || !feats) return LW_EINVAL;
  if (c->nd <= 0) {
    c->err = "directions not set";
    return LW_ESTATE;
  }
  if (b->n_particles == 0) return LW_OK;
  if (!b->offsets || !b->bx || !b->by || !b->bz || !b->ax || !b->ay || !b->az || !b->dt) {
    c->err = "batch pointer is NULL";
    return LW_EINVAL;
  }
  lw::BatchView v = lw::view_of(b);
  const int64_t blocks = b->n_particles * (int64_t)((c->nd + lw::kDirGroup - 1) / lw::kDirGroup);
  if (blocks > 0x7fffffffLL) {
    c->err = "too many particles for one feature launch";
    return LW_ERANGE;
  }
  hipLaunchKernelGGL(lw::lw_features_kernel, dim3((unsigned)blocks), dim3(lw::kFeatThreads), 0, c->stream, v,
                     c->d_dirs, c->nd, feats, c->d_err);
  if (hipGetLastError() != hipSuccess) {
    c->err = "launch lw_features";
    return LW_EDEVICE;
  }
  return LW_OK;
}

lw_status lw_surrogate_accumulate(lw_ctx* c, const lw_batch* b, const float* ylog, const float* calib,
                                  const float* err, float threshold, int32_t* flags, int64_t* flagged,
                                  int64_t* n_flagged, void* ws, size_t ws_bytes) {
  if (!c || !b || !ylog || !flags) return LW_EINVAL;
  if (c->nd <= 0 || c->nw <= 0) {
    c->err = "grids not set";
    return LW_ESTATE;
  }
  if (c->coherent) {
    c->err = "the surrogate estimates incoherent spectra only";
    return LW_EUNSUPPORTED;
  }
  const int64_t P = b->n_particles;
  if (P == 0) return LW_OK;
  const int64_t cols = (int64_t)c->nd * c->nw;
  // slices of 128 particles: ~8 work-groups per compute unit on a chunk of 1e5 particles
  // (with 1024 the sum waited on its loads and exponentials, 0.71 ms per 1e5 x 4 x 256)
  const int64_t per_slice = 128;
  const int64_t slices = (P + per_slice - 1) / per_slice;
  if (cols > 65535LL * 256) {
    c->err = "at most 65535 x 256 (direction, frequency) columns per surrogate call";
    return LW_ERANGE;
  }
  if ((flagged == nullptr) != (n_flagged == nullptr)) {
    c->err = "flagged and n_flagged go together";
    return LW_EINVAL;
  }
  const size_t need = (size_t)slices * c->ns * cols * sizeof(double);
  if (!ws || ws_bytes < need) {
    c->err = "workspace too small for the surrogate reduction (" + std::to_string(need) + " bytes)";
    return LW_ENOMEM;
  }
  hipStream_t s = c->stream;
  hipLaunchKernelGGL(lw::lw_flag_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, err, P, c->nd,
                     threshold, flags);
  hipLaunchKernelGGL(lw::lw_surrogate_sum_kernel, dim3((unsigned)slices, (unsigned)((cols + 255) / 256)),
                     dim3(256), 0, s, ylog, calib, flags, b->species, b->charge, b->weight, P, c->nd, c->nw,
                     c->ns, per_slice, (double*)ws);
  if (lw::launch_reduce_partials((double*)ws, slices, (int64_t)c->ns * cols, c->d_S, s) != hipSuccess ||
      hipGetLastError() != hipSuccess) {
    c->err = "launch surrogate reduction";
    return LW_EDEVICE;
  }
  if (flagged && n_flagged) {
    hipLaunchKernelGGL(lw::lw_compact_kernel, dim3(1), dim3(1024), 0, s, flags, P, flagged, n_flagged);
    if (hipGetLastError() != hipSuccess) {
      c->err = "launch flag compaction";
      return LW_EDEVICE;
    }
  }
  return LW_OK;
}

lw_status lw_surrogate_targets(lw_ctx* c, const lw_batch* b, const float* per_particle, double floor_value,
                               float* out) {
  if (!c || !b || !per_particle || !out || !(floor_value > 0.0)) return LW_EINVAL;
  const int64_t P = b->n_particles, cols = (int64_t)c->nd * c->nw;
  if (P == 0 || cols == 0) return LW_OK;
  const int64_t n = P * cols;
  hipLaunchKernelGGL(lw::lw_log_targets_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream,
                     per_particle, b->charge, b->weight, P, cols, floor_value, out);
  if (hipGetLastError() != hipSuccess) {
    c->err = "launch lw_log_targets";
    return LW_EDEVICE;
  }
  return LW_OK;
}

lw_status lw_mlp_create(lw_ctx* c, int32_t n_in, int32_t hidden, int32_t n_hidden, int32_t n_out,
                        uint64_t seed, lw_mlp** out) {
  if (!c || !out || n_in <= 0 || hidden <= 0 || n_hidden < 0 || n_out <= 0) return LW_EINVAL;
  lw_mlp* n = new lw_mlp();
  n->c = c;
  n->n_in = n_in;
  n->hidden = hidden;
  n->n_hidden = n_hidden;
  n->n_out = n_out;
  int64_t off = 0;
  for (int l = 0; l <= n_hidden; ++l) {
    const int din = width(n, l), dout = l < n_hidden ? hidden : n_out;
    n->w_off.push_back(off);
    off += (int64_t)dout * din;
    n->b_off.push_back(off);
    off += dout;
  }
  n->n_params = off;
  // initial weights: normal with variance 1/fan_in (Box-Muller on a 64-bit LCG), zero biases
  std::vector<float> h(off, 0.0f);
  uint64_t st = seed * 6364136223846793005ull + 1442695040888963407ull;
  auto uni = [&]() {
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    return ((st >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  };
  for (int l = 0; l <= n_hidden; ++l) {
    const int din = width(n, l), dout = l < n_hidden ? hidden : n_out;
    const double sd = 1.0 / sqrt((double)din);
    for (int64_t i = 0; i < (int64_t)dout * din; ++i) {
      const double u1 = uni(), u2 = uni();
      h[n->w_off[l] + i] = (float)(sd * sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2));
    }
  }
  lw_status rc = LW_OK;
  auto alloc = [&](float** p, int64_t cnt) {
    if (rc == LW_OK && hipMalloc(p, (size_t)cnt * sizeof(float)) != hipSuccess) rc = LW_ENOMEM;
  };
  alloc(&n->p, off);
  alloc(&n->m, off);
  alloc(&n->v, off);
  alloc(&n->g, off);
  alloc(&n->hp, hidden + 1);
  alloc(&n->hm, hidden + 1);
  alloc(&n->hv, hidden + 1);
  alloc(&n->hg, hidden + 1);
  int64_t largest = 0;  // the largest layer's weights: the split partial products of its gradient
  for (int l = 0; l <= n_hidden; ++l) largest = std::max<int64_t>(largest, n->b_off[l] - n->w_off[l]);
  alloc(&n->splitk, (int64_t)lw::kMaxSplits * largest);
  if (rc == LW_OK && hipMalloc(&n->wbf, (size_t)off * sizeof(__bf16)) != hipSuccess) rc = LW_ENOMEM;
  if (rc == LW_OK) {
    std::vector<float> zeros(std::max<int64_t>(off, hidden + 1), 0.0f);
    (void)hipMemcpy(n->p, h.data(), off * sizeof(float), hipMemcpyHostToDevice);
    (void)hipMemcpy(n->m, zeros.data(), off * sizeof(float), hipMemcpyHostToDevice);
    (void)hipMemcpy(n->v, zeros.data(), off * sizeof(float), hipMemcpyHostToDevice);
    (void)hipMemcpy(n->hp, zeros.data(), (hidden + 1) * sizeof(float), hipMemcpyHostToDevice);
    (void)hipMemcpy(n->hm, zeros.data(), (hidden + 1) * sizeof(float), hipMemcpyHostToDevice);
    (void)hipMemcpy(n->hv, zeros.data(), (hidden + 1) * sizeof(float), hipMemcpyHostToDevice);
  }
  if (rc != LW_OK) {
    lw_mlp_destroy(n);
    c->err = "hipMalloc failed for the network";
    return rc;
  }
  *out = n;
  return LW_OK;
}

void lw_mlp_destroy(lw_mlp* n) {
  if (!n) return;
  if (n->c) (void)hipStreamSynchronize(n->c->stream);
  for (void* p : {(void*)n->p, (void*)n->m, (void*)n->v, (void*)n->g, (void*)n->hp, (void*)n->hm,
                  (void*)n->hv, (void*)n->hg, (void*)n->act, (void*)n->loss_part, (void*)n->err_buf,
                  (void*)n->col_part, (void*)n->splitk, (void*)n->wbf,
                  (void*)n->norm})
    if (p) (void)hipFree(p);
  delete n;
}

lw_status lw_mlp_num_params(const lw_mlp* n, int64_t* count) {
  if (!n || !count) return LW_EINVAL;
  *count = n->n_params;
  return LW_OK;
}

lw_status lw_mlp_get_params(lw_mlp* n, float* host, int64_t count, float* host_head) {
  if (!n || !host || count != n->n_params) return LW_EINVAL;
  MLP_HIP(hipStreamSynchronize(n->c->stream), "sync");
  MLP_HIP(hipMemcpy(host, n->p, count * sizeof(float), hipMemcpyDeviceToHost), "copy params");
  if (host_head) MLP_HIP(hipMemcpy(host_head, n->hp, (n->hidden + 1) * sizeof(float), hipMemcpyDeviceToHost), "copy head");
  return LW_OK;
}

lw_status lw_mlp_set_params(lw_mlp* n, const float* host, int64_t count, const float* host_head) {
  if (!n || !host || count != n->n_params) return LW_EINVAL;
  MLP_HIP(hipStreamSynchronize(n->c->stream), "sync");
  MLP_HIP(hipMemcpy(n->p, host, count * sizeof(float), hipMemcpyHostToDevice), "copy params");
  if (host_head) MLP_HIP(hipMemcpy(n->hp, host_head, (n->hidden + 1) * sizeof(float), hipMemcpyHostToDevice), "copy head");
  return LW_OK;
}

lw_status lw_mlp_save(lw_mlp* n, const char* path) {
  if (!n || !path) return LW_EINVAL;
  MLP_HIP(hipStreamSynchronize(n->c->stream), "sync");
  const int64_t np = n->n_params, nh = n->hidden + 1;
  std::vector<float> buf((size_t)std::max(np, nh));
  lw::Bytes b;
  const float* main_arrays[3] = {n->p, n->m, n->v};
  const float* head_arrays[3] = {n->hp, n->hm, n->hv};
  for (const float* a : main_arrays) {
    MLP_HIP(hipMemcpy(buf.data(), a, np * sizeof(float), hipMemcpyDeviceToHost), "copy network");
    b.put(buf.data(), np * sizeof(float));
  }
  for (const float* a : head_arrays) {
    MLP_HIP(hipMemcpy(buf.data(), a, nh * sizeof(float), hipMemcpyDeviceToHost), "copy error head");
    b.put(buf.data(), nh * sizeof(float));
  }
  b.put(&n->step, sizeof(int64_t));
  b.put(&n->head_step, sizeof(int64_t));
  const int64_t has_norm = n->norm ? 1 : 0;
  b.put(&has_norm, sizeof(has_norm));
  if (has_norm) {
    std::vector<float> nm(2 * (size_t)n->n_in);
    MLP_HIP(hipMemcpy(nm.data(), n->norm, nm.size() * sizeof(float), hipMemcpyDeviceToHost), "copy norm");
    b.put(nm.data(), nm.size() * sizeof(float));
  }
  const int64_t skip = n->skip_index;
  b.put(&skip, sizeof(skip));
  b.put(&n->skip_coeff, sizeof(float));
  const int64_t f[5] = {n->n_in, n->hidden, n->n_hidden, n->n_out, np};
  if (!lw::write_lw_file(path, "LWMLP001", f, b)) return mlp_fail(n, LW_EINVAL, std::string("cannot write ") + path);
  return LW_OK;
}

lw_status lw_mlp_load(lw_mlp* n, const char* path) {
  if (!n || !path) return LW_EINVAL;
  lw::FileHeader h;
  lw::Bytes b;
  std::string why;
  if (!lw::read_lw_file(path, "LWMLP001", &h, &b, &why)) return mlp_fail(n, LW_EINVAL, std::string(path) + ": " + why);
  const int64_t np = n->n_params, nh = n->hidden + 1;
  if (h.f[0] != n->n_in || h.f[1] != n->hidden || h.f[2] != n->n_hidden || h.f[3] != n->n_out || h.f[4] != np)
    return mlp_fail(n, LW_EINVAL, std::string(path) + ": network shape differs");
  std::vector<float> arr[6];
  for (int i = 0; i < 6; ++i) {
    arr[i].resize(i < 3 ? np : nh);
    if (!b.get(arr[i].data(), arr[i].size() * sizeof(float))) return mlp_fail(n, LW_EINVAL, std::string(path) + ": short payload");
  }
  int64_t step = 0, head_step = 0, has_norm = 0, skip = -1;
  float coeff = 0.0f;
  std::vector<float> nm;
  bool ok = b.get(&step, 8) && b.get(&head_step, 8) && b.get(&has_norm, 8);
  if (ok && has_norm) {
    nm.resize(2 * (size_t)n->n_in);
    ok = b.get(nm.data(), nm.size() * sizeof(float));
  }
  ok = ok && b.get(&skip, 8) && b.get(&coeff, sizeof(float)) && b.at == b.v.size();
  if (!ok || skip < -1 || skip >= n->n_in) return mlp_fail(n, LW_EINVAL, std::string(path) + ": malformed payload");
  MLP_HIP(hipStreamSynchronize(n->c->stream), "sync");
  float* main_arrays[3] = {n->p, n->m, n->v};
  float* head_arrays[3] = {n->hp, n->hm, n->hv};
  for (int i = 0; i < 3; ++i) {
    MLP_HIP(hipMemcpy(main_arrays[i], arr[i].data(), np * sizeof(float), hipMemcpyHostToDevice), "load network");
    MLP_HIP(hipMemcpy(head_arrays[i], arr[3 + i].data(), nh * sizeof(float), hipMemcpyHostToDevice), "load head");
  }
  n->step = step;
  n->head_step = head_step;
  lw_status st = has_norm ? lw_mlp_set_input_norm(n, nm.data(), nm.data() + n->n_in)
                          : lw_mlp_set_input_norm(n, nullptr, nullptr);
  if (st != LW_OK) return st;
  return lw_mlp_set_output_skip(n, (int32_t)skip, coeff);
}

lw_status lw_mlp_set_input_norm(lw_mlp* n, const float* shift, const float* scale) {
  if (!n || (!shift) != (!scale)) return LW_EINVAL;
  MLP_HIP(hipStreamSynchronize(n->c->stream), "sync");
  if (!shift) {
    if (n->norm) (void)hipFree(n->norm);
    n->norm = nullptr;
    return LW_OK;
  }
  if (!n->norm) MLP_HIP(hipMalloc(&n->norm, 2 * (size_t)n->n_in * sizeof(float)), "hipMalloc(norm)");
  MLP_HIP(hipMemcpy(n->norm, shift, n->n_in * sizeof(float), hipMemcpyHostToDevice), "copy shift");
  MLP_HIP(hipMemcpy(n->norm + n->n_in, scale, n->n_in * sizeof(float), hipMemcpyHostToDevice), "copy scale");
  return LW_OK;
}

lw_status lw_mlp_set_output_skip(lw_mlp* n, int32_t input_index, float coeff) {
  if (!n || input_index < -1 || input_index >= n->n_in) return LW_EINVAL;
  n->skip_index = input_index;
  n->skip_coeff = input_index >= 0 ? coeff : 0.0f;
  return LW_OK;
}

lw_status lw_mlp_forward(lw_mlp* n, const float* x, int64_t rows, float* y, float* err_head) {
  if (!n || !x || !y || rows < 0) return LW_EINVAL;
  if (err_head && n->n_hidden < 1) return mlp_fail(n, LW_EINVAL, "the error head needs a hidden layer");
  if (rows == 0) return LW_OK;
  if (fused_shape(n) && ((uintptr_t)x & 15) == 0 && ((uintptr_t)y & 15) == 0) {
    const int64_t np = n->n_params;
    hipLaunchKernelGGL(lw::lw_round_bf16_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, n->c->stream,
                       n->p, np, n->wbf);
    MLP_HIP(hipGetLastError(), "round weights");
    lw::FusedMlp f;
    f.x = x;
    f.norm = n->norm;
    f.p = n->p;
    f.w = n->wbf;
    for (int l = 0; l <= n->n_hidden; ++l) {
      f.w_off[l] = n->w_off[l];
      f.b_off[l] = n->b_off[l];
    }
    f.n_in = n->n_in;
    f.hidden = n->hidden;
    f.n_hidden = n->n_hidden;
    f.n_out = n->n_out;
    f.rows = rows;
    f.y = y;
    f.head = err_head ? n->hp : nullptr;
    f.e = err_head;
    f.skip_index = n->skip_index;
    f.skip_coeff = n->skip_coeff;
    hipLaunchKernelGGL(lw::lw_mlp_fused_forward_kernel, dim3((unsigned)((rows + lw::kFusedRows - 1) / lw::kFusedRows)),
                       dim3(lw::kFusedThreads), 0, n->c->stream, f);
    MLP_HIP(hipGetLastError(), "fused forward");
    return LW_OK;
  }
  lw_status st = ensure_rows(n, rows);
  const float* in = nullptr;
  if (st == LW_OK) st = input_of(n, x, rows, &in);
  if (st == LW_OK) st = forward(n, x, in, rows, y, false);
  if (st != LW_OK) return st;
  if (err_head) {
    hipLaunchKernelGGL(lw::lw_head_fwd_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0,
                       n->c->stream, h_of(n, n->n_hidden - 1, rows), rows, n->hidden, n->hp, err_head);
    MLP_HIP(hipGetLastError(), "head forward");
  }
  return LW_OK;
}

lw_status lw_mlp_loss_grad(lw_mlp* n, const float* x, const float* t, int64_t rows, float* grad_host,
                           double* loss) {
  if (!n || !x || !t || rows <= 0) return LW_EINVAL;
  lw_status st = ensure_rows(n, rows);
  const float* in = nullptr;
  if (st == LW_OK) st = input_of(n, x, rows, &in);
  if (st == LW_OK) st = forward(n, x, in, rows, y_of(n, rows));
  if (st == LW_OK) st = mse(n, y_of(n, rows), t, dy_of(n, rows), rows * n->n_out, loss);
  if (st == LW_OK) st = backward(n, in, rows);
  if (st == LW_OK && grad_host) {
    MLP_HIP(hipStreamSynchronize(n->c->stream), "sync");
    MLP_HIP(hipMemcpy(grad_host, n->g, n->n_params * sizeof(float), hipMemcpyDeviceToHost), "copy grad");
  }
  return st;
}

lw_status lw_mlp_train_step(lw_mlp* n, const float* x, const float* t, int64_t rows, float lr, float wd,
                            double* loss) {
  lw_status st = lw_mlp_loss_grad(n, x, t, rows, nullptr, loss);
  if (st != LW_OK) return st;
  n->step += 1;
  return adamw(n, n->p, n->m, n->v, n->g, n->n_params, n->step, lr, wd);
}

lw_status lw_mlp_train_head_step(lw_mlp* n, const float* x, const float* err_target, int64_t rows,
                                 float lr, double* loss) {
  if (!n || !x || !err_target || rows <= 0 || n->n_hidden < 1) return LW_EINVAL;
  lw_status st = ensure_rows(n, rows);
  const float* in = nullptr;
  if (st == LW_OK) st = input_of(n, x, rows, &in);
  if (st == LW_OK) st = forward(n, x, in, rows, y_of(n, rows), false);  // the head reads h only
  if (st != LW_OK) return st;
  hipStream_t s = n->c->stream;
  const float* hlast = h_of(n, n->n_hidden - 1, rows);
  hipLaunchKernelGGL(lw::lw_head_fwd_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s,
                     hlast, rows, n->hidden, n->hp, n->err_buf);
  MLP_HIP(hipGetLastError(), "head forward");
  if (loss) {
    st = mse(n, n->err_buf, err_target, dy_of(n, rows), rows, loss);
    if (st != LW_OK) return st;
  }
  // gradient of mean (e - t)^2: weights and bias as weighted column sums of [h | 1]
  st = colsum(n, hlast, rows, n->hidden, n->hidden + 1, n->err_buf, err_target, 2.0 / (double)rows, n->hg);
  if (st != LW_OK) return st;
  n->head_step += 1;
  return adamw(n, n->hp, n->hm, n->hv, n->hg, n->hidden + 1, n->head_step, lr, 0.0f);
}

lw_status lw_column_stats(lw_ctx* c, const float* x, int64_t rows, int32_t cols, int32_t groups,
                          const float* row_add, int64_t row_add_stride, double row_add_coeff, int32_t exp10,
                          const float* err, float threshold, double* out, void* ws, size_t ws_bytes) {
  if (!c || !x || !out || cols <= 0 || groups <= 0 || rows < 0) return LW_EINVAL;
  if (rows % groups != 0) {
    c->err = "column statistics: rows must be a multiple of groups";
    return LW_EINVAL;
  }
  if (groups > 65535) {
    c->err = "column statistics: at most 65535 groups";
    return LW_ERANGE;
  }
  const int64_t P = rows / groups;
  const int64_t slices = std::max<int64_t>(1, (P + lw::kStatSlice - 1) / lw::kStatSlice);
  if (slices > 65535) {
    c->err = "column statistics: at most 65535 x 256 particles per call";
    return LW_ERANGE;
  }
  const size_t need = (size_t)slices * groups * cols * 3 * sizeof(double);
  if (!ws || ws_bytes < need) {
    c->err = "workspace too small for the column statistics (" + std::to_string(need) + " bytes)";
    return LW_ENOMEM;
  }
  hipStream_t s = c->stream;
  hipLaunchKernelGGL(lw::lw_column_stats_stage1_kernel, dim3((unsigned)((cols + 63) / 64), (unsigned)slices,
                     (unsigned)groups), dim3(256), 0, s, x, P, cols, groups, row_add, row_add_stride,
                     row_add_coeff, exp10, err, threshold, (double*)ws);
  const int64_t n = (int64_t)groups * cols;
  hipLaunchKernelGGL(lw::lw_column_stats_stage2_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                     (const double*)ws, slices, groups, cols, out);
  if (hipGetLastError() != hipSuccess) {
    c->err = "launch column statistics";
    return LW_EDEVICE;
  }
  return LW_OK;
}

lw_status lw_error_share(lw_ctx* c, const float* pred, const float* y, int64_t rows, int32_t cols, int32_t groups,
                         const double* smean, int64_t smean_stride, double floor_value, float* share) {
  if (!c || !pred || !y || !smean || !share || rows < 0 || cols <= 0 || groups <= 0 || smean_stride <= 0 ||
      !(floor_value >= 0.0))
    return LW_EINVAL;
  if (rows == 0) return LW_OK;
  if (rows > 0x7FFFFFFFLL) {
    c->err = "error share: at most 2^31 - 1 rows per call";
    return LW_ERANGE;
  }
  hipLaunchKernelGGL(lw::lw_error_share_kernel, dim3((unsigned)rows), dim3(64), 0, c->stream, pred, y, rows, cols,
                     groups, smean, smean_stride, floor_value, share);
  if (hipGetLastError() != hipSuccess) {
    c->err = "launch error share";
    return LW_EDEVICE;
  }
  return LW_OK;
}

lw_status lw_quantile_of_maxima(lw_ctx* c, const float* v, int64_t n, int32_t groups, double q, double* host_out,
                                void* ws, size_t ws_bytes) {
  if (!c || !v || !host_out || n <= 0 || groups <= 0 || !(q >= 0.0 && q <= 1.0)) return LW_EINVAL;
  const size_t need = ((size_t)n * sizeof(uint32_t) + 255) / 256 * 256 + 256 * sizeof(unsigned) + 256;
  if (!ws || ws_bytes < need) {
    c->err = "workspace too small for the quantile (" + std::to_string(need) + " bytes)";
    return LW_ENOMEM;
  }
  uint32_t* keys = (uint32_t*)ws;
  unsigned* hist = (unsigned*)((char*)ws + ((size_t)n * sizeof(uint32_t) + 255) / 256 * 256);
  double* dval = (double*)(hist + 256);
  hipStream_t s = c->stream;
  hipLaunchKernelGGL(lw::lw_max_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, n, groups, keys);
  // the k-th smallest key by four byte-wise histogram passes
  auto select = [&](int64_t k, double* value) -> lw_status {
    uint32_t prefix = 0, mask = 0;
    for (int shift = 24; shift >= 0; shift -= 8) {
      if (lw::launch_fill_u32(hist, 256, 0u, s) != hipSuccess) {
        c->err = "quantile histogram clear";
        return LW_EDEVICE;
      }
      const unsigned blocks = (unsigned)std::min<int64_t>((n + 255) / 256, 1024);
      hipLaunchKernelGGL(lw::lw_radix_hist_kernel, dim3(blocks), dim3(256), 0, s, keys, n, prefix, mask, shift, hist);
      unsigned h[256];
      if (hipMemcpyAsync(h, hist, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess) {
        c->err = "quantile histogram";
        return LW_EDEVICE;
      }
      int b = 0;
      while (b < 255 && (int64_t)h[b] <= k) k -= h[b++];
      prefix |= (uint32_t)b << shift;
      mask |= 255u << shift;
    }
    // the selected key's value, converted on the device
    uint32_t* kd = (uint32_t*)(dval + 1);
    if (hipMemcpyAsync(kd, &prefix, sizeof(prefix), hipMemcpyHostToDevice, s) != hipSuccess) {
      c->err = "quantile key";
      return LW_EDEVICE;
    }
    hipLaunchKernelGGL(lw::lw_key_to_value_kernel, dim3(1), dim3(1), 0, s, kd, dval);
    if (hipMemcpyAsync(value, dval, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      c->err = "quantile value";
      return LW_EDEVICE;
    }
    return LW_OK;
  };
  // linear interpolation between the order statistics around q (n - 1)
  const double pos = q * (double)(n - 1);
  const int64_t lo = (int64_t)floor(pos), hi = std::min<int64_t>(lo + 1, n - 1);
  double a = 0.0, b = 0.0;
  lw_status st = select(lo, &a);
  if (st == LW_OK) st = hi == lo ? (b = a, LW_OK) : select(hi, &b);
  if (st != LW_OK) return st;
  const double t = pos - (double)lo;
  *host_out = t == 0.0 ? a : a + (b - a) * t;
  return LW_OK;
}

lw_status lw_log_ratio(lw_ctx* c, const double* num, int64_t num_stride, const double* den, int64_t den_stride,
                       int64_t n, float* out) {
  if (!c || !num || !den || !out || n < 0 || num_stride <= 0 || den_stride <= 0) return LW_EINVAL;
  if (n == 0) return LW_OK;
  hipLaunchKernelGGL(lw::lw_log_ratio_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, c->stream, num,
                     num_stride, den, den_stride, n, out);
  if (hipGetLastError() != hipSuccess) {
    c->err = "launch log ratio";
    return LW_EDEVICE;
  }
  return LW_OK;
}


}  // extern "C"
