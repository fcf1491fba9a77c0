// filaments_gpu.hip -- device twin of filaments.c (workload generator, not the method),
// and the in-situ stand-in that advances the same particles window by window in a field
// of evolving amplitude.
//
// One thread per particle: the same Philox4x32-10 draws, beam initial conditions,
// random-filament field and Boris push as filaments.c, writing the same
// structure-of-arrays sample layout directly into device memory, so large
// ensembles never pass through the host.  Device libm (log, sin, cos, sqrt) may
// round differently from the host's, and the orbits are chaotic, so the two
// generators agree to rounding over short horizons, not bit for bit over long ones.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

extern "C" {
typedef struct {
  uint64_t seed;
  double dt, kT, delta, box, kmin, kmax;
  int32_t n_gamma;
  double gamma0[4];
  double frac_pos, frac_ion, ion_mass;
  int32_t len_min, len_max;
  int32_t two_d;
} wl_recipe_gpu;
}

namespace {

constexpr int kI = 16;  // field lattice |i|, |j| <= 16 (k0 = 0.5, kmax = 8)

__device__ __host__ inline void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ inline void draws(uint64_t seed, uint64_t id, uint32_t stream, uint32_t out[4]) {
  out[0] = (uint32_t)id;
  out[1] = (uint32_t)(id >> 32);
  out[2] = stream;
  out[3] = 0u;
  philox(out, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ inline double u01(uint32_t a, uint32_t b) {
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

__device__ void meta(const wl_recipe_gpu& r, uint64_t id, int32_t* len, int32_t* species,
                     double* g0, float* q, float* m) {
  uint32_t w[4], w2[4];
  draws(r.seed, id, 0u, w);
  const double us = u01(w[0], w[1]), ug = u01(w[2], w[3]);
  draws(r.seed, id, 4u, w2);
  const double ul = u01(w2[0], w2[1]);
  int32_t s = 0;
  if (us >= 1.0 - r.frac_ion)
    s = 2;
  else if (us >= 1.0 - r.frac_ion - r.frac_pos)
    s = 1;
  int32_t gi = (int32_t)(ug * r.n_gamma);
  if (gi >= r.n_gamma) gi = r.n_gamma - 1;
  const int32_t span = r.len_max - r.len_min + 1;
  int32_t L = r.len_min + (int32_t)(ul * span);
  if (L > r.len_max) L = r.len_max;
  *len = L;
  *species = s;
  *g0 = r.gamma0[gi];
  *q = s == 0 ? -1.0f : 1.0f;
  *m = s == 2 ? (float)r.ion_mass : 1.0f;
}

struct Field {
  double k0;
  const double* __restrict__ cre;  // [(kI+1)][(2 kI+1)], uniform across the wave
  const double* __restrict__ cim;
};

// B_y = Re sum_i X^i S_i,  S_i = sum_j C_ij Z^j,  X = e^{i k0 x}, Z = e^{i k0 z};
// j runs outermost so only the 17 partial sums S_i live in registers.
__device__ double field_by(const Field& f, double x, double z) {
  constexpr int W = 2 * kI + 1;
  const double cz = cos(f.k0 * z), sz = sin(f.k0 * z);
  // Z^{-kI} = conj(Z^kI)
  double pr = 1.0, pi = 0.0;
  for (int j = 0; j < kI; ++j) {
    const double t = pr * cz - pi * sz;
    pi = pr * sz + pi * cz;
    pr = t;
  }
  double zr = pr, zi = -pi;
  double sr[kI + 1], si[kI + 1];
#pragma unroll
  for (int i = 0; i <= kI; ++i) sr[i] = si[i] = 0.0;
  for (int j = 0; j < W; ++j) {
#pragma unroll
    for (int i = 0; i <= kI; ++i) {
      const double cr = f.cre[i * W + j], ci = f.cim[i * W + j];
      sr[i] += cr * zr - ci * zi;
      si[i] += cr * zi + ci * zr;
    }
    const double t = zr * cz - zi * sz;
    zi = zr * sz + zi * cz;
    zr = t;
  }
  const double cx = cos(f.k0 * x), sx = sin(f.k0 * x);
  double xr = 1.0, xi = 0.0, by = 0.0;
#pragma unroll
  for (int i = 0; i <= kI; ++i) {
    by += xr * sr[i] - xi * si[i];
    const double t = xr * cx - xi * sx;
    xi = xr * sx + xi * cx;
    xr = t;
  }
  return by;
}

// Initial position and momentum of particle `id` (beam of its species, thermal spread).
__device__ void initial_state(const wl_recipe_gpu& r, uint64_t id, double g0, float m, double* pos,
                              double* u) {
  uint32_t w[4];
  draws(r.seed, id, 1u, w);
  double px = r.box * u01(w[0], w[1]);
  double pz = r.box * u01(w[2], w[3]);
  draws(r.seed, id, 5u, w);
  double py = r.two_d ? 0.0 : r.box * u01(w[0], w[1]);
  double nrm[4];
  for (int h = 0; h < 2; ++h) {
    draws(r.seed, id, 2u + h, w);
    const double u1 = u01(w[0], w[1]), u2 = u01(w[2], w[3]);
    const double rr = sqrt(-2.0 * log(1.0 - u1));
    nrm[2 * h] = rr * cos(2.0 * M_PI * u2);
    nrm[2 * h + 1] = rr * sin(2.0 * M_PI * u2);
  }
  const double sig = sqrt(r.kT / (double)m);
  const double upx = sig * nrm[0], upy = r.two_d ? 0.0 : sig * nrm[1], upz = sig * nrm[2];
  const double gp = sqrt(1.0 + upx * upx + upy * upy + upz * upz);
  const double sgn = (id & 1u) ? -1.0 : 1.0;
  const double b0 = sgn * sqrt(1.0 - 1.0 / (g0 * g0));
  pos[0] = px;
  pos[1] = py;
  pos[2] = pz;
  u[0] = g0 * (upx + b0 * gp);
  u[1] = upy;
  u[2] = upz;
}

// One Boris step of length dt in B = (0, Bf(pos), 0) scaled by amp, writing the sample
// (position before the step, mean velocity, velocity change over dt) at idx.
__device__ inline void boris_sample(const Field& f, double amp, double qm, double dt, double* pos,
                                    double* u, int64_t idx, double* x, double* y, double* z,
                                    double* bx, double* by, double* bz, float* ax, float* ay,
                                    float* az) {
  const double px = pos[0], py = pos[1], pz = pos[2];
  const double ux = u[0], uy = u[1], uz = u[2];
  {
    const double gm = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
    const double Bf = amp * field_by(f, px, pz);
    const double ty = qm * Bf * dt / (2.0 * gm);
    const double sy = 2.0 * ty / (1.0 + ty * ty);
    const double vx = ux - uz * ty, vz = uz + ux * ty;
    const double nx = ux - vz * sy, nz = uz + vx * sy, ny = uy;
    const double gpl = sqrt(1.0 + nx * nx + ny * ny + nz * nz);
    const double bmx = ux / gm, bmy = uy / gm, bmz = uz / gm;
    const double bpx = nx / gpl, bpy = ny / gpl, bpz = nz / gpl;
    x[idx] = px;
    y[idx] = py;
    z[idx] = pz;
    bx[idx] = 0.5 * (bmx + bpx);
    by[idx] = 0.5 * (bmy + bpy);
    bz[idx] = 0.5 * (bmz + bpz);
    ax[idx] = (float)((bpx - bmx) / dt);
    ay[idx] = (float)((bpy - bmy) / dt);
    az[idx] = (float)((bpz - bmz) / dt);
    pos[0] = px + bpx * dt;
    pos[1] = py + bpy * dt;
    pos[2] = pz + bpz * dt;
    u[0] = nx;
    u[1] = ny;
    u[2] = nz;
  }
}

__global__ void wl_generate_kernel(wl_recipe_gpu r, int64_t first_id, int64_t n,
                                   const int64_t* offsets, Field f, double* x, double* y, double* z,
                                   double* bx, double* by, double* bz, float* ax, float* ay,
                                   float* az, double* t0, double* dtp, float* charge, float* weight,
                                   int32_t* species, int* status) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t id = (uint64_t)(first_id + i);
  int32_t len, s;
  double g0;
  float q, m;
  meta(r, id, &len, &s, &g0, &q, &m);
  const int64_t o = offsets[i] - offsets[0];
  const int64_t L = offsets[i + 1] - offsets[i];
  if (L != len) {
    atomicExch(status, -1);
    return;
  }
  double pos[3], u[3];
  initial_state(r, id, g0, m, pos, u);
  const double qm = (double)q / (double)m;
  const double dt = r.dt;
  for (int64_t k = 0; k < L; ++k)
    boris_sample(f, 1.0, qm, dt, pos, u, o + k, x, y, z, bx, by, bz, ax, ay, az);
  t0[i] = 0.0;
  dtp[i] = dt;
  charge[i] = q;
  weight[i] = 1.0f;
  species[i] = s;
}

// ---- in-situ stand-in: persistent particles in a field whose amplitude evolves in time
// State [6][n]: x, y, z, ux, uy, uz (FP64), advanced window by window.
__global__ void wl_insitu_init_kernel(wl_recipe_gpu r, int64_t first_id, int64_t n, double* state,
                                      float* charge, float* mass) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t id = (uint64_t)(first_id + i);
  int32_t len, s;
  double g0;
  float q, m;
  meta(r, id, &len, &s, &g0, &q, &m);
  double pos[3], u[3];
  initial_state(r, id, g0, m, pos, u);
  for (int c = 0; c < 3; ++c) {
    state[c * n + i] = pos[c];
    state[(3 + c) * n + i] = u[c];
  }
  charge[i] = q;
  mass[i] = m;
}

// One window: n_steps simulation steps, each sub-cycled n_sub times with synthesis step dt.
// The field amplitude is given at the n_steps + 1 simulation step boundaries and
// interpolated linearly inside a step (as a PIC code's particle sub-cycling interpolates
// its fields in time).  Writes n_steps * n_sub samples per particle, particle-major, and
// per particle t0 = t_start, dt, charge, weight 1 and the collection region: the z-slab
// (of n_regions equal slabs of the periodic box, across the beams) holding the particle at
// the window start.
__global__ void wl_insitu_push_kernel(Field f, int64_t n, double* state, const float* charge_in,
                                      const float* mass, const double* amp, int32_t n_steps,
                                      int32_t n_sub, double dt, double t_start, double box,
                                      int32_t n_regions, double* x, double* y, double* z,
                                      double* bx, double* by, double* bz, float* ax, float* ay,
                                      float* az, double* t0, double* dtp, float* charge,
                                      float* weight, int32_t* species) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double pos[3], u[3];
  for (int c = 0; c < 3; ++c) {
    pos[c] = state[c * n + i];
    u[c] = state[(3 + c) * n + i];
  }
  const double zm = pos[2] - box * floor(pos[2] / box);
  const int reg = min(n_regions - 1, max(0, (int)(zm / box * n_regions)));
  const double qm = (double)charge_in[i] / (double)mass[i];
  const int64_t L = (int64_t)n_steps * n_sub;
  for (int32_t st = 0; st < n_steps; ++st) {
    const double a0 = amp[st], da = amp[st + 1] - amp[st];
    for (int32_t k = 0; k < n_sub; ++k)
      boris_sample(f, a0 + da * ((double)k / (double)n_sub), qm, dt, pos, u,
                   i * L + (int64_t)st * n_sub + k, x, y, z, bx, by, bz, ax, ay, az);
  }
  for (int c = 0; c < 3; ++c) {
    state[c * n + i] = pos[c];
    state[(3 + c) * n + i] = u[c];
  }
  t0[i] = t_start;
  dtp[i] = dt;
  charge[i] = charge_in[i];
  weight[i] = 1.0f;
  species[i] = reg;
}

}  // namespace

extern "C" {

// Generate particles first_id .. first_id+n-1 into device arrays laid out by the device
// offsets (offsets[i+1]-offsets[i] must equal each particle's length).  cre/cim: device
// field coefficients [(imax+1)][(2 imax+1)] from wl_field_coeffs.  status: device int,
// set to -1 on a length mismatch.  Asynchronous on `stream`.
int wl_generate_gpu(const wl_recipe_gpu* r, int64_t first_id, int64_t n, const int64_t* offsets,
                    int32_t imax, double k0, const double* cre, const double* cim, double* x,
                    double* y, double* z, double* bx, double* by, double* bz, float* ax, float* ay,
                    float* az, double* t0, double* dtp, float* charge, float* weight,
                    int32_t* species, int* status, void* stream) {
  if (!r || n < 0 || imax != kI) return -1;
  if (n == 0) return 0;
  Field f{k0, cre, cim};
  dim3 grid((unsigned)((n + 63) / 64)), block(64);
  hipLaunchKernelGGL(wl_generate_kernel, grid, block, 0, (hipStream_t)stream, *r, first_id, n,
                     offsets, f, x, y, z, bx, by, bz, ax, ay, az, t0, dtp, charge, weight, species,
                     status);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// In-situ stand-in, initial state of particles first_id .. first_id+n-1: state [6][n]
// device FP64 (positions, momenta), charge and mass [n] device FP32.
int wl_insitu_init_gpu(const wl_recipe_gpu* r, int64_t first_id, int64_t n, double* state,
                       float* charge, float* mass, void* stream) {
  if (!r || n < 0) return -1;
  if (n == 0) return 0;
  dim3 grid((unsigned)((n + 63) / 64)), block(64);
  hipLaunchKernelGGL(wl_insitu_init_kernel, grid, block, 0, (hipStream_t)stream, *r, first_id, n,
                     state, charge, mass);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Advance the state by one window (see wl_insitu_push_kernel) and write its samples into
// device arrays of n * n_steps * n_sub samples; amp: device [n_steps + 1].
int wl_insitu_push_gpu(int32_t imax, double k0, const double* cre, const double* cim, int64_t n,
                       double* state, const float* charge_in, const float* mass, const double* amp,
                       int32_t n_steps, int32_t n_sub, double dt, double t_start, double box,
                       int32_t n_regions, double* x, double* y, double* z, double* bx, double* by,
                       double* bz, float* ax, float* ay, float* az, double* t0, double* dtp,
                       float* charge, float* weight, int32_t* species, void* stream) {
  if (imax != kI || n < 0 || n_steps < 1 || n_sub < 1 || n_regions < 1 || !(dt > 0.0) ||
      !(box > 0.0))
    return -1;
  if (n == 0) return 0;
  Field f{k0, cre, cim};
  dim3 grid((unsigned)((n + 63) / 64)), block(64);
  hipLaunchKernelGGL(wl_insitu_push_kernel, grid, block, 0, (hipStream_t)stream, f, n, state,
                     charge_in, mass, amp, n_steps, n_sub, dt, t_start, box, n_regions, x, y, z, bx,
                     by, bz, ax, ay, az, t0, dtp, charge, weight, species);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"
