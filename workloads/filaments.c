/*
 * filaments.c -- seeded synthetic particle trajectories (workload generator).
 *
 * Holds no part of the radiation computation: it only produces the sampled
 * trajectories (r_k, beta_k, betadot_k) that both the HIP library and the
 * CPU oracle consume.  It stands in for the PIC particle data of the paper
 * (Section 2.1), which is not available: beams of electrons (optionally
 * positrons and ions) counter-streaming along +-x through a static transverse
 * magnetic field B_y(x, z) made of random Fourier filaments, in the same
 * spirit as the paper's "frozen field" radiation runs (Section 2.1).
 *
 * Units are the paper's PIC units (c = m_e = q_e = 1; t in 1/omega_p,
 * lengths in c/omega_p).
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random
 * numbers: as easy as 1, 2, 3", SC'11), keyed by the workload seed, with the
 * particle index in the counter, so any particle can be regenerated alone.
 *
 * Field: B_y(x,z) = sum_k a_k cos(k_x x + k_z z + phi_k) over every lattice
 * vector k = (2 pi / L)(i, j) of a half plane with k_min <= |k| <= k_max;
 * a_k ~ 1/|k| (power per mode ~ k^-2), phi_k uniform.  The amplitude is set by
 * the jitter deflection parameter delta = |q| B_rms / (m c kbar) for electrons,
 * kbar = sum a_k^2 |k| / sum a_k^2, B_rms^2 = sum a_k^2 / 2.
 *
 * Push: Boris rotation in the static magnetic field (no electric field).
 * Samples: r_k = x^k, beta_k = (beta^{k-1/2} + beta^{k+1/2}) / 2,
 * betadot_k = (beta^{k+1/2} - beta^{k-1/2}) / dt, so straight motion gives
 * betadot == 0 exactly.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------- Philox4x32-10 ---------------- */
static void philox_round(uint32_t c[4], const uint32_t k[2]) {
  uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c[0];
  uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c[2];
  uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  uint32_t n0 = hi1 ^ c[1] ^ k[0];
  uint32_t n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

void wl_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
  uint32_t k[2] = {key_in[0], key_in[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += 0x9E3779B9u;
      k[1] += 0xBB67AE85u;
    }
    philox_round(c, k);
  }
  memcpy(out, c, sizeof(c));
}

/* Four draws for (particle id, stream). */
static void draws(uint64_t seed, uint64_t id, uint32_t stream, uint32_t out[4]) {
  uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), stream, 0u};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  wl_philox4x32_10(ctr, key, out);
}

/* 53-bit uniform in [0, 1) from two 32-bit words. */
static double u01(uint32_t a, uint32_t b) {
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

/* Two standard normals (Box-Muller) from four words. */
static void normals2(const uint32_t w[4], double out[2]) {
  double u1 = u01(w[0], w[1]);
  double u2 = u01(w[2], w[3]);
  double r = sqrt(-2.0 * log(1.0 - u1));
  out[0] = r * cos(2.0 * M_PI * u2);
  out[1] = r * sin(2.0 * M_PI * u2);
}

/* ---------------- workload recipe ---------------- */
typedef struct {
  uint64_t seed;
  double dt;          /* sample spacing */
  double kT;          /* beam rest-frame temperature, units of m_e c^2 */
  double delta;       /* jitter deflection parameter for electrons */
  double box;         /* field period L in x and z */
  double kmin, kmax;  /* field wavenumber range */
  int32_t n_gamma;    /* number of bulk-Lorentz-factor populations (equal parts) */
  double gamma0[4];
  double frac_pos;    /* fraction of positrons */
  double frac_ion;    /* fraction of ions (charge +1) */
  double ion_mass;    /* ion mass in m_e */
  int32_t len_min, len_max; /* trajectory length, uniform integers in [min, max] */
  int32_t two_d;      /* 2D2V: motion in the x-z plane (y = 0, no y momentum) */
} wl_recipe;

#define WL_SPECIES_ELECTRON 0
#define WL_SPECIES_POSITRON 1
#define WL_SPECIES_ION 2

/* Per-particle choices that fix the batch layout. */
void wl_particle_meta(const wl_recipe* r, int64_t first_id, int64_t n, int32_t* len,
                      int32_t* species, double* gamma0, float* charge, float* mass) {
  for (int64_t i = 0; i < n; ++i) {
    uint64_t id = (uint64_t)(first_id + i);
    uint32_t w[4];
    draws(r->seed, id, 0u, w);
    double us = u01(w[0], w[1]);
    double ug = u01(w[2], w[3]);
    uint32_t w2[4];
    draws(r->seed, id, 4u, w2);
    double ul = u01(w2[0], w2[1]);
    int32_t s = WL_SPECIES_ELECTRON;
    if (us >= 1.0 - r->frac_ion)
      s = WL_SPECIES_ION;
    else if (us >= 1.0 - r->frac_ion - r->frac_pos)
      s = WL_SPECIES_POSITRON;
    int32_t gi = (int32_t)(ug * r->n_gamma);
    if (gi >= r->n_gamma) gi = r->n_gamma - 1;
    int32_t span = r->len_max - r->len_min + 1;
    int32_t L = r->len_min + (int32_t)(ul * span);
    if (L > r->len_max) L = r->len_max;
    if (len) len[i] = L;
    if (species) species[i] = s;
    if (gamma0) gamma0[i] = r->gamma0[gi];
    if (charge) charge[i] = (s == WL_SPECIES_ELECTRON) ? -1.0f : 1.0f;
    if (mass) mass[i] = (s == WL_SPECIES_ION) ? (float)r->ion_mass : 1.0f;
  }
}

/* ---------------- field ---------------- */
typedef struct {
  int32_t imax;      /* |i|, |j| <= imax */
  double k0;         /* 2 pi / L */
  double* cre;       /* [(imax+1)][(2 imax+1)] complex coefficients a e^{i phi} */
  double* cim;
  int32_t n_modes;
  double brms, kbar;
} wl_field;

static int field_build(const wl_recipe* r, wl_field* f) {
  f->k0 = 2.0 * M_PI / r->box;
  f->imax = (int32_t)floor(r->kmax / f->k0 + 1e-9);
  int32_t W = 2 * f->imax + 1;
  size_t cells = (size_t)(f->imax + 1) * (size_t)W;
  f->cre = (double*)calloc(cells, sizeof(double));
  f->cim = (double*)calloc(cells, sizeof(double));
  if (!f->cre || !f->cim) return -1;
  double sum_a2 = 0.0, sum_a2k = 0.0;
  f->n_modes = 0;
  for (int32_t i = 0; i <= f->imax; ++i) {
    for (int32_t j = -f->imax; j <= f->imax; ++j) {
      if (i == 0 && j <= 0) continue; /* half plane */
      double kk = f->k0 * sqrt((double)(i * i + j * j));
      if (kk < r->kmin * (1 - 1e-12) || kk > r->kmax * (1 + 1e-12)) continue;
      uint32_t w[4];
      uint64_t mode_id = ((uint64_t)(uint32_t)i << 16) | (uint64_t)(uint32_t)(j + 4096);
      draws(r->seed, mode_id, 7u, w);
      double phi = 2.0 * M_PI * u01(w[0], w[1]);
      double a = 1.0 / kk;
      f->cre[(size_t)i * W + (j + f->imax)] = a * cos(phi);
      f->cim[(size_t)i * W + (j + f->imax)] = a * sin(phi);
      sum_a2 += a * a;
      sum_a2k += a * a * kk;
      f->n_modes++;
    }
  }
  double kbar = sum_a2k / sum_a2;
  double brms_unit = sqrt(0.5 * sum_a2);
  double scale = r->delta * kbar / brms_unit; /* electrons: |q| = m = 1 */
  for (size_t c = 0; c < cells; ++c) {
    f->cre[c] *= scale;
    f->cim[c] *= scale;
  }
  f->brms = brms_unit * scale;
  f->kbar = kbar;
  return 0;
}

static void field_free(wl_field* f) {
  free(f->cre);
  free(f->cim);
}

/* B_y at (x, z): Re sum_i X^i sum_j C_ij Z^j with X = e^{i k0 x}, Z = e^{i k0 z}. */
static double field_by(const wl_field* f, double x, double z, double* xr, double* xi, double* zr,
                       double* zi) {
  int32_t M = f->imax, W = 2 * M + 1;
  double cx = cos(f->k0 * x), sx = sin(f->k0 * x);
  double cz = cos(f->k0 * z), sz = sin(f->k0 * z);
  xr[0] = 1.0;
  xi[0] = 0.0;
  for (int32_t i = 1; i <= M; ++i) {
    xr[i] = xr[i - 1] * cx - xi[i - 1] * sx;
    xi[i] = xr[i - 1] * sx + xi[i - 1] * cx;
  }
  zr[M] = 1.0;
  zi[M] = 0.0;
  for (int32_t j = 1; j <= M; ++j) {
    zr[M + j] = zr[M + j - 1] * cz - zi[M + j - 1] * sz;
    zi[M + j] = zr[M + j - 1] * sz + zi[M + j - 1] * cz;
    zr[M - j] = zr[M + j];
    zi[M - j] = -zi[M + j];
  }
  double by = 0.0;
  for (int32_t i = 0; i <= M; ++i) {
    const double* cr = f->cre + (size_t)i * W;
    const double* ci = f->cim + (size_t)i * W;
    double sr = 0.0, si = 0.0;
    for (int32_t j = 0; j < W; ++j) {
      sr += cr[j] * zr[j] - ci[j] * zi[j];
      si += cr[j] * zi[j] + ci[j] * zr[j];
    }
    by += xr[i] * sr - xi[i] * si;
  }
  return by;
}

/* Field diagnostics: number of modes, B_rms and kbar. */
int wl_field_info(const wl_recipe* r, int32_t* n_modes, double* brms, double* kbar) {
  wl_field f;
  if (field_build(r, &f) != 0) return -2;
  *n_modes = f.n_modes;
  *brms = f.brms;
  *kbar = f.kbar;
  field_free(&f);
  return 0;
}

/* Field coefficients C_ij = a e^{i phi} on the [(imax+1)][(2 imax+1)] lattice table
 * (for the device generator).  Returns imax, or a negative value if cap is too small. */
int wl_field_coeffs(const wl_recipe* r, double* cre, double* cim, int64_t cap, double* k0) {
  wl_field f;
  if (field_build(r, &f) != 0) return -2;
  int64_t cells = (int64_t)(f.imax + 1) * (2 * f.imax + 1);
  int imax = f.imax;
  if (cells > cap) {
    field_free(&f);
    return -1;
  }
  memcpy(cre, f.cre, sizeof(double) * (size_t)cells);
  memcpy(cim, f.cim, sizeof(double) * (size_t)cells);
  *k0 = f.k0;
  field_free(&f);
  return imax;
}

/* B_y sampled at given points (for tests of the field statistics). */
int wl_field_eval(const wl_recipe* r, int64_t n, const double* x, const double* z, double* by) {
  wl_field f;
  if (field_build(r, &f) != 0) return -2;
  int32_t M = f.imax;
  double* buf = (double*)malloc(sizeof(double) * (size_t)(6 * M + 6));
  for (int64_t i = 0; i < n; ++i)
    by[i] = field_by(&f, x[i], z[i], buf, buf + (M + 1), buf + 2 * (M + 1),
                     buf + 2 * (M + 1) + (2 * M + 1));
  free(buf);
  field_free(&f);
  return 0;
}

/*
 * Generate particles first_id .. first_id+n-1 into SoA arrays.  offsets[0..n]
 * must already hold the sample layout (offsets[i+1]-offsets[i] = length of
 * particle i, normally from wl_particle_meta).  Outputs are written at
 * offsets[i] - offsets[0].
 */
int wl_generate(const wl_recipe* r, int64_t first_id, int64_t n, const int64_t* offsets,
                double* x, double* y, double* z, double* bx, double* by, double* bz,
                float* ax, float* ay, float* az, double* t0, double* dtp, float* charge,
                float* weight, int32_t* species, int nthreads) {
  wl_field f;
  if (field_build(r, &f) != 0) return -2;
  int32_t M = f.imax;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
  int status = 0;
#pragma omp parallel
  {
    double* buf = (double*)malloc(sizeof(double) * (size_t)(6 * M + 6));
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < n; ++i) {
      uint64_t id = (uint64_t)(first_id + i);
      int32_t len, s;
      double g0;
      float q, m;
      wl_particle_meta(r, first_id + i, 1, &len, &s, &g0, &q, &m);
      int64_t o = offsets[i] - offsets[0];
      int64_t L = offsets[i + 1] - offsets[i];
      if (L != len) {
#pragma omp critical
        status = -1;
        continue;
      }
      uint32_t w[4];
      draws(r->seed, id, 1u, w);
      double px = r->box * u01(w[0], w[1]);
      double pz = r->box * u01(w[2], w[3]);
      draws(r->seed, id, 5u, w);
      double py = r->two_d ? 0.0 : r->box * u01(w[0], w[1]);
      /* rest-frame thermal four-velocity, then boost along +-x */
      double nrm[4];
      draws(r->seed, id, 2u, w);
      normals2(w, nrm);
      draws(r->seed, id, 3u, w);
      normals2(w, nrm + 2);
      double sig = sqrt(r->kT / (double)m);
      double upx = sig * nrm[0], upy = r->two_d ? 0.0 : sig * nrm[1], upz = sig * nrm[2];
      double gp = sqrt(1.0 + upx * upx + upy * upy + upz * upz);
      double sgn = (id & 1u) ? -1.0 : 1.0;
      double b0 = sgn * sqrt(1.0 - 1.0 / (g0 * g0));
      double ux = g0 * (upx + b0 * gp);
      double uy = upy, uz = upz;
      double qm = (double)q / (double)m;
      double dt = r->dt;
      for (int64_t k = 0; k < L; ++k) {
        double gm = sqrt(1.0 + ux * ux + uy * uy + uz * uz);
        double Bf = field_by(&f, px, pz, buf, buf + (M + 1), buf + 2 * (M + 1),
                             buf + 2 * (M + 1) + (2 * M + 1));
        double ty = qm * Bf * dt / (2.0 * gm);
        double sy = 2.0 * ty / (1.0 + ty * ty);
        /* u' = u + u x t, t = (0, ty, 0) */
        double vx = ux - uz * ty, vz = uz + ux * ty;
        /* u+ = u + u' x s */
        double nx = ux - vz * sy, nz = uz + vx * sy, ny = uy;
        double gpl = sqrt(1.0 + nx * nx + ny * ny + nz * nz);
        double bmx = ux / gm, bmy = uy / gm, bmz = uz / gm;
        double bpx = nx / gpl, bpy = ny / gpl, bpz = nz / gpl;
        x[o + k] = px;
        y[o + k] = py;
        z[o + k] = pz;
        bx[o + k] = 0.5 * (bmx + bpx);
        by[o + k] = 0.5 * (bmy + bpy);
        bz[o + k] = 0.5 * (bmz + bpz);
        ax[o + k] = (float)((bpx - bmx) / dt);
        ay[o + k] = (float)((bpy - bmy) / dt);
        az[o + k] = (float)((bpz - bmz) / dt);
        px += bpx * dt;
        py += bpy * dt;
        pz += bpz * dt;
        ux = nx;
        uy = ny;
        uz = nz;
      }
      t0[i] = 0.0;
      dtp[i] = dt;
      charge[i] = q;
      weight[i] = 1.0f;
      species[i] = s;
    }
    free(buf);
  }
  field_free(&f);
  return status;
}
