/*
 * mlp_oracle.c -- FP64 reference of the spectrum surrogate network.
 *
 * TEST INFRASTRUCTURE: used by tests/ to check the GPU BF16 kernels' forward
 * pass and gradients.  Shares nothing with the HIP library.
 *
 * Network: x (n_in) -> [Linear, GELU] x n_hidden -> Linear -> y (n_out), all
 * hidden widths equal.  GELU(z) = z * Phi(z) with Phi the standard normal CDF
 * (erf form).  Loss = mean over rows and outputs of (y - t)^2.
 *
 * Flat parameter layout (the library uses the same order): for each layer l,
 * W_l [out_l][in_l] row-major, then b_l [out_l].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static double gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }

static double gelu_grad(double z) {
  const double cdf = 0.5 * (1.0 + erf(z / sqrt(2.0)));
  const double pdf = exp(-0.5 * z * z) / sqrt(2.0 * M_PI);
  return cdf + z * pdf;
}

int64_t mlpo_num_params(int32_t n_in, int32_t hidden, int32_t n_hidden, int32_t n_out) {
  int64_t n = 0, in = n_in;
  for (int32_t l = 0; l < n_hidden; ++l) {
    n += (int64_t)hidden * in + hidden;
    in = hidden;
  }
  n += (int64_t)n_out * in + n_out;
  return n;
}

/* GELU of a vector (exposed for tests). */
void mlpo_gelu(const double* z, double* out, int64_t n) {
  for (int64_t i = 0; i < n; ++i) out[i] = gelu(z[i]);
}

/*
 * Forward (and, when grad != NULL, backward) over `rows` samples.
 * x [rows][n_in], t [rows][n_out] (may be NULL without grad), y [rows][n_out].
 * grad [num_params] receives dLoss/dparams.  hid_out (may be NULL) receives the
 * last hidden activations [rows][hidden].  Returns the loss (0 if t is NULL).
 */
double mlpo_forward_backward(int32_t n_in, int32_t hidden, int32_t n_hidden, int32_t n_out,
                             const double* params, const double* x, const double* t, int64_t rows,
                             double* y, double* grad, double* hid_out) {
  const int32_t L = n_hidden + 1;
  /* activations: a[0] = x, z[l] pre-activation of layer l, a[l+1] = gelu(z[l]) */
  double** z = (double**)calloc(L, sizeof(double*));
  double** a = (double**)calloc(L + 1, sizeof(double*));
  int32_t* width = (int32_t*)calloc(L + 1, sizeof(int32_t));
  width[0] = n_in;
  for (int32_t l = 1; l <= n_hidden; ++l) width[l] = hidden;
  width[L] = n_out;
  a[0] = (double*)x;
  const double** W = (const double**)calloc(L, sizeof(double*));
  const double** b = (const double**)calloc(L, sizeof(double*));
  int64_t off = 0;
  for (int32_t l = 0; l < L; ++l) {
    W[l] = params + off;
    off += (int64_t)width[l + 1] * width[l];
    b[l] = params + off;
    off += width[l + 1];
  }
  for (int32_t l = 0; l < L; ++l) {
    const int32_t in = width[l], out = width[l + 1];
    z[l] = (double*)malloc(sizeof(double) * rows * out);
    for (int64_t r = 0; r < rows; ++r)
      for (int32_t o = 0; o < out; ++o) {
        double s = b[l][o];
        for (int32_t i = 0; i < in; ++i) s += W[l][(int64_t)o * in + i] * a[l][r * in + i];
        z[l][r * out + o] = s;
      }
    if (l < n_hidden) {
      a[l + 1] = (double*)malloc(sizeof(double) * rows * out);
      for (int64_t i = 0; i < rows * out; ++i) a[l + 1][i] = gelu(z[l][i]);
    } else {
      a[l + 1] = y;
      memcpy(y, z[l], sizeof(double) * rows * out);
    }
  }
  if (hid_out) memcpy(hid_out, a[n_hidden], sizeof(double) * rows * width[n_hidden]);
  double loss = 0.0;
  if (t) {
    for (int64_t i = 0; i < rows * n_out; ++i) loss += (y[i] - t[i]) * (y[i] - t[i]);
    loss /= (double)(rows * n_out);
  }
  if (grad && t) {
    memset(grad, 0, sizeof(double) * off);
    /* d = dLoss/dz of the current layer */
    double* d = (double*)malloc(sizeof(double) * rows * n_out);
    for (int64_t i = 0; i < rows * n_out; ++i) d[i] = 2.0 * (y[i] - t[i]) / (double)(rows * n_out);
    int64_t goff = off;
    for (int32_t l = L - 1; l >= 0; --l) {
      const int32_t in = width[l], out = width[l + 1];
      goff -= (int64_t)out * in + out;
      double* gW = grad + goff;
      double* gb = gW + (int64_t)out * in;
      for (int64_t r = 0; r < rows; ++r)
        for (int32_t o = 0; o < out; ++o) {
          const double dv = d[r * out + o];
          gb[o] += dv;
          for (int32_t i = 0; i < in; ++i) gW[(int64_t)o * in + i] += dv * a[l][r * in + i];
        }
      if (l > 0) {
        double* dn = (double*)malloc(sizeof(double) * rows * in);
        for (int64_t r = 0; r < rows; ++r)
          for (int32_t i = 0; i < in; ++i) {
            double s = 0.0;
            for (int32_t o = 0; o < out; ++o) s += d[r * out + o] * W[l][(int64_t)o * in + i];
            dn[r * in + i] = s * gelu_grad(z[l - 1][r * in + i]);
          }
        free(d);
        d = dn;
      }
    }
    free(d);
  }
  for (int32_t l = 0; l < L; ++l) {
    free(z[l]);
    if (l < n_hidden) free(a[l + 1]);
  }
  free(z);
  free(a);
  free(width);
  free(W);
  free(b);
  return loss;
}
