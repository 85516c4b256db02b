/*
 * mlp.c - FP64 reference of the Fourier-feature MLP used as a learned control
 * variate (TEST INFRASTRUCTURE ONLY; no code shared with the HIP library).
 *
 * Network (the control-variate function is not in the paper):
 *   z0 = [sin(2 pi B y), cos(2 pi B y)]            (2 K features, B is K x dim)
 *   h_l = silu(W_l h_{l-1} + b_l),  l = 1..L        (hidden width H)
 *   f   = W_{L+1} h_L + b_{L+1}                     (scalar)
 * silu(s) = s / (1 + exp(-s)).  Parameters are one flat array in the order
 * W_1, b_1, ..., W_{L+1}, b_{L+1}, each W row-major [out][in].
 *
 * With bf16 != 0 the values that a bfloat16 matrix unit would consume are
 * rounded to bfloat16 (round to nearest even, via binary32) at the same points
 * as the GPU kernels: the features, every hidden activation, every weight
 * matrix, and in the backward pass every pre-activation gradient that feeds a
 * matrix product.  Biases, accumulations and everything else stay in binary64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MLP_PI 3.14159265358979323846

static double to_bf16(double x) {
  float f = (float)x; /* binary64 -> binary32, round to nearest even */
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf / nan unchanged */
  uint32_t lsb = (u >> 16) & 1u;
  u = (u + 0x7fffu + lsb) & 0xffff0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

double orc_bf16_round(double x) { return to_bf16(x); }

int64_t orc_mlp_n_params(int n_freq, int hidden, int layers) {
  int64_t n = (int64_t)hidden * (2 * n_freq) + hidden;
  n += (int64_t)(layers - 1) * ((int64_t)hidden * hidden + hidden);
  n += hidden + 1;
  return n;
}

static double silu(double s) { return s / (1.0 + exp(-s)); }
static double silu_grad(double s) {
  double sg = 1.0 / (1.0 + exp(-s));
  return sg * (1.0 + s * (1.0 - sg));
}

typedef struct {
  int K, H, L, dim;
} shape;

/* forward for one input; keeps pre-activations s[l][*] and inputs a[l][*] */
static double forward_one(const double* P, const double* B, shape sh, const double* y, int bf16,
                          double* a /* (L+1) x max(2K, H) */, double* s /* L x H */) {
  const int K = sh.K, H = sh.H, L = sh.L, W0 = 2 * K;
  const int stride = W0 > H ? W0 : H;
  for (int k = 0; k < K; ++k) {
    double arg = 0.0;
    for (int d = 0; d < sh.dim; ++d) arg += B[k * sh.dim + d] * y[d];
    double sv = sin(2.0 * MLP_PI * arg), cv = cos(2.0 * MLP_PI * arg);
    a[k] = bf16 ? to_bf16(sv) : sv;
    a[K + k] = bf16 ? to_bf16(cv) : cv;
  }
  const double* p = P;
  int in = W0;
  for (int l = 0; l < L; ++l) {
    const double* W = p;
    const double* b = p + (int64_t)H * in;
    for (int o = 0; o < H; ++o) {
      double acc = 0.0;
      for (int i = 0; i < in; ++i) acc += (bf16 ? to_bf16(W[o * in + i]) : W[o * in + i]) * a[l * stride + i];
      acc += b[o];
      s[l * H + o] = acc;
      double h = silu(acc);
      a[(l + 1) * stride + o] = bf16 ? to_bf16(h) : h;
    }
    p = b + H;
    in = H;
  }
  double f = p[H];
  for (int i = 0; i < H; ++i) f += (bf16 ? to_bf16(p[i]) : p[i]) * a[L * stride + i];
  return f;
}

void orc_mlp_forward(const double* params, const double* Bmat, int n_freq, int hidden, int layers,
                     int dim, int64_t n, const double* y, int bf16, double* out) {
  shape sh = {n_freq, hidden, layers, dim};
  const int stride = 2 * n_freq > hidden ? 2 * n_freq : hidden;
  double* a = (double*)malloc(sizeof(double) * (size_t)(layers + 1) * stride);
  double* s = (double*)malloc(sizeof(double) * (size_t)layers * hidden);
  for (int64_t r = 0; r < n; ++r) out[r] = forward_one(params, Bmat, sh, y + r * dim, bf16, a, s);
  free(a);
  free(s);
}

/* Mean squared error over the batch and its gradient w.r.t. every parameter. */
double orc_mlp_loss_grad(const double* params, const double* Bmat, int n_freq, int hidden,
                         int layers, int dim, int64_t n, const double* y, const double* target,
                         int bf16, double* grad) {
  shape sh = {n_freq, hidden, layers, dim};
  const int K = n_freq, H = hidden, L = layers, W0 = 2 * K;
  const int stride = W0 > H ? W0 : H;
  const int64_t np = orc_mlp_n_params(K, H, L);
  memset(grad, 0, sizeof(double) * (size_t)np);
  double* a = (double*)malloc(sizeof(double) * (size_t)(L + 1) * stride);
  double* s = (double*)malloc(sizeof(double) * (size_t)L * H);
  double* da = (double*)malloc(sizeof(double) * (size_t)stride);
  double* ds = (double*)malloc(sizeof(double) * (size_t)H);
  /* offsets of each layer's W and b */
  int64_t* offW = (int64_t*)malloc(sizeof(int64_t) * (size_t)(L + 1));
  int64_t* offb = (int64_t*)malloc(sizeof(int64_t) * (size_t)(L + 1));
  int64_t o = 0;
  for (int l = 0; l <= L; ++l) {
    const int in = l == 0 ? W0 : H, out = l == L ? 1 : H;
    offW[l] = o;
    offb[l] = o + (int64_t)out * in;
    o = offb[l] + out;
  }
  double loss = 0.0;
  for (int64_t r = 0; r < n; ++r) {
    /* a non-finite target (a boundary point whose every path was non-finite)
       has no weight: it adds nothing to the loss or the gradient, whose
       normalisation stays 1 / n */
    if (!isfinite(target[r])) continue;
    const double f = forward_one(params, Bmat, sh, y + r * dim, bf16, a, s);
    const double e = f - target[r];
    loss += e * e;
    const double g = 2.0 * e / (double)n; /* dL/df */
    /* output layer */
    grad[offb[L]] += g;
    for (int i = 0; i < H; ++i) {
      grad[offW[L] + i] += g * a[L * stride + i];
      const double w = params[offW[L] + i];
      da[i] = g * (bf16 ? to_bf16(w) : w);
    }
    /* hidden layers L..1 (index l = L-1..0) */
    for (int l = L - 1; l >= 0; --l) {
      const int in = l == 0 ? W0 : H;
      for (int j = 0; j < H; ++j) ds[j] = da[j] * silu_grad(s[l * H + j]);
      for (int j = 0; j < H; ++j) {
        const double dq = bf16 ? to_bf16(ds[j]) : ds[j];
        grad[offb[l] + j] += ds[j];
        for (int i = 0; i < in; ++i) grad[offW[l] + (int64_t)j * in + i] += dq * a[l * stride + i];
      }
      if (l > 0) {
        for (int i = 0; i < in; ++i) {
          double acc = 0.0;
          for (int j = 0; j < H; ++j) {
            const double w = params[offW[l] + (int64_t)j * in + i];
            const double dq = bf16 ? to_bf16(ds[j]) : ds[j];
            acc += dq * (bf16 ? to_bf16(w) : w);
          }
          da[i] = acc;
        }
      }
    }
  }
  free(a);
  free(s);
  free(da);
  free(ds);
  free(offW);
  free(offb);
  return loss / (double)n;
}

/* Adam (Kingma and Ba): m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
   p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t = step >= 1. */
void orc_adam_step(double* params, double* m, double* v, const double* grad, int64_t n, int64_t step,
                   double lr, double b1, double b2, double eps) {
  const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
    v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
    params[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}
