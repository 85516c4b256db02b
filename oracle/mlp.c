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

/* ------------------------------------------------------------------------ */
/* Error bound of a bfloat16 evaluation of the network.                      */
/*                                                                          */
/* A device evaluation that rounds to bfloat16 at the same points as the     */
/* forward pass above, but sums each layer's products in binary32 in its own */
/* order, differs from it in two ways, both propagated layer by layer as an  */
/* interval half-width d per value:                                         */
/* (i) accumulation: a pre-activation carries at most acc u32 times the      */
/*     magnitude sum of its terms (bias included), `acc` given per layer     */
/*     kind (first hidden layer, other hidden layers, output layer) by the   */
/*     caller from the device's summation, on top of its inputs' own         */
/*     half-widths through |W|;                                             */
/* (ii) flips: an activation h whose distance to a boundary where its        */
/*     rounding (to binary32, then bfloat16) changes is within its           */
/*     half-width dh (|silu'| d_s to first order, plus d_s^2 / 2 with        */
/*     |silu''| <= 1/2) may round to another bfloat16 value; its rounded     */
/*     value then differs by at most dh plus one bfloat16 spacing.  Away     */
/*     from a boundary both sides round alike and the half-width is 0.       */
/* Flips that cascade (a flip widening a later pre-activation past a         */
/* boundary) are included; the bound is therefore a worst case over every    */
/* combination of flips, loose where many activations are near boundaries.  */
/* Features are exact up to the row's input half-width dy (each coordinate   */
/* of y may differ by dy; NULL: 0): they are sines and cosines of a binary64 */
/* argument rounded like the activations, moved by at most 2 pi sum|B| dy.   */
/* For each row: out = f, scale = sum |w_i a_i| + |b| of the output layer,   */
/* bound = the output's half-width, risk = activations near a boundary.      */
/* ------------------------------------------------------------------------ */

#define MLP_U32 (1.0 / 16777216.0)

/* distance from x to the nearest boundary at which its rounding to bfloat16
   (via binary32, as to_bf16) changes, and the larger bfloat16 spacing there */
static void bf16_margin(double x, double* dist, double* spacing) {
  const double r = fabs(to_bf16(x));
  float fr = (float)r, fu, fd;
  uint32_t u;
  memcpy(&u, &fr, 4);
  const uint32_t uu = u + 0x10000u, ud = u >= 0x10000u ? u - 0x10000u : 0u;
  memcpy(&fu, &uu, 4);
  memcpy(&fd, &ud, 4);
  const double up = 0.5 * (r + (double)fu), dn = 0.5 * (r + (double)fd);
  const double ax = fabs(x);
  *dist = fmin(fabs(ax - up), fabs(ax - dn));
  *spacing = fmax((double)fu - r, r - (double)fd);
}

void orc_mlp_forward_bound(const double* P, const double* Bm, int n_freq, int hidden, int layers, int dim,
                           int64_t n, const double* y, const double* dy, double acc_first, double acc_hidden,
                           double acc_out, double* out, double* scale, double* bound, int32_t* risk) {
  const int K = n_freq, H = hidden, L = layers, W0 = 2 * K;
  const int stride = W0 > H ? W0 : H;
  double* a = (double*)malloc(sizeof(double) * (size_t)2 * stride);
  double* da = (double*)malloc(sizeof(double) * (size_t)2 * stride);
  for (int64_t r = 0; r < n; ++r) {
    const double* yr = y + r * dim;
    int nrisk = 0;
    double *cur = a, *dcur = da, *nxt = a + stride, *dnxt = da + stride;
    for (int k = 0; k < K; ++k) {
      double arg = 0.0, darg = 0.0;
      for (int d = 0; d < dim; ++d) {
        arg += Bm[k * dim + d] * yr[d];
        darg += fabs(Bm[k * dim + d]) * (dy ? dy[r] : 0.0);
      }
      const double f2[2] = {sin(2.0 * MLP_PI * arg), cos(2.0 * MLP_PI * arg)};
      for (int q = 0; q < 2; ++q) {
        const double df = 2.0 * MLP_PI * darg;
        double dist, sp;
        bf16_margin(f2[q], &dist, &sp);
        cur[q * K + k] = to_bf16(f2[q]);
        dcur[q * K + k] = (df > 0.0 && dist <= df + MLP_U32 * fabs(f2[q])) ? df + sp : 0.0;
      }
    }
    const double* p = P;
    int in = W0;
    for (int l = 0; l < L; ++l) {
      const double* W = p;
      const double* b = p + (int64_t)H * in;
      const double acc = l == 0 ? acc_first : acc_hidden;
      for (int o = 0; o < H; ++o) {
        double s = b[o], mag = fabs(b[o]), prop = 0.0;
        for (int i = 0; i < in; ++i) {
          const double w = to_bf16(W[o * in + i]);
          s += w * cur[i];
          mag += fabs(w) * (fabs(cur[i]) + dcur[i]);
          prop += fabs(w) * dcur[i];
        }
        const double ds = prop + acc * MLP_U32 * mag;
        const double sg = 1.0 / (1.0 + exp(-s));
        const double h = s * sg;
        const double dh = (fabs(sg * (1.0 + s * (1.0 - sg))) + 0.25 * ds) * ds;
        double dist, sp;
        bf16_margin(h, &dist, &sp);
        nxt[o] = to_bf16(h);
        if (dist <= dh + MLP_U32 * fabs(h)) {
          ++nrisk;
          dnxt[o] = dh + sp;
        } else {
          dnxt[o] = 0.0;
        }
      }
      double* t = cur; cur = nxt; nxt = t;
      t = dcur; dcur = dnxt; dnxt = t;
      p = b + H;
      in = H;
    }
    double f = p[H], mag = fabs(p[H]), mag_dev = fabs(p[H]), prop = 0.0;
    for (int i = 0; i < H; ++i) {
      const double w = to_bf16(p[i]);
      f += w * cur[i];
      mag += fabs(w * cur[i]);
      mag_dev += fabs(w) * (fabs(cur[i]) + dcur[i]);
      prop += fabs(w) * dcur[i];
    }
    out[r] = f;
    scale[r] = mag;
    bound[r] = prop + acc_out * MLP_U32 * mag_dev;
    risk[r] = nrisk;
  }
  free(a);
  free(da);
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
