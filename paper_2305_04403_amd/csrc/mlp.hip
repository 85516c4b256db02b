// Fourier-feature MLP for the learned control variate, on the gfx950 matrix
// cores: forward, backward (mean-squared error), deterministic gradient
// reduction and Adam.  Architecture fixed at compile time: 16 frequencies
// (32 features), 4 hidden layers of 128 with SiLU, scalar output.
//
// Matrix products use v_mfma_f32_16x16x32_bf16: bfloat16 operands, binary32
// accumulation.  Rounding to bfloat16 happens at: the features, each hidden
// activation, each weight matrix (a bfloat16 copy refreshed by Adam) and each
// pre-activation gradient that enters a product; biases, accumulators, the
// output layer and all element-wise math stay in binary32.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/wob.h"

namespace {

constexpr int KF = 16;        // Fourier frequencies
constexpr int F0 = 2 * KF;    // features
constexpr int HD = 128;       // hidden width
constexpr int NL = 4;         // hidden layers
constexpr int TR = 64;        // rows per workgroup
constexpr int NT = 256;       // threads per workgroup (4 wavefronts)
constexpr int kFwdGrid = 1024;  // forward-pass workgroups (256 CUs x 4)

// parameter offsets (floats): W_l [out][in] then b_l, layers 0..NL (NL = output)
constexpr int in_of(int l) { return l == 0 ? F0 : HD; }
constexpr int out_of(int l) { return l == NL ? 1 : HD; }
constexpr int offW(int l) { return l == 0 ? 0 : offW(l - 1) + out_of(l - 1) * in_of(l - 1) + out_of(l - 1); }
constexpr int offB(int l) { return offW(l) + out_of(l) * in_of(l); }
constexpr int NP = offB(NL) + 1;
static_assert(NP == 53889, "parameter count");

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

struct Net {
  int dim;
  float* p;       // binary32 master parameters
  float* m;       // Adam first moment
  float* v;       // Adam second moment
  __bf16* wq;     // bfloat16 copy, [out][in] per layer (bias slots unused)
  __bf16* wt;     // bfloat16 transposed copy, [in][out] per layer
  float* fourier; // KF x dim
};

// SiLU with the hardware reciprocal (1 ulp; the result is rounded to bfloat16
// or multiplies a bfloat16-rounded gradient, so an IEEE division buys nothing)
__device__ __forceinline__ float sigmoid_(float s) { return __builtin_amdgcn_rcpf(1.f + __expf(-s)); }
// The activation that is rounded to bfloat16: s / (1 + e^-s) correctly
// rounded to binary32 wherever that decides the bfloat16 rounding.  The fast
// binary32 evaluation (hardware exp2 of s log2 e, hardware reciprocal) is
// within (|s| + 3) ulp of the exact value (the product s log2 e carries |s| u
// of absolute error into the exponent); its bfloat16 rounding can differ from
// that of the exact value only when it lies that close to a bfloat16 rounding
// boundary (low half-word 0x8000), and there the value is recomputed in
// binary64 and rounded once to binary32.  The rounded activation then departs
// from exact arithmetic only through the accumulation of s.
__device__ __forceinline__ float silu_rounded(float s) {
  const float h = s * sigmoid_(s);
  const int lo = (int)(__float_as_uint(h) & 0xffffu);
  const float win = 8.f + 2.f * fabsf(s);  // ulps, twice the error bound
  if (fabsf((float)(lo - 0x8000)) <= win) {
    const double d = (double)s;
    return (float)(d / (1.0 + exp(-d)));
  }
  return h;
}
__device__ __forceinline__ float silu_grad(float s) {
  const float sg = sigmoid_(s);
  return sg * (1.f + s * (1.f - sg));
}

// MFMA 16x16x32 operand fragments.  Lane l holds rows/cols (l % 16) and the
// eight k values 8 (l / 16) .. +7; the accumulator holds rows 4 (l / 16) + v.
__device__ __forceinline__ bf16x8 frag_rows(const __bf16* a, int ld, int row, int k0) {
  // a[row][k0 .. k0 + 7], contiguous
  bf16x8 f;
#pragma unroll
  for (int e = 0; e < 8; ++e) f[e] = a[row * ld + k0 + e];
  return f;
}
__device__ __forceinline__ bf16x8 frag_cols(const __bf16* a, int ld, int k0, int col) {
  // a[k0 .. k0 + 7][col], strided
  bf16x8 f;
#pragma unroll
  for (int e = 0; e < 8; ++e) f[e] = a[(k0 + e) * ld + col];
  return f;
}
__device__ __forceinline__ floatx4 mfma(bf16x8 a, bf16x8 b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Shared memory of one workgroup.
struct Smem {
  __bf16 a0[TR * F0];
  __bf16 act[NL][TR * HD];  // activations h_1 .. h_4 (bfloat16)
  __bf16 dq[TR * HD];       // bfloat16 pre-activation gradient of the current layer
  float ds[TR * HD];        // binary32 pre-activation gradient
  float g5[TR];
  float red[NT];
};

// The forward pass alone: two activation buffers (layer l writes buffer l % 2)
// whose rows are padded by 8 elements, so that the 16 rows of an operand
// fragment start 16 bytes apart and spread over the LDS banks.  About 40 KiB.
constexpr int LDA0 = F0 + 8, LDH = HD + 8;
struct FwdSmem {
  __bf16 a0[TR * LDA0];
  __bf16 act[2][TR * LDH];
  float w5[HD];  // the output layer's weights (their bfloat16 values)
};

// Features and the four hidden layers for rows r0 .. r0 + 63 into LDS (the
// backward pass): the features to a0, layer l's activations to act + l TR HD.
// Pre-activations go to `sbuf` (4 x 64 x 128 floats) when it is not null.
// Returns the last layer's buffer.
// The Fourier features of rows r0 .. r0 + 63 into a0 (row stride lda; rows
// past n are zero).
__device__ void features_tile(const Net& net, const float* y, int64_t n, int64_t r0, __bf16* a0, int lda) {
  for (int idx = threadIdx.x; idx < TR * KF; idx += NT) {
    const int r = idx / KF, k = idx % KF;
    const int64_t row = r0 + r;
    float sv = 0.f, cv = 0.f;
    if (row < n) {
      // B y in binary64 (each product of two binary32 values is exact), the
      // period taken out exactly, sin and cos of 2 pi (B y) in binary64: the
      // features are then the binary32 roundings of the exact values except
      // within ~1e-16 of a rounding boundary
      double arg = 0.0;
      for (int d = 0; d < net.dim; ++d) arg += (double)net.fourier[k * net.dim + d] * (double)y[row * net.dim + d];
      const double r = arg - rint(arg);  // exact (Sterbenz), in [-1/2, 1/2]
      double sd, cd;
      sincospi(2.0 * r, &sd, &cd);
      sv = (float)sd;
      cv = (float)cd;
    }
    a0[r * lda + k] = (__bf16)sv;
    a0[r * lda + KF + k] = (__bf16)cv;
  }
}

template <bool ALL>
__device__ const __bf16* forward_tile(const Net& net, const float* y, int64_t n, int64_t r0,
                                      __bf16* a0, __bf16* act, float* sbuf) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  features_tile(net, y, n, r0, a0, F0);
  __syncthreads();
  for (int l = 0; l < NL; ++l) {
    const int K = in_of(l);
    const __bf16* A = l == 0 ? a0 : act + (ALL ? l - 1 : (l - 1) & 1) * TR * HD;
    __bf16* O = act + (ALL ? l : l & 1) * TR * HD;
    const __bf16* W = net.wq + offW(l);
    const int ldw = K;
    const float* b = net.p + offB(l);
    floatx4 acc[8];
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) acc[cb] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int row = wave * 16 + (lane & 15);
    for (int k0 = 0; k0 < K; k0 += 32) {
      const bf16x8 af = frag_rows(A, K, row, k0 + 8 * (lane >> 4));
#pragma unroll
      for (int cb = 0; cb < 8; ++cb) {
        // B[k][o] = W[o][k]: eight consecutive k of row o of W
        const int o = cb * 16 + (lane & 15);
        const bf16x8 bf = *(const bf16x8*)(W + o * ldw + k0 + 8 * (lane >> 4));
        acc[cb] = mfma(af, bf, acc[cb]);
      }
    }
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) {
      const int col = cb * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wave * 16 + 4 * (lane >> 4) + v;
        const float s = acc[cb][v] + b[col];
        if (sbuf) sbuf[(l * TR + r) * HD + col] = s;
        O[r * HD + col] = (__bf16)silu_rounded(s);
      }
    }
    __syncthreads();
  }
  return act + (ALL ? NL - 1 : (NL - 1) & 1) * TR * HD;
}

// Output layer f = W5 . h4 + b5 for the 64 rows; 4 lanes per row.
__device__ float output_row(const Net& net, const __bf16* h4, int& r_out) {
  const int tid = threadIdx.x;
  const int r = tid >> 2, part = tid & 3;
  float acc = 0.f;
  for (int i = part * 32; i < part * 32 + 32; ++i)
    acc += (float)net.wq[offW(NL) + i] * (float)h4[r * HD + i];
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  r_out = r;
  return acc + net.p[offB(NL)];
}

// Forward pass, weight-stationary: wavefront w computes output columns
// 32 w .. 32 w + 31 of every hidden layer, and holds those columns of every
// layer's bfloat16 weights in registers as MFMA operand fragments (26
// fragments, 104 registers), loaded once per workgroup; the workgroups then
// take 64-row tiles in turn.  Per layer and tile a wavefront reads the four
// row blocks' activation fragments from LDS and issues 4 x 2 MFMAs per 32-wide
// k step.  The accumulation order of each output (k ascending in steps of 32),
// the bias, the activation and its rounding are those of the backward pass's
// forward tile.
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) mlp_forward_kernel(Net net, const float* y,
                                                                                        int64_t n, float* out) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  FwdSmem& sm = *reinterpret_cast<FwdSmem*>(smem_raw);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kq = 8 * (lane >> 4);  // the lane's eight k values within a 32-wide step
  // weight fragments: B[k][o] = W[o][k], o = 32 wave + 16 cb + lane % 16
  bf16x8 w0[2], wh[NL - 1][2][HD / 32];
  float bias[NL][2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int o = 32 * wave + 16 * cb + (lane & 15);
    w0[cb] = *(const bf16x8*)(net.wq + offW(0) + o * F0 + kq);
#pragma unroll
    for (int l = 1; l < NL; ++l)
#pragma unroll
      for (int ks = 0; ks < HD / 32; ++ks) wh[l - 1][cb][ks] = *(const bf16x8*)(net.wq + offW(l) + o * HD + 32 * ks + kq);
#pragma unroll
    for (int l = 0; l < NL; ++l) bias[l][cb] = net.p[offB(l) + o];
  }
  if (tid < HD) sm.w5[tid] = (float)net.wq[offW(NL) + tid];
  const float b5 = net.p[offB(NL)];
  const int64_t n_tiles = (n + TR - 1) / TR;
  for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const int64_t r0 = t * TR;
    features_tile(net, y, n, r0, sm.a0, LDA0);
    __syncthreads();
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const __bf16* A = l == 0 ? sm.a0 : sm.act[(l - 1) & 1];
      const int lda = l == 0 ? LDA0 : LDH;
      __bf16* O = sm.act[l & 1];
      floatx4 acc[4][2];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < in_of(l) / 32; ++ks) {
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          const bf16x8 af = *(const bf16x8*)(A + (16 * rb + (lane & 15)) * lda + 32 * ks + kq);
#pragma unroll
          for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = mfma(af, l == 0 ? w0[cb] : wh[l - 1][cb][ks], acc[rb][cb]);
        }
      }
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) {
          const int col = 32 * wave + 16 * cb + (lane & 15);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * rb + 4 * (lane >> 4) + v;
            O[r * LDH + col] = (__bf16)silu_rounded(acc[rb][cb][v] + bias[l][cb]);
          }
        }
      __syncthreads();
    }
    // output layer, as output_row computes it (4 lanes per row, 32 terms each
    // in order, then two butterfly steps), with the weights from LDS
    {
      const int r = tid >> 2, part = tid & 3;
      const __bf16* h4 = sm.act[(NL - 1) & 1] + r * LDH;
      float acc = 0.f;
      for (int i = part * 32; i < part * 32 + 32; ++i) acc += sm.w5[i] * (float)h4[i];
      acc += __shfl_xor(acc, 1, 64);
      acc += __shfl_xor(acc, 2, 64);
      if (part == 0 && r0 + r < n) out[r0 + r] = acc + b5;
    }
    __syncthreads();  // the next tile's features and layers overwrite a0 and act
  }
}

// Target transform t -> (t - shift) inv_scale, clamped to [-clip, clip] when clip > 0.
struct TargetMap {
  int on;
  float shift, inv_scale, clip;
};

// Loss and gradient of one tile: writes the tile's partial gradient (NP floats)
// and partial loss (sum of squared errors).  scale = 1 / (rows in the batch).
__global__ void __launch_bounds__(NT) mlp_grad_kernel(Net net, const float* y, const float* target,
                                                      TargetMap tm, int64_t n, float scale,
                                                      float* part_grad, float* part_loss,
                                                      float* sbuf_all) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  Smem& sm = *reinterpret_cast<Smem*>(smem_raw);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * TR;
  float* sbuf = sbuf_all + (int64_t)blockIdx.x * NL * TR * HD;
  float* G = part_grad + (int64_t)blockIdx.x * NP;
  const __bf16* h4 = forward_tile<true>(net, y, n, r0, sm.a0, sm.act[0], sbuf);
  int r;
  const float f = output_row(net, h4, r);
  float e = 0.f;
  if (r0 + r < n) {
    float tv = target[r0 + r];
    // a non-finite target (a boundary point whose every path was non-finite)
    // has no weight in the loss: e = 0 (clamping would turn NaN into -clip)
    if (isfinite(tv)) {
      if (tm.on) {
        tv = (tv - tm.shift) * tm.inv_scale;
        if (tm.clip > 0.f) tv = fminf(fmaxf(tv, -tm.clip), tm.clip);
      }
      e = f - tv;
    }
  }
  if ((tid & 3) == 0) sm.g5[r] = 2.f * e * scale;
  sm.red[tid] = (tid & 3) == 0 ? e * e : 0.f;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (tid < s) sm.red[tid] += sm.red[tid + s];
    __syncthreads();
  }
  if (tid == 0) part_loss[blockIdx.x] = sm.red[0];

  // output layer: dW5[i] = sum_r g5 h4[r][i]; db5 = sum_r g5; dh4 = g5 W5q
  if (tid < HD) {
    float acc = 0.f;
    for (int rr = 0; rr < TR; ++rr) acc += sm.g5[rr] * (float)sm.act[NL - 1][rr * HD + tid];
    G[offW(NL) + tid] = acc;
  }
  if (tid == HD) {
    float acc = 0.f;
    for (int rr = 0; rr < TR; ++rr) acc += sm.g5[rr];
    G[offB(NL)] = acc;
  }
  // ds for the last hidden layer: dh4 * silu'(s4)
  for (int idx = tid; idx < TR * HD; idx += NT) {
    const int rr = idx / HD, o = idx % HD;
    const float dh = sm.g5[rr] * (float)net.wq[offW(NL) + o];
    sm.ds[idx] = dh * silu_grad(sbuf[((NL - 1) * TR + rr) * HD + o]);
  }
  __syncthreads();

  for (int l = NL - 1; l >= 0; --l) {
    const int K = in_of(l);  // input width of layer l
    // bfloat16 copy of ds for the products; bias gradient from binary32 ds
    for (int idx = tid; idx < TR * HD; idx += NT) sm.dq[idx] = (__bf16)sm.ds[idx];
    if (tid < HD) {
      float acc = 0.f;
      for (int rr = 0; rr < TR; ++rr) acc += sm.ds[rr * HD + tid];
      G[offB(l) + tid] = acc;
    }
    __syncthreads();
    // dW_l[o][i] = sum_r dq[r][o] a_{l-1}[r][i]: (HD x TR) x (TR x K)
    {
      const __bf16* A = l == 0 ? sm.a0 : sm.act[l - 1];
      const int tiles_i = K / 16, n_tiles = 8 * tiles_i;
      for (int t = wave; t < n_tiles; t += 4) {
        const int ob = t / tiles_i, ib = t % tiles_i;
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < TR; k0 += 32) {
          const int kk = k0 + 8 * (lane >> 4);
          const bf16x8 af = frag_cols(sm.dq, HD, kk, ob * 16 + (lane & 15));  // A[o][r] = dq[r][o]
          const bf16x8 bf = frag_cols(A, K, kk, ib * 16 + (lane & 15));        // B[r][i] = a[r][i]
          acc = mfma(af, bf, acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int o = ob * 16 + 4 * (lane >> 4) + v, i = ib * 16 + (lane & 15);
          G[offW(l) + o * K + i] = acc[v];
        }
      }
    }
    if (l == 0) break;
    // dh_{l-1}[r][i] = sum_o dq[r][o] W_l[o][i]: (TR x HD) x (HD x HD), B from the transposed copy
    floatx4 acc[8];
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) acc[cb] = floatx4{0.f, 0.f, 0.f, 0.f};
    {
      const __bf16* Wt = net.wt + offW(l);  // [i][o]
      const int row = wave * 16 + (lane & 15);
      for (int k0 = 0; k0 < HD; k0 += 32) {
        const bf16x8 af = frag_rows(sm.dq, HD, row, k0 + 8 * (lane >> 4));
#pragma unroll
        for (int cb = 0; cb < 8; ++cb) {
          const int i = cb * 16 + (lane & 15);
          const bf16x8 bf = *(const bf16x8*)(Wt + i * HD + k0 + 8 * (lane >> 4));
          acc[cb] = mfma(af, bf, acc[cb]);
        }
      }
    }
    __syncthreads();  // everyone is done with dq and ds of layer l
#pragma unroll
    for (int cb = 0; cb < 8; ++cb) {
      const int i = cb * 16 + (lane & 15);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = wave * 16 + 4 * (lane >> 4) + v;
        sm.ds[rr * HD + i] = acc[cb][v] * silu_grad(sbuf[((l - 1) * TR + rr) * HD + i]);
      }
    }
    __syncthreads();
  }
}

// The tiles' partial gradients are summed in slices of kSlice tiles (tiles
// s kSlice .. s kSlice + kSlice - 1 in order, the sum written over the
// slice's first tile), then the slice sums in order: a fixed order, so the
// gradient is deterministic, with kSlice times more threads at work than one
// sum per parameter.
constexpr int kSlice = 32;
__global__ void slice_grad_kernel(float* part, int n_tiles) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int t0 = blockIdx.y * kSlice, t1 = t0 + kSlice < n_tiles ? t0 + kSlice : n_tiles;
  if (p >= NP) return;
  float acc = 0.f;
  for (int t = t0; t < t1; ++t) acc += part[(int64_t)t * NP + p];
  part[(int64_t)t0 * NP + p] = acc;
}

// grad[p] = sum over slices of the slice sums (fixed order), loss = sum part_loss * scale.
__global__ void reduce_grad_kernel(const float* part, int n_tiles, float* grad, const float* part_loss,
                                   float* loss, float scale) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NP) {
    float acc = 0.f;
    for (int t = 0; t < n_tiles; t += kSlice) acc += part[(int64_t)t * NP + p];
    grad[p] = acc;
  }
  if (p == 0 && loss) {
    float acc = 0.f;
    for (int t = 0; t < n_tiles; ++t) acc += part_loss[t];
    *loss = acc * scale;
  }
}

// Adam on the binary32 master copy, then the bfloat16 copies for the products.
__global__ void adam_kernel(Net net, const float* grad, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  const float g = grad[p];
  const float m = b1 * net.m[p] + (1.f - b1) * g;
  const float v = b2 * net.v[p] + (1.f - b2) * g * g;
  net.m[p] = m;
  net.v[p] = v;
  const float w = net.p[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  net.p[p] = w;
  // bfloat16 copies
  int l = 0;
  while (l < NL && p >= offW(l + 1)) ++l;
  const int q = p - offW(l);
  const int K = in_of(l), O = out_of(l);
  if (q < O * K) {
    const int o = q / K, i = q % K;
    net.wq[p] = (__bf16)w;
    net.wt[offW(l) + i * O + o] = (__bf16)w;
  }
}

__global__ void refresh_bf16_kernel(Net net) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  int l = 0;
  while (l < NL && p >= offW(l + 1)) ++l;
  const int q = p - offW(l);
  const int K = in_of(l), O = out_of(l);
  if (q < O * K) {
    const int o = q / K, i = q % K;
    net.wq[p] = (__bf16)net.p[p];
    net.wt[offW(l) + i * O + o] = (__bf16)net.p[p];
  }
}

}  // namespace

struct wob_mlp_s {
  Net net{};
  int64_t max_batch = 0;
  int n_tiles_max = 0;
  float* part = nullptr;      // n_tiles_max x NP
  float* part_loss = nullptr; // n_tiles_max
  float* sbuf = nullptr;      // n_tiles_max x NL x TR x HD
  float* grad = nullptr;      // NP
};

namespace {

void mlp_destroy(wob_mlp_s* h) {
  if (!h) return;
  void* ptrs[] = {h->net.p, h->net.m, h->net.v, h->net.wq, h->net.wt, h->net.fourier,
                  h->part, h->part_loss, h->sbuf, h->grad};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  delete h;
}

wob_status refresh(wob_mlp_s* h, hipStream_t st) {
  hipLaunchKernelGGL(refresh_bf16_kernel, dim3((NP + 255) / 256), dim3(256), 0, st, h->net);
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

}  // namespace

extern "C" {

int64_t wob_mlp_n_params(void) { return NP; }

wob_status wob_mlp_create(int32_t dim, const float* fourier, const float* params, int64_t max_batch,
                          wob_mlp* out) {
  if (!out) return WOB_E_ARG;
  *out = nullptr;
  if ((dim != 2 && dim != 3) || !fourier || !params || max_batch < 0) return WOB_E_ARG;
  for (int i = 0; i < KF * dim; ++i)
    if (!std::isfinite(fourier[i])) return WOB_E_ARG;
  for (int i = 0; i < NP; ++i)
    if (!std::isfinite(params[i])) return WOB_E_ARG;
  // the backward pass keeps every activation of its 64 rows in LDS (> 64 KiB)
  if (hipFuncSetAttribute((const void*)mlp_forward_kernel,
                          hipFuncAttributeMaxDynamicSharedMemorySize, sizeof(FwdSmem)) != hipSuccess ||
      hipFuncSetAttribute((const void*)mlp_grad_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          sizeof(Smem)) != hipSuccess)
    return WOB_E_DEVICE;
  wob_mlp_s* h = new (std::nothrow) wob_mlp_s();
  if (!h) return WOB_E_ALLOC;
  h->net.dim = dim;
  h->max_batch = max_batch;
  h->n_tiles_max = (int)((max_batch + TR - 1) / TR);
  bool ok = hipMalloc((void**)&h->net.p, NP * 4) == hipSuccess &&
            hipMalloc((void**)&h->net.m, NP * 4) == hipSuccess &&
            hipMalloc((void**)&h->net.v, NP * 4) == hipSuccess &&
            hipMalloc((void**)&h->net.wq, NP * 2) == hipSuccess &&
            hipMalloc((void**)&h->net.wt, NP * 2) == hipSuccess &&
            hipMalloc((void**)&h->net.fourier, KF * dim * 4) == hipSuccess &&
            hipMalloc((void**)&h->grad, NP * 4) == hipSuccess;
  if (ok && h->n_tiles_max > 0)
    ok = hipMalloc((void**)&h->part, (size_t)h->n_tiles_max * NP * 4) == hipSuccess &&
         hipMalloc((void**)&h->part_loss, (size_t)h->n_tiles_max * 4) == hipSuccess &&
         hipMalloc((void**)&h->sbuf, (size_t)h->n_tiles_max * NL * TR * HD * 4) == hipSuccess;
  if (!ok) {
    mlp_destroy(h);
    return WOB_E_ALLOC;
  }
  std::vector<float> zeros(NP, 0.f);
  ok = hipMemcpy(h->net.p, params, NP * 4, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(h->net.m, zeros.data(), NP * 4, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(h->net.v, zeros.data(), NP * 4, hipMemcpyHostToDevice) == hipSuccess &&
       hipMemcpy(h->net.fourier, fourier, KF * dim * 4, hipMemcpyHostToDevice) == hipSuccess &&
       refresh(h, nullptr) == WOB_OK && hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    mlp_destroy(h);
    return WOB_E_DEVICE;
  }
  *out = h;
  return WOB_OK;
}

void wob_mlp_free(wob_mlp h) { mlp_destroy(h); }

wob_status wob_mlp_get_params(wob_mlp h, float* params) {
  if (!h || !params) return WOB_E_ARG;
  return hipMemcpy(params, h->net.p, NP * 4, hipMemcpyDeviceToHost) == hipSuccess ? WOB_OK
                                                                                  : WOB_E_DEVICE;
}

wob_status wob_mlp_set_params(wob_mlp h, const float* params) {
  if (!h || !params) return WOB_E_ARG;
  std::vector<float> zeros(NP, 0.f);
  if (hipMemcpy(h->net.p, params, NP * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->net.m, zeros.data(), NP * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->net.v, zeros.data(), NP * 4, hipMemcpyHostToDevice) != hipSuccess)
    return WOB_E_DEVICE;
  if (refresh(h, nullptr) != WOB_OK || hipDeviceSynchronize() != hipSuccess) return WOB_E_DEVICE;
  return WOB_OK;
}

wob_status wob_mlp_get_moments(wob_mlp h, float* m, float* v) {
  if (!h || !m || !v) return WOB_E_ARG;
  return hipMemcpy(m, h->net.m, NP * 4, hipMemcpyDeviceToHost) == hipSuccess &&
                 hipMemcpy(v, h->net.v, NP * 4, hipMemcpyDeviceToHost) == hipSuccess
             ? WOB_OK
             : WOB_E_DEVICE;
}

wob_status wob_mlp_set_moments(wob_mlp h, const float* m, const float* v) {
  if (!h || !m || !v) return WOB_E_ARG;
  if (hipMemcpy(h->net.m, m, NP * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->net.v, v, NP * 4, hipMemcpyHostToDevice) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
    return WOB_E_DEVICE;
  return WOB_OK;
}

wob_status wob_mlp_forward(wob_mlp h, const float* y, int64_t n, float* out, void* stream) {
  if (!h || n < 0 || (n > 0 && (!y || !out))) return WOB_E_ARG;
  if (n == 0) return WOB_OK;
  const int64_t tiles = (n + TR - 1) / TR;
  // persistent workgroups, their weight fragments loaded once (two resident per CU)
  const int64_t grid = tiles < kFwdGrid ? tiles : kFwdGrid;
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)grid), dim3(NT), sizeof(FwdSmem),
                     (hipStream_t)stream, h->net, y, n, out);
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

wob_status wob_mlp_backward(wob_mlp h, const float* y, const float* target,
                            const wob_target_map* tmap, int64_t n, float* grad, float* loss,
                            void* stream) {
  if (!h || n <= 0 || n > h->max_batch || !y || !target || !grad) return WOB_E_ARG;
  TargetMap tm{0, 0.f, 1.f, 0.f};
  if (tmap) {
    if (!std::isfinite(tmap->shift) || !(tmap->scale > 0.f) || !std::isfinite(tmap->scale) ||
        !(tmap->clip >= 0.f))
      return WOB_E_ARG;
    tm = TargetMap{1, tmap->shift, 1.f / tmap->scale, tmap->clip};
  }
  hipStream_t st = (hipStream_t)stream;
  const int tiles = (int)((n + TR - 1) / TR);
  const float scale = 1.f / (float)n;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(tiles), dim3(NT), sizeof(Smem), st, h->net, y, target, tm,
                     n, scale, h->part, h->part_loss, h->sbuf);
  hipLaunchKernelGGL(slice_grad_kernel, dim3((NP + 255) / 256, (unsigned)((tiles + kSlice - 1) / kSlice)), dim3(256),
                     0, st, h->part, (int)tiles);
  hipLaunchKernelGGL(reduce_grad_kernel, dim3((NP + 255) / 256), dim3(256), 0, st, h->part, tiles,
                     grad, h->part_loss, loss, scale);
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

wob_status wob_mlp_adam_step(wob_mlp h, const float* grad, int64_t step, float lr, float b1, float b2,
                             float eps, void* stream) {
  if (!h || !grad || step < 1 || !(lr > 0.f) || !std::isfinite(lr) || !(b1 >= 0.f && b1 < 1.f) ||
      !(b2 >= 0.f && b2 < 1.f) || !(eps > 0.f))
    return WOB_E_ARG;
  const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
  hipLaunchKernelGGL(adam_kernel, dim3((NP + 255) / 256), dim3(256), 0, (hipStream_t)stream, h->net,
                     grad, lr, b1, b2, eps, c1, c2);
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

wob_status wob_mlp_train_step(wob_mlp h, const float* y, const float* target,
                              const wob_target_map* tmap, int64_t n, int64_t step, float lr,
                              float* loss, void* stream) {
  wob_status s = wob_mlp_backward(h, y, target, tmap, n, h ? h->grad : nullptr, loss, stream);
  if (s != WOB_OK) return s;
  return wob_mlp_adam_step(h, h->grad, step, lr, 0.9f, 0.999f, 1e-8f, stream);
}

}  // extern "C"
