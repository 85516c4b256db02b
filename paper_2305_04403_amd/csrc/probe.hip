// Measurement helpers.  wob_gather_probe: random 32-byte gathers from a buffer of a given size,
// the access pattern of the traversal's node and triangle records, to
// calibrate the gather bandwidth of the memory level a scene lives in (LDS-,
// L2-, MALL- or HBM-sized working sets).  wob_mfma_probe: one bfloat16
// matrix instruction per tile, to bound its binary32 accumulation error.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/wob.h"

namespace {

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// Each lane reads `reads` records (two 16-byte loads) at independent
// pseudo-random record indices and writes the sum of all words of every
// record it read (so that every load is whole and none is dead).
__global__ void __launch_bounds__(256) gather_probe_kernel(const float4* __restrict__ buf, uint32_t n_rec,
                                                           int32_t reads, uint32_t seed,
                                                           float* __restrict__ out, int64_t lanes) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= lanes) return;
  uint32_t h = mix32((uint32_t)t * 0x9e3779b9u ^ seed);
  float acc = 0.0f;
  for (int r = 0; r < reads; ++r) {
    h = mix32(h + 0x632be5abu);
    const uint32_t i = (uint32_t)(((uint64_t)h * n_rec) >> 32);  // uniform in [0, n_rec)
    const float4 a = buf[2 * (uint64_t)i], b = buf[2 * (uint64_t)i + 1];
    acc += ((a.x + a.y) + (a.z + a.w)) + ((b.x + b.y) + (b.z + b.w));
  }
  out[t] = acc;
}

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

// One wavefront per tile: D = A B + C with v_mfma_f32_16x16x32_bf16 (the
// network's matrix instruction).  Lane l supplies row (l % 16) of A and
// column (l % 16) of B over k = 8 (l / 16) .. +7, and holds rows
// 4 (l / 16) .. +3 of column (l % 16) of C and D.
__global__ void __launch_bounds__(64) mfma_probe_kernel(const __bf16* __restrict__ A, const __bf16* __restrict__ B,
                                                        const float* __restrict__ C, float* __restrict__ D) {
  const int64_t t = blockIdx.x;
  const int l = threadIdx.x, rc = l & 15, k0 = 8 * (l >> 4);
  const __bf16* a = A + t * 512;
  const __bf16* b = B + t * 512;
  bf16x8 af, bf;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    af[j] = a[rc * 32 + k0 + j];
    bf[j] = b[(k0 + j) * 16 + rc];
  }
  floatx4 c;
#pragma unroll
  for (int v = 0; v < 4; ++v) c[v] = C[t * 256 + (4 * (l >> 4) + v) * 16 + rc];
  const floatx4 d = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, bf, c, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) D[t * 256 + (4 * (l >> 4) + v) * 16 + rc] = d[v];
}

}  // namespace

extern "C" wob_status wob_mfma_probe(const void* a, const void* b, const float* c, float* d, int64_t n_tiles,
                                     void* stream) {
  if (!a || !b || !c || !d || n_tiles < 1 || n_tiles > 0x7fffffffll) return WOB_E_ARG;
  hipLaunchKernelGGL(mfma_probe_kernel, dim3((unsigned)n_tiles), dim3(64), 0, (hipStream_t)stream,
                     (const __bf16*)a, (const __bf16*)b, c, d);
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

extern "C" wob_status wob_gather_probe(const void* buf, int64_t bytes, int64_t lanes, int32_t reads,
                                       uint32_t seed, float* out, void* stream) {
  if (!buf || !out || bytes < 32 || bytes % 32 != 0 || bytes / 32 > 0xffffffffll || lanes < 1 ||
      lanes > ((int64_t)1 << 31) * 256 || reads < 1)
    return WOB_E_ARG;
  if ((uintptr_t)buf % 16 != 0) return WOB_E_ARG;
  const dim3 grid((unsigned)((lanes + 255) / 256)), block(256);
  hipLaunchKernelGGL(gather_probe_kernel, grid, block, 0, (hipStream_t)stream, (const float4*)buf,
                     (uint32_t)(bytes / 32), reads, seed, out, lanes);
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}
