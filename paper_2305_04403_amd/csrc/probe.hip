// Measurement helper: random 32-byte gathers from a buffer of a given size,
// the access pattern of the traversal's node and triangle records, to
// calibrate the gather bandwidth of the memory level a scene lives in (LDS-,
// L2-, MALL- or HBM-sized working sets).
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

}  // namespace

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
