// Locality order of evaluation points for the ordered solve: Morton keys of the
// points in their bounding box, a stable radix sort of (key, index), the points
// gathered into that order, and the per-point results scattered back.
//
// The walk of a point's paths reads the BVH nodes and triangles around the
// point and along its lines; the lanes of a wavefront, and the wavefronts of a
// CU, then share more of their L1 and L2 lines when they hold nearby points.
// The order changes nothing in what is computed: each point keeps its own
// random-number index (its position in the caller's array).
#include <hip/hip_runtime.h>
#include <hipcub/device/device_radix_sort.hpp>

#include <cmath>
#include <cstdint>

#include "internal.hpp"

namespace wobi {
namespace {

constexpr int kBoxBlocks = 256;     // partial bounding boxes
constexpr int kOrderThreads = 256;  // threads per workgroup of every kernel here

constexpr size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Partial bounding boxes: block b writes min x, y, z then max x, y, z of the
// points it visits (grid stride) to part[6 b ..].  NaN coordinates are skipped
// (fminf / fmaxf return the other operand).
template <typename R, int D>
__global__ void __launch_bounds__(kOrderThreads) bbox_kernel(const R* pts, int64_t n, float* part) {
  __shared__ float sh[6][kOrderThreads];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * kOrderThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kOrderThreads) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const float v = (float)pts[i * D + d];
      lo[d] = fminf(lo[d], v);
      hi[d] = fmaxf(hi[d], v);
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    sh[d][threadIdx.x] = lo[d];
    sh[3 + d][threadIdx.x] = hi[d];
  }
  __syncthreads();
  for (int w = kOrderThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        sh[d][threadIdx.x] = fminf(sh[d][threadIdx.x], sh[d][threadIdx.x + w]);
        sh[3 + d][threadIdx.x] = fmaxf(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + w]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// Morton key of each point: its cell in a 2^B per axis grid over the bounding
// box (B = 10 in 3D, 15 in 2D: 30 bits), axis bits interleaved; idx = i.  A
// degenerate or non-finite extent, or a NaN coordinate, gives cell 0 on that
// axis: the stable sort then keeps such points in input order.
template <typename R, int D>
__global__ void __launch_bounds__(kOrderThreads) morton_kernel(const R* pts, int64_t n, const float* part,
                                                               uint32_t* keys, uint32_t* idx) {
  __shared__ float box[6];
  if (threadIdx.x < 6) {
    const int q = threadIdx.x;
    float v = q < 3 ? INFINITY : -INFINITY;
    for (int b = 0; b < kBoxBlocks; ++b) v = q < 3 ? fminf(v, part[6 * b + q]) : fmaxf(v, part[6 * b + q]);
    box[q] = v;
  }
  __syncthreads();
  constexpr int B = D == 3 ? 10 : 15;
  constexpr uint32_t cells = 1u << B;
  float lo[D], scale[D];
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const float span = box[3 + d] - box[d];
    lo[d] = box[d];
    scale[d] = (span > 0.f && span < INFINITY) ? (float)cells / span : 0.f;
  }
  for (int64_t i = (int64_t)blockIdx.x * kOrderThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kOrderThreads) {
    uint32_t code = 0;
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const float t = ((float)pts[i * D + d] - lo[d]) * scale[d];
      const uint32_t c = t >= 0.f ? (t < (float)cells ? (uint32_t)t : cells - 1) : 0u;
#pragma unroll
      for (int b = 0; b < B; ++b) code |= ((c >> b) & 1u) << (D * b + d);
    }
    keys[i] = code;
    idx[i] = (uint32_t)i;
  }
}

// The points (and their primitive ids) in the sorted order.
template <typename R, int D>
__global__ void __launch_bounds__(kOrderThreads) gather_kernel(const R* pts, const int32_t* prim,
                                                               const uint32_t* order, int64_t n, R* pts_s,
                                                               int32_t* prim_s) {
  for (int64_t i = (int64_t)blockIdx.x * kOrderThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kOrderThreads) {
    const int64_t j = order[i];
#pragma unroll
    for (int d = 0; d < D; ++d) pts_s[i * D + d] = pts[j * D + d];
    if (prim) prim_s[i] = prim[j];
  }
}

// Results of sorted position i back to the caller's point order[i].
template <typename R>
__global__ void __launch_bounds__(kOrderThreads) scatter_kernel(const uint32_t* order, int64_t n,
                                                                const R* mean_s, const R* var_s, R* mean,
                                                                R* var) {
  for (int64_t i = (int64_t)blockIdx.x * kOrderThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kOrderThreads) {
    const int64_t j = order[i];
    mean[j] = mean_s[i];
    if (var) var[j] = var_s[i];
  }
}

unsigned grid_for(int64_t n) {
  const int64_t b = (n + kOrderThreads - 1) / kOrderThreads;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

template <typename R, int D>
wob_status order_impl(const OrderLayout& L, unsigned char* ws, const void* points,
                      const int32_t* point_prim, int64_t n, hipStream_t st, OrderBuffers* out) {
  float* part = (float*)(ws + L.part);
  uint32_t* keys = (uint32_t*)(ws + L.keys);
  uint32_t* keys_s = (uint32_t*)(ws + L.keys_s);
  uint32_t* idx = (uint32_t*)(ws + L.idx);
  uint32_t* order = (uint32_t*)(ws + L.order);
  R* pts_s = (R*)(ws + L.pts);
  int32_t* prim_s = (int32_t*)(ws + L.prim);
  const R* pts = (const R*)points;
  hipLaunchKernelGGL((bbox_kernel<R, D>), dim3(kBoxBlocks), dim3(kOrderThreads), 0, st, pts, n, part);
  hipLaunchKernelGGL((morton_kernel<R, D>), dim3(grid_for(n)), dim3(kOrderThreads), 0, st, pts, n, part, keys,
                     idx);
  size_t temp = L.temp_bytes;
  if (hipcub::DeviceRadixSort::SortPairs(ws + L.temp, temp, keys, keys_s, idx, order, (int)n, 0, 30, st) !=
      hipSuccess)
    return WOB_E_DEVICE;
  hipLaunchKernelGGL((gather_kernel<R, D>), dim3(grid_for(n)), dim3(kOrderThreads), 0, st, pts, point_prim,
                     order, n, pts_s, prim_s);
  out->order = order;
  out->points = pts_s;
  out->point_prim = point_prim ? prim_s : nullptr;
  out->mean = ws + L.mean;
  out->var = ws + L.var;
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

}  // namespace

OrderLayout order_layout(int dim, int precision, int64_t n) {
  OrderLayout L{};
  const size_t rs = precision == WOB_F64 ? 8 : 4;
  const size_t un = (size_t)(n > 0 ? n : 1);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  L.part = take(sizeof(float) * 6 * kBoxBlocks);
  L.keys = take(4 * un);
  L.keys_s = take(4 * un);
  L.idx = take(4 * un);
  L.order = take(4 * un);
  L.pts = take(rs * dim * un);
  L.prim = take(4 * un);
  L.mean = take(rs * un);
  L.var = take(rs * un);
  size_t temp = 0;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, temp, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (const uint32_t*)nullptr, (uint32_t*)nullptr, (int)un, 0, 30);
  L.temp_bytes = temp;
  L.temp = take(temp);
  L.total = off;
  return L;
}

wob_status order_points(int dim, int precision, const OrderLayout& L, void* workspace, const void* points,
                        const int32_t* point_prim, int64_t n, void* stream, OrderBuffers* out) {
  unsigned char* ws = (unsigned char*)workspace;
  hipStream_t st = (hipStream_t)stream;
  if (precision == WOB_F32)
    return dim == 3 ? order_impl<float, 3>(L, ws, points, point_prim, n, st, out)
                    : order_impl<float, 2>(L, ws, points, point_prim, n, st, out);
  return dim == 3 ? order_impl<double, 3>(L, ws, points, point_prim, n, st, out)
                  : order_impl<double, 2>(L, ws, points, point_prim, n, st, out);
}

wob_status scatter_results(int precision, const OrderBuffers& b, int64_t n, void* mean_out, void* var_out,
                           void* stream) {
  hipStream_t st = (hipStream_t)stream;
  if (precision == WOB_F32)
    hipLaunchKernelGGL((scatter_kernel<float>), dim3(grid_for(n)), dim3(kOrderThreads), 0, st, b.order, n,
                       (const float*)b.mean, (const float*)b.var, (float*)mean_out, (float*)var_out);
  else
    hipLaunchKernelGGL((scatter_kernel<double>), dim3(grid_for(n)), dim3(kOrderThreads), 0, st, b.order, n,
                       (const double*)b.mean, (const double*)b.var, (double*)mean_out, (double*)var_out);
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

}  // namespace wobi
