// C ABI of the forward (adjoint) single-layer estimator: start tables, the
// path kernel (the walk kernel in its forward form) and the connection of
// evaluation points to every path vertex.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <new>
#include <vector>

#include "../../include/wob.h"
#include "internal.hpp"

struct wob_starts_s {
  const wob_scene_s* scene = nullptr;
  int32_t device = 0;
  int64_t n_prims = 0;
  float* d_cdf = nullptr;  // binary32 cumulative weight fraction, caller-id order
};

using namespace wobi;

namespace {

// Connection of evaluation points to the vertices of forward paths: per point
// and path j, c_j(x) = sum_k w_jk G(x, y_jk); the mean over paths and the
// unbiased variance of c_j.  G is singular at distance zero: a point exactly at
// a vertex gets a non-finite value (records of ended paths sit far away with
// strength 0, so they add exactly 0; no per-pair distance test).
//
// A workgroup holds 64 * PPL points (PPL per lane) and its four
// wavefronts split the paths in four contiguous ranges; the vertex records are
// read at wavefront-uniform addresses (scalar loads, shared by all lanes), so
// the inner loop is register arithmetic only.  G is accumulated without its
// constant factor: 3D sum w / rho, 2D sum w log2(rho^2); per path the value is
// summed in R over chunks of kGatherChunk paths and the chunk sums in binary64.
constexpr int kGatherPPL = 2;  // points per lane of the launch
constexpr int kGatherChunk = 32;

template <typename R>
__device__ __forceinline__ R inv_dist(R r2) {
  if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rsqf(r2);
  else return (R)1 / sqrt(r2);
}

template <typename R>
__device__ __forceinline__ R log2_dist2(R r2) {
  if constexpr (sizeof(R) == 4) return __log2f(r2);
  else return log2(r2);
}

template <typename R, int D, int PPL>
__global__ void __launch_bounds__(256) gather_kernel(const R* __restrict__ vtx, int64_t n_paths, int32_t M,
                                                     const R* __restrict__ points, int64_t n_points,
                                                     R* __restrict__ mean_out, R* __restrict__ var_out) {
  __shared__ double red[4][64 * PPL][2];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t base = (int64_t)blockIdx.x * (64 * PPL);
  R px[PPL], py[PPL], pz[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    int64_t i = base + lane + 64 * q;
    if (i >= n_points) i = n_points - 1;
    px[q] = points[i * D + 0];
    py[q] = points[i * D + 1];
    pz[q] = D == 3 ? points[i * D + 2] : (R)0;
  }
  const int64_t per = (n_paths + 3) / 4;
  const int64_t j0 = wave * per < n_paths ? wave * per : n_paths;
  const int64_t j1 = j0 + per < n_paths ? j0 + per : n_paths;
  double S[PPL], Q[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) S[q] = Q[q] = 0.0;
  for (int64_t j = j0; j < j1; j += kGatherChunk) {
    const int64_t je = j + kGatherChunk < j1 ? j + kGatherChunk : j1;
    R s[PPL], s2[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) s[q] = s2[q] = (R)0;
    for (int64_t jj = j; jj < je; ++jj) {
      const R* v = vtx + jj * M * 4;
      R c[PPL];
#pragma unroll
      for (int q = 0; q < PPL; ++q) c[q] = (R)0;
      for (int k = 0; k < M; ++k) {
        const R vx = v[4 * k + 0], vy = v[4 * k + 1], vz = v[4 * k + 2], w = v[4 * k + 3];
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
          const R dx = px[q] - vx, dy = py[q] - vy;
          R r2 = dx * dx + dy * dy;
          if constexpr (D == 3) {
            const R dz = pz[q] - vz;
            r2 += dz * dz;
            c[q] += w * inv_dist(r2);
          } else {
            c[q] += w * log2_dist2(r2);
          }
        }
      }
#pragma unroll
      for (int q = 0; q < PPL; ++q) {
        s[q] += c[q];
        s2[q] += c[q] * c[q];
      }
    }
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      S[q] += (double)s[q];
      Q[q] += (double)s2[q];
    }
  }
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    red[wave][lane + 64 * q][0] = S[q];
    red[wave][lane + 64 * q][1] = Q[q];
  }
  __syncthreads();
  if (wave != 0) return;
  // G's constant: 3D 1 / (4 pi); 2D -ln 2 / (4 pi) (G = -ln(rho^2) / (4 pi))
  const double kc = D == 3 ? 0.25 / 3.14159265358979323846 : -0.69314718055994530942 * 0.25 / 3.14159265358979323846;
  const double n = (double)n_paths;
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    const int64_t i = base + lane + 64 * q;
    if (i >= n_points) continue;
    double ts = 0.0, tq = 0.0;
    for (int w = 0; w < 4; ++w) {
      ts += red[w][lane + 64 * q][0];
      tq += red[w][lane + 64 * q][1];
    }
    const double mean = ts / n;
    mean_out[i] = (R)(kc * mean);
    if (var_out) {
      const double v = n > 1.0 ? (tq - ts * mean) / (n - 1.0) : 0.0;
      var_out[i] = (R)(kc * kc * (v > 0.0 ? v : 0.0));
    }
  }
}

// Per primitive (caller-id order): |q(c_T)| A_T, the datum of bc at the
// centroid times the area (the start weight of data-proportional starts), and
// A_T.
template <typename R, int D>
__global__ void __launch_bounds__(256) data_weight_kernel(wob::SceneView<R, D> s, wob::ProgramView<R> prog,
                                                          double* __restrict__ out) {
  const int32_t j = blockIdx.x * 256 + threadIdx.x;
  if (j >= s.n_prims) return;
  const wob::PrimGeo<R> g = wob::load_prim<R, D>(s, j);
  R n[3], c[3] = {0, 0, 0}, area;
  wob::load_normal<R, D>(s, j, n);
  if constexpr (D == 3) {
    R x[3];
    wob::cross3(g.e1, g.e2, x);
    area = (R)0.5 * sqrt(wob::dot3(x, x));
    for (int a = 0; a < 3; ++a) c[a] = g.v0[a] + (g.e1[a] + g.e2[a]) / (R)3;
  } else {
    area = sqrt(g.e1[0] * g.e1[0] + g.e1[1] * g.e1[1]);
    for (int a = 0; a < 2; ++a) c[a] = g.v0[a] + g.e1[a] / (R)2;
  }
  out[2 * (int64_t)g.id] = (double)(fabs(wob::boundary_datum<R, D>(prog, g, n, c)) * area);
  out[2 * (int64_t)g.id + 1] = (double)area;
}

template <typename R, int D>
wob_status data_weights(const wob_scene_s* sc, const wob_bc* bc, double* d_out) {
  const wob::ProgramView<R> prog = make_program<R>(sc, bc);
  const dim3 grid((unsigned)((sc->n_prims + 255) / 256)), block(256);
  hipLaunchKernelGGL((data_weight_kernel<R, D>), grid, block, 0, 0, view<R, D>(sc), prog, d_out);
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

template <typename R, int D>
wob_status launch_paths(const wob_scene_s* sc, const wob_bc* bc, const float* cdf, int64_t n_paths,
                        int32_t walk_len, uint64_t seed, void* vtx_out, int32_t* vtx_prim,
                        int32_t* vtx_m, hipStream_t st) {
  wob::WalkArgs<R, D> a;
  std::memset(&a, 0, sizeof(a));
  a.scene = view<R, D>(sc);
  a.prog = make_program<R>(sc, bc);
  // one lane per group of kFwdPathsPerLane paths: forward paths are short
  // (M - 1 lines from the boundary), so fewer per lane keep enough waves in
  // flight (2^20 paths of 4 vertices: 2.7 ms with 4 per lane, 4.0 ms with 8)
  constexpr int kFwdPathsPerLane = 4;
  a.n_points = (n_paths + kFwdPathsPerLane - 1) / kFwdPathsPerLane;
  a.N = kFwdPathsPerLane;
  a.M = walk_len;
  a.L = walk_len - 1;
  a.phi = (R)bc->domain;
  a.k0 = (uint32_t)(seed & 0xffffffffu);
  a.k1 = (uint32_t)(seed >> 32);
  a.lpp_shift = 0;
  a.form = wob::F_FWD;
  a.fwd_cdf = cdf;
  a.fwd_paths = n_paths;
  a.fwd_vtx = (R*)vtx_out;
  a.vtx_prim = vtx_prim;
  a.vtx_m = vtx_m;
  constexpr int B = kSolveBlock;
  const dim3 grid((unsigned)((a.n_points + B - 1) / B)), block(B);
  if (a.prog.type == wob::P_VERTEX)
    hipLaunchKernelGGL((wob::walk_kernel<R, D, wob::F_FWD, false, false, B, wob::X_VDATA>), grid, block,
                       wob::walk_lds_bytes(a.scene.stack_cap, B), st, a);
  else
    hipLaunchKernelGGL((wob::walk_kernel<R, D, wob::F_FWD, false, false, B>), grid, block,
                       wob::walk_lds_bytes(a.scene.stack_cap, B), st, a);
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

template <typename R, int D>
wob_status launch_gather(const void* vtx, int64_t n_paths, int32_t walk_len, const void* points,
                         int64_t n_points, void* mean_out, void* var_out, hipStream_t st) {
  const int64_t per_block = 64 * kGatherPPL;
  const dim3 grid((unsigned)((n_points + per_block - 1) / per_block)), block(256);
  hipLaunchKernelGGL((gather_kernel<R, D, kGatherPPL>), grid, block, 0, st, (const R*)vtx, n_paths, walk_len,
                     (const R*)points, n_points, (R*)mean_out, (R*)var_out);
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

bool on_device(int32_t device) {
  int dev = -1;
  return hipGetDevice(&dev) == hipSuccess && dev == device;
}

}  // namespace

extern "C" {

wob_status wob_starts_create(wob_scene sc, const double* weight, wob_starts* out) {
  if (!out) return WOB_E_ARG;
  *out = nullptr;
  if (!sc || !weight) return WOB_E_ARG;
  const int64_t T = sc->n_prims;
  double tot = 0.0;
  for (int64_t j = 0; j < T; ++j) {
    if (!(weight[j] >= 0.0) || !std::isfinite(weight[j])) return WOB_E_ARG;
    tot += weight[j];
  }
  if (!(tot > 0.0) || !std::isfinite(tot)) return WOB_E_ARG;
  if (!on_device(sc->device)) return WOB_E_DEVICE;
  // binary64 running sum in id order, rounded once per entry; last entry 1
  std::vector<float> cdf((size_t)T);
  double run = 0.0;
  for (int64_t j = 0; j < T; ++j) {
    run += weight[j];
    cdf[(size_t)j] = (float)(run / tot);
  }
  cdf[(size_t)T - 1] = 1.0f;
  wob_starts_s* s = new (std::nothrow) wob_starts_s();
  if (!s) return WOB_E_ALLOC;
  s->scene = sc;
  s->device = sc->device;
  s->n_prims = T;
  if (hipMalloc((void**)&s->d_cdf, sizeof(float) * (size_t)T) != hipSuccess) {
    delete s;
    return WOB_E_ALLOC;
  }
  if (hipMemcpy(s->d_cdf, cdf.data(), sizeof(float) * (size_t)T, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(s->d_cdf);
    delete s;
    return WOB_E_DEVICE;
  }
  *out = s;
  return WOB_OK;
}

wob_status wob_starts_from_data(wob_scene sc, const wob_bc* bc, double floor, wob_starts* out) {
  if (!out) return WOB_E_ARG;
  *out = nullptr;
  if (!sc || !bc || !(floor >= 0.0) || !std::isfinite(floor)) return WOB_E_ARG;
  if (check_data(bc) != WOB_OK) return WOB_E_ARG;
  if (!on_device(sc->device)) return WOB_E_DEVICE;
  const int64_t T = sc->n_prims;
  double* d_w = nullptr;
  if (hipMalloc((void**)&d_w, 2 * sizeof(double) * (size_t)T) != hipSuccess) return WOB_E_ALLOC;
  wob_status st;
  if (sc->precision == WOB_F32)
    st = sc->dim == 3 ? data_weights<float, 3>(sc, bc, d_w) : data_weights<float, 2>(sc, bc, d_w);
  else
    st = sc->dim == 3 ? data_weights<double, 3>(sc, bc, d_w) : data_weights<double, 2>(sc, bc, d_w);
  std::vector<double> wa(2 * (size_t)T);
  if (st == WOB_OK &&
      hipMemcpy(wa.data(), d_w, 2 * sizeof(double) * (size_t)T, hipMemcpyDeviceToHost) != hipSuccess)
    st = WOB_E_DEVICE;
  (void)hipFree(d_w);
  if (st != WOB_OK) return st;
  // w_T = (|q(c_T)| + floor * mean |q|) A_T, mean |q| = sum |q(c_T)| A_T / sum A_T:
  // the floor keeps every primitive's density positive
  double wsum = 0.0, asum = 0.0;
  for (int64_t j = 0; j < T; ++j) {
    wsum += wa[2 * (size_t)j];
    asum += wa[2 * (size_t)j + 1];
  }
  const double k = floor * wsum / asum;
  std::vector<double> w((size_t)T);
  for (int64_t j = 0; j < T; ++j) w[(size_t)j] = wa[2 * (size_t)j] + k * wa[2 * (size_t)j + 1];
  return wob_starts_create(sc, w.data(), out);
}

void wob_starts_free(wob_starts s) {
  if (!s) return;
  if (s->d_cdf) (void)hipFree(s->d_cdf);
  delete s;
}

wob_status wob_forward_paths(wob_scene sc, const wob_bc* bc, wob_starts starts, int64_t n_paths,
                             int32_t walk_len, uint64_t seed, void* vtx_out, int32_t* vtx_prim,
                             int32_t* vtx_m, void* stream) {
  if (!sc || !bc) return WOB_E_ARG;
  if (bc->domain != 1 && bc->domain != -1) return WOB_E_ARG;
  if (check_data(bc) != WOB_OK) return WOB_E_ARG;
  if (bc->formulation != WOB_F_AUTO && bc->formulation != WOB_F_SINGLE_LAYER) return WOB_E_UNSUPPORTED;
  if (bc->density != 0 || bc->sampling != WOB_SAMPLE_LINE) return WOB_E_UNSUPPORTED;
  if (bc->path_offset != 0) return WOB_E_UNSUPPORTED;  // forward paths have ids of their own
  if (sc->n_neumann != sc->n_prims) return WOB_E_UNSUPPORTED;  // Neumann data only
  if (walk_len < 1 || walk_len >= 65535) return WOB_E_ARG;
  if (n_paths < 0 || n_paths >= ((int64_t)1 << 32)) return WOB_E_ARG;  // path id is a 32-bit counter word
  if (n_paths > 0 && !vtx_out) return WOB_E_ARG;
  const size_t rec = 4 * (sc->precision == WOB_F32 ? sizeof(float) : sizeof(double));
  if ((uintptr_t)vtx_out % rec != 0) return WOB_E_ARG;  // records are stored whole
  if (starts && (starts->scene != sc || starts->n_prims != sc->n_prims)) return WOB_E_ARG;
  if (n_paths == 0) return WOB_OK;
  if (!on_device(sc->device)) return WOB_E_DEVICE;
  const float* cdf = starts ? starts->d_cdf : sc->d_area_cdf;
  hipStream_t st = (hipStream_t)stream;
  if (sc->precision == WOB_F32)
    return sc->dim == 3 ? launch_paths<float, 3>(sc, bc, cdf, n_paths, walk_len, seed, vtx_out, vtx_prim, vtx_m, st)
                        : launch_paths<float, 2>(sc, bc, cdf, n_paths, walk_len, seed, vtx_out, vtx_prim, vtx_m, st);
  return sc->dim == 3 ? launch_paths<double, 3>(sc, bc, cdf, n_paths, walk_len, seed, vtx_out, vtx_prim, vtx_m, st)
                      : launch_paths<double, 2>(sc, bc, cdf, n_paths, walk_len, seed, vtx_out, vtx_prim, vtx_m, st);
}

wob_status wob_forward_gather(wob_scene sc, const void* vtx, int64_t n_paths, int32_t walk_len,
                              const void* points, int64_t n_points, void* mean_out, void* var_out,
                              void* stream) {
  if (!sc || n_paths < 1 || walk_len < 1 || walk_len >= 65535 || n_points < 0) return WOB_E_ARG;
  if (n_points > 0 && (!vtx || !points || !mean_out)) return WOB_E_ARG;
  if (var_out && n_paths < 2) return WOB_E_ARG;
  if (n_points == 0) return WOB_OK;
  if (!on_device(sc->device)) return WOB_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  if (sc->precision == WOB_F32)
    return sc->dim == 3 ? launch_gather<float, 3>(vtx, n_paths, walk_len, points, n_points, mean_out, var_out, st)
                        : launch_gather<float, 2>(vtx, n_paths, walk_len, points, n_points, mean_out, var_out, st);
  return sc->dim == 3 ? launch_gather<double, 3>(vtx, n_paths, walk_len, points, n_points, mean_out, var_out, st)
                      : launch_gather<double, 2>(vtx, n_paths, walk_len, points, n_points, mean_out, var_out, st);
}

}  // extern "C"
