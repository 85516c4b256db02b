// C ABI of the walk-on-boundary library: argument validation, scene upload and
// kernel dispatch.  The kernels themselves live in walk.hpp / device.hpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <new>
#include <vector>

#include "../../include/wob.h"
#include "bvh_build.hpp"
#include "internal.hpp"


using namespace wobi;

namespace {

// Leaves of at most two primitives: a leaf test loops over the most
// primitives any parked lane has, so small leaves keep the lanes busy
// (icosphere benchmark, leaves of at most 1 / 2 / 4: 72.5 / 68.9 / 71.2 ms).
constexpr int kMaxLeaf = 2;

// Round a double to binary16 toward -inf / +inf (|v| well inside the range).
_Float16 step_h(_Float16 h, bool up) {
  uint16_t u;
  std::memcpy(&u, &h, 2);
  if ((u & 0x7fff) == 0) u = up ? 0x0001 : 0x8001;  // +-0 -> the smallest subnormal
  else if ((u & 0x8000) != 0) u = up ? u - 1 : u + 1;
  else u = up ? u + 1 : u - 1;
  std::memcpy(&h, &u, 2);
  return h;
}
_Float16 down_h(double v) {
  _Float16 h = (_Float16)v;
  if ((double)h > v) h = step_h(h, false);
  return h;
}
_Float16 up_h(double v) {
  _Float16 h = (_Float16)v;
  if ((double)h < v) h = step_h(h, true);
  return h;
}

// Frame of the stored boxes: y' = (y - c) k with c the root box's centre
// (rounded to R, as the kernels use it) and k a power of two, |y'| <= 1.
template <typename R>
void box_frame(const wobhost::Box& root, int dim, double c[3], double& k) {
  double half = 0.0;
  for (int a = 0; a < 3; ++a) {
    c[a] = a < dim ? (double)(R)(0.5 * (root.lo[a] + root.hi[a])) : 0.0;
    if (a < dim) half = std::fmax(half, std::fmax(std::fabs(root.lo[a] - c[a]), std::fabs(root.hi[a] - c[a])));
  }
  k = half > 0.0 ? std::ldexp(1.0, -std::ilogb(half) - 1) : 1.0;
}

// A box in the frame, padded so that the FMA slab test in R precision never
// misses a primitive that the exact test would hit, stored rounded outward
// into slot `which` (FP32 scenes: binary16 pairs, lo in the low half of each
// word).
template <typename R, int D, typename Node>
void store_box(const wobhost::Box& b, const double c[3], double k, Node& n, int which) {
  double l[3], h[3], mag = 0.0;
  for (int a = 0; a < D; ++a) {
    l[a] = (b.lo[a] - c[a]) * k;
    h[a] = (b.hi[a] - c[a]) * k;
    mag = std::fmax(mag, std::fmax(std::fabs(l[a]), std::fabs(h[a])));
  }
  const double pad = (sizeof(R) == 4 ? 0x1p-19 : 0x1p-45) * (mag + 1.0);
  for (int a = 0; a < D; ++a) {
    if constexpr (sizeof(R) == 4) {
      const _Float16 lo = down_h(l[a] - pad), hi = up_h(h[a] + pad);
      uint16_t ul, uh;
      std::memcpy(&ul, &lo, 2);
      std::memcpy(&uh, &hi, 2);
      n.box[which][a] = (uint32_t)ul | ((uint32_t)uh << 16);
    } else {
      n.lo[which][a] = (R)(l[a] - pad);
      n.hi[which][a] = (R)(h[a] + pad);
    }
  }
}

// An unused slot: an empty box (lo above hi on every axis), which no line
// crosses, whatever the signs of its direction (both slab tests take the near
// side by the direction's sign), and the entry kPop, so that even a crossed
// empty slot would only pop the stack.
template <typename R, typename Node>
void store_empty(Node& n, int which) {
  for (int a = 0; a < 3; ++a) {
    if constexpr (sizeof(R) == 4) {
      n.box[which][a] = 0x7bffu | (0xfbffu << 16);  // lo = +65504, hi = -65504 (binary16)
    } else {
      n.lo[which][a] = (R)1e300;
      n.hi[which][a] = (R)-1e300;
    }
  }
  n.child[which] = wob::kPop;
}

template <typename R, int D>
wob_status upload_scene(wob_scene_s* sc, const std::vector<double>& v, const int32_t* prims,
                        const uint8_t* kind, const double* alpha, const wobhost::Bvh& bvh,
                        hipStream_t st) {
  using Node = typename wob::Rec<R, D>::Node;
  using Prim = typename wob::Rec<R, D>::Prim;
  const int64_t T = sc->n_prims;
  // 4-wide interior records, in pre-order (a record's first interior child is
  // the next record).  A record takes its binary node's two children and
  // opens the interior entry of largest box measure until it holds kArity
  // entries; every interior entry it keeps becomes a record of its own.  In
  // the builder's flat array the first child of node i is node i + 1, the
  // second the first node after the first child's subtree.
  const auto& fn = bvh.nodes;
  const int dim = D;
  double fc[3], fk;
  box_frame<R>(fn[0].box, D, fc, fk);
  std::vector<Node> nodes;
  int max_ent = wob::kArity;
  // deepest stack a line can need below a record: its own pushes (entries - 1)
  // plus the deepest of its interior children
  std::function<int32_t(size_t, int32_t*)> emit = [&](size_t i, int32_t* need) -> int32_t {
    std::vector<size_t> ent = {(size_t)fn[i].child, (size_t)fn[(size_t)fn[i].child].skip};
    while ((int)ent.size() < max_ent) {
      int best = -1;
      double bm = -1.0;
      for (int q = 0; q < (int)ent.size(); ++q)
        if (fn[ent[q]].child >= 0) {
          const double mq = wobhost::box_measure(fn[ent[q]].box, dim);
          if (mq > bm) {
            bm = mq;
            best = q;
          }
        }
      if (best < 0) break;
      const size_t c = ent[best];
      ent.erase(ent.begin() + best);
      ent.insert(ent.begin() + best, {(size_t)fn[c].child, (size_t)fn[(size_t)fn[c].child].skip});
    }
    const int32_t r = (int32_t)nodes.size();
    nodes.emplace_back();
    std::memset(&nodes[r], 0, sizeof(Node));
    int32_t deepest = 0;
    int32_t child[wob::kArity];
    for (int q = 0; q < (int)ent.size(); ++q) {
      if (fn[ent[q]].child >= 0) {
        int32_t sub = 0;
        child[q] = emit(ent[q], &sub);
        deepest = std::max(deepest, sub);
      } else {
        child[q] = fn[ent[q]].child;  // leaf code
      }
    }
    Node& n = nodes[r];
    for (int q = 0; q < wob::kArity; ++q) {
      if (q < (int)ent.size()) {
        store_box<R, D>(fn[ent[q]].box, fc, fk, n, q);
        n.child[q] = child[q];
      } else {
        store_empty<R>(n, q);
      }
    }
    *need = (int32_t)ent.size() - 1 + deepest;
    return r;
  };
  int32_t need = 0;
  int32_t root = fn[0].child >= 0 ? emit(0, &need) : fn[0].child;
  if (need > wob::kMaxDepth) {
    // a degenerate tree whose 4-wide records could push more than a lane's
    // stack holds: two entries per record (the binary tree, whose stack needs
    // at most its depth - 1 entries)
    nodes.clear();
    max_ent = 2;
    need = 0;
    root = emit(0, &need);
  }
  const int32_t n_inner = (int32_t)nodes.size();
  // every interior entry points to a later record (pre-order), so a traversal
  // never returns to a record it left: the walk ends on every line
  for (int32_t r = 0; r < n_inner; ++r)
    for (int q = 0; q < wob::kArity; ++q) {
      const int32_t c = nodes[r].child[q];
      if (c >= 0 && (c <= r || c >= n_inner)) return WOB_E_MESH;
    }
  // the traversal addresses records by a 32-bit byte offset
  if ((uint64_t)n_inner * sizeof(Node) > 0xffffffffull) return WOB_E_ARG;
  sc->n_inner = n_inner;
  for (int a = 0; a < 3; ++a) sc->frame_c[a] = fc[a];
  sc->frame_k = fk;
  sc->root = root;
  sc->stack_cap = std::max(need, 1);
  if (sc->stack_cap > wob::kMaxDepth) return WOB_E_MESH;
  std::vector<Prim> recs((size_t)T);
  std::vector<R> normals((size_t)T * 4, (R)0);
  std::vector<int32_t> leaf_of_id((size_t)T);
  std::vector<double> area((size_t)T, 0.0);
  for (int64_t j = 0; j < T; ++j) {
    const int32_t id = bvh.order[j];
    leaf_of_id[id] = (int32_t)j;
    Prim& p = recs[j];
    std::memset(&p, 0, sizeof(Prim));
    const int32_t* ix = prims + (int64_t)id * D;
    const int k = kind ? kind[id] : 0;
    p.idkind = id | (k << wob::kIdBits);
    p.alpha = alpha ? (R)alpha[id] : (R)0;
    double e1d[3] = {0, 0, 0}, e2d[3] = {0, 0, 0};
    if constexpr (D == 3) {
      for (int a = 0; a < 3; ++a) {
        const double v0 = v[(int64_t)ix[0] * 3 + a], v1 = v[(int64_t)ix[1] * 3 + a],
                     v2 = v[(int64_t)ix[2] * 3 + a];
        p.v0[a] = (R)v0;
        e1d[a] = v1 - v0;
        e2d[a] = v2 - v0;
        p.e1[a] = (R)e1d[a];
        p.e2[a] = (R)e2d[a];
      }
      double n[3] = {e1d[1] * e2d[2] - e1d[2] * e2d[1], e1d[2] * e2d[0] - e1d[0] * e2d[2],
                     e1d[0] * e2d[1] - e1d[1] * e2d[0]};
      const double l = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      for (int a = 0; a < 3; ++a) normals[4 * j + a] = (R)(n[a] / l);
      area[id] = 0.5 * l;
    } else {
      for (int a = 0; a < 2; ++a) {
        const double v0 = v[(int64_t)ix[0] * 2 + a], v1 = v[(int64_t)ix[1] * 2 + a];
        p.v0[a] = (R)v0;
        e1d[a] = v1 - v0;
        p.e[a] = (R)e1d[a];
      }
      const double l = std::sqrt(e1d[0] * e1d[0] + e1d[1] * e1d[1]);
      normals[4 * j + 0] = (R)(e1d[1] / l);
      normals[4 * j + 1] = (R)(-e1d[0] / l);
      area[id] = l;
    }
  }
  sc->node_bytes = sizeof(Node);
  sc->prim_bytes = sizeof(Prim);
  // cumulative area fraction in caller-id order: summed in binary64, rounded
  // once to binary32 (an area-uniform pick compares a binary32 uniform with it)
  std::vector<float> cdf((size_t)T);
  double tot = 0.0;
  for (int64_t j = 0; j < T; ++j) tot += area[j];
  double run = 0.0;
  for (int64_t j = 0; j < T; ++j) {
    run += area[j];
    cdf[j] = (float)(run / tot);
  }
  cdf[T - 1] = 1.0f;
  sc->area_total = tot;
  // a guide to the area CDF: with K = 2^shift >= T buckets (at most 2^24),
  // guide[b] is the first index whose cdf exceeds b / K, so the first index
  // whose cdf exceeds a binary32 uniform u lies in [guide[b], guide[b + 1]]
  // for b = floor(u K) (exact: K is a power of two); the area-uniform pick
  // searches there and finds the same index as a search of the whole CDF
  int shift = 0;
  while ((int64_t)1 << shift < T && shift < 24) ++shift;
  const int64_t K = (int64_t)1 << shift;
  std::vector<int32_t> guide((size_t)K + 1);
  {
    int64_t i = 0;
    for (int64_t b = 0; b <= K; ++b) {
      const double t = (double)b / (double)K;
      while (i < T - 1 && !((double)cdf[i] > t)) ++i;
      guide[b] = (int32_t)i;
    }
  }
  sc->guide_shift = shift;
  // the vertices (already rounded to R) and each primitive's vertex ids, for
  // per-vertex boundary data
  std::vector<R> verts_r(v.size());
  for (size_t i = 0; i < v.size(); ++i) verts_r[i] = (R)v[i];
  const size_t nb = std::max(nodes.size(), (size_t)1) * sizeof(Node), pb = recs.size() * sizeof(Prim),
               lb = leaf_of_id.size() * sizeof(int32_t), qb = normals.size() * sizeof(R),
               cb = sizeof(float) * T, vb = verts_r.size() * sizeof(R),
               ib = (size_t)T * D * sizeof(int32_t), sb = sizeof(unsigned long long),
               gb = guide.size() * sizeof(int32_t);
  if (hipMalloc(&sc->d_nodes, nb) != hipSuccess) return WOB_E_ALLOC;
  if (hipMalloc(&sc->d_prims, pb) != hipSuccess) return WOB_E_ALLOC;
  if (hipMalloc(&sc->d_normals, qb) != hipSuccess) return WOB_E_ALLOC;
  if (hipMalloc((void**)&sc->d_leaf_of_id, lb) != hipSuccess) return WOB_E_ALLOC;
  if (hipMalloc((void**)&sc->d_area_cdf, cb) != hipSuccess) return WOB_E_ALLOC;
  if (hipMalloc((void**)&sc->d_area_guide, gb) != hipSuccess) return WOB_E_ALLOC;
  if (hipMalloc(&sc->d_verts, vb) != hipSuccess) return WOB_E_ALLOC;
  if (hipMalloc((void**)&sc->d_vid, ib) != hipSuccess) return WOB_E_ALLOC;
  if (hipMalloc((void**)&sc->d_status, sb) != hipSuccess) return WOB_E_ALLOC;
  // copies on the caller's stream, waited for before the host arrays go
  const auto put = [st](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st) == hipSuccess;
  };
  bool ok = put(sc->d_normals, normals.data(), qb) && put(sc->d_prims, recs.data(), pb) &&
            put(sc->d_leaf_of_id, leaf_of_id.data(), lb) && put(sc->d_area_cdf, cdf.data(), cb) &&
            put(sc->d_area_guide, guide.data(), gb) &&
            put(sc->d_verts, verts_r.data(), vb) && put(sc->d_vid, prims, ib) &&
            hipMemsetAsync(sc->d_status, 0, sb, st) == hipSuccess;
  if (ok && !nodes.empty()) ok = put(sc->d_nodes, nodes.data(), nodes.size() * sizeof(Node));
  // the copies must end before the host arrays are released, also on failure
  if (hipStreamSynchronize(st) != hipSuccess || !ok) return WOB_E_DEVICE;
  sc->n_verts = (int64_t)(v.size() / D);
  sc->device_bytes = (int64_t)(nb + pb + lb + qb + cb + vb + ib + sb + gb);
  return WOB_OK;
}

enum Mode { MODE_SOLVE = 0, MODE_TRACE = 1, MODE_COUNT = 2 };

// VX: X_VDATA for per-vertex data (its own instantiation of each kernel)
template <typename R, int D, int FORM, int VX>
void launch_form(const wob::WalkArgs<R, D>& a0, int mode, hipStream_t st) {
  constexpr int B = kSolveBlock;
  // plain single-layer solves pool two points per lane group: at most 32
  // lanes per point (the kernel instantiation decides, by the same rule)
  const bool pooled = mode == MODE_SOLVE && !(a0.grad_out || a0.path_grad_out) && !a0.cv_g &&
                      wob::pools_points(FORM, VX, false, false);
  wob::WalkArgs<R, D> a = a0;
  a.lpp_shift = lpp_shift_for(a0.N, B, pooled);
  const int ppb = B >> a.lpp_shift;
  const dim3 grid((unsigned)((a.n_points + ppb - 1) / ppb)), block(B);
  const size_t lds = wob::walk_lds_bytes(a.scene.stack_cap, B);  // traversal stacks, held leaves
  if constexpr (FORM != wob::F_FWD) {
    if (a.grad_out || a.path_grad_out) {  // value and gradient along the same paths
      if (mode == MODE_TRACE)
        hipLaunchKernelGGL((wob::walk_kernel<R, D, FORM, true, false, B, wob::X_GRAD | VX>), grid, block, lds, st,
                           a);
      else
        hipLaunchKernelGGL((wob::walk_kernel<R, D, FORM, false, false, B, wob::X_GRAD | VX>), grid, block, lds,
                           st, a);
      return;
    }
  }
  if constexpr (D == 3 && (FORM == wob::F_SL || FORM == wob::F_SL_RIS)) {
    if (a.cv_g) {
      if (mode == MODE_SOLVE)
        hipLaunchKernelGGL((wob::walk_kernel<R, D, FORM, false, false, B, wob::X_CV | VX>), grid, block, lds, st,
                           a);
      else if (mode == MODE_TRACE)
        hipLaunchKernelGGL((wob::walk_kernel<R, D, FORM, true, false, B, wob::X_CV | VX>), grid, block, lds, st, a);
      else
        hipLaunchKernelGGL((wob::walk_kernel<R, D, FORM, false, true, B, wob::X_CV | VX>), grid, block, lds, st, a);
      return;
    }
  }
  if (mode == MODE_SOLVE)
    hipLaunchKernelGGL((wob::walk_kernel<R, D, FORM, false, false, B, VX>), grid, block, lds, st, a);
  else if (mode == MODE_TRACE)
    hipLaunchKernelGGL((wob::walk_kernel<R, D, FORM, true, false, B, VX>), grid, block, lds, st, a);
  else
    hipLaunchKernelGGL((wob::walk_kernel<R, D, FORM, false, true, B, VX>), grid, block, lds, st, a);
}

template <typename R, int D, int VX>
void launch_walk_vx(const wob::WalkArgs<R, D>& a, int mode, hipStream_t st) {
  if (a.form == wob::F_DL) launch_form<R, D, wob::F_DL, VX>(a, mode, st);
  else if (a.form == wob::F_DIRECT) launch_form<R, D, wob::F_DIRECT, VX>(a, mode, st);
  else if (a.form == wob::F_SL_RIS) launch_form<R, D, wob::F_SL_RIS, VX>(a, mode, st);
  else launch_form<R, D, wob::F_SL, VX>(a, mode, st);
}

template <typename R, int D>
void launch_walk(const wob::WalkArgs<R, D>& a, int mode, hipStream_t st) {
  if (a.prog.type == wob::P_VERTEX) launch_walk_vx<R, D, wob::X_VDATA>(a, mode, st);
  else launch_walk_vx<R, D, wob::X_NONE>(a, mode, st);
}

wob_status run_walk(wob_scene sc, const void* points, const int32_t* point_prim, int64_t n_points,
                    const wob_bc* bc, int32_t samples, int32_t walk_len, uint64_t seed,
                    const uint32_t* point_ids, void* mean_out, void* var_out, void* path_out,
                    int32_t* vtx_prim, int32_t* vtx_m, uint64_t* counters, int mode,
                    void* stream, const float* cv_g = nullptr, const float* cv_g0 = nullptr,
                    void* grad_out = nullptr, void* grad_var_out = nullptr, void* path_grad_out = nullptr,
                    const void* anchor_pts = nullptr, const int32_t* anchor_prim = nullptr) {
  Plan pl;
  wob_status s = plan_walk(sc, bc, samples, walk_len, &pl);
  if (s != WOB_OK) return s;
  if (cv_g && (sc->dim != 3 || sc->precision != WOB_F32 || pl.form != WOB_F_SINGLE_LAYER ||
               bc->density || sc->n_dirichlet > 0))
    return WOB_E_UNSUPPORTED;
  const bool grad = grad_out || path_grad_out;
  // gradients: evaluation points inside the domain, no density mode, no control variate
  if (grad && (point_prim || bc->density || cv_g)) return WOB_E_UNSUPPORTED;
  // the boundary split: both arrays or neither, gradients of the double layer only
  if ((anchor_pts != nullptr) != (anchor_prim != nullptr)) return WOB_E_ARG;
  if (anchor_prim && (!grad || pl.form != WOB_F_DOUBLE_LAYER)) return WOB_E_UNSUPPORTED;
  if (grad && mode == MODE_SOLVE && n_points > 0 && !grad_out) return WOB_E_ARG;
  if (mode == MODE_SOLVE && grad_var_out && samples < 2) return WOB_E_ARG;
  if (n_points < 0 || (n_points > 0 && !points)) return WOB_E_ARG;
  if (n_points >= (int64_t)1 << 32) return WOB_E_ARG;  // point index is a 32-bit counter word
  if (mode == MODE_SOLVE && n_points > 0 && !mean_out) return WOB_E_ARG;
  if (mode == MODE_SOLVE && var_out && samples < 2) return WOB_E_ARG;
  if (mode == MODE_TRACE && n_points > 0 && !path_out) return WOB_E_ARG;
  if (mode == MODE_COUNT && !counters) return WOB_E_ARG;
  if (n_points == 0) return WOB_OK;
  hipStream_t st = (hipStream_t)stream;
  if (sc->precision == WOB_F32) {
    if (sc->dim == 3) {
      auto a = make_args<float, 3>(sc, pl, points, point_prim, n_points, bc, samples, walk_len, seed);
      a.mean_out = (float*)mean_out; a.var_out = (float*)var_out; a.path_out = (float*)path_out;
      a.grad_out = (float*)grad_out; a.grad_var_out = (float*)grad_var_out; a.path_grad_out = (float*)path_grad_out;
      a.vtx_prim = vtx_prim; a.vtx_m = vtx_m; a.counters = (unsigned long long*)counters;
      a.point_ids = point_ids;
      a.cv_g = cv_g;
      a.cv_g0 = cv_g0 ? cv_g0 : cv_g;
      a.anchor_pts = (const float*)anchor_pts;
      a.anchor_prim = anchor_prim;
      launch_walk<float, 3>(a, mode, st);
    } else {
      auto a = make_args<float, 2>(sc, pl, points, point_prim, n_points, bc, samples, walk_len, seed);
      a.mean_out = (float*)mean_out; a.var_out = (float*)var_out; a.path_out = (float*)path_out;
      a.grad_out = (float*)grad_out; a.grad_var_out = (float*)grad_var_out; a.path_grad_out = (float*)path_grad_out;
      a.vtx_prim = vtx_prim; a.vtx_m = vtx_m; a.counters = (unsigned long long*)counters;
      a.point_ids = point_ids;
      a.anchor_pts = (const float*)anchor_pts;
      a.anchor_prim = anchor_prim;
      launch_walk<float, 2>(a, mode, st);
    }
  } else {
    if (sc->dim == 3) {
      auto a = make_args<double, 3>(sc, pl, points, point_prim, n_points, bc, samples, walk_len, seed);
      a.mean_out = (double*)mean_out; a.var_out = (double*)var_out; a.path_out = (double*)path_out;
      a.grad_out = (double*)grad_out; a.grad_var_out = (double*)grad_var_out; a.path_grad_out = (double*)path_grad_out;
      a.vtx_prim = vtx_prim; a.vtx_m = vtx_m; a.counters = (unsigned long long*)counters;
      a.point_ids = point_ids;
      a.anchor_pts = (const double*)anchor_pts;
      a.anchor_prim = anchor_prim;
      launch_walk<double, 3>(a, mode, st);
    } else {
      auto a = make_args<double, 2>(sc, pl, points, point_prim, n_points, bc, samples, walk_len, seed);
      a.mean_out = (double*)mean_out; a.var_out = (double*)var_out; a.path_out = (double*)path_out;
      a.grad_out = (double*)grad_out; a.grad_var_out = (double*)grad_var_out; a.path_grad_out = (double*)path_grad_out;
      a.vtx_prim = vtx_prim; a.vtx_m = vtx_m; a.counters = (unsigned long long*)counters;
      a.point_ids = point_ids;
      a.anchor_pts = (const double*)anchor_pts;
      a.anchor_prim = anchor_prim;
      launch_walk<double, 2>(a, mode, st);
    }
  }
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

}  // namespace

extern "C" {

const char* wob_status_string(wob_status s) {
  switch (s) {
    case WOB_OK: return "ok";
    case WOB_E_ARG: return "invalid argument";
    case WOB_E_ALLOC: return "allocation failed";
    case WOB_E_DEVICE: return "HIP runtime error";
    case WOB_E_MESH: return "invalid mesh";
    case WOB_E_UNSUPPORTED: return "unsupported combination";
    case WOB_E_TOO_LARGE: return "beyond the capacity of an allocation-free entry point";
  }
  return "unknown status";
}

}  // extern "C"

namespace {

// wob_build_bvh on host arrays, the scene's copies on `st`.
wob_status build_scene(int32_t dim, int32_t precision, const double* verts, int64_t n_verts,
                       const int32_t* prims, int64_t n_prims, const uint8_t* kind, const double* alpha,
                       hipStream_t st, wob_scene* out) {
  // vertices rounded to the scene precision: both the walk and any external
  // checker then see the same geometry
  std::vector<double> v((size_t)(n_verts * dim));
  for (int64_t i = 0; i < n_verts * dim; ++i) {
    const double x = verts[i];
    if (!std::isfinite(x)) return WOB_E_MESH;
    v[i] = precision == WOB_F32 ? (double)(float)x : x;
    if (!std::isfinite(v[i])) return WOB_E_MESH;
  }
  std::vector<wobhost::Box> boxes((size_t)n_prims);
  int32_t nd = 0, nn = 0, nr = 0;
  for (int64_t j = 0; j < n_prims; ++j) {
    wobhost::Box b;
    for (int a = 0; a < 3; ++a) {
      b.lo[a] = INFINITY;
      b.hi[a] = -INFINITY;
    }
    double p[3][3] = {{0}};
    for (int c = 0; c < dim; ++c) {
      const int32_t ix = prims[j * dim + c];
      if (ix < 0 || ix >= n_verts) return WOB_E_MESH;
      for (int a = 0; a < dim; ++a) {
        p[c][a] = v[(int64_t)ix * dim + a];
        b.lo[a] = std::fmin(b.lo[a], p[c][a]);
        b.hi[a] = std::fmax(b.hi[a], p[c][a]);
      }
    }
    for (int a = dim; a < 3; ++a) b.lo[a] = b.hi[a] = 0.0;
    // zero-length segment / zero-area triangle
    if (dim == 2) {
      if (p[0][0] == p[1][0] && p[0][1] == p[1][1]) return WOB_E_MESH;
    } else {
      const double e1[3] = {p[1][0] - p[0][0], p[1][1] - p[0][1], p[1][2] - p[0][2]};
      const double e2[3] = {p[2][0] - p[0][0], p[2][1] - p[0][1], p[2][2] - p[0][2]};
      const double c0 = e1[1] * e2[2] - e1[2] * e2[1], c1 = e1[2] * e2[0] - e1[0] * e2[2],
                   c2 = e1[0] * e2[1] - e1[1] * e2[0];
      if (c0 == 0.0 && c1 == 0.0 && c2 == 0.0) return WOB_E_MESH;
    }
    boxes[j] = b;
    const int k = kind ? kind[j] : WOB_BC_DIRICHLET;
    if (k == WOB_BC_DIRICHLET) ++nd;
    else if (k == WOB_BC_NEUMANN) ++nn;
    else if (k == WOB_BC_ROBIN) ++nr;
    else return WOB_E_ARG;
    if (alpha && !std::isfinite(alpha[j])) return WOB_E_ARG;
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return WOB_E_DEVICE;
  wobhost::Bvh bvh = wobhost::build_bvh(dim, boxes, kMaxLeaf);
  wob_scene_s* sc = new (std::nothrow) wob_scene_s();
  if (!sc) return WOB_E_ALLOC;
  sc->dim = dim;
  sc->precision = precision;
  sc->device = dev;
  sc->n_prims = n_prims;
  sc->n_nodes = (int64_t)bvh.nodes.size();
  sc->n_leaves = bvh.n_leaves;
  sc->depth = bvh.depth;
  sc->max_leaf = bvh.max_leaf;
  sc->n_dirichlet = nd;
  sc->n_neumann = nn;
  sc->n_robin = nr;
  wob_status s;
  if (precision == WOB_F32)
    s = dim == 3 ? upload_scene<float, 3>(sc, v, prims, kind, alpha, bvh, st)
                 : upload_scene<float, 2>(sc, v, prims, kind, alpha, bvh, st);
  else
    s = dim == 3 ? upload_scene<double, 3>(sc, v, prims, kind, alpha, bvh, st)
                 : upload_scene<double, 2>(sc, v, prims, kind, alpha, bvh, st);
  if (s != WOB_OK) {
    wob_free(sc);
    return s;
  }
  *out = sc;
  return WOB_OK;
}

wob_status check_build_args(int32_t dim, int32_t precision, const double* verts, int64_t n_verts,
                            const int32_t* prims, int64_t n_prims, wob_scene* out) {
  if (!out) return WOB_E_ARG;
  *out = nullptr;
  if (dim != 2 && dim != 3) return WOB_E_ARG;
  if (precision != WOB_F32 && precision != WOB_F64) return WOB_E_ARG;
  if (!verts || !prims || n_verts <= 0 || n_prims <= 0) return WOB_E_ARG;
  if (n_prims >= ((int64_t)1 << 27)) return WOB_E_ARG;  // leaf entries pack the first index in 27 bits
  if (n_verts > ((int64_t)1 << 31) - 1) return WOB_E_ARG;  // vertex ids are int32
  return WOB_OK;
}

}  // namespace

extern "C" {

wob_status wob_build_bvh(int32_t dim, int32_t precision, const double* verts, int64_t n_verts,
                         const int32_t* prims, int64_t n_prims, const uint8_t* kind,
                         const double* alpha, wob_scene* out) {
  const wob_status a = check_build_args(dim, precision, verts, n_verts, prims, n_prims, out);
  if (a != WOB_OK) return a;
  return build_scene(dim, precision, verts, n_verts, prims, n_prims, kind, alpha, nullptr, out);
}

wob_status wob_build_bvh_ex(int32_t dim, int32_t precision, const double* verts, int64_t n_verts,
                            const int32_t* prims, int64_t n_prims, const uint8_t* kind,
                            const double* alpha, int32_t inputs_on_device, void* stream,
                            wob_scene* out) {
  const wob_status a = check_build_args(dim, precision, verts, n_verts, prims, n_prims, out);
  if (a != WOB_OK) return a;
  if (inputs_on_device != 0 && inputs_on_device != 1) return WOB_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (!inputs_on_device)
    return build_scene(dim, precision, verts, n_verts, prims, n_prims, kind, alpha, st, out);
  // the tree is built on the host: bring the mesh over on the caller's stream
  std::vector<double> hv((size_t)(n_verts * dim)), ha(alpha ? (size_t)n_prims : 0);
  std::vector<int32_t> hp((size_t)(n_prims * dim));
  std::vector<uint8_t> hk(kind ? (size_t)n_prims : 0);
  const auto get = [st](void* dst, const void* src, size_t bytes) {
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st) == hipSuccess;
  };
  bool ok = get(hv.data(), verts, hv.size() * sizeof(double)) &&
            get(hp.data(), prims, hp.size() * sizeof(int32_t));
  if (ok && kind) ok = get(hk.data(), kind, hk.size());
  if (ok && alpha) ok = get(ha.data(), alpha, ha.size() * sizeof(double));
  // wait also after a failed enqueue: the host arrays are released on return
  if (hipStreamSynchronize(st) != hipSuccess || !ok) return WOB_E_DEVICE;
  return build_scene(dim, precision, hv.data(), n_verts, hp.data(), n_prims, kind ? hk.data() : nullptr,
                     alpha ? ha.data() : nullptr, st, out);
}

void wob_free(wob_scene sc) {
  if (!sc) return;
  if (sc->d_nodes) (void)hipFree(sc->d_nodes);
  if (sc->d_prims) (void)hipFree(sc->d_prims);
  if (sc->d_normals) (void)hipFree(sc->d_normals);
  if (sc->d_area_cdf) (void)hipFree(sc->d_area_cdf);
  if (sc->d_area_guide) (void)hipFree(sc->d_area_guide);
  if (sc->d_leaf_of_id) (void)hipFree(sc->d_leaf_of_id);
  if (sc->d_status) (void)hipFree(sc->d_status);
  if (sc->d_verts) (void)hipFree(sc->d_verts);
  if (sc->d_vid) (void)hipFree(sc->d_vid);
  delete sc;
}

wob_status wob_last_device_status(wob_scene sc, uint64_t* nonfinite_paths, void* stream) {
  if (!sc || !nonfinite_paths) return WOB_E_ARG;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != sc->device) return WOB_E_DEVICE;
  hipStream_t st = (hipStream_t)stream;
  unsigned long long v = 0;
  if (hipMemcpyAsync(&v, sc->d_status, sizeof(v), hipMemcpyDeviceToHost, st) != hipSuccess)
    return WOB_E_DEVICE;
  if (hipMemsetAsync(sc->d_status, 0, sizeof(v), st) != hipSuccess) return WOB_E_DEVICE;
  if (hipStreamSynchronize(st) != hipSuccess) return WOB_E_DEVICE;
  *nonfinite_paths = (uint64_t)v;
  return WOB_OK;
}

wob_status wob_get_scene_info(wob_scene sc, wob_scene_info* info) {
  if (!sc || !info) return WOB_E_ARG;
  std::memset(info, 0, sizeof(*info));
  info->dim = sc->dim;
  info->precision = sc->precision;
  info->n_prims = sc->n_prims;
  info->n_nodes = sc->n_nodes;
  info->n_leaves = sc->n_leaves;
  info->depth = sc->depth;
  info->max_leaf = sc->max_leaf;
  info->device_bytes = sc->device_bytes;
  info->node_bytes = sc->node_bytes;
  info->prim_bytes = sc->prim_bytes;
  info->n_dirichlet = sc->n_dirichlet;
  info->n_neumann = sc->n_neumann;
  info->n_robin = sc->n_robin;
  info->n_verts = sc->n_verts;
  return WOB_OK;
}

int32_t wob_lines_per_path(wob_scene sc, const wob_bc* bc, int32_t walk_len) {
  Plan pl;
  if (plan_walk(sc, bc, 1, walk_len, &pl) != WOB_OK) return -1;
  return pl.L;
}

wob_status wob_solve(wob_scene sc, const void* points, const int32_t* point_prim, int64_t n_points,
                     const wob_bc* bc, int32_t samples, int32_t walk_len, uint64_t seed,
                     void* mean_out, void* var_out, void* stream) {
  return run_walk(sc, points, point_prim, n_points, bc, samples, walk_len, seed, nullptr, mean_out,
                  var_out, nullptr, nullptr, nullptr, nullptr, MODE_SOLVE, stream);
}

wob_status wob_solve_ordered_workspace(wob_scene sc, int64_t n_points, size_t* bytes) {
  if (!sc || !bytes || n_points < 0 || n_points > INT32_MAX) return WOB_E_ARG;
  *bytes = order_layout(sc->dim, sc->precision, n_points).total;
  return WOB_OK;
}

wob_status wob_solve_ordered(wob_scene sc, const void* points, const int32_t* point_prim, int64_t n_points,
                             const wob_bc* bc, int32_t samples, int32_t walk_len, uint64_t seed,
                             void* mean_out, void* var_out, void* workspace, size_t workspace_bytes,
                             void* stream) {
  Plan pl;
  wob_status s = plan_walk(sc, bc, samples, walk_len, &pl);
  if (s != WOB_OK) return s;
  if (n_points < 0 || n_points > INT32_MAX || (n_points > 0 && (!points || !mean_out))) return WOB_E_ARG;
  if (var_out && samples < 2) return WOB_E_ARG;
  if (n_points == 0) return WOB_OK;
  const OrderLayout L = order_layout(sc->dim, sc->precision, n_points);
  if (!workspace || (uintptr_t)workspace % 256 != 0 || workspace_bytes < L.total) return WOB_E_ARG;
  OrderBuffers b;
  s = order_points(sc->dim, sc->precision, L, workspace, points, point_prim, n_points, stream, &b);
  if (s != WOB_OK) return s;
  // the walk in locality order; each point keeps its own random-number index
  s = run_walk(sc, b.points, b.point_prim, n_points, bc, samples, walk_len, seed, b.order, b.mean,
               var_out ? b.var : nullptr, nullptr, nullptr, nullptr, nullptr, MODE_SOLVE, stream);
  if (s != WOB_OK) return s;
  return scatter_results(sc->precision, b, n_points, mean_out, var_out, stream);
}

wob_status wob_trace(wob_scene sc, const void* points, const int32_t* point_prim, int64_t n_points,
                     const wob_bc* bc, int32_t samples, int32_t walk_len, uint64_t seed,
                     const uint32_t* point_ids, void* path_out, int32_t* vtx_prim, int32_t* vtx_m,
                     void* stream) {
  return run_walk(sc, points, point_prim, n_points, bc, samples, walk_len, seed, point_ids, nullptr,
                  nullptr, path_out, vtx_prim, vtx_m, nullptr, MODE_TRACE, stream);
}

wob_status wob_solve_grad(wob_scene sc, const void* points, int64_t n_points, const wob_bc* bc,
                          int32_t samples, int32_t walk_len, uint64_t seed, const void* anchor_points,
                          const int32_t* anchor_prim, void* mean_out, void* var_out, void* grad_out,
                          void* grad_var_out, void* stream) {
  if (n_points > 0 && !grad_out) return WOB_E_ARG;
  return run_walk(sc, points, nullptr, n_points, bc, samples, walk_len, seed, nullptr, mean_out, var_out,
                  nullptr, nullptr, nullptr, nullptr, MODE_SOLVE, stream, nullptr, nullptr,
                  n_points > 0 ? grad_out : nullptr, grad_var_out, nullptr, anchor_points, anchor_prim);
}

wob_status wob_trace_grad(wob_scene sc, const void* points, int64_t n_points, const wob_bc* bc,
                          int32_t samples, int32_t walk_len, uint64_t seed, const void* anchor_points,
                          const int32_t* anchor_prim, void* path_out, void* path_grad_out, void* stream) {
  if (n_points > 0 && (!path_out || !path_grad_out)) return WOB_E_ARG;
  return run_walk(sc, points, nullptr, n_points, bc, samples, walk_len, seed, nullptr, nullptr, nullptr,
                  path_out, nullptr, nullptr, nullptr, MODE_TRACE, stream, nullptr, nullptr, nullptr, nullptr,
                  n_points > 0 ? path_grad_out : nullptr, anchor_points, anchor_prim);
}

wob_status wob_count_work(wob_scene sc, const void* points, const int32_t* point_prim,
                          int64_t n_points, const wob_bc* bc, int32_t samples, int32_t walk_len,
                          uint64_t seed, uint64_t* counters, void* stream) {
  return run_walk(sc, points, point_prim, n_points, bc, samples, walk_len, seed, nullptr, nullptr,
                  nullptr, nullptr, nullptr, nullptr, counters, MODE_COUNT, stream);
}

wob_status wob_cv_addback(wob_scene sc, const float* g, const void* points, int64_t n_points,
                          uint64_t seed, void* out, void* stream) {
  if (!sc || n_points < 0 || (n_points > 0 && (!g || !points || !out))) return WOB_E_ARG;
  if (sc->dim != 3 || sc->precision != WOB_F32) return WOB_E_UNSUPPORTED;
  if (n_points == 0) return WOB_OK;
  const int64_t blocks = (n_points + 1023) / 1024;
  hipLaunchKernelGGL((wob::cv_addback_kernel<float>), dim3((unsigned)blocks), dim3(256), 0,
                     (hipStream_t)stream, view<float, 3>(sc), g, (const float*)points, n_points,
                     (uint32_t)(seed & 0xffffffffu), (float*)out, 0);
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

wob_status wob_solve_cv(wob_scene sc, const void* points, const int32_t* point_prim,
                        int64_t n_points, const wob_bc* bc, int32_t samples, int32_t walk_len,
                        uint64_t seed, const float* g, const float* g0, void* mean_out,
                        void* var_out, void* stream) {
  if (!g) return WOB_E_ARG;
  if (!g0) g0 = g;
  wob_status s = run_walk(sc, points, point_prim, n_points, bc, samples, walk_len, seed, nullptr,
                          mean_out, var_out, nullptr, nullptr, nullptr, nullptr, MODE_SOLVE, stream,
                          g, g0);
  if (s != WOB_OK || n_points == 0 || walk_len < 2) return s;
  const int64_t blocks = (n_points + 1023) / 1024;
  hipLaunchKernelGGL((wob::cv_addback_kernel<float>), dim3((unsigned)blocks), dim3(256), 0,
                     (hipStream_t)stream, view<float, 3>(sc), g0, (const float*)points, n_points,
                     (uint32_t)(seed & 0xffffffffu), (float*)mean_out, 1);
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

wob_status wob_trace_cv(wob_scene sc, const void* points, const int32_t* point_prim,
                        int64_t n_points, const wob_bc* bc, int32_t samples, int32_t walk_len,
                        uint64_t seed, const float* g, const float* g0, void* path_out,
                        void* stream) {
  if (!g) return WOB_E_ARG;
  return run_walk(sc, points, point_prim, n_points, bc, samples, walk_len, seed, nullptr, nullptr,
                  nullptr, path_out, nullptr, nullptr, nullptr, MODE_TRACE, stream, g, g0 ? g0 : g);
}

wob_status wob_cv_emission(wob_scene sc, const wob_bc* bc, const float* g, float* g0_out,
                           void* stream) {
  if (!sc || !bc || !g0_out) return WOB_E_ARG;
  if (sc->dim != 3 || sc->precision != WOB_F32) return WOB_E_UNSUPPORTED;
  Plan pl;
  wob_status s = plan_walk(sc, bc, 2, 2, &pl);
  if (s != WOB_OK) return s;
  if (pl.form != WOB_F_SINGLE_LAYER || bc->density || sc->n_dirichlet > 0) return WOB_E_UNSUPPORTED;
  const auto a = make_args<float, 3>(sc, pl, nullptr, nullptr, 0, bc, 2, 2, 0);
  hipLaunchKernelGGL((wob::emission_table_kernel<float>), dim3((unsigned)((sc->n_prims + 255) / 256)),
                     dim3(256), 0, (hipStream_t)stream, view<float, 3>(sc), a.prog, a.phi, g, g0_out);
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

wob_status wob_sample_boundary(wob_scene sc, int64_t n, uint64_t seed, void* points_out,
                               int32_t* prim_out, void* stream) {
  if (!sc || n < 0 || (n > 0 && (!points_out || !prim_out))) return WOB_E_ARG;
  if (n >= ((int64_t)1 << 32)) return WOB_E_ARG;
  if (n == 0) return WOB_OK;
  const dim3 grid((unsigned)((n + 255) / 256)), block(256);
  hipStream_t st = (hipStream_t)stream;
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  if (sc->precision == WOB_F32) {
    if (sc->dim == 3)
      hipLaunchKernelGGL((wob::sample_boundary_kernel<float, 3>), grid, block, 0, st, view<float, 3>(sc),
                         (const float*)sc->d_area_cdf, n, k0, k1, (float*)points_out, prim_out);
    else
      hipLaunchKernelGGL((wob::sample_boundary_kernel<float, 2>), grid, block, 0, st, view<float, 2>(sc),
                         (const float*)sc->d_area_cdf, n, k0, k1, (float*)points_out, prim_out);
  } else {
    if (sc->dim == 3)
      hipLaunchKernelGGL((wob::sample_boundary_kernel<double, 3>), grid, block, 0, st, view<double, 3>(sc),
                         (const float*)sc->d_area_cdf, n, k0, k1, (double*)points_out, prim_out);
    else
      hipLaunchKernelGGL((wob::sample_boundary_kernel<double, 2>), grid, block, 0, st, view<double, 2>(sc),
                         (const float*)sc->d_area_cdf, n, k0, k1, (double*)points_out, prim_out);
  }
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

wob_status wob_cv_table(wob_scene sc, wob_mlp net, float* g_out, void* stream) {
  if (!sc || !net || !g_out) return WOB_E_ARG;
  if (sc->dim != 3 || sc->precision != WOB_F32) return WOB_E_UNSUPPORTED;
  float* cen = nullptr;
  if (hipMalloc((void**)&cen, sizeof(float) * 3 * sc->n_prims) != hipSuccess) return WOB_E_ALLOC;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL((wob::centroid_kernel<float>), dim3((unsigned)((sc->n_prims + 255) / 256)),
                     dim3(256), 0, st, view<float, 3>(sc), cen);
  wob_status s = hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
  if (s == WOB_OK) s = wob_mlp_forward(net, cen, sc->n_prims, g_out, stream);
  if (hipStreamSynchronize(st) != hipSuccess && s == WOB_OK) s = WOB_E_DEVICE;
  (void)hipFree(cen);
  return s;
}

wob_status wob_intersect_all(wob_scene sc, const void* orig, const void* dir,
                             const int32_t* exclude, int64_t n_lines, int32_t max_hits,
                             int32_t* n_hits, int32_t* hit_prim, void* hit_t, void* stream) {
  if (!sc || n_lines < 0 || max_hits < 0) return WOB_E_ARG;
  if (n_lines == 0) return WOB_OK;
  if (!orig || !dir || !n_hits || (max_hits > 0 && !hit_prim)) return WOB_E_ARG;
  hipStream_t st = (hipStream_t)stream;
  const dim3 grid((unsigned)((n_lines + 255) / 256)), block(256);
  if (sc->precision == WOB_F32) {
    if (sc->dim == 3)
      hipLaunchKernelGGL((wob::intersect_kernel<float, 3>), grid, block, 0, st, view<float, 3>(sc),
                         (const float*)orig, (const float*)dir, exclude, n_lines, max_hits, n_hits,
                         hit_prim, (float*)hit_t);
    else
      hipLaunchKernelGGL((wob::intersect_kernel<float, 2>), grid, block, 0, st, view<float, 2>(sc),
                         (const float*)orig, (const float*)dir, exclude, n_lines, max_hits, n_hits,
                         hit_prim, (float*)hit_t);
  } else {
    if (sc->dim == 3)
      hipLaunchKernelGGL((wob::intersect_kernel<double, 3>), grid, block, 0, st, view<double, 3>(sc),
                         (const double*)orig, (const double*)dir, exclude, n_lines, max_hits, n_hits,
                         hit_prim, (double*)hit_t);
    else
      hipLaunchKernelGGL((wob::intersect_kernel<double, 2>), grid, block, 0, st, view<double, 2>(sc),
                         (const double*)orig, (const double*)dir, exclude, n_lines, max_hits, n_hits,
                         hit_prim, (double*)hit_t);
  }
  return hipGetLastError() == hipSuccess ? WOB_OK : WOB_E_DEVICE;
}

}  // extern "C"
