// Internal helpers shared by the ABI translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "../../include/wob.h"
#include "walk.hpp"

struct wob_scene_s {
  int32_t dim = 0, precision = 0, device = 0;
  int64_t n_prims = 0, n_nodes = 0, n_leaves = 0, n_verts = 0;
  int32_t n_inner = 0;    // interior records on the device
  int32_t root = 0;       // root entry (record 0, or a leaf)
  int32_t stack_cap = 1;  // traversal stack entries per lane
  double frame_c[3] = {0, 0, 0}, frame_k = 1;  // frame of the stored boxes
  int32_t depth = 0, max_leaf = 0;
  void* d_nodes = nullptr;
  void* d_prims = nullptr;
  void* d_normals = nullptr;
  int32_t* d_leaf_of_id = nullptr;
  void* d_verts = nullptr;       // the rounded vertices (n_verts x dim, scene precision)
  int32_t* d_vid = nullptr;      // each primitive's vertex ids, caller-id order (n_prims x dim)
  float* d_area_cdf = nullptr;  // caller-id order, cumulative area / total (last entry 1)
  int32_t* d_area_guide = nullptr;  // 2^guide_shift + 1 entries: the search range of each bucket
  int32_t guide_shift = 0;
  unsigned long long* d_status = nullptr;  // non-finite path values excluded from solves (sticky)
  double area_total = 0.0;      // |Gamma|
  int64_t node_bytes = 0, prim_bytes = 0, device_bytes = 0;
  int32_t n_dirichlet = 0, n_neumann = 0, n_robin = 0;
};

namespace wobi {

// Lanes per workgroup of the single-problem solve: one wavefront, so a
// wavefront whose points end early (exterior points whose lines miss the
// boundary) frees its slot at once instead of waiting for the slowest
// wavefront of a larger workgroup (three-tori workload, 1M points x 512 paths:
// 256 / 128 / 64 lanes 723 / 621 / 522 ms; icosphere slice 58.9 / 58.8 / 58.7).
constexpr int kSolveBlock = 64;

// Paths per lane, on average (the lanes of a point share its paths and take
// the next one as theirs end): fixes the lanes per point.  Measured with 4, 8
// and 16: three-tori workload (512 paths) 1,301 / 1,300 / 1,110 M path
// samples/s, icosphere slice (256 paths) 747 / 767 / 769 M.
constexpr int kPathsPerLane = 8;

// log2 of the lanes that share one point: the smallest power of two >=
// ceil(N / kPathsPerLane), at most the block (a wavefront holds several points
// when that is below 64), and at most 32 for solves whose lane groups pool
// two points (wob::pools_points: a group of 2 x 32 lanes is one wavefront)
inline int lpp_shift_for(int32_t samples, int block, bool pooled = false) {
  const int32_t lanes = (samples + kPathsPerLane - 1) / kPathsPerLane;
  const int cap = pooled ? (block < 32 ? block : 32) : block;
  int s = 0;
  while ((1 << s) < lanes && (1 << s) < cap) ++s;
  return s;
}

template <typename R, int D>
wob::SceneView<R, D> view(const wob_scene_s* sc) {
  wob::SceneView<R, D> s;
  s.nodes = (const typename wob::Rec<R, D>::Node*)sc->d_nodes;
  s.prims = (const typename wob::Rec<R, D>::Prim*)sc->d_prims;
  s.normals = (const R*)sc->d_normals;
  s.leaf_of_id = sc->d_leaf_of_id;
  s.area_cdf = sc->d_area_cdf;
  s.area_guide = sc->d_area_guide;
  s.guide_shift = sc->guide_shift;
  s.area_total = (R)sc->area_total;
  s.n_nodes = sc->n_inner;
  s.n_prims = (int32_t)sc->n_prims;
  s.root = sc->root;
  s.stack_cap = sc->stack_cap;
  for (int a = 0; a < 3; ++a) s.fc[a] = (R)sc->frame_c[a];
  s.fk = (R)sc->frame_k;
  return s;
}

inline int resolve_formulation(const wob_scene_s* sc, int f) {
  const bool d = sc->n_dirichlet > 0, n = sc->n_neumann > 0, r = sc->n_robin > 0;
  if (f == WOB_F_AUTO) {
    if (!n && !r) return WOB_F_DOUBLE_LAYER;
    if (!d && !r) return WOB_F_DIRECT;
    return WOB_F_SINGLE_LAYER;  // Robin parts or mixed kinds (Dirichlet parts: first-kind rows)
  }
  if (f == WOB_F_DOUBLE_LAYER) return (!n && !r) ? f : -1;
  if (f == WOB_F_DIRECT) return (!d && !r) ? f : -1;
  if (f == WOB_F_SINGLE_LAYER) return f;
  return -2;
}

struct Plan {
  int form;
  int32_t L;
  uint32_t self_thr;
  double self_p;
  int32_t ris_c;  // RIS candidates, 0 = line sampling
  uint32_t mixed_thr;
  double mixed_p, mixed_k;
};

// The data program of a solve: the analytic program, or the per-vertex data.
template <typename R>
wob::ProgramView<R> make_program(const wob_scene_s* sc, const wob_bc* bc) {
  wob::ProgramView<R> g;
  std::memset(&g, 0, sizeof(g));
  g.type = bc->data_mode == WOB_DATA_VERTEX ? wob::P_VERTEX : bc->program;
  for (int k = 0; k < 8; ++k) g.p[k] = (R)bc->params[k];
  g.vdata = (const R*)bc->vertex_data;
  g.vid = sc->d_vid;
  g.verts = (const R*)sc->d_verts;
  return g;
}

// Data mode and program of a wob_bc.
inline wob_status check_data(const wob_bc* bc) {
  if (bc->data_mode != WOB_DATA_PROGRAM && bc->data_mode != WOB_DATA_VERTEX) return WOB_E_ARG;
  if (bc->path_offset < 0) return WOB_E_ARG;
  if (bc->data_mode == WOB_DATA_VERTEX) return bc->vertex_data ? WOB_OK : WOB_E_ARG;
  if (bc->program < WOB_PROG_CONST || bc->program > WOB_PROG_INVDIST) return WOB_E_ARG;
  return WOB_OK;
}

inline wob_status plan_walk(const wob_scene_s* sc, const wob_bc* bc, int32_t samples, int32_t walk_len,
                     Plan* p) {
  if (!sc || !bc) return WOB_E_ARG;
  if (check_data(bc) != WOB_OK) return WOB_E_ARG;
  if (bc->domain != 1 && bc->domain != -1) return WOB_E_ARG;
  if (bc->density != 0 && bc->density != 1) return WOB_E_ARG;
  if (samples < 1 || walk_len < 1 || walk_len >= 65535) return WOB_E_ARG;
  if ((int64_t)bc->path_offset + samples > INT32_MAX) return WOB_E_ARG;
  const int f = resolve_formulation(sc, bc->formulation);
  if (f == -2) return WOB_E_ARG;
  if (f < 0) return WOB_E_UNSUPPORTED;
  if (bc->density && f == WOB_F_DIRECT) return WOB_E_UNSUPPORTED;
  double ps = bc->self_panel_p == 0.0 ? 1.0 / 16.0 : bc->self_panel_p;
  if (!(ps > 0.0 && ps < 1.0)) return WOB_E_ARG;
  p->form = f;
  p->L = f == WOB_F_DIRECT ? walk_len + 1 : walk_len;
  p->self_thr = (uint32_t)std::floor(ps * 16777216.0);
  if (p->self_thr == 0) return WOB_E_ARG;
  p->self_p = p->self_thr / 16777216.0;
  const double mk = bc->mixed_k == 0.0 ? 4.0 : bc->mixed_k;
  const double mp = bc->mixed_p == 0.0 ? 2.0 / 3.0 : bc->mixed_p;
  if (!std::isfinite(mk) || !(mp > 0.0 && mp < 1.0)) return WOB_E_ARG;
  p->mixed_k = mk;
  p->mixed_thr = (uint32_t)std::floor(mp * 16777216.0);
  if (p->mixed_thr == 0) return WOB_E_ARG;
  p->mixed_p = p->mixed_thr / 16777216.0;
  if (bc->sampling != WOB_SAMPLE_LINE && bc->sampling != WOB_SAMPLE_RIS) return WOB_E_ARG;
  p->ris_c = 0;
  if (bc->sampling == WOB_SAMPLE_RIS) {
    if (f != WOB_F_SINGLE_LAYER) return WOB_E_UNSUPPORTED;
    const int32_t c = bc->candidates == 0 ? 16 : bc->candidates;
    if (c < 1 || c > 64) return WOB_E_ARG;
    p->ris_c = c;
  }
  return WOB_OK;
}

template <typename R, int D>
wob::WalkArgs<R, D> make_args(const wob_scene_s* sc, const Plan& pl, const void* points,
                              const int32_t* point_prim, int64_t n_points, const wob_bc* bc,
                              int32_t samples, int32_t walk_len, uint64_t seed) {
  wob::WalkArgs<R, D> a;
  std::memset(&a, 0, sizeof(a));
  a.scene = view<R, D>(sc);
  a.prog = make_program<R>(sc, bc);
  a.points = (const R*)points;
  a.point_prim = point_prim;
  a.n_points = n_points;
  a.N = samples;
  a.M = walk_len;
  a.L = pl.L;
  a.phi = (R)bc->domain;
  a.self_thr = pl.self_thr;
  a.self_p = (R)pl.self_p;
  a.k0 = (uint32_t)(seed & 0xffffffffu);
  a.k1 = (uint32_t)(seed >> 32);
  a.problem = 0;
  a.path_offset = bc->path_offset;
  a.lpp_shift = lpp_shift_for(samples, kSolveBlock);
  a.density = bc->density;
  a.status = sc->d_status;
  a.ris_c = pl.ris_c;
  a.mixed_thr = pl.mixed_thr;
  a.mixed_p = (R)pl.mixed_p;
  a.mixed_k = (R)pl.mixed_k;
  a.form = pl.form == WOB_F_DOUBLE_LAYER ? wob::F_DL
           : pl.form == WOB_F_DIRECT    ? wob::F_DIRECT
           : pl.ris_c > 0               ? wob::F_SL_RIS
                                        : wob::F_SL;
  return a;
}


// Workspace of the ordered solve (byte offsets, each 256-aligned): partial
// bounding boxes, Morton keys (in, sorted), indices (in, sorted = the order),
// the sorted points and primitive ids, the sorted-order results, the radix
// sort's temporary storage.
struct OrderLayout {
  size_t part, keys, keys_s, idx, order, pts, prim, mean, var, temp, temp_bytes, total;
};
// The walk's inputs in locality order: order[i] is the caller's index of
// sorted point i (also its random-number point index).
struct OrderBuffers {
  const uint32_t* order;
  const void* points;
  const int32_t* point_prim;
  void* mean;
  void* var;
};
OrderLayout order_layout(int dim, int precision, int64_t n);
// Enqueues the Morton keys, the stable sort and the gather on `stream`.
wob_status order_points(int dim, int precision, const OrderLayout& L, void* workspace, const void* points,
                        const int32_t* point_prim, int64_t n, void* stream, OrderBuffers* out);
// Enqueues mean_out[order[i]] = mean[i] (and var) on `stream`.
wob_status scatter_results(int precision, const OrderBuffers& b, int64_t n, void* mean_out, void* var_out,
                           void* stream);

}  // namespace wobi
