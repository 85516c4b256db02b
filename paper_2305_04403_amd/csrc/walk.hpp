// The fused walk-on-boundary path kernel: one lane = one path, all vertices of
// the path in registers, per-point mean / variance reduced in the same launch.
#pragma once

#include "device.hpp"

namespace wob {

// Dynamic LDS of the path kernels: the lanes' traversal stacks and held
// leaves, stack_cap + kLeafSlots entries of 4 bytes per thread of the block,
// then one more row (the path counters of the lane groups) and one word (the
// path offset; sized at launch).
extern __shared__ int32_t wob_stack[];
constexpr int kLeafSlots = 4;
inline size_t walk_lds_bytes(int stack_cap, int block) {
  return ((size_t)(stack_cap + kLeafSlots + 1) * (size_t)block + 1) * sizeof(int32_t);
}

template <typename R, int D>
struct WalkArgs {
  SceneView<R, D> scene;
  ProgramView<R> prog;
  const R* points;
  const int32_t* point_prim;  // caller ids, -1 off the boundary; may be null
  const uint32_t* point_ids;  // random-number point index per point; null = position
  int64_t n_points;
  int32_t N, M, L;            // paths per point, boundary vertices, lines per path
  R phi;                      // +1 interior, -1 exterior
  uint32_t self_thr;          // mixture branch threshold floor(p_s 2^24)
  R self_p;                   // floor(p_s 2^24) / 2^24
  uint32_t k0, k1;            // Philox key
  uint32_t problem;           // problem index (counter word 2, bits 24..31)
  int32_t lpp_shift;          // log2 of lanes per point (0 .. log2 of the block size)
  int32_t path_offset;        // path k of a point draws the random numbers of path path_offset + k
  int32_t form;               // F_DL / F_DIRECT / F_SL / F_SL_RIS (read by the batched kernel)
  int32_t density;            // estimate the boundary unknown at boundary points (no own emission)
  int32_t ris_c;              // single layer: RIS candidates per vertex, 0 = line sampling
  uint32_t mixed_thr;         // single layer, Dirichlet vertices: floor(p_k 2^24)
  R mixed_p, mixed_k;         // p_k (as floor(p_k 2^24) / 2^24) and k
  const float* fwd_cdf;       // forward walk: start table, binary32 cumulative weight fraction (caller-id order)
  int64_t fwd_paths;          // forward walk: number of paths (path id = point * N + k)
  R* fwd_vtx;                 // forward walk: per path and vertex (y, strength), 4 values each
  const R* cv_g;              // control-variate table per caller primitive id (single layer), or null
  const R* cv_g0;             // its line-0 table (the add-back's), set whenever cv_g is
  R* mean_out;
  R* var_out;
  R* path_out;
  R* grad_out;                // gradient walk: per point, D components of the mean gradient
  R* grad_var_out;            // and their variances (or null)
  R* path_grad_out;           // gradient walk, trace mode: per path, D components
  const R* anchor_pts;        // gradient walk, double layer: per point a boundary point (D values) and
  const int32_t* anchor_prim; // its caller primitive id (-1: no boundary split), or both null
  int32_t* vtx_prim;
  int32_t* vtx_m;
  unsigned long long* counters;
  unsigned long long* status;  // solves: count of non-finite path values (excluded from the statistics)
};

// One path estimates u_hat(x_0):
//
// Double layer (Table 1, Dirichlet; eq. mc_dirichlet_interior_sol and
// eq. indirect_double_boundary_reordered2):  first weight -dG/dn_y / p, then
// 2 phi dG/dn_y / p; emission 2 phi g at x_1..x_{M-1} and phi g at x_M.
// With line sampling these weights are (m/2) sgn(cos) and -phi m sgn(cos).
//
// Direct BIE (Table 1, Neumann; eq. mc_cbie_neumann2, eq. mc_cbie_neumann):
// first weight -phi dG/dn_y / p = phi (m/2) sgn(cos), then
// -2 phi dG/dn_y / p = phi m sgn(cos).  Source phi int G q (off the boundary)
// or 2 phi int G q (on it), estimated from all hits of the same line plus the
// in-plane sample of the own primitive; the source of x_M (its own line) is
// halved.
//
// Single layer (Table 1, Neumann / Robin rows): first weight G / p =
// m rho / (2 |cos|) (3D), then -2 phi (dG/dn_x + alpha G) / p =
// -phi m (cos_x + alpha rho) / |cos_y| (3D); where G acts on the own primitive
// (boundary x_0, Robin vertices) the line sample is mixed with the in-plane
// sample with probability p_s.  Emission 2 phi s, halved at x_M.
//
// A lane runs its paths as a state machine: begin_step draws the vertex's
// direction (and performs in-plane self-panel steps, which trace nothing)
// until a line has to be traced; the walk loop (walk_block) steps through the
// BVH nodes of that line and hands each crossed leaf to leaf_work; end_step
// consumes the line's hits and calls begin_step for the next vertex.  The
// lanes of a wavefront therefore trace lines independently instead of every
// line waiting for the wavefront's longest one.

enum { ST_NONE = 0, ST_LINE = 1, ST_DONE = 2 };

// Extensions of the walk: the corrected walk of the control variate, and the
// gradient in the evaluation point carried along the same paths.
// X_VDATA is a flag on top of either: the boundary data may be given per
// vertex (a separate instantiation, so the program-data kernels do not carry
// the interpolation's registers).
enum Ext { X_NONE = 0, X_CV = 1, X_GRAD = 2, X_VDATA = 4 };
constexpr int ext_kind(int ext) { return ext & 3; }
constexpr bool ext_vdata(int ext) { return (ext & X_VDATA) != 0; }

// Solves whose lane groups pool the paths of two points (the plain
// single-layer walks, lines and RIS, and the direct BIE: the second point's
// statistics fit their register budget of four waves per SIMD; the double
// layer's five would not hold them); the host gives them at most 32 lanes per
// point.
constexpr bool pools_points(int form, int ext, bool trace, bool count) {
  return (form == F_SL || form == F_SL_RIS || form == F_DIRECT) && ext == X_NONE && !trace && !count;
}

// Single-layer emission at vertex y on primitive g, before the running
// weight: 2 phi s(y) on Neumann / Robin parts (Table 1), k u_D(y) on Dirichlet
// parts (eq. mixed_second_kind_ish); half of it at the last vertex x_M.
template <typename R, int D, bool VD>
__device__ __forceinline__ R sl_emission(const WalkArgs<R, D>& a, const PrimGeo<R>& g, const R n[3],
                                         const R y[3], bool last_vertex) {
  const R sv = boundary_datum<R, D, VD>(a.prog, g, n, y);
  const R e = g.kind == K_DIRICHLET ? a.mixed_k * sv : (R)2 * a.phi * sv;
  return last_vertex ? (R)0.5 * e : e;
}

template <typename R, int D>
struct PathState {
  uint32_t point, path;  // random-number indices
  R x0[3];
  int32_t prim0;
  R x[3], W, acc;
  int32_t cur_idx, i;
  int32_t* vp;           // per-line records (trace mode)
  int32_t* vm;
  uint32_t z;            // counter word 2 of the current line
  bool first, on_gamma, mixture, last, select;
  bool sum;              // corrected walk: accumulate the all-hits sum of a(h) F(y_h)
  R gscale;              // single layer: factor of the G kernel (1, or -k / p_k at a Dirichlet vertex)
  PrimGeo<R> gc;         // the primitive the vertex lies on (direct, single layer)
  R nc[3];
  R d[3], inv[3], ox[3];
  uint32_t rot[3];        // slab-test rotations of packed box words
  HitAcc<R> h;
  int32_t ni;            // traversal position: an entry, kPop or kDone
  R Wg[3], gacc[3];      // gradient walk: d W / d x0 and the gradient sum
  R Wg0[3];              // gradient walk: the step-0 derivative weight w'
  R acc_main;            // boundary split: the path's value while its coupled walk runs
  bool coupled;          // boundary split: the coupled walk from the anchor is running
};

// Forward walk: vertex k of the current path, (y_k, c_{k-1} W_k) with
// c = (1, ..., 1, 1/2), its caller id and the hits of the line that reached it.
template <typename R, int D>
__device__ __forceinline__ void fwd_record(const WalkArgs<R, D>& a, const PathState<R, D>& s, int k,
                                           int32_t id, int32_t m) {
  const int64_t v = (int64_t)s.path * a.M + k;
  const R c = k + 1 < a.M ? (R)1 : (R)0.5;
  struct alignas(4 * sizeof(R)) R4 { R x, y, z, w; };
  *reinterpret_cast<R4*>(a.fwd_vtx + v * 4) = R4{s.x[0], s.x[1], D == 3 ? s.x[2] : (R)0, c * s.W};
  if (a.vtx_prim) a.vtx_prim[v] = id;
  if (a.vtx_m) a.vtx_m[v] = m;
}

// Forward walk: the path ended at vertex k - 1 (its line found no hit); the
// remaining vertices carry nothing: strength 0 at a far position (1e18 in each
// coordinate), where the connection adds exactly 0 * (a finite kernel value)
// without a test for zero distance.
template <typename R, int D>
__device__ __forceinline__ void fwd_end(const WalkArgs<R, D>& a, const PathState<R, D>& s, int k) {
  struct alignas(4 * sizeof(R)) R4 { R x, y, z, w; };
  const R far = (R)1e18;
  for (; k < a.M; ++k) {
    const int64_t v = (int64_t)s.path * a.M + k;
    *reinterpret_cast<R4*>(a.fwd_vtx + v * 4) = R4{far, far, D == 3 ? far : (R)0, (R)0};
    if (a.vtx_prim) a.vtx_prim[v] = -1;
    if (a.vtx_m) a.vtx_m[v] = 0;
  }
}

// One single-layer vertex by resampled importance sampling (the paper's
// sampling for Robin and mixed problems, Results): C candidates uniform by
// area on the boundary (Philox block 3, w = j: word 0 the primitive through
// the binary32 cumulative area fraction in caller-id order, words 1, 2 the
// point, word 3 the reservoir uniform), target |k| with k = G on the first step
// and -2 phi (dG/dn_x + alpha G) on the recursion; a weighted reservoir keeps
// candidate j when u_j S_j < |k_j|; weight sign(k) S |Gamma| / C.  Moves the
// path to the kept point and adds its emission; returns false when no
// candidate carries kernel mass (the path ends).
// CV (corrected walk, 3D single layer): given the candidates, the pick's
// expected contribution w F(y_pick) is (|Gamma| / C) sum_j k(y_j) F(y_j); the
// step adds that sum and subtracts w F(y_pick), with F as for line sampling
// (line 0: the table g0, restored by the add-back; lines 1..M-2: 2 phi s + g;
// the last line: phi s, with no pick).
template <typename R, int D, bool TRACE, bool GRAD, bool VD, bool CV>
__device__ __forceinline__ bool ris_step(const WalkArgs<R, D>& a, PathState<R, D>& s) {
  const SceneView<R, D>& sc = a.scene;
  const R phi = a.phi;
  const R inv4pi = (R)(0.25 / 3.14159265358979323846), inv2pi = (R)(0.5 / 3.14159265358979323846);
  R S = 0, kpick = 0, ypick[3] = {0, 0, 0};
  int32_t lpick = -1;
  const bool last = s.i == a.L - 1;
  const bool sum = CV && (s.i > 0 || last);
  R csum = 0;
  for (int j = 0; j < a.ris_c; ++j) {
    const U4 rj = philox(s.path, s.point, s.z | 3u, (uint32_t)j, a.k0, a.k1);
    const float u = unit<float>(rj.x);
    // the first caller id whose cdf exceeds u, searched in its guide bucket
    const uint32_t bkt = (uint32_t)(u * (float)(1u << sc.guide_shift));
    int32_t lo = sc.area_guide[bkt], hi = sc.area_guide[bkt + 1];
    while (lo < hi) {
      const int32_t mid = (lo + hi) >> 1;
      if (sc.area_cdf[mid] > u) hi = mid;
      else lo = mid + 1;
    }
    const int32_t leaf = sc.leaf_of_id[lo];
    const PrimGeo<R> g = load_prim<R, D>(sc, leaf);
    R bu = unit<R>(rj.y), bv = D == 3 ? unit<R>(rj.z) : (R)0;
    if (bu + bv > (R)1) {
      bu = (R)1 - bu;
      bv = (R)1 - bv;
    }
    R y[3];
    hit_point(g, bu, bv, y);
    const R r[3] = {y[0] - s.x[0], y[1] - s.x[1], D == 3 ? y[2] - s.x[2] : (R)0};
    const R rr = dot3(r, r);
    R k = 0;
    if (rr > (R)0) {
      const R rho = sqrt(rr);
      if (s.gscale != (R)0) {  // first step, or a Dirichlet vertex: the G kernel
        k = s.gscale * (D == 3 ? inv4pi / rho : -inv2pi * log(rho));
      } else {
        // (y - x) . n_x from the candidate's own vertex and edges: x lies in
        // the plane of its primitive, so (y - x) . n_x = (v0_y - v0_x) . n_x +
        // a e1_y . n_x + b e2_y . n_x, free of the cancellation of y - x (whose
        // binary32 rounding would swamp the small normal component of nearby,
        // nearly coplanar candidates); zero on the own primitive
        R rn = 0;
        if (g.id != s.gc.id) {
          const R dv[3] = {g.v0[0] - s.gc.v0[0], g.v0[1] - s.gc.v0[1],
                           D == 3 ? g.v0[2] - s.gc.v0[2] : (R)0};
          rn = dot3(dv, s.nc) + bu * dot3(g.e1, s.nc) + (D == 3 ? bv * dot3(g.e2, s.nc) : (R)0);
        }
        k = D == 3 ? (R)-2 * phi * (inv4pi * rn / (rr * rho) + s.gc.alpha * inv4pi / rho)
                   : (R)-2 * phi * (inv2pi * rn / rr - s.gc.alpha * inv2pi * log(rho));
      }
    }
    const R pk = fabs(k);
    S += pk;
    if (unit<R>(rj.w) * S < pk) {
      lpick = leaf;
      kpick = k;
      ypick[0] = y[0];
      ypick[1] = y[1];
      ypick[2] = y[2];
    }
    if constexpr (CV) {
      if (sum) {  // the candidate's term of the all-candidates sum
        R cn[3];
        load_normal<R, D>(sc, leaf, cn);
        const R e = sl_emission<R, D, VD>(a, g, cn, y, s.i + 1 >= a.M);
        csum += k * (last ? e : e + a.cv_g[g.id]);
      }
    }
  }
  if constexpr (CV) {
    if (sum) s.acc += s.W * csum * sc.area_total / (R)a.ris_c;
    if (last) return false;  // the last line needs no pick
  }
  if (lpick < 0 || !(S > (R)0)) return false;
  const R w = (kpick > (R)0 ? (R)1 : (R)-1) * S * sc.area_total / (R)a.ris_c;
  if constexpr (GRAD) {
    if (s.first) {
      // RIS estimate of int grad_x G mu: grad_x G(y) / |G(y)| S |Gamma| / C,
      // grad_x G = r / (S_D rho^D), r = y - x
      const R r[3] = {ypick[0] - s.x[0], ypick[1] - s.x[1], D == 3 ? ypick[2] - s.x[2] : (R)0};
      const R rr = dot3(r, r);
      const R gr = (D == 3 ? inv4pi / (rr * sqrt(rr)) : inv2pi / rr) * S * sc.area_total /
                   ((R)a.ris_c * fabs(kpick));
#pragma unroll
      for (int k = 0; k < 3; ++k) s.Wg[k] = s.Wg[k] * w + s.W * gr * r[k];
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k) s.Wg[k] *= w;
    }
  }
  s.W *= w;
  s.x[0] = ypick[0];
  s.x[1] = ypick[1];
  s.x[2] = ypick[2];
  s.cur_idx = lpick;
  const PrimGeo<R> gn = load_prim<R, D>(sc, lpick);
  R nn[3];
  load_normal<R, D>(sc, lpick, nn);
  if (TRACE && s.vp) s.vp[s.i] = gn.id;
  if constexpr (CV) {
    if (s.i == 0) {  // the line-0 table subtracted, the emission kept
      s.acc += s.W * (sl_emission<R, D, VD>(a, gn, nn, s.x, false) - a.cv_g0[gn.id]);
    } else {  // the picked emission is inside the sum
      s.acc -= s.W * a.cv_g[gn.id];
    }
    return true;
  }
  const R e = sl_emission<R, D, VD>(a, gn, nn, s.x, s.i + 1 >= a.M);
  s.acc += s.W * e;
  if constexpr (GRAD) {
#pragma unroll
    for (int k = 0; k < 3; ++k) s.gacc[k] += s.Wg[k] * e;
  }
  return true;
}

template <typename R, int D, int FORM, bool TRACE, bool COUNT, int EXT>
__device__ __forceinline__ int begin_step(const WalkArgs<R, D>& a, PathState<R, D>& s, WorkCount& wc) {
  constexpr bool CV = ext_kind(EXT) == X_CV, GRAD = ext_kind(EXT) == X_GRAD, VD = ext_vdata(EXT);
  const R phi = a.phi;
  for (;;) {
    if (s.i >= a.L) return ST_DONE;
    s.on_gamma = s.cur_idx >= 0;
    s.z = (a.problem << 24) | ((uint32_t)s.i << 8);
    if (s.on_gamma && FORM != F_DL && FORM != F_FWD) {
      s.gc = load_prim<R, D>(a.scene, s.cur_idx);
      load_normal<R, D>(a.scene, s.cur_idx, s.nc);
    }
    // step 0 from an evaluation point uses the representation formula; in
    // density mode x0 is itself a vertex of the boundary recursion
    s.first = FORM != F_FWD && s.i == 0 && !a.density;
    if constexpr (is_sl(FORM)) {
      // Table 1: on a Dirichlet part the solution is the given value (tested
      // here, where the primitive is loaded anyway, rather than in start_path:
      // a second load there costs the single-layer kernel ~35 registers)
      if (s.first && s.on_gamma && s.gc.kind == K_DIRICHLET) {
        const R nz[3] = {0, 0, 0};
        s.acc = boundary_datum<R, D, VD>(a.prog, s.gc, nz, s.x);
        return ST_DONE;
      }
    }
    U4 r0;
    bool have_r0 = false;
    if constexpr (is_sl(FORM)) {
      // a Dirichlet vertex (mixed problems): the transformed first-kind row
      // mu = mu - k int G mu + k u_D, one term at a time (eq.
      // mixed_second_kind_ish_mc): with probability p_k the next point is
      // sampled from k G (weight -k G / (p p_k)), otherwise the walk stays at x
      // (weight 1 / (1 - p_k)); the p_k decision is word 3 of block 0
      const bool dvert = s.on_gamma && !s.first && s.gc.kind == K_DIRICHLET;
      s.gscale = s.first ? (R)1 : (R)0;
      if (dvert) {
        r0 = philox(s.path, s.point, s.z, 0u, a.k0, a.k1);
        have_r0 = true;
        if ((r0.w >> 8) >= a.mixed_thr) {
          const R ws = (R)1 / ((R)1 - a.mixed_p);
          s.W *= ws;
          if (TRACE && s.vp) s.vp[s.i] = -2 - s.gc.id;
          const R e = sl_emission<R, D, VD>(a, s.gc, s.nc, s.x, s.i + 1 >= a.M);
          s.acc += s.W * e;
          if constexpr (GRAD) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
              s.Wg[k] *= ws;
              s.gacc[k] += s.Wg[k] * e;
            }
          }
          ++s.i;
          continue;
        }
        s.gscale = -a.mixed_k / a.mixed_p;
      }
      if constexpr (FORM == F_SL_RIS) {
        if (!ris_step<R, D, TRACE, GRAD, VD, CV>(a, s)) return ST_DONE;
        ++s.i;
        continue;
      }
    }
    if (!have_r0) r0 = philox(s.path, s.point, s.z, 0u, a.k0, a.k1);
    direction<R, D>(r0.x, r0.y, s.d);
    bool use_self = false;
    s.mixture = false;
    if constexpr (is_sl(FORM)) {
      s.mixture = s.on_gamma && (s.gscale != (R)0 || s.gc.kind == K_ROBIN);
      use_self = s.mixture && (r0.z >> 8) < a.self_thr;
    }
    if (use_self) {
      const U4 r1 = philox(s.path, s.point, s.z | 1u, 0u, a.k0, a.k1);
      R y[3];
      const R gp = self_panel<R, D>(s.gc, s.nc, s.x, unit<R>(r1.x), unit<R>(r1.y), y);
      const R w = (s.gscale != (R)0 ? s.gscale * gp : (R)-2 * phi * s.gc.alpha * gp) / a.self_p;
      if (TRACE && s.vp) s.vp[s.i] = -2 - s.gc.id;
      s.W *= w;
      // control variate, line 0: subtract the line-0 table at the own primitive
      if (CV && s.i == 0 && s.i + 1 < a.M) s.acc -= s.W * a.cv_g0[s.gc.id];
      s.x[0] = y[0];
      s.x[1] = y[1];
      s.x[2] = y[2];
      // emission at the new vertex (same primitive)
      const R e = sl_emission<R, D, VD>(a, s.gc, s.nc, s.x, s.i + 1 >= a.M);
      s.acc += s.W * e;
      if constexpr (GRAD) {  // a vertex on the boundary: never the first step
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          s.Wg[k] *= w;
          s.gacc[k] += s.Wg[k] * e;
        }
      }
      ++s.i;
      continue;
    }
    s.last = s.i == a.L - 1;
    // the direct BIE's last line and the corrected walk's last line need no pick
    s.select = !((FORM == F_DIRECT || CV) && s.last);
    s.sum = CV && (s.i > 0 || s.last);
    line_slabs<R, D>(a.scene, s.x, s.d, s.inv, s.ox, s.rot);
    s.h.m = 0;
    s.h.key = 0xffffffffu;
    s.h.id = 0x7fffffff;
    s.h.idx = -1;
    s.h.t = 0;
    s.h.src = 0;
    if constexpr (GRAD) s.h.srcg[0] = s.h.srcg[1] = s.h.srcg[2] = 0;
    s.ni = a.scene.root;
    if (COUNT) wc.lines += 1;
    return ST_LINE;
  }
}

// couple >= 0 (gradient walks of the double layer): instead of path `path`'s
// walk from its evaluation point, start the coupled walk of the boundary split
// from the anchor on primitive `couple` (see walk_block); the path's value is
// kept aside.  Both starts end in the same begin_step call, so that its code
// is inlined once.
template <typename R, int D, int FORM, bool TRACE, bool COUNT, int EXT>
__device__ __forceinline__ int start_path(const WalkArgs<R, D>& a, PathState<R, D>& s, uint32_t path,
                                          int64_t item, WorkCount& wc, int32_t couple = -1,
                                          int64_t point = 0) {
  constexpr bool GRAD = ext_kind(EXT) == X_GRAD, VD = ext_vdata(EXT);
  s.path = path;
  bool coupled_start = false;
  if constexpr (GRAD && FORM == F_DL) coupled_start = couple >= 0;
  if (coupled_start) {
    // the coupled walk: x* as vertex 1, then the path's own lines 1, 2, ...
    s.acc_main = s.acc;
    s.coupled = true;
    if (couple >= a.scene.n_prims) {  // a caller error: the gradient is NaN
      s.acc = (R)NAN;
      return ST_DONE;
    }
    if (TRACE) s.vp = s.vm = nullptr;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      s.x[k] = k < D ? a.anchor_pts[point * D + k] : (R)0;
      s.Wg[k] = 0;
    }
    s.cur_idx = a.scene.leaf_of_id[couple];
    s.W = 1;
    s.i = 1;
    // the double layer's emission at vertex 1 (halved when it is x_M)
    const PrimGeo<R> g = load_prim<R, D>(a.scene, s.cur_idx);
    R n[3];
    load_normal<R, D>(a.scene, s.cur_idx, n);
    s.acc = ((1 < a.M) ? (R)2 * a.phi : a.phi) * boundary_datum<R, D, VD>(a.prog, g, n, s.x);
  } else {
    if constexpr (GRAD) {
#pragma unroll
      for (int k = 0; k < 3; ++k) s.Wg0[k] = 0;
      s.coupled = false;
    }
    if constexpr (FORM == F_FWD) {
      // y_1 on the boundary: primitive T from the start table (Philox
      // (id, 0xfffffffe, (problem << 24) | 0xffff03, 0): word 0 against the
      // binary32 table, words 1, 2 the point, reflected into the triangle), with
      // density p_0 = P_T / A_T; W_1 = 2 phi q(y_1) / p_0
      if (item >= a.fwd_paths) return ST_NONE;
      s.path = (uint32_t)item;
      const SceneView<R, D>& sc = a.scene;
      const U4 r = philox(s.path, s.point, (a.problem << 24) | 0xffff03u, 0u, a.k0, a.k1);
      const float u = unit<float>(r.x);
      int32_t lo = 0, hi = sc.n_prims - 1;
      while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (a.fwd_cdf[mid] > u) hi = mid;
        else lo = mid + 1;
      }
      const int32_t leaf = sc.leaf_of_id[lo];
      const PrimGeo<R> g = load_prim<R, D>(sc, leaf);
      R bu = unit<R>(r.y), bv = D == 3 ? unit<R>(r.z) : (R)0;
      if (bu + bv > (R)1) {
        bu = (R)1 - bu;
        bv = (R)1 - bv;
      }
      hit_point(g, bu, bv, s.x);
      R n[3];
      load_normal<R, D>(sc, leaf, n);
      R area;
      if constexpr (D == 3) {
        R c[3];
        cross3(g.e1, g.e2, c);
        area = (R)0.5 * sqrt(dot3(c, c));
      } else {
        area = sqrt(g.e1[0] * g.e1[0] + g.e1[1] * g.e1[1]);
      }
      const R pt = (R)a.fwd_cdf[lo] - (lo > 0 ? (R)a.fwd_cdf[lo - 1] : (R)0);
      s.W = (R)2 * a.phi * boundary_datum<R, D, VD>(a.prog, g, n, s.x) * area / pt;
      s.acc = 0;
      s.i = 0;
      s.cur_idx = leaf;
      fwd_record<R, D>(a, s, 0, g.id, 0);
      return begin_step<R, D, FORM, TRACE, COUNT, EXT>(a, s, wc);
    }
    if (TRACE) {
      s.vp = a.vtx_prim ? a.vtx_prim + item * a.L : nullptr;
      s.vm = a.vtx_m ? a.vtx_m + item * a.L : nullptr;
      for (int i = 0; i < a.L; ++i) {
        if (s.vp) s.vp[i] = -1;
        if (s.vm) s.vm[i] = 0;
      }
    }
    // a primitive id outside [-1, n_prims) is a caller error: the path is NaN;
    // so is a density-mode point off the boundary (it has no boundary unknown)
    if (s.prim0 < -1 || s.prim0 >= a.scene.n_prims || (a.density && s.prim0 < 0)) {
      s.acc = (R)NAN;
      return ST_DONE;
    }
    s.cur_idx = s.prim0 >= 0 ? a.scene.leaf_of_id[s.prim0] : -1;
    s.x[0] = s.x0[0];
    s.x[1] = s.x0[1];
    s.x[2] = s.x0[2];
    if (FORM == F_DL && s.cur_idx >= 0 && !a.density) {
      // Table 1: on the boundary the Dirichlet solution is the given value
      const PrimGeo<R> g = load_prim<R, D>(a.scene, s.cur_idx);
      const R nz[3] = {0, 0, 0};
      s.acc = boundary_datum<R, D, VD>(a.prog, g, nz, s.x);
      return ST_DONE;
    }
    s.W = 1;
    s.acc = 0;
    s.i = 0;
    if constexpr (GRAD) {
  #pragma unroll
      for (int k = 0; k < 3; ++k) s.Wg[k] = s.gacc[k] = 0;
    }
  }
  return begin_step<R, D, FORM, TRACE, COUNT, EXT>(a, s, wc);
}


// The primitives of the crossed leaves a lane holds (one to four) on the
// current line.  The primitive loop
// only tests and records the accepted primitives in a bit mask; the hits are
// then handled in a loop of their own, so that the lanes with a hit in this
// leaf phase do that work together instead of one or two at a time inside the
// primitive loop.  Per hit: count it; with `select`, draw its key (Philox
// block 2, w = caller id) and keep the smallest (key, id) -- the line
// parameter and barycentrics of the kept hit are computed once, in end_step;
// for the direct BIE add G q / p_all to the source sum; for the corrected walk
// add a(h) F(y_h).
template <typename R, int D, int FORM, bool COUNT, int EXT>
__device__ __forceinline__ void leaf_work(const WalkArgs<R, D>& a, PathState<R, D>& s, int32_t code,
                                          int32_t code2, int32_t code3, int32_t code4, WorkCount& wc) {
  static_assert(kLeafSlots == 4, "leaf_work takes four leaf codes");
  constexpr bool CV = ext_kind(EXT) == X_CV, GRAD = ext_kind(EXT) == X_GRAD, VD = ext_vdata(EXT);
  const SceneView<R, D>& sc = a.scene;
  {
    // one to four leaves (codes -1 = none after the first): primitive b of the
    // row is first + b (b < count), then the second leaf's, and so on
    const int32_t first = code >> 3, count = (code & 7) + 1;
    const int32_t c2 = code2 >= 0 ? (code2 & 7) + 1 : 0, c3 = code3 >= 0 ? (code3 & 7) + 1 : 0;
    const int32_t first2 = (code2 >> 3) - count, first3 = (code3 >> 3) - count - c2;
    const int32_t first4 = (code4 >> 3) - count - c2 - c3;
    const int32_t total = count + c2 + c3 + (code4 >= 0 ? (code4 & 7) + 1 : 0);
    constexpr bool GEO = FORM == F_DIRECT || CV;  // per-hit work needs the hit's geometry
    uint32_t accepted = 0;  // bit b: primitive b of the leaves is hit
    int32_t id0 = 0;        // caller id of the first hit (no reload for it)
    for (int32_t b = 0; b < total; ++b) {
      const int32_t j = (b < count ? first : (b < count + c2 ? first2 : (b < count + c2 + c3 ? first3 : first4))) + b;
      if (j == s.cur_idx) continue;
      if (COUNT) wc.prims += 1;
      const PrimGeo<R> g = load_prim<R, D>(sc, j);
      R t, u, v;
      if (hit_prim<R, D>(g, s.x, s.d, t, u, v)) {
        if (!accepted) id0 = g.id;
        accepted |= 1u << b;
      }
    }
    bool later = false;
    while (accepted) {
      const int32_t b = __builtin_ctz(accepted);
      const int32_t j = (b < count ? first : (b < count + c2 ? first2 : (b < count + c2 + c3 ? first3 : first4))) + b;
      accepted &= accepted - 1;
      PrimGeo<R> g;
      if (GEO || later) g = load_prim<R, D>(sc, j);
      const int32_t id = (GEO || later) ? g.id : id0;
      later = true;
      if (COUNT) wc.hits += 1;
      s.h.m += 1;
      if (s.select) {
        const uint32_t key = philox(s.path, s.point, s.z | 2u, (uint32_t)id, a.k0, a.k1).x;
        if (key < s.h.key || (key == s.h.key && id < s.h.id)) {
          s.h.key = key;
          s.h.id = id;
          s.h.idx = j;
        }
      }
      if constexpr (FORM == F_DIRECT) {
        R y[3], n[3];
        load_normal<R, D>(sc, j, n);
        const R t = plane_hit<R, D>(g, n, s.x, s.d, y);
        const R q = boundary_datum<R, D, VD>(a.prog, g, n, y);  // Neumann data
        // y - x = t d: distance and cosine from the line itself, free of the
        // cancellation in y - x when the hit is close to x
        const R rho = fabs(t);
        const R ac = fabs(dot3(s.d, n));  // |cos theta_y|
        // G q / p_all: 3D rho q / (2 |c|); 2D -rho ln(rho) q / (2 |c|)
        const R gp = D == 3 ? rho / ((R)2 * ac) : -rho * log(rho) / ((R)2 * ac);
        s.h.src += gp * q;
        if constexpr (GRAD) {
          // grad_x G q / p_all = q sgn(t) d / (2 |c|) in 2D and 3D (line 0 only:
          // later sources do not depend on x0)
          if (s.i == 0) {
            const R gq = (t > (R)0 ? q : -q) / ((R)2 * ac);
#pragma unroll
            for (int k = 0; k < 3; ++k) s.h.srcg[k] += gq * s.d[k];
          }
        }
      }
      if constexpr (CV && FORM == F_SL && D == 3) {
        if (s.sum) {
          // a(h) F(y_h): the weight of hit h without the 1/m of the pick
          R y[3], n[3];
          load_normal<R, D>(sc, j, n);
          const R t = plane_hit<R, D>(g, n, s.x, s.d, y);
          const R rho = fabs(t);
          const R acy = fabs(dot3(s.d, n));
          const R sgn_t = t > (R)0 ? (R)1 : (R)-1;
          R ah = s.first ? rho / ((R)2 * acy)
                         : -a.phi * (sgn_t * dot3(s.d, s.nc) + s.gc.alpha * rho) / acy;
          if (s.mixture) ah /= ((R)1 - a.self_p);
          const R sh = boundary_datum<R, D, VD>(a.prog, g, n, y);
          const R F = s.last ? a.phi * sh : (R)2 * a.phi * sh + a.cv_g[g.id];
          s.h.src += ah * F;
        }
      }
    }
  }
}

template <typename R, int D, int FORM, bool TRACE, bool COUNT, int EXT>
__device__ __forceinline__ int end_step(const WalkArgs<R, D>& a, PathState<R, D>& s, WorkCount& wc) {
  constexpr bool CV = ext_kind(EXT) == X_CV, GRAD = ext_kind(EXT) == X_GRAD, VD = ext_vdata(EXT);
  const R phi = a.phi;
  HitAcc<R>& h = s.h;
  if (TRACE) {
    if (s.vm) s.vm[s.i] = h.m;
    if (s.vp) s.vp[s.i] = (s.select && h.m > 0) ? h.id : -1;
  }
  if constexpr (FORM == F_DIRECT) {
    R S;
    if (s.on_gamma) {
      const U4 r1 = philox(s.path, s.point, s.z | 1u, 0u, a.k0, a.k1);
      R ys[3];
      const R gp = self_panel<R, D>(s.gc, s.nc, s.x, unit<R>(r1.x), unit<R>(r1.y), ys);
      S = (R)2 * phi * (h.src + gp * boundary_datum<R, D, VD>(a.prog, s.gc, s.nc, ys));
    } else {
      S = phi * h.src;
    }
    const R cl = s.last ? (R)0.5 : (R)1;
    s.acc += s.W * S * cl;
    if constexpr (GRAD) {
      // line 0 from x0 off the boundary: the source phi int G q depends on x0
#pragma unroll
      for (int k = 0; k < 3; ++k)
        s.gacc[k] += (s.Wg[k] * S + (s.i == 0 ? s.W * phi * h.srcg[k] : (R)0)) * cl;
    }
    if (s.last) return ST_DONE;
  }
  if (h.m == 0) {
    if constexpr (FORM == F_FWD) fwd_end<R, D>(a, s, s.i + 1);
    return ST_DONE;
  }
  if (CV && s.last) {
    // the all-hits mean of the last emission
    s.acc += s.W * h.src;
    return ST_DONE;
  }
  const PrimGeo<R> gy = load_prim<R, D>(a.scene, h.idx);
  R y[3], w, ny[3];
  // the kept hit: where the line crosses its primitive's plane
  load_normal<R, D>(a.scene, h.idx, ny);
  h.t = plane_hit<R, D>(gy, ny, s.x, s.d, y);
  // y - x = t d: the unit direction to the hit is sign(t) d and rho = |t|
  const R sgn_t = h.t > (R)0 ? (R)1 : (R)-1;
  const R mm = (R)h.m;
  if constexpr (FORM == F_DL || FORM == F_DIRECT || FORM == F_FWD) {
    const R sg = sgn_t * dot3(s.d, ny) > (R)0 ? (R)1 : (R)-1;  // sgn(cos theta_y)
    if constexpr (FORM == F_DL)
      w = (s.first && !s.on_gamma) ? (R)0.5 * mm * sg : -phi * mm * sg;
    else if constexpr (FORM == F_DIRECT)
      w = s.on_gamma ? phi * mm * sg : (R)0.5 * phi * mm * sg;
    else  // the Neumann row's kernel with its arguments swapped, over the line density
      w = phi * mm * sg;
  } else {
    const R rho = fabs(h.t);
    const R acy = fabs(dot3(s.d, ny));
    if (s.gscale != (R)0) {
      // G / p (times -k / p_k at a Dirichlet vertex)
      w = s.gscale * (D == 3 ? mm * rho / ((R)2 * acy) : -mm * rho * log(rho) / ((R)2 * acy));
    } else {
      const R cx = sgn_t * dot3(s.d, s.nc);
      w = D == 3 ? -phi * mm * (cx + s.gc.alpha * rho) / acy
                 : -phi * mm * (cx - s.gc.alpha * rho * log(rho)) / acy;
    }
    if (s.mixture) w /= ((R)1 - a.self_p);
  }
  if (CV && s.i > 0) s.acc += s.W * h.src;  // all-hits sum of a(h) F(y_h), emissions included
  if constexpr (GRAD) {
    if (s.i == 0) {
      // line 0 from x0 off the boundary: w' = grad_x kernel / p, with
      // rhat = sgn(t) d, rho = |t|, c = rhat . n_y (2D and 3D alike):
      //   single layer  grad G / p           = m rhat / (2 |c|)
      //   double layer  -grad dG/dn_y / p    = -m (n_y - D c rhat) / (2 rho |c|)
      //   direct BIE    -phi grad dG/dn_y / p (the same times phi)
      const R* n = ny;
      R wg[3];
      const R c = sgn_t * dot3(s.d, n), ac = fabs(c), rho = fabs(h.t);
      if constexpr (is_sl(FORM)) {
        const R f = s.gscale * mm * sgn_t / ((R)2 * ac);
#pragma unroll
        for (int k = 0; k < 3; ++k) wg[k] = f * s.d[k];
      } else {
        const R f = (FORM == F_DL ? (R)-1 : -phi) * mm / ((R)2 * rho * ac);
#pragma unroll
        for (int k = 0; k < 3; ++k) wg[k] = f * (n[k] - (R)D * c * sgn_t * s.d[k]);
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        s.Wg[k] = s.Wg[k] * w + s.W * wg[k];
        s.Wg0[k] = wg[k];
      }
    } else {
#pragma unroll
      for (int k = 0; k < 3; ++k) s.Wg[k] *= w;
    }
  }
  s.W *= w;
  s.x[0] = y[0];
  s.x[1] = y[1];
  s.x[2] = y[2];
  s.cur_idx = h.idx;
  if constexpr (CV) {
    // subtract the table at the picked hit (line 0: the line-0 table, whose
    // exact mean the add-back restores; the emission of line 0 stays as is)
    if (s.i == 0) {
      s.acc -= s.W * a.cv_g0[gy.id];
      s.acc += s.W * (R)2 * phi * boundary_datum<R, D, VD>(a.prog, gy, ny, s.x);
    } else {
      s.acc -= s.W * a.cv_g[gy.id];
    }
  } else if constexpr (is_sl(FORM)) {
    const R e = sl_emission<R, D, VD>(a, gy, ny, s.x, s.i + 1 >= a.M);
    s.acc += s.W * e;
    if constexpr (GRAD) {
#pragma unroll
      for (int k = 0; k < 3; ++k) s.gacc[k] += s.Wg[k] * e;
    }
  } else if constexpr (FORM == F_DL) {
    const R e = ((s.i + 1 < a.M) ? (R)2 * phi : phi) * boundary_datum<R, D, VD>(a.prog, gy, ny, s.x);
    s.acc += s.W * e;
    if constexpr (GRAD) {
#pragma unroll
      for (int k = 0; k < 3; ++k) s.gacc[k] += s.Wg[k] * e;
    }
  } else if constexpr (FORM == F_FWD) {
    fwd_record<R, D>(a, s, s.i + 1, gy.id, h.m);
  }
  ++s.i;
  return begin_step<R, D, FORM, TRACE, COUNT, EXT>(a, s, wc);
}


// Learned control variate, single layer, 3D (not in the paper): the same
// paths as the plain walk (same draws, same picks) plus, at every line, a term
// with zero mean given the line (the pick is uniform over the m hits):
//   line 0:        - w(j) g0(T_j); its mean sum_T g0_T int_T G(x0, y) dA is
//                  added per point by the add-back kernel (a self-panel
//                  sample at a boundary x0 subtracts w g0(T0) the same way);
//   lines 1..M-2:  sum_h a(h) [2 phi s(y_h) + g(T_h)] - w(j) g(T_j)
//                  (the picked emission is inside the sum);
//   line M-1:      sum_h a(h) phi s(y_h), the exact conditional mean of the
//                  last emission, so no pick is needed;
// with a(h) = w(h) / m the weight of hit h without the 1/m of the pick.

__device__ __forceinline__ void chan_merge(double& n, double& mean, double& m2, double nb,
                                           double meanb, double m2b) {
  if (nb == 0.0) return;
  if (n == 0.0) {
    n = nb;
    mean = meanb;
    m2 = m2b;
    return;
  }
  const double nn = n + nb;
  const double delta = meanb - mean;
  mean += delta * (nb / nn);
  m2 += m2b + delta * delta * (n * nb / nn);
  n = nn;
}

// One block's share of a solve: BLOCK lanes cover BLOCK >> lpp_shift points,
// the N paths of a point on lpp = 1 << lpp_shift consecutive lanes.  The lanes
// of a point inside one wavefront (G = min(lpp, 64) of them, the first at
// L0 within the point) share the paths L0 + (c mod G) + (c / G) lpp, c = 0,
// 1, ...: each takes the next free c when its path ends, so the wavefront's
// lanes finish together instead of waiting for the lane whose share of paths
// ran longest.  Pooled solves (pools_points) share across two points: the
// 2 lpp lanes of points 2j, 2j + 1 take c = 0 .. 2N - 1 as (point c >= N,
// path c mod N), which halves the time the lanes wait for the group's last
// paths.  A path's value depends on its index only, not on the lane.
// `red` is BLOCK / 64 x red_stride<EXT, D>() doubles of LDS.
template <int EXT, int D>
constexpr int red_stride() { return ext_kind(EXT) == X_GRAD ? 3 + 2 * D : 3; }

template <typename R, int D, int FORM, bool TRACE, bool COUNT, int BLOCK, int EXT = X_NONE>
__device__ __forceinline__ void walk_block(const WalkArgs<R, D>& a, int64_t block_index, double* red) {
  const int tid = threadIdx.x;
  const int lpp = 1 << a.lpp_shift;
  constexpr bool POOL = pools_points(FORM, EXT, TRACE, COUNT);
  // the lane group that shares a pool of paths: G lanes, a power of two,
  // aligned; its first point point0
  const int gshift = POOL ? a.lpp_shift + 1 : (a.lpp_shift < 6 ? a.lpp_shift : 6);
  const int G = 1 << gshift;
  const int64_t point0 =
      block_index * (BLOCK >> a.lpp_shift) + (POOL ? ((tid >> a.lpp_shift) & ~1) : (tid >> a.lpp_shift));
  const int lane_in_point = tid & (lpp - 1);
  // the group's next free counter, in LDS after the stacks and held leaves
  // (the first G counters start at once); only this wavefront reads and
  // writes it
  if ((tid & (G - 1)) == 0)
    __hip_atomic_store(wob_stack + (a.scene.stack_cap + kLeafSlots) * BLOCK + tid, G, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_WAVEFRONT);
  // the path offset, read back at each path's start: kept in LDS rather than
  // in a scalar register across the loops (the kernel's scalar registers are
  // all in use; one more spills others into the hot loops).  Every wavefront
  // writes the same value before it reads it.
  int32_t* const offset_word = wob_stack + (a.scene.stack_cap + kLeafSlots + 1) * BLOCK;
  if ((tid & 63) == 0) *offset_word = a.path_offset;
  // counter c of the group -> the path's point (0 or 1 within the pool) and
  // index; false past the group's last path (c is taken in increasing order,
  // and so are the paths it names)
  auto path_of = [&](int c, int& pl_, int& k_) -> bool {
    if constexpr (POOL) {
      pl_ = c >= a.N ? 1 : 0;
      k_ = c - pl_ * a.N;
      return c < 2 * a.N && point0 + pl_ < a.n_points;
    } else {
      pl_ = 0;
      k_ = (lane_in_point & ~(G - 1)) + (c & (G - 1)) + (c >> gshift) * lpp;
      return k_ < a.N && point0 < a.n_points;
    }
  };
  double n = 0.0, mean = 0.0, m2 = 0.0;
  // pooled: the statistics of the pool's second point
  double n1 = 0.0, mean1 = 0.0, m21 = 0.0;
  constexpr bool GRAD = ext_kind(EXT) == X_GRAD;
  constexpr int GD = GRAD ? D : 1;  // gradient statistics per component (unused otherwise)
  double gmean[GD], gm2[GD];
#pragma unroll
  for (int c = 0; c < GD; ++c) gmean[c] = gm2[c] = 0.0;
  WorkCount wc = {0, 0, 0, 0};
  // the corrected walk exists for the 3D single layer only (lines and RIS)
  constexpr int KEXT =
      (ext_kind(EXT) == X_CV && !(D == 3 && (FORM == F_SL || FORM == F_SL_RIS))) ? (EXT & X_VDATA) : EXT;
  {
    // The lane's paths (first the one of counter c = its place in the group,
    // then the group's next free ones) run as one state machine.  Lanes step
    // through BVH nodes; a lane that has reached four crossed leaves parks
    // until half of the stepping lanes have parked, and the lanes holding
    // leaves then test them together; a lane at the end of its line parks
    // until a quarter of the working lanes have, and those lanes then take
    // their path steps together.  That code thus runs on many lanes at
    // once instead of on the one or two lanes that stand at a leaf or a line
    // end in a given node step.
    PathState<R, D> s;
    int k = 0, pl = 0;
    int64_t point = point0;  // the point of the lane's path
    int st = ST_NONE;
    // the lane's traversal stack: LDS, entry k at wob_stack[k * BLOCK + tid]
    // (consecutive lanes in consecutive banks); empty between lines.  After
    // its stack_cap entries come kLeafSlots more: the crossed leaves the lane
    // holds (nq of them) until the leaf test; a lane holding fewer than
    // kLeafSlots keeps stepping
    int32_t* const stk = wob_stack + tid;
    int32_t* const leafq = stk + a.scene.stack_cap * BLOCK;
    int sp = 0, nq = 0;
    auto load_point = [&]() {
      if constexpr (FORM == F_FWD) {
        s.point = 0xfffffffeu;  // forward paths: no evaluation point
      } else {
        s.x0[0] = a.points[point * D + 0];
        s.x0[1] = a.points[point * D + 1];
        s.x0[2] = D == 3 ? a.points[point * D + 2] : (R)0;
        s.prim0 = a.point_prim ? a.point_prim[point] : -1;
        s.point = a.point_ids ? a.point_ids[point] : (uint32_t)point;
      }
    };
    if (path_of(tid & (G - 1), pl, k)) {
      point = point0 + pl;
      load_point();
      st = start_path<R, D, FORM, TRACE, COUNT, KEXT>(a, s, (uint32_t)(*offset_word + k), point * (int64_t)a.N + k,
                                                      wc);
    }
    for (;;) {
      // finished paths: record, start the lane's next one
      while (st == ST_DONE) {
        // boundary split (gradient walks of the double layer): a path whose
        // point has an anchor and whose line 0 met the boundary runs the
        // coupled walk from the anchor next, then subtracts w' times its value
        int32_t couple = -1;
        bool take = false;
        {
          if constexpr (GRAD && FORM == F_DL) {
            if (s.coupled) {
#pragma unroll
              for (int c = 0; c < 3; ++c) s.gacc[c] -= s.Wg0[c] * s.acc;
              s.acc = s.acc_main;
              s.coupled = false;
            } else if (a.anchor_prim) {
              const int32_t anchor = a.anchor_prim[point];
              if (anchor >= 0 && (s.Wg0[0] != (R)0 || s.Wg0[1] != (R)0 || s.Wg0[2] != (R)0)) couple = anchor;
              else if (anchor < -1) s.gacc[0] = (R)NAN;  // a caller error: the gradient is NaN
            }
          }
          if (couple < 0) {
            const R v = s.acc;
            if (TRACE) a.path_out[point * (int64_t)a.N + k] = v;
            bool finite = isfinite(v);
            if constexpr (GRAD) {
#pragma unroll
              for (int c = 0; c < GD; ++c) {
                if (TRACE) a.path_grad_out[(point * (int64_t)a.N + k) * D + c] = s.gacc[c];
                finite = finite && isfinite(s.gacc[c]);
              }
            }
            if (POOL && finite && pl) {
              n1 += 1.0;
              const double dv = (double)v - mean1;
              mean1 += dv / n1;
              m21 += dv * ((double)v - mean1);
            } else if (finite) {
              n += 1.0;
              const double dv = (double)v - mean;
              mean += dv / n;
              m2 += dv * ((double)v - mean);
              if constexpr (GRAD) {
#pragma unroll
                for (int c = 0; c < GD; ++c) {
                  const double dg = (double)s.gacc[c] - gmean[c];
                  gmean[c] += dg / n;
                  gm2[c] += dg * ((double)s.gacc[c] - gmean[c]);
                }
              }
            } else if (!TRACE && !COUNT && FORM != F_FWD && a.status) {
              // a non-finite path (degenerate geometry, an invalid primitive id, data
              // singular on the boundary) is counted and left out of the statistics
              atomicAdd(a.status, 1ull);
            }
            take = true;
          }
        }
        // the lanes of the group that take a path here get its next counters in
        // lane order (every lane reads the counter before the first one of
        // them writes it back)
        const uint64_t grab = __ballot(take);
        bool go = couple >= 0;
        if (take) {
          const int lane = tid & 63;
          const uint64_t mine = G == 64 ? grab : grab & (((1ull << G) - 1) << (lane & ~(G - 1)));
          const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mine >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mine, 0u));
          // atomic loads and stores: other lanes write the counter, and a plain
          // load may be hoisted out of this loop and kept in a register that
          // only the writing lane updates (stale counters, repeated paths)
          int32_t* const gnext = wob_stack + (a.scene.stack_cap + kLeafSlots) * BLOCK + (tid & ~(G - 1));
          const int c = __hip_atomic_load(gnext, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) + rank;
          if (rank == 0) __hip_atomic_store(gnext, c + __popcll(mine), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
          int pn;
          go = path_of(c, pn, k);
          if (POOL && go && pn != pl) {  // the pool's second point: its data
            pl = pn;
            point = point0 + pl;
            load_point();
          }
        }
        st = go ? start_path<R, D, FORM, TRACE, COUNT, KEXT>(a, s, (uint32_t)(*offset_word + k),
                                                             point * (int64_t)a.N + k, wc,
                                                             couple, point)
                : ST_NONE;
      }
      const int idle = __popcll(__ballot(st == ST_NONE));
      if (idle == 64) break;
      // lanes parked at the end of their line, and lanes that step through nodes
      const int ends = __popcll(__ballot(st == ST_LINE && nq == 0 && s.ni == kDone));
      const int active = 64 - idle - ends;
      // node steps until half of the stepping lanes hold four crossed leaves
      // or stand at the end of their line; a lane keeps stepping while it
      // holds fewer (measured on the icosphere benchmark: parking at the
      // first / second / third / fourth leaf 622 / 694 / 725 / 733 M path
      // samples/s; with two, a wait for 3/8, 1/2, 5/8 of the lanes: 678, 688,
      // 677; with four and the shared paths, 3/8, 1/2, 5/8 on the three-tori
      // workload: 1,284, 1,303, 1,287)
      const int want = (active * 4 + 7) >> 3;
      bool trav = st == ST_LINE && nq == 0 && s.ni != kDone;
      while (trav) {
        if (active - __popcll(__ballot(1)) >= want) break;
        // one step: take the position (or pop it), fetch an interior record by
        // a 32-bit byte offset from the uniform base, test its child boxes,
        // continue with one crossed entry and push the others; a leaf entry
        // goes to the lane's leaf queue, and the fourth one parks the lane
        int32_t e = s.ni;
        if (e == kPop) e = sp > 0 ? stk[--sp * BLOCK] : kDone;
        if (e >= 0 && e != kDone) {
          using Node = typename Rec<R, D>::Node;
          const Node node = *reinterpret_cast<const Node*>(reinterpret_cast<const char*>(a.scene.nodes) +
                                                           (uint32_t)e * (uint32_t)sizeof(Node));
          if (COUNT) wc.nodes += 1;
          const uint32_t m = child_mask<R, D>(node, s.inv, s.ox, s.rot);
          // continue with the first crossed entry, push the others
          e = kPop;
#pragma unroll
          for (int q = 0; q < kArity; ++q) {
            if (m & (1u << q)) {
              if (e == kPop) e = node.child[q];
              else if (sp < a.scene.stack_cap) stk[sp++ * BLOCK] = node.child[q];
            }
          }
        }
        const bool at_leaf = e < 0 && e != kPop;
        if (at_leaf) leafq[nq++ * BLOCK] = -1 - e;
        s.ni = at_leaf ? kPop : e;
        trav = nq < kLeafSlots && e != kDone;
      }
      // the lanes holding leaves test them together
      if (nq > 0) {
        const int32_t c1 = leafq[0], c2 = nq > 1 ? leafq[BLOCK] : -1, c3 = nq > 2 ? leafq[2 * BLOCK] : -1;
        const int32_t c4 = nq > 3 ? leafq[3 * BLOCK] : -1;
        leaf_work<R, D, FORM, COUNT, KEXT>(a, s, c1, c2, c3, c4, wc);
        nq = 0;
      }
      // path steps run once a quarter of the working lanes stand at the end of
      // their line, or when no lane steps (measured: 557, 574, 566 M path
      // samples/s for 1/8, 1/4, 3/8; with the shared paths on the three-tori
      // workload 1,279, 1,303, 1,280)
      const bool at_end = st == ST_LINE && s.ni == kDone;
      const int n_end = __popcll(__ballot(at_end));
      const int stepping = __popcll(__ballot(st == ST_LINE && s.ni != kDone));
      if (4 * n_end >= 64 - idle || stepping == 0) {
        if (at_end) st = end_step<R, D, FORM, TRACE, COUNT, KEXT>(a, s, wc);
      }
    }
  }
  if (COUNT) {
    unsigned long long c[4] = {wc.lines, wc.nodes, wc.prims, wc.hits};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      for (int off = 32; off > 0; off >>= 1) c[k] += __shfl_xor(c[k], off, 64);
      if ((tid & 63) == 0) atomicAdd(a.counters + k, c[k]);
    }
    return;
  }
  if (TRACE || FORM == F_FWD) return;

  if constexpr (POOL) {
    // each of the pool's two points: merged over the group's lanes
#pragma unroll
    for (int slot = 0; slot < 2; ++slot) {
      double tn = slot ? n1 : n, tm = slot ? mean1 : mean, ts = slot ? m21 : m2;
      for (int off = G >> 1; off > 0; off >>= 1) {
        const double nb = __shfl_xor(tn, off, 64);
        const double mb = __shfl_xor(tm, off, 64);
        const double sb = __shfl_xor(ts, off, 64);
        if (((tid & 63) & off) == 0) {
          chan_merge(tn, tm, ts, nb, mb, sb);
        } else {
          double n2 = nb, mean2 = mb, m22 = sb;
          chan_merge(n2, mean2, m22, tn, tm, ts);
          tn = n2;
          tm = mean2;
          ts = m22;
        }
      }
      const int64_t pt = point0 + slot;
      if ((tid & (G - 1)) == 0 && pt < a.n_points) {
        a.mean_out[pt] = tn > 0.0 ? (R)tm : (R)NAN;
        if (a.var_out) a.var_out[pt] = (R)(tn > 1.0 ? ts / (tn - 1.0) : 0.0);
      }
    }
    return;
  }

  // per-point0 reduction: within the point0's lanes of the wavefront, then across
  // the point0's wavefronts
  // (the gradient components merge with the same counts, in the same order)
  for (int off = (lpp < 64 ? lpp : 64) >> 1; off > 0; off >>= 1) {
    const double nb = __shfl_xor(n, off, 64);
    const double mb = __shfl_xor(mean, off, 64);
    const double sb = __shfl_xor(m2, off, 64);
    const bool low = ((tid & 63) & off) == 0;
    if constexpr (GRAD) {
#pragma unroll
      for (int c = 0; c < GD; ++c) {
        const double gmb = __shfl_xor(gmean[c], off, 64);
        const double gsb = __shfl_xor(gm2[c], off, 64);
        double n1 = n, n2 = nb;
        if (low) {
          chan_merge(n1, gmean[c], gm2[c], nb, gmb, gsb);
        } else {
          double mean2 = gmb, m22 = gsb;
          chan_merge(n2, mean2, m22, n, gmean[c], gm2[c]);
          gmean[c] = mean2;
          gm2[c] = m22;
        }
      }
    }
    if (low) {
      chan_merge(n, mean, m2, nb, mb, sb);
    } else {
      double n2 = nb, mean2 = mb, m22 = sb;
      chan_merge(n2, mean2, m22, n, mean, m2);
      n = n2;
      mean = mean2;
      m2 = m22;
    }
  }
  if (lpp <= 64) {
    if (lane_in_point == 0 && point0 < a.n_points) {
      a.mean_out[point0] = n > 0.0 ? (R)mean : (R)NAN;
      if (a.var_out) a.var_out[point0] = (R)(n > 1.0 ? m2 / (n - 1.0) : 0.0);
      if constexpr (GRAD) {
#pragma unroll
        for (int c = 0; c < GD; ++c) {
          a.grad_out[point0 * D + c] = n > 0.0 ? (R)gmean[c] : (R)NAN;
          if (a.grad_var_out) a.grad_var_out[point0 * D + c] = (R)(n > 1.0 ? gm2[c] / (n - 1.0) : 0.0);
        }
      }
    }
    return;
  }
  constexpr int RS = red_stride<EXT, D>();
  const int wave = tid >> 6;
  if ((tid & 63) == 0) {
    red[wave * RS + 0] = n;
    red[wave * RS + 1] = mean;
    red[wave * RS + 2] = m2;
    if constexpr (GRAD) {
#pragma unroll
      for (int c = 0; c < GD; ++c) {
        red[wave * RS + 3 + 2 * c] = gmean[c];
        red[wave * RS + 4 + 2 * c] = gm2[c];
      }
    }
  }
  __syncthreads();
  if (lane_in_point == 0 && point0 < a.n_points) {
    const int waves = lpp >> 6;
    double tn = red[wave * RS + 0], tm = red[wave * RS + 1], ts = red[wave * RS + 2];
    if constexpr (GRAD) {
#pragma unroll
      for (int c = 0; c < GD; ++c) {
        double gn = tn, gm = red[wave * RS + 3 + 2 * c], gs = red[wave * RS + 4 + 2 * c];
        for (int w = 1; w < waves; ++w)
          chan_merge(gn, gm, gs, red[(wave + w) * RS + 0], red[(wave + w) * RS + 3 + 2 * c],
                     red[(wave + w) * RS + 4 + 2 * c]);
        a.grad_out[point0 * D + c] = gn > 0.0 ? (R)gm : (R)NAN;
        if (a.grad_var_out) a.grad_var_out[point0 * D + c] = (R)(gn > 1.0 ? gs / (gn - 1.0) : 0.0);
      }
    }
    for (int w = 1; w < waves; ++w)
      chan_merge(tn, tm, ts, red[(wave + w) * RS + 0], red[(wave + w) * RS + 1], red[(wave + w) * RS + 2]);
    a.mean_out[point0] = tn > 0.0 ? (R)tm : (R)NAN;
    if (a.var_out) a.var_out[point0] = (R)(tn > 1.0 ? ts / (tn - 1.0) : 0.0);
  }
}

template <typename R, int D, int FORM, bool TRACE, bool COUNT, int BLOCK, int EXT = X_NONE>
__global__ void __launch_bounds__(BLOCK) walk_kernel(WalkArgs<R, D> a) {
  __shared__ double red[(BLOCK / 64) * red_stride<EXT, D>()];
  walk_block<R, D, FORM, TRACE, COUNT, BLOCK, EXT>(a, blockIdx.x, red);
}

// Add-back of the control variate: out[p] (+)= an unbiased value of
// sum_T g_T int_T G(x_p, y) dA.  Triangles whose centroid lies within four
// bounding radii of x_p ("near") use the closed form; every other triangle uses
// g_T A_T G(x_p, y_T) at one point y_T uniform in T (its expectation is the
// exact integral; G varies by at most ~30 % over a far triangle).  y_T depends
// on (seed, triangle) only, so it is drawn once per triangle when the triangle
// is staged and shared by every point:
//   h = hash32(id + 0x9e3779b9 (seed_lo + 1)),
//   u0 = unit(hash32(h ^ 0x68e31da4)), u1 = unit(hash32(h ^ 0xb5297a4d)),
//   reflected into the triangle when u0 + u1 > 1, y_T = v0 + u0 e1 + u1 e2.
// Every workgroup streams the triangles through LDS in tiles of 256; a far pair
// costs one distance test and one reciprocal square root.  Each lane keeps 4
// points in registers.  A tile whose triangles all have g_T = 0 adds exactly
// zero: its pairs are skipped (the whole sum, for g = 0).
template <typename R>
__global__ void __launch_bounds__(256) cv_addback_kernel(SceneView<R, 3> s, const R* __restrict__ g_by_id,
                                                         const R* __restrict__ points, int64_t n,
                                                         uint32_t seed, R* out, int accumulate) {
  // per triangle: [c (3), (4 r)^2] [y_T (3), g A / (4 pi)] [v (9), t (9), u (9), n (3), g, pad]
  // (the pad words of the first four records carry the wavefronts' votes)
  constexpr int TILE = 256, PPT = 4, NF = 40;
  __shared__ __align__(16) R tile[TILE * NF];
  const int tid = threadIdx.x;
  R x[PPT][3], acc[PPT];
  int64_t pidx[PPT];
#pragma unroll
  for (int k = 0; k < PPT; ++k) {
    pidx[k] = ((int64_t)blockIdx.x * PPT + k) * 256 + tid;
    const int64_t q = pidx[k] < n ? pidx[k] : 0;
    x[k][0] = points[q * 3 + 0];
    x[k][1] = points[q * 3 + 1];
    x[k][2] = points[q * 3 + 2];
    acc[k] = 0;
  }
  for (int32_t t0 = 0; t0 < s.n_prims; t0 += TILE) {
    __syncthreads();
    const int32_t j = t0 + tid;
    R* T = tile + tid * NF;
    bool nonzero = false;
    if (j < s.n_prims) {
      const PrimGeo<R> g = load_prim<R, 3>(s, j);
      R nn[3];
      load_normal<R, 3>(s, j, nn);
      R v[3][3];
      for (int k = 0; k < 3; ++k) {
        v[0][k] = g.v0[k];
        v[1][k] = g.v0[k] + g.e1[k];
        v[2][k] = g.v0[k] + g.e2[k];
      }
      R cen[3], rad2 = 0;
      for (int k = 0; k < 3; ++k) cen[k] = (v[0][k] + v[1][k] + v[2][k]) / (R)3;
      for (int c = 0; c < 3; ++c) {
        const int c1 = c == 2 ? 0 : c + 1;
        R e[3] = {v[c1][0] - v[c][0], v[c1][1] - v[c][1], v[c1][2] - v[c][2]};
        const R il = rsqrt_<R>(dot3(e, e));
        R tt[3] = {e[0] * il, e[1] * il, e[2] * il}, uu[3];
        cross3(tt, nn, uu);
        R dc[3] = {v[c][0] - cen[0], v[c][1] - cen[1], v[c][2] - cen[2]};
        rad2 = fmax(rad2, dot3(dc, dc));
        for (int k = 0; k < 3; ++k) {
          T[8 + c * 3 + k] = v[c][k];
          T[17 + c * 3 + k] = tt[k];
          T[26 + c * 3 + k] = uu[k];
        }
      }
      R cr[3];
      cross3(g.e1, g.e2, cr);
      const R gT = g_by_id[g.id];
      nonzero = gT != (R)0;
      const uint32_t h = hash32((uint32_t)g.id + 0x9e3779b9u * (seed + 1u));
      R a = unit<R>(hash32(h ^ 0x68e31da4u)), b = unit<R>(hash32(h ^ 0xb5297a4du));
      if (a + b > (R)1) {
        a = (R)1 - a;
        b = (R)1 - b;
      }
      T[0] = cen[0];
      T[1] = cen[1];
      T[2] = cen[2];
      T[3] = (R)16 * rad2;  // (4 r)^2
      for (int k = 0; k < 3; ++k) T[4 + k] = v[0][k] + a * (v[1][k] - v[0][k]) + b * (v[2][k] - v[0][k]);
      T[7] = gT * (R)0.5 * sqrt(dot3(cr, cr)) * (R)(0.25 / 3.14159265358979323846);
      T[35] = nn[0];
      T[36] = nn[1];
      T[37] = nn[2];
      T[38] = gT;
    }
    // whether any g_T of the tile is non-zero: each wavefront's vote in the
    // pad word of one of the first four records (no LDS beyond the tile's
    // 40 KiB, which lets four workgroups share a CU)
    const bool wave_nonzero = __ballot(nonzero) != 0;  // every lane of the wavefront votes
    if ((tid & 63) == 0) tile[(tid >> 6) * NF + 39] = wave_nonzero ? (R)1 : (R)0;
    __syncthreads();
    if (tile[39] == (R)0 && tile[NF + 39] == (R)0 && tile[2 * NF + 39] == (R)0 && tile[3 * NF + 39] == (R)0)
      continue;  // the same decision in every lane
    const int cnt = s.n_prims - t0 < TILE ? s.n_prims - t0 : TILE;
    for (int q = 0; q < cnt; ++q) {
      const R* P = tile + q * NF;
      const R c0 = P[0], c1 = P[1], c2 = P[2], near2 = P[3];
      const R y0 = P[4], y1 = P[5], y2 = P[6], gw = P[7];
#pragma unroll
      for (int k = 0; k < PPT; ++k) {
        const R dx = x[k][0] - c0, dy = x[k][1] - c1, dz = x[k][2] - c2;
        if (dx * dx + dy * dy + dz * dz < near2) {
          R v[3][3], tt[3][3], uu[3][3], nn[3];
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int m = 0; m < 3; ++m) {
              v[c][m] = P[8 + c * 3 + m];
              tt[c][m] = P[17 + c * 3 + m];
              uu[c][m] = P[26 + c * 3 + m];
            }
          nn[0] = P[35];
          nn[1] = P[36];
          nn[2] = P[37];
          acc[k] += P[38] * tri_potential<R>(v, tt, uu, nn, x[k]);
        } else {
          const R yx = y0 - x[k][0], yy = y1 - x[k][1], yz = y2 - x[k][2];
          acc[k] += gw * rsqrt_<R>(yx * yx + yy * yy + yz * yz);
        }
      }
    }
  }
#pragma unroll
  for (int k = 0; k < PPT; ++k)
    if (pidx[k] < n) out[pidx[k]] = accumulate ? out[pidx[k]] + acc[k] : acc[k];
}

// g0[id] = (g ? g[id] : 0) + 2 phi s(centroid of id): the line-0 table of the
// control variate with the first emission frozen per triangle (3D).
template <typename R>
__global__ void emission_table_kernel(SceneView<R, 3> s, ProgramView<R> prog, R phi, const float* g,
                                      float* g0) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= s.n_prims) return;
  const PrimGeo<R> p = load_prim<R, 3>(s, j);
  R n[3], y[3];
  load_normal<R, 3>(s, j, n);
  for (int k = 0; k < 3; ++k) y[k] = p.v0[k] + (p.e1[k] + p.e2[k]) / (R)3;
  const R e = (R)2 * phi * boundary_datum<R, 3>(prog, p, n, y);
  g0[p.id] = (float)((g ? (R)g[p.id] : (R)0) + e);
}


// Area-uniform points on the boundary: primitive by binary search of the
// area CDF, then a uniform point on it.  Philox counter (i, 0xffffffff,
// 0xffffff03, 0): block 3 of the last problem / line slot, a stream the walk
// never draws.
template <typename R, int D>
__global__ void sample_boundary_kernel(SceneView<R, D> s, const float* __restrict__ cdf, int64_t n,
                                       uint32_t k0, uint32_t k1, R* points, int32_t* prim_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const U4 r = philox((uint32_t)i, 0xffffffffu, 0xffffff03u, 0u, k0, k1);
  const float u = unit<float>(r.x);
  int32_t lo = 0, hi = s.n_prims - 1;
  while (lo < hi) {  // first caller id with cdf > u
    const int32_t mid = (lo + hi) >> 1;
    if (cdf[mid] > u) hi = mid;
    else lo = mid + 1;
  }
  const PrimGeo<R> g = load_prim<R, D>(s, s.leaf_of_id[lo]);
  R a = unit<R>(r.y), b = D == 3 ? unit<R>(r.z) : (R)0;
  if (a + b > (R)1) {
    a = (R)1 - a;
    b = (R)1 - b;
  }
  R y[3];
  hit_point(g, a, b, y);
  for (int k = 0; k < D; ++k) points[i * D + k] = y[k];
  prim_out[i] = g.id;
}

// Centroid of every primitive, written at its caller id (3D).

template <typename R>
__global__ void centroid_kernel(SceneView<R, 3> s, float* out) {
  const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= s.n_prims) return;
  const PrimGeo<R> g = load_prim<R, 3>(s, j);
  for (int k = 0; k < 3; ++k) out[(int64_t)g.id * 3 + k] = (float)(g.v0[k] + (g.e1[k] + g.e2[k]) / (R)3);
}

// Persistent batched solve: every block pulls tiles (problem, block of points)
// from a device counter until none is left.  Tiles of one problem are
// contiguous; tile_off (n_probs + 1 entries) is the prefix sum of tiles per
// problem.  With stride > 1 only every stride-th tile runs (autotuner timing).
// VX: X_VDATA when some problem gives its data per vertex.
template <typename R, int D, int BLOCK, int VX = X_NONE>
__global__ void __launch_bounds__(BLOCK) batch_kernel(const WalkArgs<R, D>* __restrict__ probs,
                                                      const int64_t* __restrict__ tile_off,
                                                      int32_t n_probs, int64_t stride,
                                                      unsigned long long* __restrict__ counter) {
  __shared__ double red[(BLOCK / 64) * 3];
  __shared__ long long s_tile;
  const int64_t n_tiles = tile_off[n_probs];
  for (;;) {
    if (threadIdx.x == 0) s_tile = (long long)atomicAdd(counter, 1ull) * stride;
    __syncthreads();
    const int64_t tile = s_tile;
    __syncthreads();
    if (tile >= n_tiles) break;
    int lo = 0, hi = n_probs - 1;
    while (lo < hi) {  // last problem whose first tile is <= tile
      const int mid = (lo + hi + 1) >> 1;
      if (tile_off[mid] <= tile) lo = mid;
      else hi = mid - 1;
    }
    const int b = __builtin_amdgcn_readfirstlane(lo);
    const WalkArgs<R, D>& a = probs[b];
    const int64_t local = tile - tile_off[b];
    const int form = __builtin_amdgcn_readfirstlane(a.form);
    if (form == F_DL) walk_block<R, D, F_DL, false, false, BLOCK, VX>(a, local, red);
    else if (form == F_DIRECT) walk_block<R, D, F_DIRECT, false, false, BLOCK, VX>(a, local, red);
    else if (form == F_SL_RIS) walk_block<R, D, F_SL_RIS, false, false, BLOCK, VX>(a, local, red);
    else walk_block<R, D, F_SL, false, false, BLOCK, VX>(a, local, red);
  }
}


// Every hit of each line, in traversal order (parity / debugging).
template <typename R, int D>
__global__ void __launch_bounds__(256) intersect_kernel(SceneView<R, D> s, const R* orig, const R* dir,
                                                        const int32_t* exclude, int64_t n_lines,
                                                        int32_t max_hits, int32_t* n_hits,
                                                        int32_t* hit_ids, R* hit_t) {
  const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= n_lines) return;
  R x[3], d[3], inv[3], ox[3];
  uint32_t rot[3];
  for (int a = 0; a < 3; ++a) {
    x[a] = a < D ? orig[l * D + a] : (R)0;
    d[a] = a < D ? dir[l * D + a] : (R)0;
  }
  line_slabs<R, D>(s, x, d, inv, ox, rot);
  const int32_t ex_id = exclude ? exclude[l] : -1;
  const int32_t ex = (ex_id >= 0 && ex_id < s.n_prims) ? s.leaf_of_id[ex_id] : -1;
  int32_t cnt = 0;
  WorkCount wc = {0, 0, 0, 0};
  for_each_leaf<R, D, false>(s, inv, ox, rot, wc, [&](int32_t first, int32_t count) {
    for (int32_t j = first; j < first + count; ++j) {
      if (j == ex) continue;
      const PrimGeo<R> g = load_prim<R, D>(s, j);
      R t, u, v;
      if (!hit_prim<R, D>(g, x, d, t, u, v)) continue;
      if (cnt < max_hits) {
        hit_ids[l * max_hits + cnt] = g.id;
        if (hit_t) {
          // the line parameter as the walk takes it: from the primitive's plane
          R n[3], y[3];
          load_normal<R, D>(s, j, n);
          hit_t[l * max_hits + cnt] = plane_hit<R, D>(g, n, x, d, y);
        }
      }
      ++cnt;
    }
  });
  n_hits[l] = cnt;
}

}  // namespace wob
