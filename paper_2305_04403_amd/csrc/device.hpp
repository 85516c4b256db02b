// Device-side building blocks of the walk-on-boundary path kernels (gfx950).
//
// Everything here runs per lane: one lane owns one Monte Carlo path.  The walk
// is not a contraction, so there is no MFMA in it; the cost is the all-hits
// line traversal, which is bound by gathers from the cache level that holds
// the scene.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wob {

// F_SL_RIS is the single layer with resampled importance sampling: its own
// kernel form, so that the line-sampling kernels carry none of its registers.
// F_FWD is the forward (adjoint) single-layer walk from the boundary.
enum Formulation { F_DL = 1, F_DIRECT = 2, F_SL = 3, F_SL_RIS = 4, F_FWD = 5 };
__host__ __device__ constexpr bool is_sl(int f) { return f == F_SL || f == F_SL_RIS; }
enum Kind { K_DIRICHLET = 0, K_NEUMANN = 1, K_ROBIN = 2 };
// P_VERTEX: data given per mesh vertex, interpolated linearly on each primitive
enum Program { P_CONST = 0, P_LINEAR = 1, P_QUAD = 2, P_INVDIST = 3, P_VERTEX = 4 };

// --------------------------------------------------------------------------
// Scene records.  Primitives are stored in BVH leaf order.  idkind packs the
// caller's primitive id (bits 0..28) and its boundary kind (bits 29..30).
// --------------------------------------------------------------------------
// The BVH is stored as 4-wide interior records: the host collapses the binary
// SAH tree (a record takes its node's two children and opens the largest
// interior ones until it holds four entries), so a line takes half the
// dependent record fetches of a binary tree and one record is one 64-byte
// line.  The traversal is bound by the rate at which the CUs' vector memory
// path serves the lanes' gathers, so records are kept small: in an FP32 scene
// the boxes are binary16 in a normalised frame (scene centre c, power-of-two
// scale k, y' = (y - c) k in [-1, 1]), rounded outward, and the slab test
// reads them with mixed-precision FMAs.  A child entry is the index of an
// interior record (>= 0) or a leaf, -1 - ((first << 3) | (count - 1)) with
// first the leaf-order index of its first primitive (< 2^27).  Unused slots
// hold an empty box (lo > hi), which no line crosses.
constexpr int kArity = 4;
template <typename R> struct alignas(32) Wide { R lo[kArity][3], hi[kArity][3]; int32_t child[kArity]; };
// FP32 scenes: one word per box and axis, binary16 lo in the low half and hi
// in the high half.  A lane rotates each word by 16 bits when its direction is
// negative on that axis, so the low half is the slab's near side and the high
// half its far side without a min / max per axis.  (2D scenes leave the third
// axis word unused.)
template <> struct alignas(64) Wide<float> { uint32_t box[kArity][3]; int32_t child[kArity]; };
// Traversal positions besides entries: take the next entry from the stack,
// and the line's traversal is over.
constexpr int32_t kPop = INT32_MIN;
constexpr int32_t kDone = INT32_MAX;
// Bound on the traversal stack: a record pushes the crossed entries it does
// not continue with (up to three), so a lane's stack never holds more than the
// largest sum of (entries - 1) over the records on a root-to-leaf path, which
// the scene upload computes (scenes above this bound are rejected); with the
// leaf queue a lane's LDS stays within 64 entries, a 256-thread workgroup's
// within 64 KB.
constexpr int kMaxDepth = 60;
// An FP32 triangle record is padded to 64 bytes so that it never straddles a
// 64-byte block: the traversal is bound by the rate of L1-miss requests, and a
// straddling record costs two.
template <typename R> struct alignas(sizeof(R) == 4 ? 64 : 32) Prim3 { R v0[3]; int32_t idkind; R e1[3]; R alpha; R e2[3]; int32_t pad; };
template <typename R> struct alignas(16) Prim2 { R v0[2]; R e[2]; R alpha; int32_t idkind; };

template <typename R, int D> struct Rec;
template <typename R> struct Rec<R, 3> { using Node = Wide<R>; using Prim = Prim3<R>; };
template <typename R> struct Rec<R, 2> { using Node = Wide<R>; using Prim = Prim2<R>; };

constexpr int kIdBits = 29;
constexpr int32_t kIdMask = (1 << kIdBits) - 1;

template <typename R, int D>
struct SceneView {
  const typename Rec<R, D>::Node* nodes;
  const typename Rec<R, D>::Prim* prims;
  const R* normals;           // 4 per primitive (leaf order): unit outward normal, 0
  const int32_t* leaf_of_id;  // caller id -> leaf-order index
  const float* area_cdf;      // caller-id order, cumulative area / |Gamma| (binary32, last 1)
  // guide[b] = the first index whose area_cdf exceeds b / 2^guide_shift
  // (b = 0 .. 2^guide_shift; the last entry n_prims - 1)
  const int32_t* area_guide;
  int32_t guide_shift;
  R area_total;               // |Gamma|
  int32_t n_nodes;            // interior records
  int32_t n_prims;
  int32_t root;               // entry of the root: record 0, or a leaf when the tree is one leaf
  int32_t stack_cap;          // traversal stack entries per lane (the tree depth, >= 1)
  R fc[3], fk;                // frame of the boxes: y' = (y - fc) fk (fc[2] = 0 in 2D)
};

template <typename R>
struct ProgramView {
  int32_t type;
  R p[8];
  // P_VERTEX: the values (caller's vertex order), each primitive's vertex ids
  // (caller-id order, D per primitive) and the scene's rounded vertices
  const R* vdata;
  const int32_t* vid;
  const R* verts;
};

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
// --------------------------------------------------------------------------
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                      uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32 x 32 -> 64-bit multiply per product (v_mad_u64_u32) instead of a
    // low and a high multiply
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

// A 32-bit integer hash (Wellons' "lowbias32" constants) for the add-back's
// far-field sample points, where a full Philox block per (point, triangle)
// pair would cost more than the geometry.
__host__ __device__ __forceinline__ uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

// u = ((w >> 9) + 1/2) 2^-23: exact in binary32 and binary64, never 0 or 1.
template <typename R>
__device__ __forceinline__ R unit(uint32_t w) {
  return ((R)(w >> 9) + (R)0.5) * (R)(1.0 / 8388608.0);
}

template <typename R> __device__ __forceinline__ void sincospi_(R x, R* s, R* c);
template <> __device__ __forceinline__ void sincospi_<float>(float x, float* s, float* c) { sincospif(x, s, c); }
template <> __device__ __forceinline__ void sincospi_<double>(double x, double* s, double* c) { sincospi(x, s, c); }

// Uniform direction on the sphere (3D) or circle (2D); the line covers +d and -d.
template <typename R, int D>
__device__ __forceinline__ void direction(uint32_t w0, uint32_t w1, R d[3]) {
  if constexpr (D == 3) {
    const R z = (R)1 - (R)2 * unit<R>(w0);
    const R s = sqrt(fmax((R)0, (R)1 - z * z));
    R sn, cs;
    sincospi_<R>((R)2 * unit<R>(w1), &sn, &cs);
    d[0] = s * cs;
    d[1] = s * sn;
    d[2] = z;
  } else {
    R sn, cs;
    sincospi_<R>((R)2 * unit<R>(w0), &sn, &cs);
    d[0] = cs;
    d[1] = sn;
    d[2] = 0;
  }
}

// --------------------------------------------------------------------------
// Small vector helpers
// --------------------------------------------------------------------------
template <typename R> __device__ __forceinline__ R dot3(const R a[3], const R b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
template <typename R> __device__ __forceinline__ void cross3(const R a[3], const R b[3], R c[3]) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
template <typename R> __device__ __forceinline__ R rsqrt_(R v);
template <> __device__ __forceinline__ float rsqrt_<float>(float v) { return rsqrtf(v); }
template <> __device__ __forceinline__ double rsqrt_<double>(double v) { return 1.0 / sqrt(v); }

// Geometry of one primitive in a uniform 3-component form (z = 0 in 2D).
template <typename R>
struct PrimGeo {
  R v0[3], e1[3], e2[3];  // 2D: e1 = segment vector, e2 unused
  R alpha;
  int32_t id, kind;
};

template <typename R, int D>
__device__ __forceinline__ PrimGeo<R> load_prim(const SceneView<R, D>& s, int32_t idx) {
  PrimGeo<R> g;
  const auto& p = s.prims[idx];
  if constexpr (D == 3) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      g.v0[a] = p.v0[a];
      g.e1[a] = p.e1[a];
      g.e2[a] = p.e2[a];
    }
  } else {
    g.v0[0] = p.v0[0]; g.v0[1] = p.v0[1]; g.v0[2] = 0;
    g.e1[0] = p.e[0]; g.e1[1] = p.e[1]; g.e1[2] = 0;
    g.e2[0] = g.e2[1] = g.e2[2] = 0;
  }
  g.alpha = p.alpha;
  g.id = p.idkind & kIdMask;
  g.kind = (p.idkind >> kIdBits) & 3;
  return g;
}

// Unit normal pointing out of Omega.  Computed on the host in binary64 from
// the rounded vertices and stored once: the cross product of two short edges
// of a sliver triangle is too ill-conditioned to normalise in binary32.
template <typename R, int D>
__device__ __forceinline__ void load_normal(const SceneView<R, D>& s, int32_t idx, R n[3]) {
  const R* p = s.normals + 4 * (int64_t)idx;
  n[0] = p[0];
  n[1] = p[1];
  n[2] = D == 3 ? p[2] : (R)0;
}

// --------------------------------------------------------------------------
// Harmonic program and boundary datum (eq. PoissonBC)
// --------------------------------------------------------------------------
template <typename R, int D>
__device__ __forceinline__ void program_eval(const ProgramView<R>& g, const R y[3], R& u, R grad[3]) {
  grad[0] = grad[1] = grad[2] = 0;
  switch (g.type) {
    case P_CONST:
      u = g.p[0];
      break;
    case P_LINEAR:
      u = g.p[0] * y[0] + g.p[1] * y[1] + (D == 3 ? g.p[2] * y[2] : (R)0) + g.p[3];
      grad[0] = g.p[0];
      grad[1] = g.p[1];
      grad[2] = D == 3 ? g.p[2] : (R)0;
      break;
    case P_QUAD:
      u = y[0] * y[0] - y[1] * y[1];
      grad[0] = (R)2 * y[0];
      grad[1] = (R)-2 * y[1];
      break;
    default: {  // P_INVDIST
      const R r0 = y[0] - g.p[0], r1 = y[1] - g.p[1], r2 = D == 3 ? y[2] - g.p[2] : (R)0;
      const R rr = r0 * r0 + r1 * r1 + r2 * r2;
      if constexpr (D == 3) {
        const R il = rsqrt_<R>(rr);
        u = il;
        const R il3 = il * il * il;
        grad[0] = -r0 * il3;
        grad[1] = -r1 * il3;
        grad[2] = -r2 * il3;
      } else {
        u = (R)0.5 * log(rr);
        const R ir = (R)1 / rr;
        grad[0] = r0 * ir;
        grad[1] = r1 * ir;
      }
    }
  }
}

// Per-vertex data interpolated linearly on primitive g at y: the barycentric
// coordinates of y from the primitive's exact (rounded-once) vertices, solved
// in binary64 (the Gram system; a sliver's ill-conditioning stays at the
// binary64 unit), then f0 + b1 (f1 - f0) + b2 (f2 - f0).
template <typename R, int D>
__device__ __forceinline__ R vertex_datum(const ProgramView<R>& prog, const PrimGeo<R>& g, const R y[3]) {
  const int32_t* ix = prog.vid + (int64_t)g.id * D;
  double v[3][3];
#pragma unroll
  for (int c = 0; c < D; ++c)
#pragma unroll
    for (int a = 0; a < 3; ++a) v[c][a] = a < D ? (double)prog.verts[(int64_t)ix[c] * D + a] : 0.0;
  const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
  const double w[3] = {(double)y[0] - v[0][0], (double)y[1] - v[0][1], D == 3 ? (double)y[2] - v[0][2] : 0.0};
  const double f0 = (double)prog.vdata[ix[0]], d1 = (double)prog.vdata[ix[1]] - f0;
  if constexpr (D == 3) {
    const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
    const double g11 = e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2];
    const double g12 = e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2];
    const double g22 = e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2];
    const double r1 = e1[0] * w[0] + e1[1] * w[1] + e1[2] * w[2];
    const double r2 = e2[0] * w[0] + e2[1] * w[1] + e2[2] * w[2];
    const double det = g11 * g22 - g12 * g12;
    const double b1 = (r1 * g22 - r2 * g12) / det, b2 = (r2 * g11 - r1 * g12) / det;
    const double d2 = (double)prog.vdata[ix[2]] - f0;
    return (R)(f0 + b1 * d1 + b2 * d2);
  } else {
    const double b1 = (e1[0] * w[0] + e1[1] * w[1]) / (e1[0] * e1[0] + e1[1] * e1[1]);
    return (R)(f0 + b1 * d1);
  }
}

// VD: whether per-vertex data can occur (the walk kernels are instantiated
// with and without it: the binary64 interpolation costs registers, and so
// occupancy, even where it is never taken).
template <typename R, int D, bool VD = true>
__device__ __forceinline__ R boundary_datum(const ProgramView<R>& prog, const PrimGeo<R>& g,
                                            const R n[3], const R y[3]) {
  if constexpr (VD) {
    if (prog.type == P_VERTEX) return vertex_datum<R, D>(prog, g, y);
  }
  R u, grad[3];
  program_eval<R, D>(prog, y, u, grad);
  if (g.kind == K_DIRICHLET) return u;
  const R q = dot3(n, grad);
  return g.kind == K_NEUMANN ? q : q + g.alpha * u;
}

// --------------------------------------------------------------------------
// In-plane sample on the primitive that contains x.  Returns G(x, y) / p(y):
// 3D, theta uniform and radius uniform in [0, R(theta)]: G/p = R(theta) / 2;
// 2D, y uniform on the segment: G/p = -L ln|y - x| / (2 pi).
// --------------------------------------------------------------------------
template <typename R, int D>
__device__ __forceinline__ R self_panel(const PrimGeo<R>& g, const R n[3], const R x[3], R u0, R u1,
                                        R y[3]) {
  if constexpr (D == 3) {
    R t1[3], t2[3];
    const R il = rsqrt_<R>(dot3(g.e1, g.e1));
    t1[0] = g.e1[0] * il; t1[1] = g.e1[1] * il; t1[2] = g.e1[2] * il;
    cross3(n, t1, t2);
    const R b[3] = {g.v0[0] - x[0], g.v0[1] - x[1], g.v0[2] - x[2]};
    R a[3][2];
    a[0][0] = dot3(b, t1);
    a[0][1] = dot3(b, t2);
    a[1][0] = a[0][0] + dot3(g.e1, t1);
    a[1][1] = a[0][1] + dot3(g.e1, t2);
    a[2][0] = a[0][0] + dot3(g.e2, t1);
    a[2][1] = a[0][1] + dot3(g.e2, t2);
    R sn, cs;
    sincospi_<R>((R)2 * u0, &sn, &cs);
    R Rt = (R)3.0e38;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int c1 = c == 2 ? 0 : c + 1;
      const R ex = a[c1][0] - a[c][0], ey = a[c1][1] - a[c][1];
      const R den = cs * ey - sn * ex;
      if (den != (R)0) {
        const R s = (a[c][0] * ey - a[c][1] * ex) / den;
        if (s > (R)0 && s < Rt) Rt = s;
      }
    }
    if (!(Rt < (R)3.0e38)) Rt = 0;
    const R rho = u1 * Rt;
#pragma unroll
    for (int k = 0; k < 3; ++k) y[k] = x[k] + rho * (cs * t1[k] + sn * t2[k]);
    return (R)0.5 * Rt;
  } else {
    y[0] = g.v0[0] + u0 * g.e1[0];
    y[1] = g.v0[1] + u0 * g.e1[1];
    y[2] = 0;
    const R L = sqrt(g.e1[0] * g.e1[0] + g.e1[1] * g.e1[1]);
    const R dx = y[0] - x[0], dy = y[1] - x[1];
    const R rho = sqrt(dx * dx + dy * dy);
    return -L * log(rho) * (R)(0.5 / 3.14159265358979323846);
  }
}

// --------------------------------------------------------------------------
// int_T G(x, y) dA over a triangle in closed form: with d = (x - v0).n, per
// edge (unit tangent t, in-plane outward normal u = t x n) the log term
// P ln((R+ + s+)/(R- + s-)) (P = A.u, s = A.t for A = vertex - x), minus |d|
// times the solid angle of the triangle seen from x (Van Oosterom-Strackee).
// Vertices v[3], edge tangents tt[3][3], edge normals uu[3][3], normal n.
// --------------------------------------------------------------------------
template <typename R>
__device__ __forceinline__ R tri_potential(const R v[3][3], const R tt[3][3], const R uu[3][3],
                                           const R n[3], const R x[3]) {
  R A[3][3], Rv[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    A[c][0] = v[c][0] - x[0];
    A[c][1] = v[c][1] - x[1];
    A[c][2] = v[c][2] - x[2];
    Rv[c] = sqrt(dot3(A[c], A[c]));
  }
  const R d = dot3(A[0], n);
  R sum_log = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int c1 = c == 2 ? 0 : c + 1;
    const R P = dot3(A[c], uu[c]);
    if (P == (R)0) continue;
    const R sm = dot3(A[c], tt[c]), sp = dot3(A[c1], tt[c]);
    // ln(R + s), for s < 0 as ln(R0^2) - ln(R - s) with R0^2 = P^2 + d^2 (R^2 = R0^2 + s^2),
    // which never subtracts nearly equal numbers
    const R r02 = P * P + d * d;
    const R lp = sp >= (R)0 ? log(Rv[c1] + sp) : log(r02) - log(Rv[c1] - sp);
    const R lm = sm >= (R)0 ? log(Rv[c] + sm) : log(r02) - log(Rv[c] - sm);
    sum_log += P * (lp - lm);
  }
  R bc[3];
  cross3(A[1], A[2], bc);
  const R num = dot3(A[0], bc);
  const R den = Rv[0] * Rv[1] * Rv[2] + dot3(A[0], A[1]) * Rv[2] + dot3(A[0], A[2]) * Rv[1] +
                dot3(A[1], A[2]) * Rv[0];
  const R omega = fabs((R)2 * atan2(num, den));
  return (sum_log - fabs(d) * omega) * (R)(0.25 / 3.14159265358979323846);
}

// --------------------------------------------------------------------------
// All-hits line traversal
// --------------------------------------------------------------------------
struct WorkCount {
  uint64_t lines, nodes, prims, hits;
};

template <typename R>
struct HitAcc {
  int32_t m;
  uint32_t key;
  int32_t id, idx;
  R t;        // line parameter of the selected hit (set when the step is taken):
              // y - x = t d, so rhat = sign(t) d and rho = |t|
  R src;      // direct BIE: sum over hits of G q / p_all
  R srcg[3];  // gradient walk, direct BIE, line 0: sum over hits of grad_x G q / p_all
};

// 1 / x for x != 0: in FP32 the hardware reciprocal (1 ulp) unless |x| is
// below 1e-30 (no denormal reaches it), in FP64 the division.
template <typename R> __device__ __forceinline__ R recip_(R x) {
  if constexpr (sizeof(R) == 4) return fabsf(x) >= 1e-30f ? __builtin_amdgcn_rcpf(x) : 1.0f / x;
  else return 1.0 / x;
}

// Test one primitive against the line x + t d (t real, inclusive edges).
// On a hit returns true and writes t and the barycentrics.
template <typename R, int D>
__device__ __forceinline__ bool hit_prim(const PrimGeo<R>& g, const R x[3], const R d[3], R& t, R& u, R& v) {
  if constexpr (D == 3) {
    // Moller-Trumbore with the barycentric tests on the numerators: with
    // U = (x - v0).(d x e2), V = d.((x - v0) x e1) and det = e1.(d x e2), the
    // hit condition u = U / det in [0, 1], v = V / det >= 0, u + v <= 1 is
    // U sd >= 0, V sd >= 0, (U + V) sd <= |det| for sd = sign(det); the
    // division is left for the accepted hits.
    R pv[3], qv[3];
    cross3(d, g.e2, pv);
    const R det = dot3(g.e1, pv);
    const R sv[3] = {x[0] - g.v0[0], x[1] - g.v0[1], x[2] - g.v0[2]};
    cross3(sv, g.e1, qv);
    const R sd = det < (R)0 ? (R)-1 : (R)1;
    const R us = dot3(sv, pv) * sd, vs = dot3(d, qv) * sd, ad = det * sd;
    if (det == (R)0 || us < (R)0 || vs < (R)0 || us + vs > ad) return false;
    const R inv = recip_(det);
    u = us * sd * inv;
    v = vs * sd * inv;
    t = dot3(g.e2, qv) * inv;
    return true;
  } else {
    const R det = d[0] * g.e1[1] - d[1] * g.e1[0];
    if (det == (R)0) return false;
    const R inv = (R)1 / det;
    const R sx = x[0] - g.v0[0], sy = x[1] - g.v0[1];
    // s = cross(x - v0, d) / cross(e, d) = -cross(x - v0, d) / det
    u = -(sx * d[1] - sy * d[0]) * inv;
    if (u < (R)0 || u > (R)1) return false;
    v = 0;
    // t = cross(v0 - x, e) / det
    t = (-sx * g.e1[1] + sy * g.e1[0]) * inv;
    return true;
  }
}

template <typename R>
__device__ __forceinline__ void hit_point(const PrimGeo<R>& g, R u, R v, R y[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) y[k] = g.v0[k] + u * g.e1[k] + v * g.e2[k];
}

// Line parameter and point where the line x + t d crosses the plane of a
// primitive it hits (unit normal n, 2D: n[2] = 0): t = (v0 - x) . n / (d . n),
// y = x + t d.  The barycentric solution of the hit test rounds with the
// primitive's shape (its error grows like |e1| |e2| / (2 A) on slivers); this
// form rounds by a few units of |x| + |t| over |d . n| whatever the shape.
// The test accepted the hit with d . n != 0; should the rounded normal still
// give 0, the barycentric solution is used.
template <typename R, int D>
__device__ __forceinline__ R plane_hit(const PrimGeo<R>& g, const R n[3], const R x[3], const R d[3], R y[3]) {
  const R w[3] = {g.v0[0] - x[0], g.v0[1] - x[1], D == 3 ? g.v0[2] - x[2] : (R)0};
  const R dn = dot3(d, n);
  R t;
  if (dn != (R)0) {
    t = dot3(w, n) / dn;
  } else {
    R u, v;
    hit_prim<R, D>(g, x, d, t, u, v);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) y[k] = x[k] + t * d[k];
  return t;
}

// Slab test of a line against a box in the scene's box frame; inv = 1 / d
// (finite), ox = -x' inv with x' the line's point in that frame.  The near side
// of each slab is lo where inv >= 0 and hi otherwise, so an empty box (lo above
// hi, an unused record slot) is never crossed.
template <typename R, int D>
__device__ __forceinline__ bool line_box(const R lo[3], const R hi[3], const R inv[3], const R ox[3]) {
  R tmin = (R)-INFINITY, tmax = (R)INFINITY;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const bool pos = inv[k] >= (R)0;
    const R tn = fma(pos ? lo[k] : hi[k], inv[k], ox[k]), tf = fma(pos ? hi[k] : lo[k], inv[k], ox[k]);
    tmin = fmax(tmin, tn);
    tmax = fmin(tmax, tf);
  }
  return tmin <= tmax;
}

// 1 / d for the slab tests, a large finite value for d = 0.  In FP32 the
// hardware reciprocal (1 ulp) serves: the boxes are padded by far more than
// the resulting error in the slab parameters; components below 1e-30 count as
// zero (no denormal reaches the reciprocal).
template <typename R> __device__ __forceinline__ R safe_inv(R d) {
  if constexpr (sizeof(R) == 4) return fabsf(d) < 1e-30f ? 1e30f : __builtin_amdgcn_rcpf(d);
  else return d == 0.0 ? 1e300 : 1.0 / d;
}

// Slab-test constants of the line x + t d: inv = 1 / d, ox = -x' inv, and
// the rotation that puts a packed box word's near side in its low half.
template <typename R, int D>
__device__ __forceinline__ void line_slabs(const SceneView<R, D>& s, const R x[3], const R d[3], R inv[3],
                                           R ox[3], uint32_t rot[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    inv[k] = safe_inv(d[k]);
    ox[k] = -((x[k] - s.fc[k]) * s.fk) * inv[k];
    rot[k] = inv[k] < (R)0 ? 16u : 0u;
  }
}

typedef _Float16 half2_t __attribute__((ext_vector_type(2)));

// Slab test against a packed binary16 box (FP32 scenes).
template <int D>
__device__ __forceinline__ bool packed_box(const uint32_t b[3], const float inv[3], const float ox[3],
                                           const uint32_t rot[3]) {
  float tn[3], tf[3];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const half2_t v = __builtin_bit_cast(half2_t, __builtin_amdgcn_alignbit(b[k], b[k], rot[k]));
    tn[k] = fmaf((float)v.x, inv[k], ox[k]);
    tf[k] = fmaf((float)v.y, inv[k], ox[k]);
  }
  const float tmin = D == 3 ? fmaxf(fmaxf(tn[0], tn[1]), tn[2]) : fmaxf(tn[0], tn[1]);
  const float tmax = D == 3 ? fminf(fminf(tf[0], tf[1]), tf[2]) : fminf(tf[0], tf[1]);
  return tmin <= tmax;
}

// Which of an interior record's child boxes the line crosses: bit k for slot k.
template <typename R, int D>
__device__ __forceinline__ uint32_t child_mask(const typename Rec<R, D>::Node& n, const R inv[3], const R ox[3],
                                               const uint32_t rot[3]) {
  uint32_t m = 0;
#pragma unroll
  for (int k = 0; k < kArity; ++k) {
    bool h;
    if constexpr (sizeof(R) == 4) h = packed_box<D>(n.box[k], inv, ox, rot);
    else h = line_box<R, D>(n.lo[k], n.hi[k], inv, ox);
    m |= h ? (1u << k) : 0u;
  }
  return m;
}

// Calls leaf(first, count) for every leaf whose box the line crosses, depth
// first with a private stack (one line per thread: the hit-list query).  The
// path kernel runs the same traversal in its own loop, with the stack in LDS,
// where lanes park at crossed leaves and test them together.
template <typename R, int D, bool COUNT, typename Leaf>
__device__ __forceinline__ void for_each_leaf(const SceneView<R, D>& s, const R inv[3], const R ox[3],
                                              const uint32_t rot[3], WorkCount& wc, Leaf&& leaf) {
  int32_t stk[kMaxDepth];
  int sp = 0;
  int32_t e = s.root;
  for (;;) {
    if (e >= 0) {
      const typename Rec<R, D>::Node n = s.nodes[e];
      if (COUNT) wc.nodes += 1;
      uint32_t m = child_mask<R, D>(n, inv, ox, rot);
      // continue with the first crossed entry, push the others
      e = kPop;
#pragma unroll
      for (int k = 0; k < kArity; ++k) {
        if (m & (1u << k)) {
          if (e == kPop) e = n.child[k];
          else if (sp < kMaxDepth) stk[sp++] = n.child[k];
        }
      }
    } else if (e != kPop) {
      const int32_t code = -1 - e;
      leaf(code >> 3, (code & 7) + 1);
      e = kPop;
    }
    if (e == kPop) {
      if (sp == 0) break;
      e = stk[--sp];
    }
  }
}

}  // namespace wob
