/*
 * oracle.h - FP64 brute-force walk-on-boundary (WoB) reference estimator.
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the independent checker for the HIP
 * library: it shares no source with it and is never called by the product
 * path.  Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.
 *
 * What it computes (Sugimoto et al., "A Practical Walk-on-Boundary Method for
 * Boundary Value Problems"):
 *   - Dirichlet problems, double-layer indirect BIE (Sec. 4.1, Table 1 rows
 *     "Dirichlet"), recursive estimator of eq. indirect_double_boundary_reordered2
 *     and eq. mc_dirichlet_interior_sol, truncated with the halved last term
 *     (Sec. 4.1.2 "Path truncation").
 *   - Neumann problems, direct BIE (Sec. 4.2, eq. cbie_neumann, eq.
 *     mc_cbie_neumann, eq. mc_cbie_neumann2, Table 1 rows "Neumann").
 *   - Neumann / Robin problems, single-layer indirect BIE (Sec. 4.3, Table 1
 *     rows "Mixed or degenerate problem", Neumann and Robin boundary rows).
 *   - Interior (phi = +1) and exterior (phi = -1) domains (Sec. 4.5.1).
 *   - Line sampling with all hits, one hit picked uniformly, pdf times 1/m
 *     (Sec. 4.4.1 "Ray sampling").
 *   Kernels G, dG/dn_y, dG/dn_x are taken verbatim from Appendix A.
 *
 * Every intersection query loops over EVERY primitive (no acceleration
 * structure).  All arithmetic is double precision.  Random numbers come from
 * Philox4x32-10 (Salmon et al., SC'11), implemented here from its published
 * definition; the stream layout is documented in oracle.c.
 */
#ifndef WOB_ORACLE_H
#define WOB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* primitive boundary-condition kinds (eq. PoissonBC) */
enum { ORC_DIRICHLET = 0, ORC_NEUMANN = 1, ORC_ROBIN = 2 };
/* formulations (Table 1) */
enum { ORC_AUTO = 0, ORC_DOUBLE_LAYER = 1, ORC_DIRECT = 2, ORC_SINGLE_LAYER = 3 };
/* analytic harmonic functions u from which boundary data are derived */
enum { ORC_PROG_CONST = 0, ORC_PROG_LINEAR = 1, ORC_PROG_QUAD = 2, ORC_PROG_INVDIST = 3 };

typedef struct {
  int dim;                 /* 2 (segments) or 3 (triangles) */
  int64_t n_verts;
  int64_t n_prims;
  const double* verts;     /* n_verts * dim */
  const int32_t* prims;    /* n_prims * dim, oriented so the normal points out of Omega */
  const uint8_t* kind;     /* n_prims, or NULL = all Dirichlet */
  const double* alpha;     /* n_prims Robin coefficients, or NULL = 0 */
} orc_mesh;

typedef struct {
  int domain;              /* +1 interior (phi = +1), -1 exterior (phi = -1) */
  int formulation;         /* ORC_* formulation, ORC_AUTO = Table 1 mapping */
  int program;             /* ORC_PROG_* */
  double params[8];        /* program parameters */
  uint32_t self_threshold; /* self-panel mixture probability as floor(p_s * 2^24) */
  double self_p;           /* the same probability as a real number, floor(p_s*2^24)/2^24 */
  int density;             /* 1: estimate the boundary unknown (nu or mu) without its own
                              emission, at points on the boundary (double / single layer) */
  int sampling;            /* single layer: ORC_SAMPLE_LINE (line sampling of Sec. 4.4.1 with
                              the self-panel mixture) or ORC_SAMPLE_RIS (resampled importance
                              sampling over area-uniform candidates, Results) */
  int candidates;          /* RIS candidates per vertex, 1..64 */
  /* single layer with Dirichlet parts (mixed problems, eq. mixed_second_kind_ish):
     at a Dirichlet vertex the next point is sampled from k G with probability
     p_k (weight -k G / (p p_k)) and otherwise the walk stays (weight 1/(1-p_k));
     the emission there is k u_D */
  double mixed_k;
  uint32_t mixed_threshold; /* p_k as floor(p_k * 2^24) */
  double mixed_p;           /* floor(p_k * 2^24) / 2^24 */
  /* boundary data: 0 = derived from the harmonic program (u, n . grad u,
     n . grad u + alpha u by kind), 1 = given per mesh vertex and interpolated
     linearly on each primitive (the datum of the primitive's own kind: g, q
     or g_R; eq. PoissonBC) */
  int data_mode;
  const double* vertex_data; /* [n_verts] when data_mode == 1 */
} orc_bc;

enum { ORC_SAMPLE_LINE = 0, ORC_SAMPLE_RIS = 1 };

/* Per (point, path) record produced by orc_trace. Arrays may be NULL. */
typedef struct {
  double* value;           /* [n_items] per-path estimate u_hat */
  double* abs_sum;         /* [n_items] the path sum with every factor and summand replaced
                              by its magnitude (scale for relative tolerances) */
  double* graze;           /* [n_items] min over the lines' primitives of the decision margin in
                              units of its rounding scale (decision_margin, oracle.c) */
  double* err;             /* [n_items] first-order rounding-error bound of the value in units
                              of the unit roundoff u (see oracle.c): an evaluation of the same
                              path with unit roundoff u differs by about u * err at most */
  int32_t* vtx_prim;       /* [n_items * L] selected primitive per line, -1 none, -2-p self-panel */
  int32_t* vtx_m;          /* [n_items * L] number of hits per line */
  double* vtx_pos;         /* [n_items * L * dim] vertex reached by each line */
} orc_trace_out;

/* Philox4x32-10 block: out = Philox(ctr, key). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Lines per path for a formulation: M (double / single layer) or M + 1 (direct). */
int orc_lines_per_path(const orc_mesh* mesh, const orc_bc* bc, int walk_len);

/* Resolve ORC_AUTO with Table 1's mapping; returns the formulation or -1. */
int orc_resolve_formulation(const orc_mesh* mesh, int formulation);

/* Per-path estimates for an explicit list of (point index, path index) items.
 * points: [n_points * dim]; point_prim: [n_points] or NULL (-1 = off boundary).
 * Returns 0 on success, nonzero on bad arguments. */
int orc_trace(const orc_mesh* mesh, const double* points, const int32_t* point_prim,
              int64_t n_points, const orc_bc* bc, int walk_len, uint64_t seed,
              uint32_t problem, int64_t n_items, const int64_t* item_point,
              const int64_t* item_path, orc_trace_out* out, int n_threads);

/* Mean and unbiased variance over paths 0..N-1 for every point (two-pass),
 * over the finite path values (a non-finite one is left out; NaN mean when
 * none is finite). */
int orc_solve(const orc_mesh* mesh, const double* points, const int32_t* point_prim,
              int64_t n_points, const orc_bc* bc, int samples, int walk_len,
              uint64_t seed, uint32_t problem, double* mean_out, double* var_out,
              int n_threads);

/* All hits of the lines orig + t*dir (t real), excluding primitive exclude[i].
 * n_hits[i] is the full count; at most max_hits (prim, t, margin) are stored,
 * in increasing (t, prim) order. margin: the decision margin in units of its rounding
 * scale (decision_margin in oracle.c). */
int orc_intersect_all(const orc_mesh* mesh, const double* orig, const double* dir,
                      const int32_t* exclude, int64_t n_lines, int max_hits,
                      int32_t* n_hits, int32_t* hit_prim, double* hit_t,
                      double* hit_margin, double* line_graze, int n_threads);

/* Harmonic program value and boundary datum s(y) on primitive `prim`. */
double orc_program_value(const orc_mesh* mesh, const orc_bc* bc, const double* y);
double orc_boundary_datum(const orc_mesh* mesh, const orc_bc* bc, int64_t prim, const double* y);

/* Self-panel estimate of the single-layer integral over the own primitive:
 * returns G(x, y)/p(y) for the sample drawn from uniforms (u0, u1) and writes y. */
double orc_self_panel(const orc_mesh* mesh, int64_t prim, const double* x, double u0,
                      double u1, double* y_out);

/* int_T G(x, y) dA over primitive `prim` in closed form (3D: potential of a
 * uniform triangle; 2D: of a uniform segment). */
double orc_prim_potential(const orc_mesh* mesh, int64_t prim, const double* x);

/* Learned control variate, single layer (see oracle.c): per-path values of the
 * corrected estimator for per-primitive tables g (lines 1.., the network's
 * prediction of the boundary unknown minus its emission) and g0 (line 0; NULL
 * means g0 = g).  The per-point add-back sum_T g0_T int_T G(x0, y) dA comes
 * from orc_cv_addback (zero when M = 1).  abs_sum and err (may be NULL): the
 * path's magnitude sum and rounding-error bound in units of u, as in orc_trace. */
int orc_trace_cv(const orc_mesh* mesh, const double* points, const int32_t* point_prim,
                 int64_t n_points, const orc_bc* bc, int walk_len, uint64_t seed,
                 uint32_t problem, const double* g, const double* g0, int64_t n_items,
                 const int64_t* item_point, const int64_t* item_path, double* value,
                 double* abs_sum, double* err, int n_threads);
/* randomized = 0: sum_T g_T int_T G(x0, y) dA in closed form.  randomized = 1:
 * closed form only for triangles whose centroid lies within four bounding radii of
 * x0; every other triangle contributes g_T A_T G(x0, y_T) at one uniform point
 * y_T of the triangle drawn from a 32-bit integer hash of (seed, triangle) and
 * shared by all evaluation points (an unbiased value of the same sum at each
 * point). */
int orc_cv_addback(const orc_mesh* mesh, const double* g, const double* points, int64_t n_points,
                   uint32_t seed, int randomized, double* out, int n_threads);

/* Gradient estimators (Sec. 4.1.3, derivative estimators along the same paths):
 * the path of orc_trace with the kernel of its first step replaced by its
 * gradient in x0 (double layer: -grad dG/dn_y; direct BIE: -phi grad dG/dn_y
 * and phi grad G in the step-0 source; single layer: grad G), the rest of the
 * path unchanged.  Points must lie off the boundary (the gradient equations
 * hold inside the domain); no density mode.  grad: [n_items * dim];
 * grad_abs: the magnitude sum of the gradient terms (rounding scale); err,
 * grad_err: rounding-error bounds of the value and of each gradient component
 * in units of u (as orc_trace_out.err).
 * anchors, anchor_prim (double layer only; both NULL or both given): per point
 * a boundary point x* and its primitive (-1: no split at that point).  Each path's gradient w' nu^(y_1)
 * (w' the step-0 derivative weight, nu^ the rest of the path) becomes
 * w' (nu^(y_1) - nu^(x*)), nu^(x*) the coupled walk from x* with the path's
 * own random numbers of lines 1, 2, ... (the boundary split of Sec. 4.1.3;
 * unbiased because w' has mean zero for x0 off the closed boundary). */
int orc_trace_grad(const orc_mesh* mesh, const double* points, int64_t n_points, const orc_bc* bc,
                   int walk_len, uint64_t seed, uint32_t problem, int64_t n_items,
                   const int64_t* item_point, const int64_t* item_path, const double* anchors,
                   const int32_t* anchor_prim, double* value, double* grad, double* abs_sum, double* grad_abs,
                   double* graze, double* err, double* grad_err, int n_threads);
int orc_solve_grad(const orc_mesh* mesh, const double* points, int64_t n_points, const orc_bc* bc,
                   int samples, int walk_len, uint64_t seed, uint32_t problem, const double* anchors,
                   const int32_t* anchor_prim, double* mean_out, double* var_out, double* grad_out,
                   double* grad_var_out, int n_threads);

/* Forward (adjoint) estimator of the single layer, all-Neumann boundary
 * (Sec. 4.4.3 "Forward estimator"; see oracle.c for the derivation and the
 * random-number layout).  orc_forward_paths writes, per path and vertex
 * k = 1..M, the vertex y_k, its primitive, the hits of the line that reached
 * it (0 for k = 1) and its source strength c_{k-1} W_k (0 and prim -1 once the
 * path has ended).  start_weight: per-primitive start weights w_T >= 0 in id
 * order (sum > 0), or NULL for area-uniform starts. */
typedef struct {
  double* vtx_pos;         /* [n_paths * M * dim] */
  double* vtx_w;           /* [n_paths * M] */
  int32_t* vtx_prim;       /* [n_paths * M] */
  int32_t* vtx_m;          /* [n_paths * M] */
  double* graze;           /* [n_paths] min over the lines' primitives of the decision margin in
                              units of its rounding scale (decision_margin, oracle.c) */
  double* vtx_perr;        /* [n_paths * M] rounding-error bounds (units of u) of each vertex's */
  double* vtx_werr;        /* position and strength (see oracle.c) */
} orc_forward_out;
int orc_forward_paths(const orc_mesh* mesh, const orc_bc* bc, const double* start_weight,
                      int64_t n_paths, int walk_len, uint64_t seed, uint32_t problem,
                      orc_forward_out* out, int n_threads);
/* u(x_p) ~ (1 / n_paths) sum_paths sum_k w_k G(x_p, y_k): mean, unbiased variance
 * over paths, and the magnitude sum (1 / n_paths) sum |w_k| |G| (rounding scale). */
int orc_forward_gather(int dim, int64_t n_paths, int walk_len, const double* vtx_pos,
                       const double* vtx_w, const double* points, int64_t n_points,
                       double* mean_out, double* var_out, double* abs_out, int n_threads);

/* Unit outward normal of a primitive. */
void orc_prim_normal(const orc_mesh* mesh, int64_t prim, double* n_out);

#ifdef __cplusplus
}
#endif
#endif
