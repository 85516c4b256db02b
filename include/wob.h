/*
 * wob.h - C ABI of the MI355X (gfx950) walk-on-boundary library.
 *
 * Walk-on-boundary (WoB) Monte Carlo estimation of harmonic functions from
 * boundary integral equations (Sugimoto, Chen, Jiang, Batty, Hachisuka, "A
 * Practical Walk-on-Boundary Method for Boundary Value Problems"):
 *   - Dirichlet problems: indirect double-layer BIE (Sec. 4.1; Table 1,
 *     "Dirichlet" rows; estimator eq. indirect_double_boundary_reordered2 and
 *     eq. mc_dirichlet_interior_sol).
 *   - Neumann problems: direct BIE (Sec. 4.2; eq. cbie_neumann,
 *     eq. mc_cbie_neumann, eq. mc_cbie_neumann2; Table 1, "Neumann" rows).
 *   - Robin and Neumann/Robin mixtures: indirect single-layer BIE (Sec. 4.3;
 *     Table 1, "Mixed or degenerate problem" rows for Neumann and Robin parts).
 *   - Interior and exterior domains (Sec. 4.5.1; sign phi of Table 1).
 *   - Line sampling with all hits and a uniform pick among them (Sec. 4.4.1),
 *     truncated after M boundary vertices with the last emission halved
 *     (Sec. 4.1.2).
 *
 * Conventions
 *   - Every call returns a wob_status; no exception crosses the ABI.
 *   - Arrays passed to wob_solve / wob_trace / wob_intersect_all / wob_count_work
 *     are DEVICE pointers owned by the caller.  Their element type follows the
 *     scene's precision: float for WOB_F32 scenes, double for WOB_F64 scenes.
 *     The library never allocates or frees caller outputs.
 *   - Work is enqueued asynchronously on `stream` (a hipStream_t passed as
 *     void*, NULL = default stream).  Argument errors are detected on the host
 *     before anything is enqueued; a WOB_E_DEVICE return means the HIP runtime
 *     reported an error for the launch.
 *   - A scene is immutable after wob_build_bvh and may be used by any number
 *     of concurrent calls on any streams of the device it was built on.
 *   - Random numbers: Philox4x32-10 with key (seed & 0xffffffff, seed >> 32)
 *     and counter (path k, point p, (problem << 24) | (line << 8) | block, w);
 *     block 0 draws the line direction and the mixture branch, block 1 the
 *     in-plane self-panel sample, block 2 with w = primitive id the key that
 *     selects a hit (the hit with the smallest (key, id) is taken, a uniform
 *     choice among the hits).  Results are bit-reproducible for a given seed.
 */
#ifndef WOB_H
#define WOB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wob_scene_s* wob_scene;

typedef enum {
  WOB_OK = 0,
  WOB_E_ARG = 1,         /* invalid argument: NULL where required, bad size, bad enum */
  WOB_E_ALLOC = 2,       /* device or host allocation failed */
  WOB_E_DEVICE = 3,      /* HIP runtime error (no device, launch failure, copy failure) */
  WOB_E_MESH = 4,        /* index out of range, zero-length / zero-area primitive, non-finite vertex */
  WOB_E_UNSUPPORTED = 5, /* a combination this library does not implement */
  WOB_E_TOO_LARGE = 6    /* beyond the fixed capacity of an allocation-free entry point */
} wob_status;

/* Boundary-condition kind per primitive (eq. PoissonBC). */
enum { WOB_BC_DIRICHLET = 0, WOB_BC_NEUMANN = 1, WOB_BC_ROBIN = 2 };

/* BIE formulation (Table 1).  AUTO: all Dirichlet -> double layer, all Neumann
 * -> direct, anything with Robin parts or mixing kinds -> single layer (on
 * Dirichlet parts the transformed first-kind row of eq. mixed_second_kind_ish,
 * see wob_bc.mixed_k).  The double layer takes Dirichlet meshes only, the
 * direct BIE Neumann meshes only; the single layer takes any mesh. */
enum { WOB_F_AUTO = 0, WOB_F_DOUBLE_LAYER = 1, WOB_F_DIRECT = 2, WOB_F_SINGLE_LAYER = 3 };

/* Harmonic function u whose boundary traces give the data: Dirichlet u,
 * Neumann du/dn, Robin du/dn + alpha u (n = the primitive's unit normal).
 *   CONST    u = params[0]
 *   LINEAR   u = params[0] x + params[1] y + params[2] z + params[3]   (2D: no z term)
 *   QUAD     u = x^2 - y^2
 *   INVDIST  3D: u = 1 / |x - c|;  2D: u = ln |x - c|;  c = params[0..2] */
enum { WOB_PROG_CONST = 0, WOB_PROG_LINEAR = 1, WOB_PROG_QUAD = 2, WOB_PROG_INVDIST = 3 };

/* Scene precision: geometry, arithmetic of the walk and element type of arrays. */
enum { WOB_F32 = 0, WOB_F64 = 1 };

/* How the single layer samples its integrals (see wob_bc.sampling).  RIS, per
 * vertex x: C candidates y_j area-uniform on the boundary (Philox block 3,
 * w = j: word 0 picks the primitive by the binary32 cumulative area fraction in
 * id order, words 1, 2 the point, reflected into the triangle); kernel k = G on
 * the first step, -2 phi (dG/dn_x + alpha G) on the recursion; a weighted
 * reservoir keeps candidate j when u_j S_j < |k_j| (u_j from word 3, S_j the
 * running sum of |k|); weight sign(k) S |Gamma| / C.  No lines are traced. */
enum { WOB_SAMPLE_LINE = 0, WOB_SAMPLE_RIS = 1 };

typedef struct {
  int32_t domain;       /* +1 interior (phi = +1), -1 exterior (phi = -1) */
  int32_t formulation;  /* WOB_F_* */
  int32_t program;      /* WOB_PROG_* */
  int32_t density;      /* 0: the solution u at the points.  1: the boundary unknown (double
                           layer nu, single layer mu) at points ON the boundary, without its
                           own emission 2 phi s (the targets of the learned control variate);
                           not with the direct BIE; a point with point_prim -1 (or no
                           point_prim) has no boundary unknown and gets NaN paths */
  int32_t sampling;     /* single layer only: WOB_SAMPLE_LINE (line sampling of Sec. 4.4.1,
                           all hits, uniform pick, self-panel mixture) or WOB_SAMPLE_RIS
                           (resampled importance sampling over area-uniform boundary
                           candidates, as the paper does for Robin and mixed problems,
                           Results).  Other formulations: WOB_SAMPLE_LINE only */
  int32_t candidates;   /* RIS candidates per vertex, 1..64 (0 selects 16) */
  double params[8];     /* program parameters */
  double self_panel_p;  /* single layer: probability of the in-plane sample on the own
                           primitive where G acts on it (0 selects 1/16); in (0, 1) */
  double mixed_k;       /* single layer with Dirichlet parts (mixed problems): the constant k
                           of the transformed first-kind row mu = mu - k int G mu + k u_D
                           (eq. mixed_second_kind_ish); 0 selects 4 (the paper's Results) */
  double mixed_p;       /* its probability p_k of sampling the k G term (else the walk stays
                           at x), in (0, 1); 0 selects 2/3 */
  int32_t data_mode;    /* WOB_DATA_PROGRAM: the data g, q, g_R derive from `program` (the
                           traces of a harmonic u).  WOB_DATA_VERTEX: they are given, one
                           value per mesh vertex in `vertex_data`, and interpolated linearly
                           on each primitive; the value is the datum of the primitive's own
                           kind (eq. PoissonBC: g on Dirichlet, q on Neumann, g_R on Robin
                           parts) and `program` / `params` are ignored */
  int32_t path_offset;  /* >= 0: path k of every point draws the random numbers of path
                           path_offset + k (0 for a plain solve; path_offset + samples <=
                           2^31 - 1).  Solves of disjoint path ranges of the same points
                           and seed hold disjoint paths of one estimator: their per-point
                           (n, mean, M2 = (n - 1) var) merge into the solve of the union by
                           Chan's formula, n = n1 + n2, d = mean2 - mean1, mean = mean1 +
                           d n2 / n, M2 = M2_1 + M2_2 + d^2 n1 n2 / n (resume a solve, or
                           share its paths among devices).  Not with wob_forward_paths */
  const void* vertex_data; /* WOB_DATA_VERTEX: DEVICE array of the scene's n_verts values, of
                           the scene's element type, indexed like the vertices passed to
                           wob_build_bvh; caller-owned, read by enqueued work */
} wob_bc;

/* Where the boundary data come from (wob_bc.data_mode). */
enum { WOB_DATA_PROGRAM = 0, WOB_DATA_VERTEX = 1 };

typedef struct {
  int32_t dim;          /* 2 or 3 */
  int32_t precision;    /* WOB_F32 / WOB_F64 */
  int64_t n_prims;
  int64_t n_nodes;      /* tree nodes (interior + leaves); the device holds the
                           n_nodes - n_leaves interior ones, each with both
                           children's boxes */
  int64_t n_leaves;
  int32_t depth;        /* nodes on the longest root-to-leaf path (root = 1) */
  int32_t max_leaf;     /* most primitives in one leaf */
  int64_t device_bytes; /* bytes of device memory the scene holds */
  int64_t node_bytes;   /* size of one interior-node record */
  int64_t prim_bytes;   /* size of one primitive record */
  int32_t n_dirichlet, n_neumann, n_robin, reserved;
  int64_t n_verts;      /* vertices of the mesh (the length of per-vertex data) */
} wob_scene_info;

/* Build the line-query acceleration structure for a boundary mesh and upload it
 * to the current HIP device (the geometry query that Sec. 4.4.1's all-hits
 * sampling needs; the structure itself is this library's design).
 *   dim        2 (line segments) or 3 (triangles)
 *   precision  WOB_F32 or WOB_F64; vertices are rounded to that precision
 *   verts      HOST array, n_verts * dim doubles
 *   prims      HOST array, n_prims * dim vertex indices (n_prims < 2^27);
 *              orientation such that
 *              (v1 - v0) x (v2 - v0) (3D) or the tangent turned by -90 degrees
 *              (2D, counter-clockwise boundary) points OUT of the interior Omega
 *              (Sec. 4.5.1: normals stay outward from Omega for exterior problems)
 *   kind       HOST array, n_prims WOB_BC_* codes, or NULL (all Dirichlet)
 *   alpha      HOST array, n_prims Robin coefficients, or NULL (all 0)
 *   out        receives the scene handle; released with wob_free
 * Synchronous.  Errors: WOB_E_ARG, WOB_E_MESH, WOB_E_ALLOC, WOB_E_DEVICE. */
wob_status wob_build_bvh(int32_t dim, int32_t precision, const double* verts, int64_t n_verts,
                         const int32_t* prims, int64_t n_prims, const uint8_t* kind,
                         const double* alpha, wob_scene* out);

/* wob_build_bvh with the mesh arrays in host or device memory and its copies
 * on `stream`.  inputs_on_device = 1: verts, prims, kind and alpha are DEVICE
 * pointers (same layouts; kind and alpha may be NULL); they are copied to the
 * host on `stream`, which the call waits for (the tree is built on the host),
 * and the scene is uploaded on `stream`.  inputs_on_device = 0: as
 * wob_build_bvh, with the upload on `stream`.  Synchronous.  Errors: as
 * wob_build_bvh. */
wob_status wob_build_bvh_ex(int32_t dim, int32_t precision, const double* verts, int64_t n_verts,
                            const int32_t* prims, int64_t n_prims, const uint8_t* kind,
                            const double* alpha, int32_t inputs_on_device, void* stream,
                            wob_scene* out);

/* Release a scene (waits for nothing: the caller must not free a scene that
 * enqueued work still uses).  NULL is ignored. */
void wob_free(wob_scene scene);

wob_status wob_get_scene_info(wob_scene scene, wob_scene_info* info);

/* Device-side status of the solves on a scene, sticky until read: the number
 * of path values that were not finite (a degenerate primitive, an invalid
 * point_prim id, data singular at a boundary point) since the last call.  Such
 * paths are left out of the per-point statistics of wob_solve, wob_solve_cv,
 * wob_solve_grad and the batched solves (a point with no finite path gets a
 * NaN mean); wob_trace returns them as they are.  Reads the counter with an
 * asynchronous copy on `stream`, resets it, and waits for the stream: call it
 * after the solves it should cover have been enqueued on that stream, and
 * never inside a captured graph.  Errors: WOB_E_ARG, WOB_E_DEVICE. */
wob_status wob_last_device_status(wob_scene scene, uint64_t* nonfinite_paths, void* stream);

/* Number of lines traced per path: walk_len for the double and single layer,
 * walk_len + 1 for the direct BIE (the last vertex traces one more line for its
 * source integral).  Returns -1 on bad arguments. */
int32_t wob_lines_per_path(wob_scene scene, const wob_bc* bc, int32_t walk_len);

/* Solve: for every evaluation point p, average N independent WoB paths of
 * walk_len boundary vertices (Algorithm 1's EstimateSolution generalised to
 * Table 1's estimators).
 *   points      DEVICE, n_points * dim (float / double by scene precision)
 *   point_prim  DEVICE, n_points primitive ids, -1 for points off the boundary;
 *               NULL = all off the boundary.  A point with an id must lie on
 *               that primitive: it is then estimated with the boundary rows of
 *               Table 1 (Dirichlet: the given value; direct and single layer:
 *               the boundary equations).
 *   samples     N >= 1 (N >= 2 when var_out is not NULL)
 *   walk_len    M >= 1, M < 65536
 *   seed        Philox key
 *   mean_out    DEVICE, n_points: (1/N) sum of path values
 *   var_out     DEVICE, n_points: unbiased sample variance of the path values, or NULL
 * Errors: WOB_E_ARG, WOB_E_UNSUPPORTED, WOB_E_DEVICE. */
wob_status wob_solve(wob_scene scene, const void* points, const int32_t* point_prim,
                     int64_t n_points, const wob_bc* bc, int32_t samples, int32_t walk_len,
                     uint64_t seed, void* mean_out, void* var_out, void* stream);

/* wob_solve with the evaluation points walked in a locality order: the same
 * estimate (Algorithm 1's EstimateSolution under Table 1's estimators) and the
 * same paths, scheduled so that points lying close together run side by side
 * and share cached BVH nodes and triangles.  On the device, on `stream`: Morton
 * keys of the points (2^10 cells per axis in 3D, 2^15 in 2D, over the points'
 * bounding box), a stable radix sort of (key, index), the points and their
 * primitive ids gathered into that order, the walk (point i of the sorted order
 * keeps the random-number point index of its caller position), and the results
 * written back to the caller's order.  Every point's path values equal
 * wob_solve's; mean_out and var_out equal wob_solve's up to the order in which
 * a point's path values are summed (binary32 / binary64 rounding).  The result
 * does not depend on anything but the inputs: equal calls give equal bits.
 *   points ... var_out   as for wob_solve; n_points <= INT32_MAX
 *   workspace        DEVICE, 256-byte aligned, at least the size that
 *                    wob_solve_ordered_workspace gives for n_points; owned by
 *                    the caller, contents undefined after the call.  Calls that
 *                    share a workspace must be ordered on one stream.
 * Errors: WOB_E_ARG (also: workspace NULL, misaligned or too small),
 * WOB_E_UNSUPPORTED, WOB_E_DEVICE. */
wob_status wob_solve_ordered(wob_scene scene, const void* points, const int32_t* point_prim,
                             int64_t n_points, const wob_bc* bc, int32_t samples, int32_t walk_len,
                             uint64_t seed, void* mean_out, void* var_out, void* workspace,
                             size_t workspace_bytes, void* stream);

/* Device workspace bytes of wob_solve_ordered for n_points points of this
 * scene (its dimension and precision).  Errors: WOB_E_ARG (n_points < 0 or
 * above INT32_MAX, NULL scene or bytes). */
wob_status wob_solve_ordered_workspace(wob_scene scene, int64_t n_points, size_t* bytes);

/* Per-path values (parity and debugging); the same paths as wob_solve.
 *   point_ids  DEVICE, n_points uint32 point indices used in the random-number
 *              counter, or NULL (point i uses index i).  With ids, a subset of a
 *              larger solve's points reproduces that solve's paths exactly.
 *   path_out   DEVICE, n_points * samples, path k of point p at p * samples + k
 *   vtx_prim   DEVICE, n_points * samples * L int32 (L = wob_lines_per_path) or NULL:
 *              primitive id picked by each line, -1 if the line met nothing (or was
 *              the source-only last line of the direct BIE), -2 - id for an in-plane
 *              self-panel sample on primitive id; entries after a path ended are -1
 *   vtx_m      DEVICE, same shape, number of hits of each line, or NULL */
wob_status wob_trace(wob_scene scene, const void* points, const int32_t* point_prim,
                     int64_t n_points, const wob_bc* bc, int32_t samples, int32_t walk_len,
                     uint64_t seed, const uint32_t* point_ids, void* path_out, int32_t* vtx_prim,
                     int32_t* vtx_m, void* stream);

/* Every intersection of the lines orig + t dir, t real (Sec. 4.4.1 "all-hits").
 *   orig, dir    DEVICE, n_lines * dim
 *   exclude      DEVICE, n_lines primitive ids to skip (-1 none), or NULL
 *   n_hits       DEVICE, n_lines: total number of hits of each line
 *   hit_prim     DEVICE, n_lines * max_hits primitive ids, in traversal order;
 *                only the first max_hits hits of a line are stored
 *   hit_t        DEVICE, n_lines * max_hits line parameters (float / double), or NULL */
wob_status wob_intersect_all(wob_scene scene, const void* orig, const void* dir,
                             const int32_t* exclude, int64_t n_lines, int32_t max_hits,
                             int32_t* n_hits, int32_t* hit_prim, void* hit_t, void* stream);

/* Work counters for the same walk as wob_solve (measurement only).
 *   counters  DEVICE, 4 uint64: lines traced, interior nodes visited (each
 *             visit tests the boxes of both children), primitives tested,
 *             hits found; accumulated (the caller zeroes them). */
wob_status wob_count_work(wob_scene scene, const void* points, const int32_t* point_prim,
                          int64_t n_points, const wob_bc* bc, int32_t samples, int32_t walk_len,
                          uint64_t seed, uint64_t* counters, void* stream);

/* Gradient of the solution at points inside the domain, estimated along the
 * same paths as the value (Sec. 4.1.3, derivative estimators: the first step's
 * kernel replaced by its gradient in x0, the rest of each path unchanged;
 * the gradient equations of the three formulations).  Per path the gradient
 * is W' times the path's remaining sum, with, for the step from x0 to the
 * picked hit y (rhat = (y - x0) / rho, c = rhat . n_y, m hits):
 *   double layer  -grad_x dG/dn_y / p = -m (n_y - D c rhat) / (2 rho |c|)
 *   direct BIE    phi times the same, plus phi grad_x G q / p_all summed
 *                 over the hits of line 0 for the source (q sgn(t) d / (2|c|))
 *   single layer  grad_x G / p = m rhat / (2 |c|)  (RIS: grad_x G / |G| S |Gamma| / C)
 * The double-layer and direct kernels are hypersingular (1 / |c|): noisier
 * near the boundary, as the paper observes.  Every point must lie off the
 * boundary (no point_prim argument); no density mode.
 * Boundary split (double layer; Sec. 4.1.3 splits the gradient at the
 * boundary point nearest to x0): with an anchor x* on the boundary, each
 * path's gradient W' nu becomes W' (nu - nu*), nu the path's sum after its
 * step 0 and nu* that of a coupled walk which takes x* as its vertex 1 and
 * then the path's own random numbers of lines 1, 2, ...  Unbiased for any
 * anchor (W' has mean zero for x0 off the closed boundary); near the boundary
 * the two walks start close together and take the same directions, which
 * removes the hypersingular growth of the variance.  A path costs up to two
 * walks where the split is on.
 *   points        DEVICE, n_points * dim
 *   anchor_points DEVICE, n_points * dim (scene element type): x* per point, or NULL
 *   anchor_prim   DEVICE, n_points int32: the primitive (caller id) x* lies on,
 *                 -1 for no split at that point; NULL with anchor_points NULL.
 *                 An id outside [-1, n_prims) makes that point's gradient NaN.
 *   mean_out, var_out   as wob_solve (var_out may be NULL)
 *   grad_out      DEVICE, n_points * dim: mean gradient, point-major
 *   grad_var_out  DEVICE, n_points * dim: variance of each component, or NULL
 * Errors: WOB_E_ARG, WOB_E_UNSUPPORTED (anchors for another formulation),
 * WOB_E_DEVICE. */
wob_status wob_solve_grad(wob_scene scene, const void* points, int64_t n_points, const wob_bc* bc,
                          int32_t samples, int32_t walk_len, uint64_t seed, const void* anchor_points,
                          const int32_t* anchor_prim, void* mean_out, void* var_out, void* grad_out,
                          void* grad_var_out, void* stream);

/* Per-path values (n_points * samples) and gradients (n_points * samples * dim)
 * of the estimator of wob_solve_grad (the same paths, the same anchors). */
wob_status wob_trace_grad(wob_scene scene, const void* points, int64_t n_points, const wob_bc* bc,
                          int32_t samples, int32_t walk_len, uint64_t seed, const void* anchor_points,
                          const int32_t* anchor_prim, void* path_out, void* path_grad_out, void* stream);

/* Measurement helper (not part of the method): `lanes` lanes each read
 * `reads` 32-byte records (two 16-byte loads) at independent pseudo-random
 * record indices of buf (`bytes` long, a multiple of 32, 16-byte aligned) and
 * write the sum of all eight floats of the records they read to out[lane].
 * Timed around, it gives the random-gather rate of the memory level that
 * holds a working set of that size, for records read the way the traversal
 * reads its interior-node records.  Errors: WOB_E_ARG, WOB_E_DEVICE. */
wob_status wob_gather_probe(const void* buf, int64_t bytes, int64_t lanes, int32_t reads, uint32_t seed,
                            float* out, void* stream);

/* Measurement helper (not part of the method): for each of n_tiles tiles,
 * D = A B + C with the bfloat16 matrix instruction that wob_mlp_* use
 * (binary32 accumulation).  a: DEVICE bfloat16, n_tiles x 16 x 32 row-major;
 * b: DEVICE bfloat16, n_tiles x 32 x 16 row-major; c, d: DEVICE binary32,
 * n_tiles x 16 x 16 row-major.  Compared with exact dot products it bounds
 * the instruction's accumulation error, on which the network's parity bound
 * rests.  Errors: WOB_E_ARG, WOB_E_DEVICE. */
wob_status wob_mfma_probe(const void* a, const void* b, const float* c, float* d, int64_t n_tiles,
                          void* stream);

const char* wob_status_string(wob_status status);

/* ------------------------------------------------------------------------- */
/* Forward (adjoint) estimator of the single layer, Neumann boundaries        */
/* (Sec. 4.4.3 "Forward estimator"; the Neumann rows of Table 1 for the single  */
/* layer; boundary starts by the magnitude of the data as in the paper's      */
/* Neumann example, and the reuse of boundary subpaths by every evaluation    */
/* point as in its potential-flow example).                                   */
/*                                                                           */
/* The single layer reads u(x) = int G(x, y) mu(y) dA with mu = f + K mu,     */
/* f = 2 phi q (q the Neumann datum, phi = bc->domain) and K(x, y) =          */
/* -2 phi dG/dn_x(x, y).  A forward path starts at y_1 on the boundary with   */
/* density p_0 and strength W_1 = f(y_1) / p_0(y_1); y_{k+1} is the picked    */
/* hit of a uniformly random line through y_k (one of its m hits, as in the   */
/* backward walk) and W_{k+1} = W_k phi m sgn(cos theta), theta the angle at  */
/* y_{k+1} between y_{k+1} - y_k and the normal there (K with its arguments   */
/* swapped, over the line density).  Vertex k carries c_{k-1} W_k with        */
/* c = (1, ..., 1, 1/2) (the truncated series with the halved last term,      */
/* Sec. 4.1.2), and                                                           */
/*     u(x) ~ (1 / n_paths) sum_paths sum_k c_{k-1} W_k G(x, y_k),            */
/* the same truncated series as the backward single-layer walk.               */
/* ------------------------------------------------------------------------- */

/* Start distribution: primitive T with probability w_T / sum(w), uniform
 * inside T (density P_T / A_T, with P_T read from the binary32 cumulative
 * table built here: binary64 running sum in caller-id order, each entry
 * rounded once).  Weights proportional to |q| A_T put the starts where the
 * data are large; a primitive with w_T = 0 never starts a path, so its data
 * are dropped.
 *   weight  HOST, n_prims values >= 0, finite, sum > 0 (caller-id order)
 * Allocates a device table of n_prims floats.  The table refers to the scene:
 * free it before the scene.  Errors: WOB_E_ARG, WOB_E_ALLOC, WOB_E_DEVICE. */
typedef struct wob_starts_s* wob_starts;
wob_status wob_starts_create(wob_scene scene, const double* weight, wob_starts* out);

/* Starts by the magnitude of the data (the paper's boundary sampling for
 * sparse Neumann values): w_T = (|q(c_T)| + floor * qbar) A_T with q the datum
 * of bc (program and params; Neumann rows) at the centroid c_T and
 * qbar = sum |q(c_T)| A_T / sum A_T.  floor >= 0; with floor > 0 every
 * primitive can start a path, so the estimate stays unbiased where q vanishes
 * at a centroid but not elsewhere on the primitive.  The weights are computed
 * on the device in the scene's precision, the table as in wob_starts_create.
 * Errors: WOB_E_ARG (also: all weights zero), WOB_E_ALLOC, WOB_E_DEVICE. */
wob_status wob_starts_from_data(wob_scene scene, const wob_bc* bc, double floor, wob_starts* out);
void wob_starts_free(wob_starts starts);

/* Forward paths.  Scene: every primitive Neumann; bc: formulation AUTO or
 * SINGLE_LAYER, density 0, sampling LINE (program and params give q).
 *   starts     from wob_starts_create on this scene, or NULL = uniform by area
 *   n_paths    0 <= n_paths < 2^32; path j draws Philox counters
 *              (j, 0xfffffffe, (0 << 24) | 0xffff03, 0) for its start (word 0
 *              the primitive, words 1, 2 the point) and, for line i from y_{i+1},
 *              blocks 0 (direction) and 2 (hit keys) as the backward walk
 *   walk_len   M vertices per path, 1 <= M < 65535 (M - 1 lines)
 *   vtx_out    DEVICE, n_paths * M * 4 values of the scene's precision, path-major:
 *              (y_x, y_y, y_z (0 in 2D), c_{k-1} W_k); 16-byte (binary64:
 *              32-byte) aligned.  A path whose line finds no hit ends: its
 *              later vertices are (1e18, 1e18, 1e18 (0 in 2D), 0), strength 0 far
 *              from any evaluation point.
 *   vtx_prim   DEVICE, n_paths * M caller ids of the vertices (-1 after the end),
 *              or NULL
 *   vtx_m      DEVICE, n_paths * M hits of the line that reached each vertex
 *              (0 for the start and after the end), or NULL
 * Errors: WOB_E_ARG, WOB_E_UNSUPPORTED (not all Neumann, another formulation,
 * density or RIS), WOB_E_DEVICE. */
wob_status wob_forward_paths(wob_scene scene, const wob_bc* bc, wob_starts starts, int64_t n_paths,
                             int32_t walk_len, uint64_t seed, void* vtx_out, int32_t* vtx_prim,
                             int32_t* vtx_m, void* stream);

/* Every evaluation point connected to every forward-path vertex:
 * mean_out[p] = (1 / n_paths) sum_j c_j(x_p), c_j(x) = sum_k v_jk.w G(x, v_jk.y),
 * var_out[p] = unbiased variance of the c_j.  The paths' correlation across
 * points is the price of the reuse.  G is singular at distance zero: a point
 * exactly at a vertex's position gets a non-finite value (records must hold
 * finite positions; ended paths' records add exactly 0 for points within
 * 1e17 of the origin).
 *   vtx        DEVICE, as written by wob_forward_paths (n_paths * walk_len records)
 *   n_paths    >= 1 (>= 2 with var_out)
 *   points     DEVICE, n_points * dim of the scene's precision
 *   mean_out   DEVICE, n_points;  var_out DEVICE, n_points, or NULL
 * The scene gives dimension, precision and device only.
 * Errors: WOB_E_ARG, WOB_E_DEVICE. */
wob_status wob_forward_gather(wob_scene scene, const void* vtx, int64_t n_paths, int32_t walk_len,
                              const void* points, int64_t n_points, void* mean_out, void* var_out,
                              void* stream);

/* ------------------------------------------------------------------------- */
/* Batched solves: many problems (scenes, point sets, data, N, M) in one      */
/* persistent launch.  Not in the paper: its estimators are run per problem;  */
/* batching only schedules them together.                                     */
/* ------------------------------------------------------------------------- */

typedef struct {
  wob_scene scene;          /* all scenes of a batch share dim, precision and device */
  const void* points;       /* DEVICE, n_points * dim */
  const int32_t* point_prim;/* DEVICE or NULL, as in wob_solve */
  int64_t n_points;
  wob_bc bc;
  int32_t samples;          /* N >= 2 */
  int32_t walk_len;         /* M >= 1 */
  uint64_t seed;
  uint32_t stream_id;       /* random-number counter field "problem" (< 256); with the same
                               seed and stream_id 0 a problem draws exactly the paths of
                               wob_solve */
  int32_t reserved;         /* must be 0 */
  void* mean_out;           /* DEVICE, n_points */
  void* var_out;            /* DEVICE, n_points, or NULL */
} wob_problem;

/* Launch shape of the persistent kernel. */
typedef struct {
  int32_t block;            /* lanes per workgroup: 64, 128, 256 or 512 */
  int32_t blocks_per_cu;    /* persistent workgroups per compute unit, 1..32 */
} wob_tune;

typedef struct wob_batch_s* wob_batch;

/* Validate the problems, upload the problem table and capture the solve as a
 * hipGraph {reset the tile counter, persistent kernel}.  The arrays of every
 * problem must stay valid while the batch is used.  tune NULL = 256 lanes,
 * 4 workgroups per CU (128 lanes when the traversal stacks of the deepest
 * scene would not fit a 256-lane workgroup's LDS; a given tune that does not
 * fit is WOB_E_ARG).  Tiles (one workgroup's points of one problem) are
 * ordered by decreasing estimated cost and pulled from an atomic counter.
 * Errors: WOB_E_ARG, WOB_E_UNSUPPORTED, WOB_E_ALLOC, WOB_E_DEVICE. */
wob_status wob_batch_create(const wob_problem* problems, int32_t n_problems,
                            const wob_tune* tune, wob_batch* out);

/* Replay the captured graph on `stream`: solves every problem. */
wob_status wob_batch_launch(wob_batch batch, void* stream);

/* Autotuner: time every candidate launch shape on a strided subset of the
 * tiles (every sample_stride-th tile, >= 1) and keep the fastest; re-captures
 * the graph.  With cache_path (or NULL), a text file of
 * "<workload signature> <block> <blocks_per_cu>" lines is read first (a hit
 * skips the timing) and appended after tuning.  Overwrites the problems'
 * outputs.  chosen may be NULL.  Synchronous on `stream`. */
wob_status wob_batch_autotune(wob_batch batch, int32_t sample_stride, const char* cache_path,
                              wob_tune* chosen, void* stream);

/* Current launch shape and total tiles. */
wob_status wob_batch_get_tune(wob_batch batch, wob_tune* tune, int64_t* n_tiles);

void wob_batch_free(wob_batch batch);

/* One-shot: create, launch, wait on `stream`, free. */
wob_status wob_solve_batched(const wob_problem* problems, int32_t n_problems,
                             const wob_tune* tune, void* stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): wob_solve_batched without any device
 * allocation.  The problem table, the tile offsets and the tile counter live
 * in a fixed, file-scope device array of the library (one per device, about
 * WOB_STATIC_MAX_PROBLEMS * 0.5 KB, held until the process ends), so at most
 * WOB_STATIC_MAX_PROBLEMS problems per call (more: WOB_E_TOO_LARGE, nothing
 * launched).  Same problems, tune and results as wob_solve_batched (bitwise:
 * the same kernel and launch shape; tune NULL = 256 lanes x 4 per CU, or the
 * same fallback); no autotuning and no graph.  The table is copied from host
 * memory the call owns, so the call waits for `stream` before it returns.
 * Every call on a device shares that device's array and overwrites it (the
 * counter is reset by a kernel each call): calls that overlap on one device,
 * from several threads or on several streams, race and must be serialised by
 * the caller.  Errors: as wob_batch_create, and WOB_E_TOO_LARGE. */
#define WOB_STATIC_MAX_PROBLEMS 256
wob_status wob_solve_batched_static(const wob_problem* problems, int32_t n_problems,
                                    const wob_tune* tune, void* stream);

/* ------------------------------------------------------------------------- */
/* Learned control variate (not in the paper; an exact control variate for   */
/* the single-layer estimator of Sec. 4.3, Table 1 Neumann / Robin rows).    */
/* ------------------------------------------------------------------------- */

/* Fourier-feature MLP on the matrix cores: z0 = [sin(2 pi B y), cos(2 pi B y)]
 * (16 frequencies, B is 16 x dim), four hidden layers of 128 with SiLU, scalar
 * output; bfloat16 weights and activations, binary32 accumulation.  Parameters
 * are one flat binary32 array: W_1 [128][32], b_1, W_2..W_4 [128][128], b_2..b_4,
 * W_5 [1][128], b_5 (53,889 values). */
typedef struct wob_mlp_s* wob_mlp;

int64_t wob_mlp_n_params(void);

/* fourier: HOST 16 x dim; params: HOST wob_mlp_n_params() values; max_batch: the
 * largest batch wob_mlp_backward / wob_mlp_train_step accept (0 = inference only).
 * The library owns the device copies (parameters, Adam moments, bfloat16 copies,
 * workspace).  Synchronous.  Errors: WOB_E_ARG, WOB_E_ALLOC, WOB_E_DEVICE. */
wob_status wob_mlp_create(int32_t dim, const float* fourier, const float* params, int64_t max_batch,
                          wob_mlp* out);
void wob_mlp_free(wob_mlp net);
/* HOST copies of the binary32 parameters (set also resets the Adam moments). */
wob_status wob_mlp_get_params(wob_mlp net, float* params);
wob_status wob_mlp_set_params(wob_mlp net, const float* params);
/* HOST copies of the Adam moments (first and second, wob_mlp_n_params() values
 * each; binary32).  With the parameters they are the whole training state (the
 * step count is the caller's, passed to each Adam step): a fit checkpointed by
 * get_params + get_moments and restored by set_params then set_moments goes on
 * exactly as without the break.  Synchronous with the null stream: wait for
 * work enqueued on other streams first.  Errors: WOB_E_ARG, WOB_E_DEVICE. */
wob_status wob_mlp_get_moments(wob_mlp net, float* m, float* v);
wob_status wob_mlp_set_moments(wob_mlp net, const float* m, const float* v);

/* out[i] = f(y_i); y DEVICE n x dim, out DEVICE n. */
wob_status wob_mlp_forward(wob_mlp net, const float* y, int64_t n, float* out, void* stream);

/* Optional transform of the targets inside the loss: t -> (t - shift) / scale,
 * then clamped to [-clip, clip] when clip > 0 (scale > 0). */
typedef struct {
  float shift;
  float scale;
  float clip;
} wob_target_map;

/* Mean squared error (1/n) sum (f(y_i) - t_i)^2, t_i = target_i mapped by tmap
 * (NULL = unchanged), and its gradient with respect to every parameter (DEVICE
 * grad, wob_mlp_n_params() floats; loss DEVICE 1 float or NULL).  Deterministic.
 * 1 <= n <= max_batch. */
wob_status wob_mlp_backward(wob_mlp net, const float* y, const float* target,
                            const wob_target_map* tmap, int64_t n, float* grad, float* loss,
                            void* stream);

/* Adam (Kingma and Ba) on the binary32 parameters with bias correction for step
 * >= 1, then refresh of the bfloat16 copies.  grad DEVICE. */
wob_status wob_mlp_adam_step(wob_mlp net, const float* grad, int64_t step, float lr, float b1,
                             float b2, float eps, void* stream);

/* backward + Adam (b1 0.9, b2 0.999, eps 1e-8) with an internal gradient buffer. */
wob_status wob_mlp_train_step(wob_mlp net, const float* y, const float* target,
                              const wob_target_map* tmap, int64_t n, int64_t step, float lr,
                              float* loss, void* stream);

/* n area-uniform points on the boundary (DEVICE n * dim, scene precision) and the
 * primitive each lies on (DEVICE n int32), from Philox counter (i, 0xffffffff,
 * 0xffffff03, 0) with key seed: the training locations of the control variate. */
wob_status wob_sample_boundary(wob_scene scene, int64_t n, uint64_t seed, void* points_out,
                               int32_t* prim_out, void* stream);

/* Control-variate table: g[id] = net(centroid of primitive id), DEVICE n_prims floats.
 * 3D binary32 scenes. */
wob_status wob_cv_table(wob_scene scene, wob_mlp net, float* g_out, void* stream);

/* Exact control variate for the single-layer estimator (3D, binary32 scenes;
 * the control variate is not part of the paper).  Same paths and picks as
 * wob_solve; every line adds a term whose mean given the line is zero because
 * the pick is uniform over the m hits (with RIS sampling: given the C
 * candidates, the pick's mean is (|Gamma| / C) sum_j k(y_j) F(y_j), and the
 * sums below run over the candidates):
 *   line 0:     the subtraction w(j) g0(T_j), whose mean sum_T g0_T int_T G(x0, y) dA
 *               is added per point (wob_cv_addback, with the solve's seed);
 *   lines 1..M-2: the all-hits sum of a(h) [2 phi s(y_h) + g(T_h)] minus the
 *               picked w(j) g(T_j);
 *   last line:  the all-hits mean of the last emission.
 * Unbiased for all tables g, g0 (DEVICE, n_prims floats by primitive id; g0 NULL
 * means g0 = g).  With g close to the boundary unknown minus its emission and
 * g0 = g + the emission at the centroid (wob_cv_emission) the variance falls.
 * Errors as wob_solve; WOB_E_UNSUPPORTED for other formulations, 2D or binary64
 * scenes. */
wob_status wob_solve_cv(wob_scene scene, const void* points, const int32_t* point_prim,
                        int64_t n_points, const wob_bc* bc, int32_t samples, int32_t walk_len,
                        uint64_t seed, const float* g, const float* g0, void* mean_out,
                        void* var_out, void* stream);

/* Per-path values of the corrected estimator WITHOUT the per-point add-back. */
wob_status wob_trace_cv(wob_scene scene, const void* points, const int32_t* point_prim,
                        int64_t n_points, const wob_bc* bc, int32_t samples, int32_t walk_len,
                        uint64_t seed, const float* g, const float* g0, void* path_out,
                        void* stream);

/* out[p] = an unbiased value of sum_T g_T int_T G(x_p, y) dA: the closed form for
 * triangles whose centroid is within four bounding radii of x_p, and for every
 * other triangle g_T A_T G(x_p, y_T) at one point y_T uniform in T drawn from a
 * 32-bit hash of (seed, triangle id), the same for every point.  DEVICE arrays
 * (points n_points x 3, out n_points). */
wob_status wob_cv_addback(wob_scene scene, const float* g, const void* points, int64_t n_points,
                          uint64_t seed, void* out, void* stream);

/* g0_out[id] = (g ? g[id] : 0) + 2 phi s(c_id), s the boundary datum of bc on
 * primitive id at its centroid c_id, phi = bc->domain: the line-0 table of
 * wob_solve_cv.  Single-layer problems, 3D binary32 scenes.  DEVICE arrays. */
wob_status wob_cv_emission(wob_scene scene, const wob_bc* bc, const float* g, float* g0_out,
                           void* stream);

#ifdef __cplusplus
}
#endif
#endif /* WOB_H */
