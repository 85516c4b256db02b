/*
 * oracle.c - FP64 brute-force walk-on-boundary reference estimator.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Plain, slow and literal on
 * purpose: every line query tests every primitive, every weight is formed as
 * "kernel / pdf" from the fundamental solution of Appendix A and the
 * line-sampling density of Sec. 4.4.1, and all arithmetic is double precision.
 *
 * Random-number streams (Philox4x32-10, key = (seed low 32 bits, seed high 32
 * bits)); counter words for path k of point p, problem q, line i:
 *     ctr = (k, p, (q << 24) | (i << 8) | block, w)
 *   block 0, w = 0     : word0, word1 -> line direction, word2 -> mixture branch
 *   block 1, w = 0     : word0, word1 -> in-plane self-panel sample
 *   block 2, w = prim  : word0 -> selection key of primitive `prim` on line i
 * Uniform variates: u = ((word >> 9) + 0.5) / 2^23, exact in binary32 and
 * binary64.  A branch with probability p is taken when (word >> 8) < floor(p 2^24).
 *
 * Hit selection (Sec. 4.4.1 picks one of the m hits uniformly at random):
 * the hit with the smallest (key, primitive id) is taken.  With independent
 * keys this is a uniform choice among the m hits and does not depend on the
 * order in which hits are found.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as    */
/* easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies, with a   */
/* Weyl key schedule between rounds.                                          */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint32_t path, uint32_t point, uint32_t problem,
                 uint32_t line, uint32_t block, uint32_t w, uint32_t out[4]) {
  uint32_t ctr[4] = {path, point, (problem << 24) | (line << 8) | block, w};
  uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
  orc_philox4x32_10(ctr, key, out);
}

static double uniform(uint32_t word) {
  return ((double)(word >> 9) + 0.5) / 8388608.0;
}

/* ------------------------------------------------------------------------- */
/* Small vector helpers (dimension 2 or 3; unused components are zero).       */
/* ------------------------------------------------------------------------- */
static double dot(const double* a, const double* b, int dim) {
  double s = 0.0;
  for (int k = 0; k < dim; ++k) s += a[k] * b[k];
  return s;
}
static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
static double cross2(const double* a, const double* b) { return a[0] * b[1] - a[1] * b[0]; }

static void prim_vertex(const orc_mesh* m, int64_t prim, int corner, double* v) {
  int64_t vi = m->prims[prim * m->dim + corner];
  v[2] = 0.0;
  for (int a = 0; a < m->dim; ++a) v[a] = m->verts[vi * m->dim + a];
}

void orc_prim_normal(const orc_mesh* m, int64_t prim, double* n) {
  double v0[3] = {0.0, 0.0, 0.0}, v1[3] = {0.0, 0.0, 0.0}, v2[3] = {0.0, 0.0, 0.0};
  n[0] = n[1] = n[2] = 0.0;
  prim_vertex(m, prim, 0, v0);
  prim_vertex(m, prim, 1, v1);
  if (m->dim == 3) {
    prim_vertex(m, prim, 2, v2);
    double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
    double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
    cross3(e1, e2, n);
    double l = sqrt(dot(n, n, 3));
    for (int a = 0; a < 3; ++a) n[a] /= l;
  } else {
    /* counter-clockwise boundary: the outward normal is the tangent turned by -90 deg */
    double e[2] = {v1[0] - v0[0], v1[1] - v0[1]};
    double l = sqrt(e[0] * e[0] + e[1] * e[1]);
    n[0] = e[1] / l;
    n[1] = -e[0] / l;
  }
}

static int prim_kind(const orc_mesh* m, int64_t prim) {
  return m->kind ? (int)m->kind[prim] : ORC_DIRICHLET;
}
static double prim_alpha(const orc_mesh* m, int64_t prim) {
  return m->alpha ? m->alpha[prim] : 0.0;
}

/* ------------------------------------------------------------------------- */
/* Fundamental solution and its derivatives, Appendix A (r = y - x).          */
/* ------------------------------------------------------------------------- */
static double G(const double* x, const double* y, int dim) {
  double r[3] = {y[0] - x[0], y[1] - x[1], dim == 3 ? y[2] - x[2] : 0.0};
  double rn = sqrt(dot(r, r, dim));
  return dim == 3 ? 1.0 / (4.0 * ORC_PI * rn) : -log(rn) / (2.0 * ORC_PI);
}
/* Error scale of a G factor for the parity tolerance (the magnitude sum of a
   path): |G| in 3D; in 2D max(|ln rho|, 1) / (2 pi), because ln rho carries an
   absolute rounding error of order one unit of the arithmetic, which does not
   vanish where G itself does (rho near 1). */
static double G_mag(const double* x, const double* y, int dim) {
  if (dim == 3) return fabs(G(x, y, dim));
  double r[2] = {y[0] - x[0], y[1] - x[1]};
  return fmax(fabs(log(sqrt(r[0] * r[0] + r[1] * r[1]))), 1.0) / (2.0 * ORC_PI);
}

static double dG_dny(const double* x, const double* y, const double* ny, int dim) {
  double r[3] = {y[0] - x[0], y[1] - x[1], dim == 3 ? y[2] - x[2] : 0.0};
  double rn = sqrt(dot(r, r, dim));
  double rdn = dot(r, ny, dim);
  return dim == 3 ? -rdn / (4.0 * ORC_PI * rn * rn * rn) : -rdn / (2.0 * ORC_PI * rn * rn);
}
static double dG_dnx(const double* x, const double* y, const double* nx, int dim) {
  double r[3] = {y[0] - x[0], y[1] - x[1], dim == 3 ? y[2] - x[2] : 0.0};
  double rn = sqrt(dot(r, r, dim));
  double rdn = dot(r, nx, dim);
  return dim == 3 ? rdn / (4.0 * ORC_PI * rn * rn * rn) : rdn / (2.0 * ORC_PI * rn * rn);
}

/* Gradients in x (the evaluation point) of G and of dG/dn_y, for the gradient
 * estimators (Sec. 4.1.3, derivative estimators; the gradient equations of
 * the three formulations of Table 1 and Sec. 4.3).  With r = y - x, rho = |r| and S_D = 4 pi (3D), 2 pi (2D):
 *   grad_x G        = r / (S_D rho^D)
 *   grad_x dG/dn_y  = (n_y / rho^D - D (r . n_y) r / rho^(D+2)) / S_D        */
static void grad_G(const double* x, const double* y, int dim, double* g) {
  double r[3] = {y[0] - x[0], y[1] - x[1], dim == 3 ? y[2] - x[2] : 0.0};
  const double rho = sqrt(dot(r, r, dim));
  const double c = dim == 3 ? 1.0 / (4.0 * ORC_PI * rho * rho * rho) : 1.0 / (2.0 * ORC_PI * rho * rho);
  for (int a = 0; a < 3; ++a) g[a] = c * r[a];
}
static void grad_dG_dny(const double* x, const double* y, const double* ny, int dim, double* g) {
  double r[3] = {y[0] - x[0], y[1] - x[1], dim == 3 ? y[2] - x[2] : 0.0};
  const double rr = dot(r, r, dim), rho = sqrt(rr), rdn = dot(r, ny, dim);
  const double sd = dim == 3 ? 4.0 * ORC_PI : 2.0 * ORC_PI;
  const double rd = dim == 3 ? rr * rho : rr; /* rho^D */
  for (int a = 0; a < 3; ++a) g[a] = (ny[a] / rd - (double)dim * rdn * r[a] / (rd * rr)) / sd;
  if (dim == 2) g[2] = 0.0;
}

/* Area density of the point y reached by a uniformly random line through x
 * that is one of m hits picked uniformly: the line direction is uniform on the
 * sphere (circle) and covers +d and -d, so the density per unit solid angle is
 * 2/(4 pi) (per radian 2/(2 pi)); converting solid angle to area gives
 * |cos theta_y| / r^2 (2D: / r).  Sec. 4.4.1: picking one of m multiplies by 1/m. */
static double line_pdf(const double* x, const double* y, const double* ny, int m, int dim) {
  double r[3] = {y[0] - x[0], y[1] - x[1], dim == 3 ? y[2] - x[2] : 0.0};
  double rn = sqrt(dot(r, r, dim));
  double c = fabs(dot(r, ny, dim)) / rn;
  if (dim == 3) return (2.0 / (4.0 * ORC_PI)) * c / (rn * rn) / (double)m;
  return (2.0 / (2.0 * ORC_PI)) * c / rn / (double)m;
}

/* ------------------------------------------------------------------------- */
/* Harmonic programs u(x) and the boundary datum derived from them.           */
/* ------------------------------------------------------------------------- */
static void program_eval(const orc_mesh* m, const orc_bc* bc, const double* y, double* u,
                         double* grad) {
  const double* p = bc->params;
  int dim = m->dim;
  grad[0] = grad[1] = grad[2] = 0.0;
  switch (bc->program) {
    case ORC_PROG_CONST:
      *u = p[0];
      break;
    case ORC_PROG_LINEAR:
      *u = p[0] * y[0] + p[1] * y[1] + (dim == 3 ? p[2] * y[2] : 0.0) + p[3];
      grad[0] = p[0];
      grad[1] = p[1];
      grad[2] = dim == 3 ? p[2] : 0.0;
      break;
    case ORC_PROG_QUAD:
      *u = y[0] * y[0] - y[1] * y[1];
      grad[0] = 2.0 * y[0];
      grad[1] = -2.0 * y[1];
      break;
    case ORC_PROG_INVDIST: {
      double r[3] = {y[0] - p[0], y[1] - p[1], dim == 3 ? y[2] - p[2] : 0.0};
      double rr = dot(r, r, dim);
      if (dim == 3) {
        double rn = sqrt(rr);
        *u = 1.0 / rn;
        for (int a = 0; a < 3; ++a) grad[a] = -r[a] / (rr * rn);
      } else {
        *u = 0.5 * log(rr);
        for (int a = 0; a < 2; ++a) grad[a] = r[a] / rr;
      }
      break;
    }
    default:
      *u = NAN;
  }
}

double orc_program_value(const orc_mesh* m, const orc_bc* bc, const double* y) {
  double u, g[3];
  program_eval(m, bc, y, &u, g);
  return u;
}

/* Barycentric coordinates of y on primitive prim (the least-squares point of
   its plane): solve [e1.e1 e1.e2; e1.e2 e2.e2] (b1, b2) = (e1.w, e2.w), w = y - v0
   (2D: b1 = e.w / e.e); b0 = 1 - b1 - b2. */
static void prim_bary(const orc_mesh* m, int64_t prim, const double* y, double b[3]) {
  double v0[3] = {0.0, 0.0, 0.0}, v1[3] = {0.0, 0.0, 0.0}, v2[3] = {0.0, 0.0, 0.0};
  prim_vertex(m, prim, 0, v0);
  prim_vertex(m, prim, 1, v1);
  const int dim = m->dim;
  double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], dim == 3 ? v1[2] - v0[2] : 0.0};
  double w[3] = {y[0] - v0[0], y[1] - v0[1], dim == 3 ? y[2] - v0[2] : 0.0};
  if (dim == 2) {
    b[1] = dot(e1, w, 2) / dot(e1, e1, 2);
    b[2] = 0.0;
  } else {
    prim_vertex(m, prim, 2, v2);
    double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
    const double g11 = dot(e1, e1, 3), g12 = dot(e1, e2, 3), g22 = dot(e2, e2, 3);
    const double r1 = dot(e1, w, 3), r2 = dot(e2, w, 3), det = g11 * g22 - g12 * g12;
    b[1] = (r1 * g22 - r2 * g12) / det;
    b[2] = (r2 * g11 - r1 * g12) / det;
  }
  b[0] = 1.0 - b[1] - b[2];
}

/* Per-vertex data interpolated linearly on primitive prim at y. */
static double vertex_datum(const orc_mesh* m, const orc_bc* bc, int64_t prim, const double* y) {
  double b[3];
  prim_bary(m, prim, y, b);
  double f = 0.0;
  for (int c = 0; c < m->dim; ++c) f += b[c] * bc->vertex_data[m->prims[prim * m->dim + c]];
  return f;
}

/* eq. PoissonBC: Dirichlet value u, Neumann flux du/dn, Robin du/dn + alpha u;
   with per-vertex data, the interpolated value is the datum of the primitive's
   own kind. */
double orc_boundary_datum(const orc_mesh* m, const orc_bc* bc, int64_t prim, const double* y) {
  if (bc->data_mode == 1) return vertex_datum(m, bc, prim, y);
  double u, g[3], n[3];
  program_eval(m, bc, y, &u, g);
  int kind = prim_kind(m, prim);
  if (kind == ORC_DIRICHLET) return u;
  orc_prim_normal(m, prim, n);
  double q = dot(n, g, m->dim);
  if (kind == ORC_NEUMANN) return q;
  return q + prim_alpha(m, prim) * u;
}

/* ------------------------------------------------------------------------- */
/* Line / primitive intersection (line x + t d, t real).                      */
/* Returns 1 on a hit.  *margin is the signed smallest barycentric coordinate  */
/* (negative outside), *cosv = |d . n| of the primitive.                       */
/* ------------------------------------------------------------------------- */
static int line_prim_b(const orc_mesh* m, int64_t j, const double* x, const double* d,
                       double* t, double* y, double* margin, double* cosv, double* bary);

static int line_prim(const orc_mesh* m, int64_t j, const double* x, const double* d,
                     double* t, double* y, double* margin, double* cosv) {
  double b[2];
  return line_prim_b(m, j, x, d, t, y, margin, cosv, b);
}

/* As line_prim; also writes the barycentric coordinates of y along e1, e2
   (2D: along the segment, and 0). */
static int line_prim_b(const orc_mesh* m, int64_t j, const double* x, const double* d,
                       double* t, double* y, double* margin, double* cosv, double* bary) {
  double v0[3] = {0.0, 0.0, 0.0}, v1[3] = {0.0, 0.0, 0.0}, v2[3] = {0.0, 0.0, 0.0};
  prim_vertex(m, j, 0, v0);
  prim_vertex(m, j, 1, v1);
  if (m->dim == 3) {
    /* Moeller-Trumbore in double precision, inclusive edges */
    prim_vertex(m, j, 2, v2);
    double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2]};
    double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
    double pv[3], qv[3], nn[3];
    cross3(d, e2, pv);
    double det = dot(e1, pv, 3);
    cross3(e1, e2, nn);
    double nl = sqrt(dot(nn, nn, 3));
    *cosv = fabs(dot(d, nn, 3)) / nl;
    if (det == 0.0) {
      *margin = 0.0;
      return 0;
    }
    double s[3] = {x[0] - v0[0], x[1] - v0[1], x[2] - v0[2]};
    double u = dot(s, pv, 3) / det;
    cross3(s, e1, qv);
    double v = dot(d, qv, 3) / det;
    *t = dot(e2, qv, 3) / det;
    double w = 1.0 - u - v;
    double mg = u < v ? u : v;
    mg = mg < w ? mg : w;
    *margin = mg;
    for (int a = 0; a < 3; ++a) y[a] = v0[a] + u * e1[a] + v * e2[a];
    bary[0] = u;
    bary[1] = v;
    return mg >= 0.0;
  } else {
    double e[2] = {v1[0] - v0[0], v1[1] - v0[1]};
    double det = cross2(d, e);
    double el = sqrt(e[0] * e[0] + e[1] * e[1]);
    *cosv = fabs(cross2(d, e)) / el; /* |d . n| with n the unit normal of e */
    if (det == 0.0) {
      *margin = 0.0;
      return 0;
    }
    double xa[2] = {x[0] - v0[0], x[1] - v0[1]};
    double ax[2] = {v0[0] - x[0], v0[1] - x[1]};
    double s = cross2(xa, d) / cross2(e, d);
    *t = cross2(ax, e) / det;
    double mg = s < 1.0 - s ? s : 1.0 - s;
    *margin = mg;
    y[0] = v0[0] + s * e[0];
    y[1] = v0[1] + s * e[1];
    y[2] = 0.0;
    bary[0] = s;
    bary[1] = 0.0;
    return mg >= 0.0;
  }
}

/* Grazing measure of a line / primitive decision: the smallest barycentric
   margin expressed in units of the rounding scale of the decision a binary
   intersection test takes.  Such a test decides on the numerators of the
   barycentric coordinates, (x - v0) . (d x e2) and d . ((x - v0) x e1) in 3D
   (-(x - v0) x d in 2D), whose rounding is of order |x - v0| |e| units, against
   the margin times |det| = 2 A cos (|e| cos in 2D); the sum test adds |e1| |e2|.
   So g = |margin| |det| / (|x - v0| (|e1| + |e2|) + |e1| |e2|) (2D:
   |margin| |e| cos / (|x - v0| + |e|)).  Near the line's start on a
   well-shaped triangle g is about |margin| cos / 3; it is far smaller on
   slivers and on primitives far from x, whose decisions are ill-conditioned. */
static double decision_margin(const orc_mesh* m, int64_t j, const double* x, double margin, double cosv) {
  double v0[3] = {0.0, 0.0, 0.0}, v1[3] = {0.0, 0.0, 0.0}, v2[3] = {0.0, 0.0, 0.0};
  prim_vertex(m, j, 0, v0);
  prim_vertex(m, j, 1, v1);
  const int dim = m->dim;
  double s[3] = {x[0] - v0[0], x[1] - v0[1], dim == 3 ? x[2] - v0[2] : 0.0};
  double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], dim == 3 ? v1[2] - v0[2] : 0.0};
  const double l1 = sqrt(dot(e1, e1, dim)), ls = sqrt(dot(s, s, dim));
  if (dim == 2) return fabs(margin) * l1 * cosv / (ls + l1);
  prim_vertex(m, j, 2, v2);
  double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]}, n[3];
  cross3(e1, e2, n);
  const double l2 = sqrt(dot(e2, e2, 3)), a2 = sqrt(dot(n, n, 3));
  return fabs(margin) * a2 * cosv / (ls * (l1 + l2) + l1 * l2);
}

/* ------------------------------------------------------------------------- */
/* In-plane sample on the primitive that contains x ("self panel").  A line   */
/* through x never meets the primitive it starts on (its plane contains the  */
/* line only with probability zero), yet G does not vanish there; this term  */
/* covers that part of every single-layer integral.                           */
/*  3D: theta uniform in [0, 2 pi), radius uniform in [0, R(theta)], where     */
/*      R(theta) is the distance from x to the triangle's boundary; the area   */
/*      density is 1 / (2 pi R(theta) rho).                                    */
/*  2D: y uniform along the segment; density 1 / length.                       */
/* Returns G(x, y) / p(y).                                                     */
/* ------------------------------------------------------------------------- */
/* The sample itself; R_out and sinb_out (3D, may be NULL) receive the
   distance R(theta) to the triangle's boundary and the sine of the angle at
   which the in-plane ray leaves through its edge (the rounding-error bound
   below needs both). */
static double self_panel_geo(const orc_mesh* m, int64_t prim, const double* x, double u0, double u1,
                             double* y, double* R_out, double* sinb_out) {
  double v[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  for (int c = 0; c < m->dim; ++c) prim_vertex(m, prim, c, v[c]);
  if (m->dim == 3) {
    double n[3], t1[3], t2[3];
    orc_prim_normal(m, prim, n);
    double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
    double l1 = sqrt(dot(e1, e1, 3));
    for (int a = 0; a < 3; ++a) t1[a] = e1[a] / l1;
    cross3(n, t1, t2);
    double loc[3][2];
    for (int c = 0; c < 3; ++c) {
      double r[3] = {v[c][0] - x[0], v[c][1] - x[1], v[c][2] - x[2]};
      loc[c][0] = dot(r, t1, 3);
      loc[c][1] = dot(r, t2, 3);
    }
    double theta = 2.0 * ORC_PI * u0;
    double dir[2] = {cos(theta), sin(theta)};
    double R = INFINITY, sinb = 1.0;
    for (int c = 0; c < 3; ++c) {
      const double* a = loc[c];
      const double* b = loc[(c + 1) % 3];
      double e[2] = {b[0] - a[0], b[1] - a[1]};
      double den = cross2(dir, e);
      if (den != 0.0) {
        double s = cross2(a, e) / den;
        if (s > 0.0 && s < R) {
          R = s;
          sinb = fabs(den) / sqrt(e[0] * e[0] + e[1] * e[1]);
        }
      }
    }
    if (!(R < INFINITY)) R = 0.0;
    if (R_out) *R_out = R;
    if (sinb_out) *sinb_out = sinb;
    double rho = u1 * R;
    for (int a = 0; a < 3; ++a) y[a] = x[a] + rho * (dir[0] * t1[a] + dir[1] * t2[a]);
    if (rho <= 0.0) return 0.0;
    double pdf = 1.0 / (2.0 * ORC_PI * R * rho);
    return G(x, y, 3) / pdf;
  } else {
    double e[2] = {v[1][0] - v[0][0], v[1][1] - v[0][1]};
    double len = sqrt(e[0] * e[0] + e[1] * e[1]);
    y[0] = v[0][0] + u0 * e[0];
    y[1] = v[0][1] + u0 * e[1];
    y[2] = 0.0;
    double pdf = 1.0 / len;
    if (R_out) *R_out = len;
    if (sinb_out) *sinb_out = 1.0;
    return G(x, y, 2) / pdf;
  }
}

double orc_self_panel(const orc_mesh* m, int64_t prim, const double* x, double u0, double u1,
                      double* y) {
  return self_panel_geo(m, prim, x, u0, u1, y, NULL, NULL);
}

/* ------------------------------------------------------------------------- */
/* Formulation mapping, Table 1: Dirichlet -> double layer, Neumann -> direct,*/
/* Robin or Neumann/Robin mixtures -> single layer.  Mixtures containing      */
/* Dirichlet parts (first-kind rows) are not handled here.                    */
/* ------------------------------------------------------------------------- */
int orc_resolve_formulation(const orc_mesh* m, int formulation) {
  int nd = 0, nn = 0, nr = 0;
  for (int64_t j = 0; j < m->n_prims; ++j) {
    int k = prim_kind(m, j);
    nd += k == ORC_DIRICHLET;
    nn += k == ORC_NEUMANN;
    nr += k == ORC_ROBIN;
  }
  if (formulation == ORC_AUTO) {
    if (nn == 0 && nr == 0) return ORC_DOUBLE_LAYER;
    if (nd == 0 && nr == 0) return ORC_DIRECT;
    return ORC_SINGLE_LAYER; /* Robin, Neumann / Robin, and mixed with Dirichlet parts */
  }
  if (formulation == ORC_DOUBLE_LAYER) return (nn == 0 && nr == 0) ? formulation : -1;
  if (formulation == ORC_DIRECT) return (nd == 0 && nr == 0) ? formulation : -1;
  if (formulation == ORC_SINGLE_LAYER) return formulation;
  return -1;
}

int orc_lines_per_path(const orc_mesh* m, const orc_bc* bc, int walk_len) {
  int f = orc_resolve_formulation(m, bc->formulation);
  return f == ORC_DIRECT ? walk_len + 1 : walk_len;
}

/* ------------------------------------------------------------------------- */
/* First-order rounding-error bound of a path.  Used only as the parity       */
/* tolerance of the tests; it plays no part in any estimate.                  */
/*                                                                           */
/* A device evaluation of the same path in a binary format with unit roundoff */
/* u rounds every vertex, weight and emission.  Their first-order effect on   */
/* the path value is bounded here in units of u (so one bound serves binary32 */
/* and binary64), from the geometry of the path alone:                        */
/*  - vertex position: the hit y of the line x + t d on a primitive met at     */
/*    incidence c = |cos theta_y| moves in the primitive's plane by the line's */
/*    own displacement over c.  The line is displaced by the error P(x) of its */
/*    start and by the rounding of x - v0, of d and of the products of the     */
/*    intersection test, whose operands have sizes |x|, |y| and rho = |t|:     */
/*        P(y) = (P(x) + |x| + |y| + rho) / c;                                 */
/*    the same displacement moves y along the line, so rho carries P(y) too.  */
/*    A self-panel sample moves with x and with R(theta), which the ray's     */
/*    exit edge fixes at incidence sin beta: dR = (P(x) + |x| + R) / sin beta; */
/*    a point drawn on a primitive by its barycentrics (RIS candidates, 2D     */
/*    self-panel points) carries |y| only.                                     */
/*  - weight w: relative error eps(w) from the errors of rho, of cos theta_y   */
/*    (one unit absolute, so 1/c relative) and of cos theta_x; a running       */
/*    product W carries the sum of the eps of its factors.  Line weights of    */
/*    the double layer and the direct BIE are +-m (times 1/2): exact.          */
/*  - emission e = k s(y) moves by |k| |grad s(y)| (P(y) + |y| + |c_p|), the    */
/*    last two the rounding of the coordinates the data program subtracts      */
/*    (c_p the program's centre).                                              */
/* The bound of a path sums over its terms T = W e: |W| (error of e) +        */
/* (sum of eps in W) |W e|, with the magnitude forms of W and e of abs_sum.    */
/* A constant of a few units per rounding is left to the test's multiplier.   */
/* ------------------------------------------------------------------------- */
static double norm_d(const double* a, int dim) { return sqrt(dot(a, a, dim)); }

/* |grad u| and the spectral norm of the Hessian of the harmonic program at y. */
static void program_sens(const orc_mesh* m, const orc_bc* bc, const double* y, double* g1,
                         double* g2) {
  const double* p = bc->params;
  const int dim = m->dim;
  *g1 = 0.0;
  *g2 = 0.0;
  if (bc->program == ORC_PROG_LINEAR) {
    *g1 = sqrt(p[0] * p[0] + p[1] * p[1] + (dim == 3 ? p[2] * p[2] : 0.0));
  } else if (bc->program == ORC_PROG_QUAD) {
    *g1 = 2.0 * sqrt(y[0] * y[0] + y[1] * y[1]);
    *g2 = 2.0;
  } else if (bc->program == ORC_PROG_INVDIST) {
    double r[3] = {y[0] - p[0], y[1] - p[1], dim == 3 ? y[2] - p[2] : 0.0};
    const double rn = norm_d(r, dim);
    /* 3D u = 1/r: |grad u| = 1/r^2, Hessian eigenvalues 2/r^3, -1/r^3 (twice);
       2D u = ln r: 1/r and +-1/r^2 */
    *g1 = dim == 3 ? 1.0 / (rn * rn) : 1.0 / rn;
    *g2 = dim == 3 ? 2.0 / (rn * rn * rn) : 1.0 / (rn * rn);
  }
}

/* |grad s| of the boundary datum of primitive prim at y (s = u, n . grad u, or
   n . grad u + alpha u), and the size of the coordinates the program
   subtracts from y's (its centre). */
static double datum_sens(const orc_mesh* m, const orc_bc* bc, int64_t prim, const double* y) {
  if (bc->data_mode == 1) {
    /* the in-plane gradient of the linear interpolant: |f(y + h) - f(y)| <= |grad| |h|
       for a displacement h in the primitive's plane */
    double v0[3] = {0.0, 0.0, 0.0}, v1[3] = {0.0, 0.0, 0.0}, v2[3] = {0.0, 0.0, 0.0};
    prim_vertex(m, prim, 0, v0);
    prim_vertex(m, prim, 1, v1);
    const int32_t* ix = m->prims + prim * m->dim;
    const double f0 = bc->vertex_data[ix[0]], df1 = bc->vertex_data[ix[1]] - f0;
    double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], m->dim == 3 ? v1[2] - v0[2] : 0.0};
    if (m->dim == 2) return fabs(df1) / sqrt(dot(e1, e1, 2));
    prim_vertex(m, prim, 2, v2);
    const double df2 = bc->vertex_data[ix[2]] - f0;
    double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2]};
    const double g11 = dot(e1, e1, 3), g12 = dot(e1, e2, 3), g22 = dot(e2, e2, 3), det = g11 * g22 - g12 * g12;
    const double a = (df1 * g22 - df2 * g12) / det, b = (df2 * g11 - df1 * g12) / det;
    double gr[3];
    for (int k = 0; k < 3; ++k) gr[k] = a * e1[k] + b * e2[k];
    return sqrt(dot(gr, gr, 3));
  }
  double g1, g2;
  program_sens(m, bc, y, &g1, &g2);
  const int kind = prim_kind(m, prim);
  if (kind == ORC_DIRICHLET) return g1;
  if (kind == ORC_NEUMANN) return g2;
  return g2 + fabs(prim_alpha(m, prim)) * g1;
}
static double program_centre(const orc_mesh* m, const orc_bc* bc) {
  return bc->data_mode == 0 && bc->program == ORC_PROG_INVDIST ? norm_d(bc->params, m->dim) : 0.0;
}

/* Error of an emission k s(y) (units of u) from the position error P of y. */
static double emission_err(const orc_mesh* m, const orc_bc* bc, int64_t prim, const double* y, double k,
                           double P) {
  return fabs(k) * datum_sens(m, bc, prim, y) * (P + norm_d(y, m->dim) + program_centre(m, bc));
}

/* ------------------------------------------------------------------------- */
/* All hits of one line, brute force.                                         */
/* ------------------------------------------------------------------------- */
typedef struct {
  int m;                 /* number of hits */
  int64_t sel;           /* selected primitive (smallest key, then id), -1 if none */
  uint32_t sel_key;
  double sel_y[3];
  double sel_b[2];       /* barycentric coordinates of the selected hit */
  double src;            /* sum over hits of G(x,y) q(y) / p_all(y) (direct Neumann) */
  double src_abs;        /* sum over hits of |G(x,y) q(y) / p_all(y)| */
  double graze;          /* min over primitives of the decision margin (decision_margin) */
  double src_grad[3];    /* sum over hits of grad_x G(x,y) q(y) / p_all(y) */
  double src_grad_abs;   /* sum over hits of |grad_x G q / p_all|, all components */
  double src_err;        /* rounding-error bound of src (units of u) */
  double src_grad_err;   /* and of src_grad, all components */
} line_hits;

/* P: position error of x (units of u), for the error bounds of the source sums. */
static void all_hits(const orc_mesh* m, const double* normals, const orc_bc* bc, int want_src,
                     int want_sel, const double* x, const double* d, int64_t exclude,
                     uint64_t seed, uint32_t path, uint32_t point, uint32_t problem,
                     uint32_t line, double P, line_hits* h) {
  h->m = 0;
  h->sel = -1;
  h->sel_key = 0xffffffffu;
  h->src = 0.0;
  h->src_abs = 0.0;
  h->graze = INFINITY;
  h->src_grad[0] = h->src_grad[1] = h->src_grad[2] = 0.0;
  h->src_grad_abs = 0.0;
  h->src_err = 0.0;
  h->src_grad_err = 0.0;
  for (int64_t j = 0; j < m->n_prims; ++j) {
    if (j == exclude) continue;
    double t, y[3], margin, cosv, b[2];
    int hit = line_prim_b(m, j, x, d, &t, y, &margin, &cosv, b);
    double g = decision_margin(m, j, x, margin, cosv);
    if (g < h->graze) h->graze = g;
    if (!hit) continue;
    h->m += 1;
    if (want_sel) {
      uint32_t r[4];
      draw(seed, path, point, problem, line, 2u, (uint32_t)j, r);
      if (h->sel < 0 || r[0] < h->sel_key || (r[0] == h->sel_key && j < h->sel)) {
        h->sel = j;
        h->sel_key = r[0];
        memcpy(h->sel_y, y, sizeof(h->sel_y));
        h->sel_b[0] = b[0];
        h->sel_b[1] = b[1];
      }
    }
    if (want_src) {
      /* all-hits estimate of the integral of G q along this line: each hit is
         weighted by 1 / p_all with p_all the density without the 1/m factor */
      const double* ny = normals + 3 * j;
      double q = orc_boundary_datum(m, bc, j, y);
      double term = G(x, y, m->dim) * q / line_pdf(x, y, ny, 1, m->dim);
      h->src += term;
      h->src_abs += fabs(term);
      double gg[3];
      grad_G(x, y, m->dim, gg);
      const double pa = line_pdf(x, y, ny, 1, m->dim);
      for (int a = 0; a < 3; ++a) {
        h->src_grad[a] += gg[a] * q / pa;
        h->src_grad_abs += fabs(gg[a] * q / pa);
      }
      /* error bound of the term: G / p_all is rho / (2c) (2D: -rho ln rho / (2c)),
         with rho and y moved by (P + |x| + |y| + rho) / c and c rounded by one
         unit; the gradient term q sgn(t) d / (2c) the same way */
      const double rho = fabs(t), c = cosv;
      const double dy = (P + norm_d(x, m->dim) + norm_d(y, m->dim) + rho) / c;
      const double gp = fabs(G(x, y, m->dim) / pa);
      const double dgp = m->dim == 3 ? 1.0 / (2.0 * c) : (fabs(log(rho)) + 1.0) / (2.0 * c);
      const double sq = datum_sens(m, bc, j, y) * (dy + norm_d(y, m->dim) + program_centre(m, bc));
      h->src_err += fabs(q) * (dgp * dy + gp / c) + gp * sq;
      h->src_grad_err += (fabs(q) * (1.0 / c + 2.0) + sq) / (2.0 * c);
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Area-uniform boundary points for resampled importance sampling.            */
/* The primitive is the first id whose cumulative area fraction exceeds a     */
/* uniform u; the fractions are summed in binary64 in id order and rounded    */
/* once to binary32, and u is a binary32 value, so the choice of primitive is */
/* an exact decision.  The point is v0 + a e1 + b e2 with (a, b) uniform on   */
/* the unit square and reflected into the triangle when a + b > 1.            */
/* ------------------------------------------------------------------------- */
typedef struct {
  float* cdf;   /* n_prims */
  double total; /* |Gamma| */
} area_table;

static double prim_area(const orc_mesh* m, int64_t j) {
  double v0[3], v1[3], v2[3] = {0.0, 0.0, 0.0};
  prim_vertex(m, j, 0, v0);
  prim_vertex(m, j, 1, v1);
  if (m->dim == 2) {
    double e[2] = {v1[0] - v0[0], v1[1] - v0[1]};
    return sqrt(e[0] * e[0] + e[1] * e[1]);
  }
  prim_vertex(m, j, 2, v2);
  double e1[3], e2[3], n[3];
  for (int a = 0; a < 3; ++a) {
    e1[a] = v1[a] - v0[a];
    e2[a] = v2[a] - v0[a];
  }
  cross3(e1, e2, n);
  return 0.5 * sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
}

static area_table make_area_table(const orc_mesh* m) {
  area_table t;
  t.cdf = (float*)malloc(sizeof(float) * (size_t)m->n_prims);
  double tot = 0.0;
  for (int64_t j = 0; j < m->n_prims; ++j) tot += prim_area(m, j);
  double run = 0.0;
  for (int64_t j = 0; j < m->n_prims; ++j) {
    run += prim_area(m, j);
    t.cdf[j] = (float)(run / tot);
  }
  t.cdf[m->n_prims - 1] = 1.0f;
  t.total = tot;
  return t;
}

static int64_t area_pick(const area_table* t, int64_t n, float u) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    int64_t mid = (lo + hi) / 2;
    if (t->cdf[mid] > u) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

/* Single-layer emission at a vertex y on primitive prim, before the running
   weight: 2 phi s(y) on Neumann / Robin parts (Table 1) and k u_D(y) on
   Dirichlet parts (eq. mixed_second_kind_ish); half of it at the last vertex
   x_M (Sec. 4.1.2). */
static double sl_emission(const orc_mesh* m, const orc_bc* bc, int64_t prim, const double* y,
                          int last_vertex) {
  const double s = orc_boundary_datum(m, bc, prim, y);
  const double e = prim_kind(m, prim) == ORC_DIRICHLET ? bc->mixed_k * s : 2.0 * (double)bc->domain * s;
  return last_vertex ? 0.5 * e : e;
}

/* ------------------------------------------------------------------------- */
/* One path (point p, path k).                                                */
/* ------------------------------------------------------------------------- */
typedef struct {
  double value, abs_sum, graze;
  double err;      /* first-order rounding-error bound of the value (units of u) */
  double grad_err; /* and of each gradient component (gradient walks) */
  /* gradient walks: the derivative weight of step 0, w' = grad_x kernel / p
     (0 when line 0 found no hit), its magnitude sum and its relative
     rounding-error bound (units of u) */
  double wg0[3], wg0_abs, wg0_eps;
} path_result;

/* i0 = 0: the path from x0 (an evaluation point, or a boundary point with
   prim0 >= 0).  i0 > 0 (double layer only): the continuation of a path from
   the boundary point x0 on prim0 taken as its vertex i0, with the random
   numbers of lines i0, i0 + 1, ... of path (point, path): the emission at x0
   and every later term, as the path itself carries them after reaching its
   vertex i0 (the coupled walk of the gradient's boundary split). */
static path_result one_path(const orc_mesh* m, const double* normals, const area_table* at,
                            const orc_bc* bc, int form, const double* x0, int64_t prim0, int M,
                            uint64_t seed, uint32_t problem, uint32_t point, uint32_t path,
                            int32_t* vprim, int32_t* vm, double* vpos, double* grad,
                            double* grad_abs, int i0) {
  const int dim = m->dim;
  const double phi = (double)bc->domain;
  const int L = form == ORC_DIRECT ? M + 1 : M;
  path_result res = {0.0, 0.0, INFINITY, 0.0, 0.0, {0.0, 0.0, 0.0}, 0.0, 0.0};
  for (int i = 0; i < L; ++i) {
    if (vprim) vprim[i] = -1;
    if (vm) vm[i] = 0;
    if (vpos)
      for (int a = 0; a < dim; ++a) vpos[i * dim + a] = NAN;
  }

  /* density mode estimates the boundary unknown at boundary points: a point
     off the boundary has none (a caller error, as in the library: NaN) */
  if (bc->density && prim0 < 0) {
    res.value = NAN;
    res.abs_sum = NAN;
    return res;
  }
  /* Table 1, Dirichlet: on the boundary the solution is the given value (also
     on the Dirichlet parts of a mixed problem) */
  if (i0 == 0 && prim0 >= 0 && !bc->density &&
      (form == ORC_DOUBLE_LAYER || (form == ORC_SINGLE_LAYER && prim_kind(m, prim0) == ORC_DIRICHLET))) {
    res.value = orc_boundary_datum(m, bc, prim0, x0);
    res.abs_sum = fabs(res.value);
    res.err = emission_err(m, bc, prim0, x0, 1.0, 0.0);
    return res;
  }

  double x[3] = {x0[0], x0[1], dim == 3 ? x0[2] : 0.0};
  int64_t cur = prim0;
  /* abs_sum: the same sum with every factor and summand replaced by its
     magnitude (the scale of the rounding error of the sum) */
  double W = 1.0, acc = 0.0, abs_sum = 0.0, Wabs = 1.0;
  /* rounding-error bound (units of u): position error P of the current vertex,
     summed relative errors of the weights in W (eW) and in Wg (eWg) */
  double P = 0.0, eW = 0.0, eWg = 0.0, err = 0.0, gerr = 0.0;
  /* gradient in x0 (x0 off the boundary): the same path with the kernel of
     the first step differentiated in x0 (the gradient estimators of Sec. 4.1.3;
     the rest of the path estimates the same boundary unknown).  Wg is the
     derivative of W: a step multiplies it by its weight w, and step 0 adds
     W w' (w' = grad_x kernel / pdf); the step-0 source of the direct BIE adds
     its own derivative; every emission e adds Wg e. */
  const int want_grad = grad != NULL;
  double Wg[3] = {0.0, 0.0, 0.0}, gacc[3] = {0.0, 0.0, 0.0}, Wgabs = 0.0, gabs = 0.0;
  if (i0 > 0) {
    /* the double layer's emission at vertex i0 = x0 (halved when it is x_M) */
    const double k = i0 < M ? 2.0 : 1.0;
    const double e = k * phi * orc_boundary_datum(m, bc, prim0, x);
    acc = e;
    abs_sum = fabs(e);
    err = emission_err(m, bc, prim0, x, k, 0.0);
  }

  for (int i = i0; i < L; ++i) {
    const int on_gamma = cur >= 0;
    const double xn = norm_d(x, dim);
    uint32_t r0[4];
    draw(seed, path, point, problem, (uint32_t)i, 0u, 0u, r0);
    double d[3] = {0.0, 0.0, 0.0};
    if (dim == 3) {
      double z = 1.0 - 2.0 * uniform(r0[0]);
      double s = sqrt(fmax(0.0, 1.0 - z * z));
      double ph = 2.0 * ORC_PI * uniform(r0[1]);
      d[0] = s * cos(ph);
      d[1] = s * sin(ph);
      d[2] = z;
    } else {
      double th = 2.0 * ORC_PI * uniform(r0[0]);
      d[0] = cos(th);
      d[1] = sin(th);
    }

    /* step 0 from an evaluation point uses the representation formula; in
       density mode x0 is itself a boundary vertex of the recursion */
    const int first = i == 0 && !bc->density;
    /* a Dirichlet vertex of the single-layer recursion (mixed problems): the
       transformed first-kind row mu = mu - k int G mu + k u_D, sampled term by
       term: with probability p_k the next point comes from k G (weight
       -k G / (p p_k)), otherwise the walk stays at x (weight 1 / (1 - p_k)) */
    const int dvert = form == ORC_SINGLE_LAYER && on_gamma && !first && prim_kind(m, cur) == ORC_DIRICHLET;
    if (dvert && (r0[3] >> 8) >= bc->mixed_threshold) {
      const double w = 1.0 / (1.0 - bc->mixed_p);
      W *= w;
      Wabs *= w;
      for (int a = 0; a < 3; ++a) Wg[a] *= w;
      Wgabs *= w;
      if (vprim) vprim[i] = (int32_t)(-2 - cur);
      if (vm) vm[i] = 0;
      if (vpos)
        for (int a = 0; a < dim; ++a) vpos[i * dim + a] = x[a];
      const double e = sl_emission(m, bc, cur, x, i + 1 >= M);
      acc += W * e;
      abs_sum += Wabs * fabs(e);
      for (int a = 0; a < 3; ++a) gacc[a] += Wg[a] * e;
      gabs += Wgabs * fabs(e);
      const double ee = emission_err(m, bc, cur, x, bc->mixed_k * (i + 1 >= M ? 0.5 : 1.0), P);
      err += Wabs * ee + eW * Wabs * fabs(e);
      gerr += Wgabs * ee + eWg * Wgabs * fabs(e);
      continue;
    }
    const double gscale = dvert ? -bc->mixed_k / bc->mixed_p : 1.0; /* kernel k G / p_k or G */

    if (form == ORC_SINGLE_LAYER && bc->sampling == ORC_SAMPLE_RIS) {
      /* Resampled importance sampling (Results: Robin and mixed problems use
         area-uniform candidates and resample them by the integral kernel).
         The kernel k(y) is G(x, y) on the first step and
         -2 phi (dG/dn_x + alpha G) on the recursion; target |k|.  Candidate j
         draws Philox block 3 with w = j: word 0 picks the primitive, words 1, 2
         the point, word 3 the resampling uniform u_j; a weighted reservoir
         keeps candidate j when u_j S_j < |k_j| (S_j the running sum of |k|),
         so the kept one has probability |k_j| / S.  Weight
         k(y) / |k(y)| * S |Gamma| / C, the RIS estimate of int k(y) (.) dy. */
      const int C = bc->candidates;
      double S = 0.0, Smag = 0.0, kpick = 0.0, ypick[3] = {0.0, 0.0, 0.0}, dS = 0.0;
      int64_t jpick = -1;
      const double* nx = on_gamma ? normals + 3 * cur : NULL;
      const double ax = on_gamma ? prim_alpha(m, cur) : 0.0;
      for (int j = 0; j < C; ++j) {
        uint32_t rj[4];
        draw(seed, path, point, problem, (uint32_t)i, 3u, (uint32_t)j, rj);
        const int64_t pj = area_pick(at, m->n_prims, (float)uniform(rj[0]));
        double a = uniform(rj[1]), b = dim == 3 ? uniform(rj[2]) : 0.0;
        if (a + b > 1.0) {
          a = 1.0 - a;
          b = 1.0 - b;
        }
        double v0[3], v1[3], v2[3] = {0.0, 0.0, 0.0}, yc[3] = {0.0, 0.0, 0.0};
        prim_vertex(m, pj, 0, v0);
        prim_vertex(m, pj, 1, v1);
        if (dim == 3) prim_vertex(m, pj, 2, v2);
        for (int c = 0; c < dim; ++c) yc[c] = v0[c] + a * (v1[c] - v0[c]) + b * (v2[c] - v0[c]);
        double r[3] = {yc[0] - x[0], yc[1] - x[1], dim == 3 ? yc[2] - x[2] : 0.0};
        double k = 0.0;
        const double rr = dot(r, r, dim);
        if (rr > 0.0) {
          if (first || dvert) {
            k = gscale * G(x, yc, dim);
          } else {
            /* dG/dn_x = (y - x) . n_x / (4 pi rho^3) (2D: / (2 pi rho^2)).  The
               vertex x lies in the plane of its primitive, so
               (y - x) . n_x = (v0_y - v0_x) . n_x + a e1_y . n_x + b e2_y . n_x,
               which keeps its accuracy when y is close to x and nearly coplanar
               (forming y - x first would lose it to cancellation); it is zero on
               the own primitive */
            double rn = 0.0;
            if (pj != cur) {
              double w0[3];
              prim_vertex(m, cur, 0, w0);
              double dv[3] = {v0[0] - w0[0], v0[1] - w0[1], dim == 3 ? v0[2] - w0[2] : 0.0};
              double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], dim == 3 ? v1[2] - v0[2] : 0.0};
              double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], dim == 3 ? v2[2] - v0[2] : 0.0};
              rn = dot(dv, nx, dim) + a * dot(e1, nx, dim) + (dim == 3 ? b * dot(e2, nx, dim) : 0.0);
            }
            const double rho = sqrt(rr);
            const double dgdn = dim == 3 ? rn / (4.0 * ORC_PI * rr * rho) : rn / (2.0 * ORC_PI * rr);
            k = -2.0 * phi * (dgdn + ax * G(x, yc, dim));
          }
        }
        const double pk = fabs(k);
        S += pk;
        if (rr > 0.0) { /* the same kernel with its error scale (G_mag) */
          /* error of k: rho moves by P + |x| + |y| (x's error and the rounding of
             y - x); the numerator (y - x) . n_x of the recursion, formed from
             vertices and edges, by |x| + |y| */
          const double rho = sqrt(rr), drho = P + xn + norm_d(yc, dim);
          if (first || dvert) {
            Smag += fabs(gscale) * G_mag(x, yc, dim);
            dS += fabs(gscale) * (dim == 3 ? 1.0 / (4.0 * ORC_PI * rr) : 1.0 / (2.0 * ORC_PI * rho)) * drho;
          } else { /* |2 dG/dn_x| + 2 |alpha| G_mag, with 2 dG/dn_x = -k / phi - 2 alpha G */
            const double dn2 = fabs(k + 2.0 * phi * ax * G(x, yc, dim));
            Smag += dn2 + 2.0 * fabs(ax) * G_mag(x, yc, dim);
            const double sd = dim == 3 ? 4.0 * ORC_PI * rr * rho : 2.0 * ORC_PI * rr;
            dS += dn2 * (double)dim * drho / rho + 2.0 * (xn + norm_d(yc, dim)) / sd +
                  2.0 * fabs(ax) * (dim == 3 ? 1.0 / (4.0 * ORC_PI * rr) : 1.0 / (2.0 * ORC_PI * rho)) * drho;
          }
        }
        const double u = uniform(rj[3]);
        if (S > 0.0) {
          double margin = fabs(u * S - pk) / S; /* distance of the keep decision from its threshold */
          if (margin < res.graze) res.graze = margin;
        }
        if (u * S < pk) {
          jpick = pj;
          kpick = k;
          memcpy(ypick, yc, sizeof(ypick));
        }
      }
      if (vm) vm[i] = 0;
      if (jpick < 0 || !(S > 0.0)) break; /* no candidate carries kernel mass */
      if (vprim) vprim[i] = (int32_t)jpick;
      const double w = (kpick > 0.0 ? 1.0 : -1.0) * S * at->total / (double)C;
      const double eps = dS / Smag;
      if (want_grad && first) {
        /* RIS estimate of int grad_x G mu: grad_x G(y) / |G(y)| S |Gamma| / C */
        double gg[3];
        grad_G(x, ypick, dim, gg);
        const double f = S * at->total / (double)C / fabs(kpick);
        Wgabs = 0.0;
        for (int a = 0; a < 3; ++a) {
          Wg[a] = Wg[a] * w + W * gg[a] * f;
          Wgabs += fabs(W * gg[a] * f);
        }
        /* grad G / |G| = r / rho^2 (2D: r / (rho^2 |ln rho|)): the picked
           point's distance carries P + |x| + |y| */
        double r[3] = {ypick[0] - x[0], ypick[1] - x[1], dim == 3 ? ypick[2] - x[2] : 0.0};
        const double rho = norm_d(r, dim);
        eWg = eps + 3.0 * (P + xn + norm_d(ypick, dim)) / rho +
              (dim == 2 ? (P + xn + norm_d(ypick, dim)) / (rho * fmax(fabs(log(rho)), 1e-300)) : 0.0);
      } else {
        for (int a = 0; a < 3; ++a) Wg[a] *= w;
        Wgabs *= Smag * at->total / (double)C;
        eWg += eps;
      }
      W *= w;
      Wabs *= Smag * at->total / (double)C;
      eW += eps;
      memcpy(x, ypick, sizeof(x));
      cur = jpick;
      P = norm_d(x, dim); /* a point drawn by its barycentrics */
      if (vpos)
        for (int a = 0; a < dim; ++a) vpos[i * dim + a] = x[a];
      const double e = sl_emission(m, bc, cur, x, i + 1 >= M);
      acc += W * e;
      abs_sum += Wabs * fabs(e);
      for (int a = 0; a < 3; ++a) gacc[a] += Wg[a] * e;
      gabs += Wgabs * fabs(e);
      const double ke = (prim_kind(m, cur) == ORC_DIRICHLET ? bc->mixed_k : 2.0) * (i + 1 >= M ? 0.5 : 1.0);
      const double ee = emission_err(m, bc, cur, x, ke, P);
      err += Wabs * ee + eW * Wabs * fabs(e);
      gerr += Wgabs * ee + eWg * Wgabs * fabs(e);
      continue;
    }

    /* single layer: where G acts on the own primitive (the first step from a
       boundary point, and the alpha G part at Robin vertices) mix the line
       sample with an in-plane self-panel sample */
    int mixture = form == ORC_SINGLE_LAYER && on_gamma &&
                  (first || dvert || prim_kind(m, cur) == ORC_ROBIN);
    int use_self = mixture && (r0[2] >> 8) < bc->self_threshold;

    double y[3] = {0.0, 0.0, 0.0};
    int64_t next = -1;
    double w, wabs, eps = 0.0, Pn = 0.0;
    if (use_self) {
      uint32_t r1[4];
      draw(seed, path, point, problem, (uint32_t)i, 1u, 0u, r1);
      double R, sinb;
      double gp = self_panel_geo(m, cur, x, uniform(r1[0]), uniform(r1[1]), y, &R, &sinb);
      if (dim == 3) {
        /* G / p = R(theta) / 2: R moves by (P + |x| + R) / sin beta, and y,
           a fraction of R from x, with it */
        const double dR = (P + xn + R) / sinb;
        eps = dR / R;
        Pn = P + dR + xn + R;
      } else {
        /* G / p = -L ln rho / (2 pi) with y on the segment by its parameter:
           rho moves by P + |x| + |y| */
        const double rho = sqrt((y[0] - x[0]) * (y[0] - x[0]) + (y[1] - x[1]) * (y[1] - x[1]));
        eps = (P + xn + norm_d(y, dim)) / (rho * fmax(fabs(log(rho)), 1.0));
        Pn = norm_d(y, dim);
      }
      if (first || dvert)
        w = gscale * gp / bc->self_p; /* u = int G mu; Dirichlet vertex: -k G / p_k */
      else
        w = -2.0 * phi * prim_alpha(m, cur) * gp / bc->self_p; /* -2 phi alpha G */
      wabs = fabs(w);
      next = cur;
      if (vprim) vprim[i] = (int32_t)(-2 - cur);
      if (vm) vm[i] = 0;
    } else {
      line_hits h;
      const int src_line = form == ORC_DIRECT;
      const int last = i == L - 1;
      all_hits(m, normals, bc, src_line, !(src_line && last), x, d, cur, seed, path, point,
               problem, (uint32_t)i, P, &h);
      if (h.graze < res.graze) res.graze = h.graze;
      if (vm) vm[i] = h.m;
      if (vprim) vprim[i] = (int32_t)h.sel;
      if (form == ORC_DIRECT) {
        /* source integral of the direct BIE: phi int G q off the boundary,
           2 phi int G q on it (Table 1, Neumann rows) */
        double S, Sabs, Serr = h.src_err;
        if (on_gamma) {
          uint32_t r1[4];
          double ys[3], R, sinb;
          draw(seed, path, point, problem, (uint32_t)i, 1u, 0u, r1);
          double gp = self_panel_geo(m, cur, x, uniform(r1[0]), uniform(r1[1]), ys, &R, &sinb);
          double qs = orc_boundary_datum(m, bc, cur, ys);
          double own = gp * qs;
          S = 2.0 * phi * (h.src + own);
          Sabs = 2.0 * (h.src_abs + fabs(own));
          /* the own-panel term as in the self-panel step above */
          double dgp, dys;
          if (dim == 3) {
            const double dR = (P + xn + R) / sinb;
            dgp = 0.5 * dR;
            dys = P + dR + xn + R;
          } else {
            const double rho = sqrt((ys[0] - x[0]) * (ys[0] - x[0]) + (ys[1] - x[1]) * (ys[1] - x[1]));
            dgp = R * (P + xn + norm_d(ys, dim)) / (2.0 * ORC_PI * rho);
            dys = norm_d(ys, dim);
          }
          Serr = 2.0 * (h.src_err + fabs(qs) * dgp + emission_err(m, bc, cur, ys, gp, dys));
        } else {
          S = phi * h.src;
          Sabs = h.src_abs;
        }
        const double cl = last ? 0.5 : 1.0;
        double term = W * S * cl;
        acc += term;
        abs_sum += Wabs * Sabs * cl;
        err += (Wabs * Serr + eW * Wabs * Sabs) * cl;
        if (want_grad) {
          /* the step-0 source phi int G q is a function of x0 (off the boundary) */
          for (int a = 0; a < 3; ++a)
            gacc[a] += (Wg[a] * S + (i == 0 ? W * phi * h.src_grad[a] : 0.0)) * cl;
          gabs += (Wgabs * Sabs + (i == 0 ? W * h.src_grad_abs : 0.0)) * cl;
          gerr += (Wgabs * Serr + eWg * Wgabs * Sabs + (i == 0 ? Wabs * h.src_grad_err : 0.0)) * cl;
        }
        if (last) break;
      }
      if (h.m == 0) break;
      memcpy(y, h.sel_y, sizeof(y));
      next = h.sel;
      const double* ny = normals + 3 * next;
      double p = line_pdf(x, y, ny, h.m, dim);
      /* the picked hit: incidence c, distance rho, and its position error */
      double ry[3] = {y[0] - x[0], y[1] - x[1], dim == 3 ? y[2] - x[2] : 0.0};
      const double rho = norm_d(ry, dim), cy = fabs(dot(ry, ny, dim)) / rho;
      Pn = (P + xn + norm_d(y, dim) + rho) / cy;
      double kern, kabs;
      if (form == ORC_DOUBLE_LAYER) {
        kern = (first && !on_gamma) ? -dG_dny(x, y, ny, dim)           /* u = -int dG/dny nu */
                                     : 2.0 * phi * dG_dny(x, y, ny, dim); /* nu = 2 phi int dG/dny nu + ... */
        kabs = fabs(kern);
      } else if (form == ORC_DIRECT) {
        kern = on_gamma ? -2.0 * phi * dG_dny(x, y, ny, dim) /* boundary row */
                        : -phi * dG_dny(x, y, ny, dim);      /* interior / exterior row */
        kabs = fabs(kern);
      } else {
        if (first || dvert) {
          kern = gscale * G(x, y, dim); /* u = int G mu; Dirichlet vertex: -k G / p_k */
          kabs = fabs(gscale) * G_mag(x, y, dim);
          /* G / p = m rho / (2c) (2D: -m rho ln rho / (2c)) */
          eps = (dim == 3 ? Pn / rho : Pn * (fabs(log(rho)) + 1.0) / (rho * fmax(fabs(log(rho)), 1.0))) +
                1.0 / cy;
        } else {
          /* dG/dn_x with its numerator (y - x) . n_x in vertex-and-edge form:
             x lies in the plane of its primitive, so (y - x) . n_x =
             (v0_y - v0_x) . n_x + b1 e1_y . n_x + b2 e2_y . n_x, accurate also
             for a hit close to x on a nearly coplanar neighbour (where forming
             y - x first loses digits to cancellation) */
          const double* nx = normals + 3 * cur;
          double w0[3] = {0.0, 0.0, 0.0}, u0[3] = {0.0, 0.0, 0.0}, u1[3] = {0.0, 0.0, 0.0},
                 u2[3] = {0.0, 0.0, 0.0};
          prim_vertex(m, cur, 0, w0);
          prim_vertex(m, next, 0, u0);
          prim_vertex(m, next, 1, u1);
          if (dim == 3) prim_vertex(m, next, 2, u2);
          double dv[3], e1[3], e2[3];
          for (int a = 0; a < 3; ++a) {
            dv[a] = u0[a] - w0[a];
            e1[a] = u1[a] - u0[a];
            e2[a] = dim == 3 ? u2[a] - u0[a] : 0.0;
          }
          const double rn = dot(dv, nx, dim) + h.sel_b[0] * dot(e1, nx, dim) +
                            (dim == 3 ? h.sel_b[1] * dot(e2, nx, dim) : 0.0);
          double r[3] = {y[0] - x[0], y[1] - x[1], dim == 3 ? y[2] - x[2] : 0.0};
          const double rr = dot(r, r, dim), rho2 = sqrt(rr);
          const double dgdn = dim == 3 ? rn / (4.0 * ORC_PI * rr * rho2) : rn / (2.0 * ORC_PI * rr);
          kern = -2.0 * phi * (dgdn + prim_alpha(m, cur) * G(x, y, dim));
          kabs = 2.0 * (fabs(dgdn) + fabs(prim_alpha(m, cur)) * G_mag(x, y, dim));
          /* w = -phi m (c_x + alpha rho) / c (2D: c_x - alpha rho ln rho): c
             rounded by one unit, rho moved by Pn, and c_x by one unit plus
             |x| / rho: a rounded vertex lies about |x| units off its
             primitive's plane, which moves (y - x) . n_x by as much */
          const double al = fabs(prim_alpha(m, cur)), cx = fabs(rn) / rho2;
          const double lr = fabs(log(rho2));
          eps = dim == 3 ? (1.0 + xn / rho2 + al * Pn) / (cx + al * rho2) + 1.0 / cy
                         : (1.0 + xn / rho2 + al * Pn * (lr + 1.0)) / (cx + al * rho2 * fmax(lr, 1.0)) +
                               1.0 / cy;
        }
      }
      w = kern / p;
      wabs = kabs / p;
      if (mixture) {
        w /= (1.0 - bc->self_p);
        wabs /= (1.0 - bc->self_p);
      }
      if (want_grad && i == 0) {
        /* step 0 from x0 off the boundary: w' = grad_x kernel / p */
        double kg[3];
        if (form == ORC_SINGLE_LAYER) {
          grad_G(x, y, dim, kg);
          for (int a = 0; a < 3; ++a) kg[a] *= gscale;
        } else {
          grad_dG_dny(x, y, ny, dim, kg);
          const double f = form == ORC_DOUBLE_LAYER ? -1.0 : -phi; /* -dG/dn_y, -phi dG/dn_y */
          for (int a = 0; a < 3; ++a) kg[a] *= f;
        }
        double wg[3], wgabs = 0.0;
        for (int a = 0; a < 3; ++a) {
          wg[a] = kg[a] / p;
          wgabs += fabs(wg[a]);
        }
        for (int a = 0; a < 3; ++a) Wg[a] = Wg[a] * w + W * wg[a];
        Wgabs = Wgabs * wabs + Wabs * wgabs;
        /* w': single layer m sgn(t) d / (2c); double layer and direct
           -m (n - D c rhat) / (2 rho c) (times phi): c rounded by one unit, rho
           moved by Pn, the D c rhat part by D units */
        eWg = form == ORC_SINGLE_LAYER ? 1.0 / cy + 2.0 : Pn / rho + (1.0 + dim) / cy + 2.0;
        for (int a = 0; a < 3; ++a) res.wg0[a] = wg[a];
        res.wg0_abs = wgabs;
        res.wg0_eps = eWg;
      } else {
        for (int a = 0; a < 3; ++a) Wg[a] *= w;
        Wgabs *= wabs;
        eWg += eps;
      }
    }
    if (use_self) {
      for (int a = 0; a < 3; ++a) Wg[a] *= w;
      Wgabs *= wabs;
      eWg += eps;
    }

    W *= w;
    Wabs *= wabs;
    eW += eps;
    P = Pn;
    memcpy(x, y, sizeof(x));
    cur = next;
    if (vpos)
      for (int a = 0; a < dim; ++a) vpos[i * dim + a] = x[a];

    if (form != ORC_DIRECT) {
      /* emission 2 phi s at x_{i+1} (single layer on Dirichlet parts: k u_D);
         the last vertex gets half of it (Sec. 4.1.2, modified Neumann series) */
      double e, k;
      if (form == ORC_SINGLE_LAYER) {
        e = sl_emission(m, bc, cur, x, i + 1 >= M);
        k = (prim_kind(m, cur) == ORC_DIRICHLET ? bc->mixed_k : 2.0) * (i + 1 >= M ? 0.5 : 1.0);
      } else {
        double s = orc_boundary_datum(m, bc, cur, x);
        k = (i + 1 < M ? 2.0 : 1.0);
        e = k * phi * s;
      }
      acc += W * e;
      abs_sum += Wabs * fabs(e);
      for (int a = 0; a < 3; ++a) gacc[a] += Wg[a] * e;
      gabs += Wgabs * fabs(e);
      const double ee = emission_err(m, bc, cur, x, k, P);
      err += Wabs * ee + eW * Wabs * fabs(e);
      gerr += Wgabs * ee + eWg * Wgabs * fabs(e);
    }
  }
  res.value = acc;
  res.abs_sum = abs_sum;
  res.err = err;
  res.grad_err = gerr;
  if (want_grad) {
    for (int a = 0; a < dim; ++a) grad[a] = gacc[a];
    if (grad_abs) *grad_abs = gabs;
  }
  return res;
}

static double* make_normals(const orc_mesh* m) {
  double* n = (double*)malloc(sizeof(double) * 3 * (size_t)(m->n_prims > 0 ? m->n_prims : 1));
  for (int64_t j = 0; j < m->n_prims; ++j) orc_prim_normal(m, j, n + 3 * j);
  return n;
}

static int check_args(const orc_mesh* m, const orc_bc* bc, int walk_len) {
  if (!m || !bc) return 1;
  if (bc->data_mode != 0 && (bc->data_mode != 1 || !bc->vertex_data)) return 1;
  if (m->dim != 2 && m->dim != 3) return 1;
  if (m->n_prims <= 0 || !m->verts || !m->prims) return 1;
  if (walk_len < 1) return 1;
  if (bc->domain != 1 && bc->domain != -1) return 1;
  if (orc_resolve_formulation(m, bc->formulation) < 0) return 1;
  if (bc->density && orc_resolve_formulation(m, bc->formulation) == ORC_DIRECT) return 1;
  if (bc->sampling != ORC_SAMPLE_LINE && bc->sampling != ORC_SAMPLE_RIS) return 1;
  if (!(bc->mixed_p > 0.0 && bc->mixed_p < 1.0) || bc->mixed_threshold == 0 || !isfinite(bc->mixed_k) ||
      bc->mixed_k == 0.0)
    return 1;
  if (bc->sampling == ORC_SAMPLE_RIS &&
      (orc_resolve_formulation(m, bc->formulation) != ORC_SINGLE_LAYER || bc->candidates < 1 ||
       bc->candidates > 64))
    return 1;
  return 0;
}

int orc_trace(const orc_mesh* m, const double* points, const int32_t* point_prim,
              int64_t n_points, const orc_bc* bc, int walk_len, uint64_t seed, uint32_t problem,
              int64_t n_items, const int64_t* item_point, const int64_t* item_path,
              orc_trace_out* out, int n_threads) {
  if (check_args(m, bc, walk_len)) return 1;
  const int form = orc_resolve_formulation(m, bc->formulation);
  const int L = form == ORC_DIRECT ? walk_len + 1 : walk_len;
  double* normals = make_normals(m);
  area_table at = make_area_table(m);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
  for (int64_t it = 0; it < n_items; ++it) {
    int64_t p = item_point[it];
    if (p < 0 || p >= n_points) continue;
    double x0[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < m->dim; ++a) x0[a] = points[p * m->dim + a];
    int64_t prim0 = point_prim ? point_prim[p] : -1;
    path_result r = one_path(m, normals, &at, bc, form, x0, prim0, walk_len, seed, problem,
                             (uint32_t)p, (uint32_t)item_path[it],
                             out->vtx_prim ? out->vtx_prim + it * L : NULL,
                             out->vtx_m ? out->vtx_m + it * L : NULL,
                             out->vtx_pos ? out->vtx_pos + it * L * m->dim : NULL, NULL, NULL, 0);
    if (out->value) out->value[it] = r.value;
    if (out->abs_sum) out->abs_sum[it] = r.abs_sum;
    if (out->graze) out->graze[it] = r.graze;
    if (out->err) out->err[it] = r.err;
  }
  free(normals);
  free(at.cdf);
  return 0;
}

int orc_solve(const orc_mesh* m, const double* points, const int32_t* point_prim,
              int64_t n_points, const orc_bc* bc, int samples, int walk_len, uint64_t seed,
              uint32_t problem, double* mean_out, double* var_out, int n_threads) {
  if (check_args(m, bc, walk_len) || samples < 1) return 1;
  const int form = orc_resolve_formulation(m, bc->formulation);
  double* normals = make_normals(m);
  area_table at = make_area_table(m);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t p = 0; p < n_points; ++p) {
    double x0[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < m->dim; ++a) x0[a] = points[p * m->dim + a];
    int64_t prim0 = point_prim ? point_prim[p] : -1;
    /* statistics over the finite path values only: a non-finite path
       (degenerate geometry, data singular at a boundary point) is left out */
    double* v = (double*)malloc(sizeof(double) * (size_t)samples);
    double sum = 0.0;
    int n = 0;
    for (int k = 0; k < samples; ++k) {
      const double val = one_path(m, normals, &at, bc, form, x0, prim0, walk_len, seed, problem,
                                  (uint32_t)p, (uint32_t)k, NULL, NULL, NULL, NULL, NULL, 0)
                             .value;
      if (!isfinite(val)) continue;
      v[n++] = val;
      sum += val;
    }
    double mean = n > 0 ? sum / n : NAN;
    double ss = 0.0;
    for (int k = 0; k < n; ++k) ss += (v[k] - mean) * (v[k] - mean);
    mean_out[p] = mean;
    if (var_out) var_out[p] = n > 1 ? ss / (n - 1) : 0.0;
    free(v);
  }
  free(normals);
  free(at.cdf);
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Forward (adjoint) estimator of the single layer on Neumann boundaries     */
/* (Sec. 4.4.3 "Forward estimator"; Table 1, single-layer Neumann rows).        */
/*                                                                           */
/* The single layer writes u(x) = int G(x, y) mu(y) dA with mu = f + K mu,    */
/* f = 2 phi q and K(x, y) = -2 phi dG/dn_x(x, y).  Truncated with the halved  */
/* last term (Sec. 4.1.2) the estimate is                                    */
/*     u(x) ~ sum_{j < M} c_j < G(x, .), K^j f >,   c = (1, ..., 1, 1/2).     */
/* The backward walk samples these integrals from x outwards.  The forward    */
/* walk samples the same sum from the data towards x: y_1 is drawn on the      */
/* boundary with density p_0 and carries W_1 = f(y_1) / p_0(y_1); y_{k+1} is  */
/* the picked hit of a uniformly random line through y_k and carries           */
/* W_{k+1} = W_k K(y_{k+1}, y_k) / p(y_{k+1} | y_k), the kernel read with its   */
/* arguments swapped (its normal derivative now acts at the sampled point,     */
/* whose |cos| the line density contains).  Then E[W_k h(y_k)] =              */
/* < K^{k-1} f, h > for every h, and vertex k of a path is a source of         */
/* strength c_{k-1} W_k at y_k that every evaluation point connects to:        */
/*     u(x) ~ (1 / n_paths) sum_paths sum_k c_{k-1} W_k G(x, y_k).             */
/*                                                                           */
/* Start density: primitive T with probability P_T from a binary32 cumulative  */
/* table of caller weights w_T in id order (binary64 running sum, rounded      */
/* once; P_T = cdf_T - cdf_{T-1} evaluated in binary64), then uniform in T, so */
/* p_0 = P_T / A_T.  Weights proportional to |q| A_T place the starts where    */
/* the data are large (the boundary sampling by the magnitude of the boundary  */
/* value in the paper's Neumann example); NULL means w_T = A_T.                */
/*                                                                           */
/* Random numbers of path j (point word 0xfffffffe):                          */
/*   start  (j, 0xfffffffe, (problem << 24) | 0xffff03, 0): word 0 the         */
/*          primitive (binary32 uniform against the table), words 1, 2 the    */
/*          point (reflected into the triangle when a + b > 1);                */
/*   line i (from y_{i+1}): blocks 0 and 2 exactly as in the backward walk.    */
/* ------------------------------------------------------------------------- */
#define ORC_FWD_POINT 0xfffffffeu

static int all_neumann(const orc_mesh* m) {
  if (!m->kind) return 0;
  for (int64_t j = 0; j < m->n_prims; ++j)
    if (m->kind[j] != ORC_NEUMANN) return 0;
  return 1;
}

int orc_forward_paths(const orc_mesh* m, const orc_bc* bc, const double* start_weight,
                      int64_t n_paths, int walk_len, uint64_t seed, uint32_t problem,
                      orc_forward_out* out, int n_threads) {
  if (!m || !bc || !out || m->dim < 2 || m->dim > 3 || m->n_prims <= 0 || walk_len < 1 ||
      walk_len >= 65535 || n_paths < 0)
    return 1;
  if (bc->domain != 1 && bc->domain != -1) return 1;
  if (!all_neumann(m)) return 1;
  const int dim = m->dim, M = walk_len;
  const double phi = (double)bc->domain;
  /* start table */
  float* cdf = (float*)malloc(sizeof(float) * (size_t)m->n_prims);
  double tot = 0.0;
  for (int64_t j = 0; j < m->n_prims; ++j) {
    const double w = start_weight ? start_weight[j] : prim_area(m, j);
    if (!(w >= 0.0) || !isfinite(w)) {
      free(cdf);
      return 1;
    }
    tot += w;
  }
  if (!(tot > 0.0)) {
    free(cdf);
    return 1;
  }
  double run = 0.0;
  for (int64_t j = 0; j < m->n_prims; ++j) {
    run += start_weight ? start_weight[j] : prim_area(m, j);
    cdf[j] = (float)(run / tot);
  }
  cdf[m->n_prims - 1] = 1.0f;
  area_table st = {cdf, tot};
  double* normals = make_normals(m);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t p = 0; p < n_paths; ++p) {
    const uint32_t path = (uint32_t)p;
    double* pos = out->vtx_pos ? out->vtx_pos + p * M * dim : NULL;
    for (int k = 0; k < M; ++k) {
      if (out->vtx_w) out->vtx_w[p * M + k] = 0.0;
      if (out->vtx_prim) out->vtx_prim[p * M + k] = -1;
      if (out->vtx_m) out->vtx_m[p * M + k] = 0;
      if (out->vtx_perr) out->vtx_perr[p * M + k] = 0.0;
      if (out->vtx_werr) out->vtx_werr[p * M + k] = 0.0;
      if (pos)
        for (int a = 0; a < dim; ++a) pos[k * dim + a] = 0.0;
    }
    /* rounding-error bounds (units of u): position of the current vertex and
       the strength's first factor 2 phi q(y_1) A_T / P_T (later steps multiply
       by the exact factors +-m) */
    double graze = INFINITY, P = 0.0, werr = 0.0;
    /* y_1 ~ p_0 */
    uint32_t r[4];
    draw(seed, path, ORC_FWD_POINT, problem, 0xffffu, 3u, 0u, r);
    const int64_t T = area_pick(&st, m->n_prims, (float)uniform(r[0]));
    double a = uniform(r[1]), b = dim == 3 ? uniform(r[2]) : 0.0;
    if (a + b > 1.0) {
      a = 1.0 - a;
      b = 1.0 - b;
    }
    double v0[3], v1[3], v2[3] = {0.0, 0.0, 0.0}, x[3] = {0.0, 0.0, 0.0};
    prim_vertex(m, T, 0, v0);
    prim_vertex(m, T, 1, v1);
    if (dim == 3) prim_vertex(m, T, 2, v2);
    for (int c = 0; c < dim; ++c) x[c] = v0[c] + a * (v1[c] - v0[c]) + b * (v2[c] - v0[c]);
    const double P_T = (double)cdf[T] - (T > 0 ? (double)cdf[T - 1] : 0.0);
    const double p0 = P_T / prim_area(m, T);
    double W = 2.0 * phi * orc_boundary_datum(m, bc, T, x) / p0;
    P = norm_d(x, dim); /* drawn by its barycentrics */
    werr = 4.0 * fabs(W) + emission_err(m, bc, T, x, 2.0 / p0, P);
    int64_t cur = T;
    for (int k = 0; k < M; ++k) {
      if (k > 0) {
        /* line k - 1 from y_k */
        uint32_t r0[4];
        draw(seed, path, ORC_FWD_POINT, problem, (uint32_t)(k - 1), 0u, 0u, r0);
        double d[3] = {0.0, 0.0, 0.0};
        if (dim == 3) {
          double z = 1.0 - 2.0 * uniform(r0[0]);
          double s = sqrt(fmax(0.0, 1.0 - z * z));
          double ph = 2.0 * ORC_PI * uniform(r0[1]);
          d[0] = s * cos(ph);
          d[1] = s * sin(ph);
          d[2] = z;
        } else {
          double th = 2.0 * ORC_PI * uniform(r0[0]);
          d[0] = cos(th);
          d[1] = sin(th);
        }
        line_hits h;
        all_hits(m, normals, bc, 0, 1, x, d, cur, seed, path, ORC_FWD_POINT, problem,
                 (uint32_t)(k - 1), P, &h);
        if (h.graze < graze) graze = h.graze;
        if (out->vtx_m) out->vtx_m[p * M + k] = h.m;
        if (h.m == 0) break;
        const double* ny = normals + 3 * h.sel;
        /* K(y_{k+1}, y_k) / p(y_{k+1} | y_k) */
        const double kern = -2.0 * phi * dG_dnx(h.sel_y, x, ny, dim);
        const double pdf = line_pdf(x, h.sel_y, ny, h.m, dim);
        {
          double rr[3] = {h.sel_y[0] - x[0], h.sel_y[1] - x[1], dim == 3 ? h.sel_y[2] - x[2] : 0.0};
          const double rho = sqrt(dot(rr, rr, dim)), c = fabs(dot(rr, ny, dim)) / rho;
          P = (P + norm_d(x, dim) + norm_d(h.sel_y, dim) + rho) / c;
        }
        W *= kern / pdf;
        werr *= (double)h.m;
        memcpy(x, h.sel_y, sizeof(x));
        cur = h.sel;
      }
      if (out->vtx_w) out->vtx_w[p * M + k] = (k + 1 < M ? 1.0 : 0.5) * W;
      if (out->vtx_perr) out->vtx_perr[p * M + k] = P;
      if (out->vtx_werr) out->vtx_werr[p * M + k] = (k + 1 < M ? 1.0 : 0.5) * werr;
      if (out->vtx_prim) out->vtx_prim[p * M + k] = (int32_t)cur;
      if (pos)
        for (int c = 0; c < dim; ++c) pos[k * dim + c] = x[c];
    }
    if (out->graze) out->graze[p] = graze;
  }
  free(normals);
  free(cdf);
  return 0;
}

/* Connection of every evaluation point to every vertex of the forward paths:
 * per point, the per-path values c_j(x) = sum_k w_jk G(x, y_jk) (a vertex at
 * distance zero contributes nothing), their mean over the n_paths paths and
 * unbiased variance, and the sum of |w G| / n_paths (the rounding scale). */
int orc_forward_gather(int dim, int64_t n_paths, int walk_len, const double* vtx_pos,
                       const double* vtx_w, const double* points, int64_t n_points,
                       double* mean_out, double* var_out, double* abs_out, int n_threads) {
  if ((dim != 2 && dim != 3) || n_paths < 1 || walk_len < 1 || n_points < 0) return 1;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
  for (int64_t p = 0; p < n_points; ++p) {
    const double* x = points + p * dim;
    double* cj = (double*)malloc(sizeof(double) * (size_t)n_paths);
    double sum = 0.0, sabs = 0.0;
    for (int64_t j = 0; j < n_paths; ++j) {
      double c = 0.0;
      for (int k = 0; k < walk_len; ++k) {
        const double* y = vtx_pos + (j * walk_len + k) * dim;
        const double w = vtx_w[j * walk_len + k];
        double r[3] = {y[0] - x[0], y[1] - x[1], dim == 3 ? y[2] - x[2] : 0.0};
        if (w == 0.0 || dot(r, r, dim) == 0.0) continue;
        const double t = w * G(x, y, dim);
        c += t;
        sabs += fabs(w) * G_mag(x, y, dim);
      }
      cj[j] = c;
      sum += c;
    }
    const double mean = sum / (double)n_paths;
    double ss = 0.0;
    for (int64_t j = 0; j < n_paths; ++j) ss += (cj[j] - mean) * (cj[j] - mean);
    free(cj);
    mean_out[p] = mean;
    if (var_out) var_out[p] = n_paths > 1 ? ss / (double)(n_paths - 1) : 0.0;
    if (abs_out) abs_out[p] = sabs / (double)n_paths;
  }
  return 0;
}

/* Per-path values and gradients in x0 for (point, path) items; every point
 * off the boundary (the gradient equations hold inside the domain only). */
/* The boundary split of the double layer's gradient (Sec. 4.1.3: near the
 * boundary the first step's kernel grad_x dG/dn_y is hypersingular; split at
 * the boundary point nearest to x0).  The kernel integrates to zero over the
 * closed boundary for x0 off it (the double-layer potential of a constant
 * density is constant on each side), so w' times any quantity independent of
 * line 0 has mean zero: each path's gradient w' nu^(y_1) becomes
 * w' (nu^(y_1) - nu^(x*)), nu^(x*) the path's coupled walk from the anchor
 * x* (on primitive prim*) with the random numbers of its own lines 1, 2, ...
 * Near x* the two walks start close together and take the same directions,
 * so the difference, not the hypersingular kernel, sets the noise. */
static void anchor_split(const orc_mesh* m, const double* normals, const area_table* at, const orc_bc* bc,
                         int form, const double* anchors, const int32_t* anchor_prim, int64_t p, int walk_len,
                         uint64_t seed, uint32_t problem, uint32_t path, path_result* r, double* grad,
                         double* gabs) {
  /* no anchor for this point, or line 0 found no hit: nothing to subtract */
  if (anchor_prim[p] < 0 || r->wg0_abs == 0.0) return;
  double xa[3] = {0.0, 0.0, 0.0};
  for (int a = 0; a < m->dim; ++a) xa[a] = anchors[p * m->dim + a];
  const path_result c = one_path(m, normals, at, bc, form, xa, anchor_prim[p], walk_len, seed, problem,
                                 (uint32_t)p, path, NULL, NULL, NULL, NULL, NULL, 1);
  for (int a = 0; a < m->dim; ++a) grad[a] -= r->wg0[a] * c.value;
  *gabs += r->wg0_abs * c.abs_sum;
  r->grad_err += r->wg0_abs * c.err + r->wg0_eps * r->wg0_abs * c.abs_sum;
  if (c.graze < r->graze) r->graze = c.graze;
}

static int check_anchors(const orc_mesh* m, const orc_bc* bc, const double* anchors,
                         const int32_t* anchor_prim, int64_t n_points) {
  if (!anchors && !anchor_prim) return 0;
  if (!anchors || !anchor_prim) return 1;
  if (orc_resolve_formulation(m, bc->formulation) != ORC_DOUBLE_LAYER) return 1;
  for (int64_t p = 0; p < n_points; ++p)
    if (anchor_prim[p] < -1 || anchor_prim[p] >= m->n_prims) return 1;
  return 0;
}

int orc_trace_grad(const orc_mesh* m, const double* points, int64_t n_points, const orc_bc* bc,
                   int walk_len, uint64_t seed, uint32_t problem, int64_t n_items,
                   const int64_t* item_point, const int64_t* item_path, const double* anchors,
                   const int32_t* anchor_prim, double* value, double* grad, double* abs_sum, double* grad_abs,
                   double* graze, double* err, double* grad_err, int n_threads) {
  if (check_args(m, bc, walk_len) || bc->density || !grad) return 1;
  if (check_anchors(m, bc, anchors, anchor_prim, n_points)) return 1;
  const int form = orc_resolve_formulation(m, bc->formulation);
  double* normals = make_normals(m);
  area_table at = make_area_table(m);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
  for (int64_t it = 0; it < n_items; ++it) {
    int64_t p = item_point[it];
    if (p < 0 || p >= n_points) continue;
    double x0[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < m->dim; ++a) x0[a] = points[p * m->dim + a];
    double gabs = 0.0;
    path_result r = one_path(m, normals, &at, bc, form, x0, -1, walk_len, seed, problem, (uint32_t)p,
                             (uint32_t)item_path[it], NULL, NULL, NULL, grad + it * m->dim, &gabs, 0);
    if (anchors)
      anchor_split(m, normals, &at, bc, form, anchors, anchor_prim, p, walk_len, seed, problem,
                   (uint32_t)item_path[it], &r, grad + it * m->dim, &gabs);
    if (value) value[it] = r.value;
    if (abs_sum) abs_sum[it] = r.abs_sum;
    if (grad_abs) grad_abs[it] = gabs;
    if (graze) graze[it] = r.graze;
    if (err) err[it] = r.err;
    if (grad_err) grad_err[it] = r.grad_err;
  }
  free(normals);
  free(at.cdf);
  return 0;
}

/* Mean and unbiased variance over paths 0..N-1 of the value and of each
 * gradient component (two-pass), every point off the boundary. */
int orc_solve_grad(const orc_mesh* m, const double* points, int64_t n_points, const orc_bc* bc,
                   int samples, int walk_len, uint64_t seed, uint32_t problem, const double* anchors,
                   const int32_t* anchor_prim, double* mean_out, double* var_out, double* grad_out,
                   double* grad_var_out, int n_threads) {
  if (check_args(m, bc, walk_len) || bc->density || samples < 1) return 1;
  if (check_anchors(m, bc, anchors, anchor_prim, n_points)) return 1;
  const int form = orc_resolve_formulation(m, bc->formulation);
  const int dim = m->dim;
  double* normals = make_normals(m);
  area_table at = make_area_table(m);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t p = 0; p < n_points; ++p) {
    double x0[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < dim; ++a) x0[a] = points[p * dim + a];
    /* finite paths only (value and every gradient component finite) */
    double* v = (double*)malloc(sizeof(double) * (size_t)samples * (1 + (size_t)dim));
    double* g = v + samples;
    int n = 0;
    for (int k = 0; k < samples; ++k) {
      path_result r = one_path(m, normals, &at, bc, form, x0, -1, walk_len, seed, problem, (uint32_t)p,
                               (uint32_t)k, NULL, NULL, NULL, g + (size_t)n * dim, NULL, 0);
      if (anchors) {
        double gabs = 0.0;
        anchor_split(m, normals, &at, bc, form, anchors, anchor_prim, p, walk_len, seed, problem, (uint32_t)k,
                     &r, g + (size_t)n * dim, &gabs);
      }
      v[n] = r.value;
      int finite = isfinite(v[n]);
      for (int c = 0; c < dim; ++c) finite = finite && isfinite(g[(size_t)n * dim + c]);
      if (finite) ++n;
    }
    for (int c = -1; c < dim; ++c) {
      double sum = 0.0, ss = 0.0;
      for (int k = 0; k < n; ++k) sum += c < 0 ? v[k] : g[(size_t)k * dim + c];
      const double mean = n > 0 ? sum / n : NAN;
      for (int k = 0; k < n; ++k) {
        const double d = (c < 0 ? v[k] : g[(size_t)k * dim + c]) - mean;
        ss += d * d;
      }
      const double var = n > 1 ? ss / (n - 1) : 0.0;
      if (c < 0) {
        if (mean_out) mean_out[p] = mean;
        if (var_out) var_out[p] = var;
      } else {
        if (grad_out) grad_out[p * dim + c] = mean;
        if (grad_var_out) grad_var_out[p * dim + c] = var;
      }
    }
    free(v);
  }
  free(normals);
  free(at.cdf);
  return 0;
}

int orc_intersect_all(const orc_mesh* m, const double* orig, const double* dir,
                      const int32_t* exclude, int64_t n_lines, int max_hits, int32_t* n_hits,
                      int32_t* hit_prim, double* hit_t, double* hit_margin, double* line_graze,
                      int n_threads) {
  if (!m || (m->dim != 2 && m->dim != 3) || max_hits < 0) return 1;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t l = 0; l < n_lines; ++l) {
    double x[3] = {0.0, 0.0, 0.0}, d[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < m->dim; ++a) {
      x[a] = orig[l * m->dim + a];
      d[a] = dir[l * m->dim + a];
    }
    int64_t ex = exclude ? exclude[l] : -1;
    int cnt = 0;
    double graze = INFINITY;
    for (int64_t j = 0; j < m->n_prims; ++j) {
      if (j == ex) continue;
      double t, y[3], margin, cosv;
      int hit = line_prim(m, j, x, d, &t, y, &margin, &cosv);
      double g = decision_margin(m, j, x, margin, cosv);
      if (g < graze) graze = g;
      if (!hit) continue;
      if (cnt < max_hits) {
        /* insertion in (t, prim) order */
        int pos = cnt;
        int32_t* hp = hit_prim + l * max_hits;
        double* ht = hit_t + l * max_hits;
        double* hm = hit_margin ? hit_margin + l * max_hits : NULL;
        while (pos > 0 && (ht[pos - 1] > t || (ht[pos - 1] == t && hp[pos - 1] > j))) {
          hp[pos] = hp[pos - 1];
          ht[pos] = ht[pos - 1];
          if (hm) hm[pos] = hm[pos - 1];
          --pos;
        }
        hp[pos] = (int32_t)j;
        ht[pos] = t;
        if (hm) hm[pos] = g;
      }
      ++cnt;
    }
    n_hits[l] = cnt;
    if (line_graze) line_graze[l] = graze;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Closed-form potential of a uniform primitive, int_T G(x, y) dA.            */
/* 3D (Wilton et al. 1984): with n the unit normal, d = (x - p1).n, rho the   */
/* projection of x on the plane, and per edge p_i -> p_i+1: unit tangent t,   */
/* outward in-plane normal u = t x n, P = (p_i - rho).u, s- / s+ = the        */
/* tangential coordinates of the edge's ends, R- / R+ their distances to x,   */
/* R0^2 = P^2 + d^2:                                                          */
/*   int_T 1/|x-y| dA = sum P ln((R+ + s+)/(R- + s-))                          */
/*                    - |d| sum [atan(P s+/(R0^2 + |d| R+)) - atan(P s-/(R0^2 + |d| R-))]. */
/* 2D: int over the segment of -ln|x - y| / (2 pi) dl in closed form.         */
/* ------------------------------------------------------------------------- */
static double log_ratio(double Rp, double sp, double Rm, double sm) {
  /* ln((R+ + s+)/(R- + s-)) = ln((R- - s-)/(R+ - s+)); take the form without
     cancellation */
  if (sp + sm >= 0.0) return log((Rp + sp) / (Rm + sm));
  return log((Rm - sm) / (Rp - sp));
}

double orc_prim_potential(const orc_mesh* m, int64_t prim, const double* x) {
  if (m->dim == 3) {
    double p[3][3], n[3];
    for (int c = 0; c < 3; ++c) prim_vertex(m, prim, c, p[c]);
    orc_prim_normal(m, prim, n);
    double xv[3] = {x[0] - p[0][0], x[1] - p[0][1], x[2] - p[0][2]};
    const double dn = dot(xv, n, 3);
    const double ad = fabs(dn);
    double rho[3] = {x[0] - dn * n[0], x[1] - dn * n[1], x[2] - dn * n[2]};
    double sum_log = 0.0, sum_atan = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double* a = p[c];
      const double* b = p[(c + 1) % 3];
      double e[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
      const double L = sqrt(dot(e, e, 3));
      double t[3] = {e[0] / L, e[1] / L, e[2] / L}, u[3];
      cross3(t, n, u);
      double ar[3] = {a[0] - rho[0], a[1] - rho[1], a[2] - rho[2]};
      double br[3] = {b[0] - rho[0], b[1] - rho[1], b[2] - rho[2]};
      const double P = dot(ar, u, 3);
      const double sm = dot(ar, t, 3), sp = dot(br, t, 3);
      double xa[3] = {x[0] - a[0], x[1] - a[1], x[2] - a[2]};
      double xb[3] = {x[0] - b[0], x[1] - b[1], x[2] - b[2]};
      const double Rm = sqrt(dot(xa, xa, 3)), Rp = sqrt(dot(xb, xb, 3));
      const double R02 = P * P + dn * dn;
      if (P != 0.0) sum_log += P * log_ratio(Rp, sp, Rm, sm);
      if (ad > 0.0) sum_atan += atan(P * sp / (R02 + ad * Rp)) - atan(P * sm / (R02 + ad * Rm));
    }
    return (sum_log - ad * sum_atan) / (4.0 * ORC_PI);
  }
  double a[3], b[3];
  prim_vertex(m, prim, 0, a);
  prim_vertex(m, prim, 1, b);
  double e[2] = {b[0] - a[0], b[1] - a[1]};
  const double L = sqrt(e[0] * e[0] + e[1] * e[1]);
  double t[2] = {e[0] / L, e[1] / L};
  double ax[2] = {x[0] - a[0], x[1] - a[1]};
  const double s0 = -(ax[0] * t[0] + ax[1] * t[1]); /* tangential coordinate of a relative to x */
  const double s1 = s0 + L;
  const double h = fabs(ax[0] * t[1] - ax[1] * t[0]);
  /* int_{s0}^{s1} ln sqrt(s^2 + h^2) ds */
  double F1 = 0.5 * s1 * log(s1 * s1 + h * h) - s1 + (h > 0.0 ? h * atan(s1 / h) : 0.0);
  double F0 = 0.5 * s0 * log(s0 * s0 + h * h) - s0 + (h > 0.0 ? h * atan(s0 / h) : 0.0);
  if (s1 == 0.0 && h == 0.0) F1 = 0.0;
  if (s0 == 0.0 && h == 0.0) F0 = 0.0;
  return -(F1 - F0) / (2.0 * ORC_PI);
}

/* 32-bit integer hash (the "lowbias32" constants of C. Wellons' hash prospector) */
static uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}

int orc_cv_addback(const orc_mesh* m, const double* g, const double* points, int64_t n_points,
                   uint32_t seed, int randomized, double* out, int n_threads) {
  if (!m || !g || m->dim != 3) return 1;
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t p = 0; p < n_points; ++p) {
    double x[3] = {points[p * 3], points[p * 3 + 1], points[p * 3 + 2]};
    double acc = 0.0;
    for (int64_t j = 0; j < m->n_prims; ++j) {
      if (!randomized) {
        acc += g[j] * orc_prim_potential(m, j, x);
        continue;
      }
      double v[3][3], c[3] = {0.0, 0.0, 0.0};
      for (int k = 0; k < 3; ++k) prim_vertex(m, j, k, v[k]);
      for (int k = 0; k < 3; ++k) c[k] = (v[0][k] + v[1][k] + v[2][k]) / 3.0;
      double r2 = 0.0;
      for (int k = 0; k < 3; ++k) {
        double dv[3] = {v[k][0] - c[0], v[k][1] - c[1], v[k][2] - c[2]};
        double q = dot(dv, dv, 3);
        if (q > r2) r2 = q;
      }
      double dx[3] = {x[0] - c[0], x[1] - c[1], x[2] - c[2]};
      if (dot(dx, dx, 3) < 16.0 * r2) {
        acc += g[j] * orc_prim_potential(m, j, x);
      } else {
        /* one point per (seed, triangle), the same for every evaluation point */
        const uint32_t h = hash32((uint32_t)j + 0x9e3779b9u * (seed + 1u));
        double a = uniform(hash32(h ^ 0x68e31da4u)), b = uniform(hash32(h ^ 0xb5297a4du));
        if (a + b > 1.0) {
          a = 1.0 - a;
          b = 1.0 - b;
        }
        double e1[3], e2[3], y[3], nn[3];
        for (int k = 0; k < 3; ++k) {
          e1[k] = v[1][k] - v[0][k];
          e2[k] = v[2][k] - v[0][k];
          y[k] = v[0][k] + a * e1[k] + b * e2[k];
        }
        cross3(e1, e2, nn);
        const double area = 0.5 * sqrt(dot(nn, nn, 3));
        acc += g[j] * area * G(x, y, 3);
      }
    }
    out[p] = acc;
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Learned control variate for the single layer (not in the paper).          */
/*                                                                           */
/* At a line with hits h (weights w(h) = m a(h), a(h) = kernel / p_all), the */
/* plain estimator continues with w(j) * (value at y_j) for the picked j.    */
/* For any function F, adding sum_h a(h) F(y_h) - w(j) F(y_j) changes        */
/* nothing in expectation given the line (the pick is uniform over the m     */
/* hits), so the estimator stays unbiased for every F:                       */
/*  - line 0 from x0: F = g0(T(y)) (a second table); the subtraction is     */
/*    kept and its exact expectation sum_T g0_T int_T G(x0, y) dA is added   */
/*    per point (orc_cv_addback) instead of the all-hits sum; a self-panel   */
/*    sample at a boundary x0 subtracts w g0(T0) too, so the add-back covers */
/*    all of Gamma.  With g0 = g + (emission at the centroid) the step-0     */
/*    emission is corrected as well, up to its variation over a triangle;    */
/*  - lines 1..M-2 (line branch): F = 2 phi s(y) + g(T(y));                  */
/*  - line M-1 (line branch): F = phi s(y), the exact rest of the path, so   */
/*    the pick is not needed at all.                                         */
/* ------------------------------------------------------------------------- */
typedef struct {
  int64_t prim;
  double y[3];
  uint32_t key;
} hit_rec;

static int collect_hits(const orc_mesh* m, const double* x, const double* d, int64_t exclude,
                        hit_rec* out, int max_out, uint64_t seed, uint32_t path, uint32_t point,
                        uint32_t problem, uint32_t line) {
  int k = 0;
  for (int64_t j = 0; j < m->n_prims; ++j) {
    if (j == exclude) continue;
    double t, y[3], margin, cosv;
    if (!line_prim(m, j, x, d, &t, y, &margin, &cosv)) continue;
    if (k < max_out) {
      uint32_t r[4];
      draw(seed, path, point, problem, line, 2u, (uint32_t)j, r);
      out[k].prim = j;
      memcpy(out[k].y, y, sizeof(out[k].y));
      out[k].key = r[0];
    }
    ++k;
  }
  return k;
}

#define CV_MAX_HITS 256

/* Value of the corrected path; *abs_out and *err_out (may be NULL) receive its
   magnitude sum and its first-order rounding-error bound in units of u (the
   bookkeeping of one_path, extended to the all-hits sums). */
static double one_path_cv(const orc_mesh* m, const double* normals, const area_table* at,
                          const orc_bc* bc, const double* g, const double* g0, const double* x0,
                          int64_t prim0, int M, uint64_t seed, uint32_t problem, uint32_t point,
                          uint32_t path, double* abs_out, double* err_out) {
  const int dim = m->dim;
  const double phi = (double)bc->domain;
  double x[3] = {x0[0], x0[1], dim == 3 ? x0[2] : 0.0};
  int64_t cur = prim0;
  double W = 1.0, acc = 0.0;
  double Wabs = 1.0, abs_sum = 0.0, P = 0.0, eW = 0.0, err = 0.0;
  hit_rec hits[CV_MAX_HITS];
  for (int i = 0; i < M; ++i) {
    const int on_gamma = cur >= 0, last = i == M - 1;
    const double xn = norm_d(x, dim);
    uint32_t r0[4];
    draw(seed, path, point, problem, (uint32_t)i, 0u, 0u, r0);
    double d[3] = {0.0, 0.0, 0.0};
    if (dim == 3) {
      double z = 1.0 - 2.0 * uniform(r0[0]);
      double sq = sqrt(fmax(0.0, 1.0 - z * z));
      double ph = 2.0 * ORC_PI * uniform(r0[1]);
      d[0] = sq * cos(ph);
      d[1] = sq * sin(ph);
      d[2] = z;
    } else {
      double th = 2.0 * ORC_PI * uniform(r0[0]);
      d[0] = cos(th);
      d[1] = sin(th);
    }
    double y[3];
    int64_t next;
    double Wn, Wnabs, eWn, Pn;
    if (bc->sampling == ORC_SAMPLE_RIS) {
      /* RIS vertex (candidates and pick as in one_path): given the C
         candidates, the pick's expected contribution w F(y_pick) is
         (|Gamma| / C) sum_j k(y_j) F(y_j); the corrected walk adds that sum
         and subtracts w F(y_pick), with F as for line sampling (line 0: the
         table g0, its mean restored by the add-back; lines 1..M-2:
         2 phi s + g; the last line, line 0 included when M = 1: phi s, with
         no pick). */
      const int C = bc->candidates;
      const double* nx = on_gamma ? normals + 3 * cur : NULL;
      const double ax = on_gamma ? prim_alpha(m, cur) : 0.0;
      const double cw = at->total / (double)C;
      double S = 0.0, Smag = 0.0, dS = 0.0, kpick = 0.0, csum = 0.0, cabs = 0.0, cerr = 0.0;
      int64_t jpick = -1;
      for (int jc = 0; jc < C; ++jc) {
        uint32_t rj[4];
        draw(seed, path, point, problem, (uint32_t)i, 3u, (uint32_t)jc, rj);
        const int64_t pj = area_pick(at, m->n_prims, (float)uniform(rj[0]));
        double ca = uniform(rj[1]), cb = dim == 3 ? uniform(rj[2]) : 0.0;
        if (ca + cb > 1.0) {
          ca = 1.0 - ca;
          cb = 1.0 - cb;
        }
        double v0[3], v1[3], v2[3] = {0.0, 0.0, 0.0}, yc[3] = {0.0, 0.0, 0.0};
        prim_vertex(m, pj, 0, v0);
        prim_vertex(m, pj, 1, v1);
        if (dim == 3) prim_vertex(m, pj, 2, v2);
        for (int c = 0; c < dim; ++c) yc[c] = v0[c] + ca * (v1[c] - v0[c]) + cb * (v2[c] - v0[c]);
        double r[3] = {yc[0] - x[0], yc[1] - x[1], dim == 3 ? yc[2] - x[2] : 0.0};
        const double rr = dot(r, r, dim);
        double k = 0.0, kmag = 0.0, dk = 0.0;
        if (rr > 0.0) {
          const double rho = sqrt(rr), drho = P + xn + norm_d(yc, dim);
          if (i == 0) {
            k = G(x, yc, dim);
            kmag = G_mag(x, yc, dim);
            dk = (dim == 3 ? 1.0 / (4.0 * ORC_PI * rr) : 1.0 / (2.0 * ORC_PI * rho)) * drho;
          } else {
            /* (y - x) . n_x from the candidate's vertex and edges (zero on the
               own primitive), as in one_path */
            double rn = 0.0;
            if (pj != cur) {
              double w0[3];
              prim_vertex(m, cur, 0, w0);
              double dv[3] = {v0[0] - w0[0], v0[1] - w0[1], dim == 3 ? v0[2] - w0[2] : 0.0};
              double e1[3] = {v1[0] - v0[0], v1[1] - v0[1], dim == 3 ? v1[2] - v0[2] : 0.0};
              double e2[3] = {v2[0] - v0[0], v2[1] - v0[1], dim == 3 ? v2[2] - v0[2] : 0.0};
              rn = dot(dv, nx, dim) + ca * dot(e1, nx, dim) + (dim == 3 ? cb * dot(e2, nx, dim) : 0.0);
            }
            const double dgdn = dim == 3 ? rn / (4.0 * ORC_PI * rr * rho) : rn / (2.0 * ORC_PI * rr);
            k = -2.0 * phi * (dgdn + ax * G(x, yc, dim));
            const double dn2 = fabs(2.0 * dgdn);
            kmag = dn2 + 2.0 * fabs(ax) * G_mag(x, yc, dim);
            const double sd = dim == 3 ? 4.0 * ORC_PI * rr * rho : 2.0 * ORC_PI * rr;
            dk = dn2 * (double)dim * drho / rho + 2.0 * (xn + norm_d(yc, dim)) / sd +
                 2.0 * fabs(ax) * (dim == 3 ? 1.0 / (4.0 * ORC_PI * rr) : 1.0 / (2.0 * ORC_PI * rho)) * drho;
          }
        }
        const double pk = fabs(k);
        S += pk;
        Smag += kmag;
        dS += dk;
        const double u = uniform(rj[3]);
        if (u * S < pk) {
          jpick = pj;
          kpick = k;
          memcpy(y, yc, sizeof(y));
        }
        if (i > 0 || last) { /* the candidate's term of the all-candidates sum */
          const double kf = last ? phi : 2.0 * phi;
          const double e = kf * orc_boundary_datum(m, bc, pj, yc);
          const double F = e + (last ? 0.0 : g[pj]);
          csum += cw * k * F;
          cabs += cw * kmag * (fabs(e) + (last ? 0.0 : fabs(g[pj])));
          cerr += cw * (kmag * emission_err(m, bc, pj, yc, kf, norm_d(yc, dim)) +
                        (eW * kmag + dk) * (fabs(e) + (last ? 0.0 : fabs(g[pj]))));
        }
      }
      if (i > 0 || last) {
        acc += W * csum;
        abs_sum += Wabs * cabs;
        err += Wabs * cerr;
      }
      if (last || jpick < 0 || !(S > 0.0)) break;
      const double w = (kpick > 0.0 ? 1.0 : -1.0) * S * cw;
      Wn = W * w;
      Wnabs = Wabs * Smag * cw;
      eWn = eW + dS / Smag;
      Pn = norm_d(y, dim); /* a point drawn by its barycentrics */
      next = jpick;
      if (i == 0) {
        const double ej = 2.0 * phi * orc_boundary_datum(m, bc, next, y);
        acc += Wn * (ej - g0[next]);
        abs_sum += Wnabs * (fabs(g0[next]) + fabs(ej));
        err += Wnabs * emission_err(m, bc, next, y, 2.0 * phi, Pn) + eWn * Wnabs * (fabs(g0[next]) + fabs(ej));
      } else {
        acc -= Wn * g[next]; /* the picked candidate's emission is inside the sum */
        abs_sum += Wnabs * fabs(g[next]);
        err += eWn * Wnabs * fabs(g[next]);
      }
      W = Wn;
      Wabs = Wnabs;
      eW = eWn;
      P = Pn;
      memcpy(x, y, sizeof(x));
      cur = next;
      continue;
    }
    const int mixture = on_gamma && (i == 0 || prim_kind(m, cur) == ORC_ROBIN);
    const int use_self = mixture && (r0[2] >> 8) < bc->self_threshold;
    if (use_self) {
      uint32_t r1[4];
      draw(seed, path, point, problem, (uint32_t)i, 1u, 0u, r1);
      double R, sinb;
      const double gp = self_panel_geo(m, cur, x, uniform(r1[0]), uniform(r1[1]), y, &R, &sinb);
      const double w = (i == 0 ? gp : -2.0 * phi * prim_alpha(m, cur) * gp) / bc->self_p;
      const double dR = (P + xn + R) / sinb;
      Wn = W * w;
      Wnabs = Wabs * fabs(w);
      eWn = eW + dR / R;
      Pn = P + dR + xn + R;
      next = cur;
      if (i == 0 && !last) {
        acc -= Wn * g0[cur];
        abs_sum += Wnabs * fabs(g0[cur]);
        err += eWn * Wnabs * fabs(g0[cur]);
      }
      const double k = last ? phi : 2.0 * phi;
      const double e = k * orc_boundary_datum(m, bc, cur, y);
      acc += Wn * e;
      abs_sum += Wnabs * fabs(e);
      err += Wnabs * emission_err(m, bc, cur, y, k, Pn) + eWn * Wnabs * fabs(e);
    } else {
      const int mh = collect_hits(m, x, d, cur, hits, CV_MAX_HITS, seed, path, point, problem,
                                  (uint32_t)i);
      if (mh == 0) break;
      if (mh > CV_MAX_HITS) return NAN;
      double a[CV_MAX_HITS], aabs[CV_MAX_HITS], aeps[CV_MAX_HITS], ap[CV_MAX_HITS];
      int j = 0;
      for (int h = 0; h < mh; ++h) {
        const double* ny = normals + 3 * hits[h].prim;
        double kern, kabs;
        double r[3] = {hits[h].y[0] - x[0], hits[h].y[1] - x[1], dim == 3 ? hits[h].y[2] - x[2] : 0.0};
        const double rho = norm_d(r, dim), cy = fabs(dot(r, ny, dim)) / rho;
        ap[h] = (P + xn + norm_d(hits[h].y, dim) + rho) / cy; /* the hit's position error */
        if (i == 0) {
          kern = G(x, hits[h].y, dim);
          kabs = G_mag(x, hits[h].y, dim);
          aeps[h] = ap[h] / rho + 1.0 / cy;
        } else {
          const double* nx = normals + 3 * cur;
          const double al = fabs(prim_alpha(m, cur));
          const double dn = dG_dnx(x, hits[h].y, nx, dim);
          kern = -2.0 * phi * (dn + prim_alpha(m, cur) * G(x, hits[h].y, dim));
          kabs = 2.0 * (fabs(dn) + al * G_mag(x, hits[h].y, dim));
          const double cx = fabs(dot(r, nx, dim)) / rho;
          aeps[h] = (1.0 + xn / rho + al * ap[h]) / (cx + al * rho) + 1.0 / cy;
        }
        const double pa = line_pdf(x, hits[h].y, ny, 1, dim) * (mixture ? 1.0 - bc->self_p : 1.0);
        a[h] = kern / pa;
        aabs[h] = kabs / pa;
        if (hits[h].key < hits[j].key || (hits[h].key == hits[j].key && hits[h].prim < hits[j].prim))
          j = h;
      }
      if (last) {
        for (int h = 0; h < mh; ++h) {
          const double e = phi * orc_boundary_datum(m, bc, hits[h].prim, hits[h].y);
          acc += W * a[h] * e;
          abs_sum += Wabs * aabs[h] * fabs(e);
          err += Wabs * aabs[h] * emission_err(m, bc, hits[h].prim, hits[h].y, phi, ap[h]) +
                 (eW + aeps[h]) * Wabs * aabs[h] * fabs(e);
        }
        break;
      }
      const double wj = a[j] * (double)mh;
      Wn = W * wj;
      Wnabs = Wabs * aabs[j] * (double)mh;
      eWn = eW + aeps[j];
      Pn = ap[j];
      memcpy(y, hits[j].y, sizeof(y));
      next = hits[j].prim;
      const double ej = 2.0 * phi * orc_boundary_datum(m, bc, next, y);
      if (i == 0) {
        acc -= Wn * g0[next];
        acc += Wn * ej;
        abs_sum += Wnabs * (fabs(g0[next]) + fabs(ej));
        err += Wnabs * emission_err(m, bc, next, y, 2.0 * phi, Pn) + eWn * Wnabs * (fabs(g0[next]) + fabs(ej));
      } else {
        for (int h = 0; h < mh; ++h) {
          const double eh = 2.0 * phi * orc_boundary_datum(m, bc, hits[h].prim, hits[h].y);
          acc += W * a[h] * (eh + g[hits[h].prim]);
          abs_sum += Wabs * aabs[h] * (fabs(eh) + fabs(g[hits[h].prim]));
          err += Wabs * aabs[h] * emission_err(m, bc, hits[h].prim, hits[h].y, 2.0 * phi, ap[h]) +
                 (eW + aeps[h]) * Wabs * aabs[h] * (fabs(eh) + fabs(g[hits[h].prim]));
        }
        acc -= Wn * g[next]; /* the picked hit's emission is kept as in the plain estimator */
        abs_sum += Wnabs * fabs(g[next]);
        err += eWn * Wnabs * fabs(g[next]);
      }
    }
    W = Wn;
    Wabs = Wnabs;
    eW = eWn;
    P = Pn;
    memcpy(x, y, sizeof(x));
    cur = next;
  }
  if (abs_out) *abs_out = abs_sum;
  if (err_out) *err_out = err;
  return acc;
}

int orc_trace_cv(const orc_mesh* m, const double* points, const int32_t* point_prim,
                 int64_t n_points, const orc_bc* bc, int walk_len, uint64_t seed, uint32_t problem,
                 const double* g, const double* g0, int64_t n_items, const int64_t* item_point,
                 const int64_t* item_path, double* value, double* abs_sum, double* err,
                 int n_threads) {
  if (check_args(m, bc, walk_len) || !g) return 1;
  if (!g0) g0 = g;
  if (orc_resolve_formulation(m, bc->formulation) != ORC_SINGLE_LAYER || bc->density) return 1;
  for (int64_t j = 0; j < m->n_prims; ++j)
    if (prim_kind(m, j) == ORC_DIRICHLET) return 1; /* the corrected walk has no Dirichlet rows */
  double* normals = make_normals(m);
  area_table at = make_area_table(m);
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 4)
#endif
  for (int64_t it = 0; it < n_items; ++it) {
    const int64_t p = item_point[it];
    if (p < 0 || p >= n_points) continue;
    double x0[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < m->dim; ++a) x0[a] = points[p * m->dim + a];
    const int64_t prim0 = point_prim ? point_prim[p] : -1;
    value[it] = one_path_cv(m, normals, &at, bc, g, g0, x0, prim0, walk_len, seed, problem,
                            (uint32_t)p, (uint32_t)item_path[it], abs_sum ? abs_sum + it : NULL,
                            err ? err + it : NULL);
  }
  free(normals);
  free(at.cdf);
  return 0;
}
