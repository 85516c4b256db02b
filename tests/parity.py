"""Shared helpers for GPU-vs-oracle parity tests (test infrastructure).

The bar, per path (the oracle's values are binary64 brute force on the same
inputs and the same random numbers):

* hit lists and picks: identical outside the grazing class;
* value: |u_gpu - u_oracle| <= RTOL * S + KAPPA * u * E, where S is the path
  sum with every factor and summand replaced by its magnitude (alternating
  double-layer sums and mixed-sign source sums can cancel to ~0), u the unit
  roundoff of the scene's format and E the oracle's first-order rounding-error
  bound of the path in units of u (oracle.c: the error of every vertex position,
  weight and emission propagated along the path from its geometry: incidence
  cosines, distances, the data's derivatives).  E is what makes 1e-5 of S
  unreachable for a binary32 evaluation of an ill-conditioned path (a line
  meeting a primitive at |cos| ~ 1e-3, a hop of 1e-4 between two vertices);
  for well-conditioned paths RTOL * S dominates.  Every test reports the share
  of its checked paths that meet RTOL * S alone.

Grazing class: a path is left out (and counted) when, on one of its lines, the
decision of some primitive's hit test lies within GRAZE of flipping, measured
in units of that decision's own rounding scale (the oracle's decision_margin:
the barycentric margin times |det| over |x - v0| |e| + |e1||e2|).  1e-6 is
about 16 binary32 roundings; binary64 scenes use 1e-14 (about 90 roundings).
"""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle
from paper_2305_04403_amd import inputs as I

GRAZE = 1e-6
GRAZE_F64 = 1e-14
RTOL_F32 = 1e-5
RTOL_F64 = 1e-12
U_F32 = 2.0 ** -24
U_F64 = 2.0 ** -53
# The bound counts every rounding of a chain of operations once, with unit
# weight; a kernel's chain (a dot product, a division, a square root) takes a
# few.  KAPPA is that factor.
KAPPA = 8.0


def is_f32(rtol: float) -> bool:
    return rtol >= 1e-7


def graze_for(rtol: float) -> float:
    return GRAZE if is_f32(rtol) else GRAZE_F64


def tolerance(abs_sum, err, rtol: float):
    """The per-path (or per-component) bar: RTOL * S + KAPPA * u * E."""
    u = U_F32 if is_f32(rtol) else U_F64
    return rtol * np.asarray(abs_sum) + KAPPA * u * np.asarray(err)


def f32(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def f32_mesh(mesh: I.Mesh) -> I.Mesh:
    return dataclasses.replace(mesh, verts=f32(mesh.verts))


@dataclasses.dataclass
class PathParity:
    n: int
    n_graze: int
    n_checked: int
    n_vertex_mismatch: int
    n_value_mismatch: int
    n_plain: int          # checked paths within RTOL * S alone
    max_rel_err: float
    max_err_over_tol: float
    worst: str

    def summary(self) -> str:
        share = self.n_plain / max(self.n_checked, 1)
        return (f"paths={self.n} grazing={self.n_graze} checked={self.n_checked} "
                f"vertex-mismatch={self.n_vertex_mismatch} value-mismatch={self.n_value_mismatch} "
                f"within-plain-bar={self.n_plain} ({share:.5f}) "
                f"max-rel-err={self.max_rel_err:.3e} max-err/tol={self.max_err_over_tol:.3f} "
                f"worst: {self.worst}")

    def assert_exact(self, max_graze_frac: float = 0.01):
        """The bar with no allowance: every checked path's picks, hit counts
        and value inside it."""
        assert self.n_graze <= max_graze_frac * self.n, self.summary()
        assert self.n_vertex_mismatch == 0, self.summary()
        assert self.n_value_mismatch == 0, self.summary()


def compare_paths(orc: dict, gpu_val: np.ndarray, gpu_vprim: np.ndarray, gpu_vm: np.ndarray,
                  rtol: float) -> PathParity:
    """orc: oracle trace dict over the same (point, path) items, flattened."""
    n = orc["value"].shape[0]
    g = orc["graze"] < graze_for(rtol)
    ok = ~g
    vmis = np.any(orc["vtx_prim"] != gpu_vprim, axis=1) | np.any(orc["vtx_m"] != gpu_vm, axis=1)
    scale = np.maximum(orc["abs_sum"], 1e-300)
    err = np.abs(gpu_val - orc["value"])
    rel = err / scale
    tol = np.maximum(tolerance(orc["abs_sum"], orc["err"], rtol), 1e-300)
    ratio = np.where(ok, err / tol, 0.0)
    rel_ok = np.where(ok, rel, 0.0)
    w = int(np.argmax(ratio)) if n else 0
    worst = (f"item={w} orc={orc['value'][w]:.9g} gpu={gpu_val[w]:.9g} abs_sum={orc['abs_sum'][w]:.3g} "
             f"err_bound={orc['err'][w]:.3g}u graze={orc['graze'][w]:.3g}") if n else ""
    return PathParity(n=n, n_graze=int(g.sum()), n_checked=int(ok.sum()),
                      n_vertex_mismatch=int((vmis & ok).sum()),
                      n_value_mismatch=int(((err > tol) & ok).sum()),
                      n_plain=int(((err <= rtol * orc["abs_sum"]) & ok).sum()),
                      max_rel_err=float(rel_ok.max()) if n else 0.0,
                      max_err_over_tol=float(ratio.max()) if n else 0.0, worst=worst)


def oracle_all_paths(om, points, point_prim, bc, N, M, seed, point_ids=None):
    P = points.shape[0]
    ip = np.repeat(np.arange(P), N)
    ik = np.tile(np.arange(N), P)
    if point_ids is not None:
        # the oracle indexes its point array by the random-number point index
        big = np.zeros((int(point_ids.max()) + 1, points.shape[1]))
        big[point_ids] = points
        bpp = None
        if point_prim is not None:
            bpp = np.full(big.shape[0], -1, dtype=np.int32)
            bpp[point_ids] = point_prim
        return oracle.trace(om, big, bpp, bc, M, seed, np.repeat(point_ids, N), ik, want_pos=False)
    return oracle.trace(om, points, point_prim, bc, M, seed, ip, ik, want_pos=False)
