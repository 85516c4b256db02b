"""Shared helpers for GPU-vs-oracle parity tests (test infrastructure)."""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle
from paper_2305_04403_amd import inputs as I

# Grazing class (the parity bar: paths agree exactly except where a hit grazes
# a primitive within 1e-6): a path is grazing when some line of it passes within 1e-6 of a
# primitive's edge, measured as |smallest barycentric coordinate| * |cos| where
# cos is the angle between the line and the primitive's normal (the factor
# 1/|cos| is how FP32 barycentric error grows towards grazing incidence).
GRAZE = 1e-6
# per-path relative tolerance, relative to the path sum with every factor and
# summand replaced by its magnitude (alternating double-layer sums and mixed-sign
# source sums can cancel to ~0)
RTOL_F32 = 1e-5
RTOL_F64 = 1e-12
# Weights and source terms that divide by |cos theta_y| amplify the rounding error
# of cos (a few ulp absolute) by 1/|cos|; the tolerance grows by COS_ULP / |cos|
# for the smallest such cosine of the path.
COS_ULP_F32 = 4e-7
COS_ULP_F64 = 1e-15


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
    max_rel_err: float
    max_err_over_tol: float
    worst: str

    def summary(self) -> str:
        return (f"paths={self.n} grazing={self.n_graze} checked={self.n_checked} "
                f"vertex-mismatch={self.n_vertex_mismatch} value-mismatch={self.n_value_mismatch} "
                f"max-rel-err={self.max_rel_err:.3e} max-err/tol={self.max_err_over_tol:.3f} "
                f"worst: {self.worst}")


def compare_paths(orc: dict, gpu_val: np.ndarray, gpu_vprim: np.ndarray, gpu_vm: np.ndarray,
                  rtol: float, graze: float = GRAZE) -> PathParity:
    """orc: oracle trace dict over the same (point, path) items, flattened."""
    n = orc["value"].shape[0]
    g = orc["graze"] < graze
    ok = ~g
    vmis = np.any(orc["vtx_prim"] != gpu_vprim, axis=1) | np.any(orc["vtx_m"] != gpu_vm, axis=1)
    scale = np.maximum(orc["abs_sum"], 1e-300)
    err = np.abs(gpu_val - orc["value"])
    rel = err / scale
    cos_ulp = COS_ULP_F32 if rtol >= 1e-7 else COS_ULP_F64
    tol = scale * (rtol + cos_ulp / np.maximum(orc["cond_cos"], 1e-300))
    ratio = np.where(ok, err / tol, 0.0)
    rel_ok = np.where(ok, rel, 0.0)
    w = int(np.argmax(ratio)) if n else 0
    worst = (f"item={w} orc={orc['value'][w]:.9g} gpu={gpu_val[w]:.9g} abs_sum={orc['abs_sum'][w]:.3g} "
             f"cond_cos={orc['cond_cos'][w]:.3g} graze={orc['graze'][w]:.3g}") if n else ""
    return PathParity(n=n, n_graze=int(g.sum()), n_checked=int(ok.sum()),
                      n_vertex_mismatch=int((vmis & ok).sum()),
                      n_value_mismatch=int(((err > tol) & ok).sum()),
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
