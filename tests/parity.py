"""Shared helpers for GPU-vs-oracle parity tests (test infrastructure)."""
from __future__ import annotations

import dataclasses

import numpy as np

import oracle
from paper_2305_04403_amd import inputs as I

# Grazing class (the north-star tolerance "exactly, except at grazing hits within
# 1e-6"): a path is grazing when some line of it passes within 1e-6 of a
# primitive's edge, measured as |smallest barycentric coordinate| * |cos| where
# cos is the angle between the line and the primitive's normal (the factor
# 1/|cos| is how FP32 barycentric error grows towards grazing incidence).
GRAZE = 1e-6
# per-path relative tolerance, relative to the sum of |terms| of the path
# (alternating double-layer sums can cancel to ~0)
RTOL_F32 = 1e-5
RTOL_F64 = 1e-12


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

    def summary(self) -> str:
        return (f"paths={self.n} grazing={self.n_graze} checked={self.n_checked} "
                f"vertex-mismatch={self.n_vertex_mismatch} value-mismatch={self.n_value_mismatch} "
                f"max-rel-err={self.max_rel_err:.3e}")


def compare_paths(orc: dict, gpu_val: np.ndarray, gpu_vprim: np.ndarray, gpu_vm: np.ndarray,
                  rtol: float, graze: float = GRAZE) -> PathParity:
    """orc: oracle trace dict over the same (point, path) items, flattened."""
    n = orc["value"].shape[0]
    g = orc["graze"] < graze
    ok = ~g
    vmis = np.any(orc["vtx_prim"] != gpu_vprim, axis=1) | np.any(orc["vtx_m"] != gpu_vm, axis=1)
    scale = np.maximum(orc["abs_sum"], 1e-300)
    rel = np.abs(gpu_val - orc["value"]) / scale
    rel_ok = np.where(ok, rel, 0.0)
    return PathParity(n=n, n_graze=int(g.sum()), n_checked=int(ok.sum()),
                      n_vertex_mismatch=int((vmis & ok).sum()),
                      n_value_mismatch=int(((rel > rtol) & ok).sum()),
                      max_rel_err=float(rel_ok.max()) if n else 0.0)


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
