"""ctypes front end of the FP64 brute-force oracle (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package.  The product library never does.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import build as _build

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB selects another build of the same sources (the sanitized one)
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

AUTO, DOUBLE_LAYER, DIRECT, SINGLE_LAYER = 0, 1, 2, 3
PROG_CONST, PROG_LINEAR, PROG_QUAD, PROG_INVDIST = 0, 1, 2, 3


class _Mesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("n_verts", C.c_int64), ("n_prims", C.c_int64),
                ("verts", C.c_void_p), ("prims", C.c_void_p), ("kind", C.c_void_p),
                ("alpha", C.c_void_p)]


class _BC(C.Structure):
    _fields_ = [("domain", C.c_int), ("formulation", C.c_int), ("program", C.c_int),
                ("params", C.c_double * 8), ("self_threshold", C.c_uint32), ("self_p", C.c_double),
                ("density", C.c_int), ("sampling", C.c_int), ("candidates", C.c_int),
                ("mixed_k", C.c_double), ("mixed_threshold", C.c_uint32), ("mixed_p", C.c_double),
                ("data_mode", C.c_int), ("vertex_data", C.c_void_p)]


class _TraceOut(C.Structure):
    _fields_ = [("value", C.c_void_p), ("abs_sum", C.c_void_p), ("graze", C.c_void_p),
                ("err", C.c_void_p), ("vtx_prim", C.c_void_p), ("vtx_m", C.c_void_p),
                ("vtx_pos", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            _build.build()
        _lib = C.CDLL(LIB_PATH)
        _lib.orc_philox4x32_10.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        vp = C.c_void_p
        _lib.orc_trace.restype = C.c_int
        _lib.orc_trace.argtypes = [vp, vp, vp, C.c_int64, vp, C.c_int, C.c_uint64, C.c_uint32,
                                   C.c_int64, vp, vp, vp, C.c_int]
        _lib.orc_solve.restype = C.c_int
        _lib.orc_solve.argtypes = [vp, vp, vp, C.c_int64, vp, C.c_int, C.c_int, C.c_uint64,
                                   C.c_uint32, vp, vp, C.c_int]
        _lib.orc_intersect_all.restype = C.c_int
        _lib.orc_intersect_all.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_int, vp, vp, vp, vp,
                                           vp, C.c_int]
        _lib.orc_self_panel.restype = C.c_double
        _lib.orc_self_panel.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_double,
                                        C.c_double, C.c_void_p]
        _lib.orc_boundary_datum.restype = C.c_double
        _lib.orc_boundary_datum.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        _lib.orc_program_value.restype = C.c_double
        _lib.orc_program_value.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.orc_resolve_formulation.restype = C.c_int
        _lib.orc_resolve_formulation.argtypes = [C.c_void_p, C.c_int]
        _lib.orc_lines_per_path.restype = C.c_int
        _lib.orc_lines_per_path.argtypes = [C.c_void_p, C.c_void_p, C.c_int]
        _lib.orc_prim_normal.argtypes = [C.c_void_p, C.c_int64, C.c_void_p]
        _lib.orc_prim_potential.argtypes = [vp, C.c_int64, vp]
        _lib.orc_prim_potential.restype = C.c_double
        _lib.orc_cv_addback.argtypes = [vp, vp, vp, C.c_int64, C.c_uint32, C.c_int, vp, C.c_int]
        _lib.orc_cv_addback.restype = C.c_int
        _lib.orc_trace_cv.argtypes = [vp, vp, vp, C.c_int64, vp, C.c_int, C.c_uint64, C.c_uint32, vp,
                                      vp, C.c_int64, vp, vp, vp, vp, vp, C.c_int]
        _lib.orc_trace_cv.restype = C.c_int
        _lib.orc_trace_grad.argtypes = [vp, vp, C.c_int64, vp, C.c_int, C.c_uint64, C.c_uint32, C.c_int64,
                                        vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, C.c_int]
        _lib.orc_trace_grad.restype = C.c_int
        _lib.orc_solve_grad.argtypes = [vp, vp, C.c_int64, vp, C.c_int, C.c_int, C.c_uint64, C.c_uint32,
                                        vp, vp, vp, vp, vp, vp, C.c_int]
        _lib.orc_solve_grad.restype = C.c_int
        _lib.orc_forward_paths.argtypes = [vp, vp, vp, C.c_int64, C.c_int, C.c_uint64, C.c_uint32, vp,
                                           C.c_int]
        _lib.orc_forward_paths.restype = C.c_int
        _lib.orc_forward_gather.argtypes = [C.c_int, C.c_int64, C.c_int, vp, vp, vp, C.c_int64, vp, vp,
                                            vp, C.c_int]
        _lib.orc_forward_gather.restype = C.c_int
        _lib.orc_mlp_n_params.argtypes = [C.c_int, C.c_int, C.c_int]
        _lib.orc_mlp_n_params.restype = C.c_int64
        _lib.orc_mlp_forward.argtypes = [vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, vp,
                                         C.c_int, vp]
        _lib.orc_mlp_forward.restype = None
        _lib.orc_mlp_forward_bound.argtypes = [vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, vp,
                                               vp, C.c_double, C.c_double, C.c_double, vp, vp, vp, vp]
        _lib.orc_mlp_forward_bound.restype = None
        _lib.orc_mlp_loss_grad.argtypes = [vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int64, vp,
                                           vp, C.c_int, vp]
        _lib.orc_mlp_loss_grad.restype = C.c_double
        _lib.orc_adam_step.argtypes = [vp, vp, vp, vp, C.c_int64, C.c_int64, C.c_double, C.c_double,
                                       C.c_double, C.c_double]
        _lib.orc_adam_step.restype = None
        _lib.orc_bf16_round.argtypes = [C.c_double]
        _lib.orc_bf16_round.restype = C.c_double
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class OracleMesh:
    """Holds contiguous float64 / int32 copies of a mesh and the C view of them."""

    def __init__(self, mesh):
        self.dim = int(mesh.dim)
        self.verts = np.ascontiguousarray(mesh.verts, dtype=np.float64)
        self.prims = np.ascontiguousarray(mesh.prims, dtype=np.int32)
        self.kind = None if mesh.kind is None else np.ascontiguousarray(mesh.kind, dtype=np.uint8)
        self.alpha = None if mesh.alpha is None else np.ascontiguousarray(mesh.alpha, dtype=np.float64)
        self.c = _Mesh(self.dim, self.verts.shape[0], self.prims.shape[0], _ptr(self.verts),
                       _ptr(self.prims), _ptr(self.kind), _ptr(self.alpha))

    @property
    def ref(self):
        return C.byref(self.c)

    def normals(self) -> np.ndarray:
        out = np.zeros((self.prims.shape[0], 3))
        for j in range(self.prims.shape[0]):
            lib().orc_prim_normal(self.ref, j, out[j].ctypes.data)
        return out[:, : self.dim]


def self_threshold(p: float) -> int:
    return int(np.floor(p * 2.0 ** 24))


SAMPLE_LINE, SAMPLE_RIS = 0, 1


def make_bc(domain: int = 1, formulation: int = AUTO, program: int = PROG_CONST,
            params=(), self_p: float = 1.0 / 16.0, density: bool = False, sampling: int = SAMPLE_LINE,
            candidates: int = 16, mixed_k: float = 4.0, mixed_p: float = 2.0 / 3.0,
            vertex_data: Optional[np.ndarray] = None) -> _BC:
    """Boundary data from the harmonic program, or, with vertex_data (one value
    per mesh vertex), given per vertex and interpolated linearly on each
    primitive (the returned structure keeps a reference to the array)."""
    b = _BC()
    if vertex_data is not None:
        vd = np.ascontiguousarray(vertex_data, dtype=np.float64)
        b.data_mode = 1
        b.vertex_data = vd.ctypes.data
        b._vd = vd
    b.mixed_k = float(mixed_k)
    b.mixed_threshold = self_threshold(mixed_p)
    b.mixed_p = b.mixed_threshold / 2.0 ** 24
    b.density = int(bool(density))
    b.sampling = int(sampling)
    b.candidates = int(candidates)
    b.domain = int(domain)
    b.formulation = int(formulation)
    b.program = int(program)
    for i, v in enumerate(params):
        b.params[i] = float(v)
    b.self_threshold = self_threshold(self_p)
    b.self_p = b.self_threshold / 2.0 ** 24
    return b


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    o = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(c.ctypes.data, k.ctypes.data, o.ctypes.data)
    return o


def resolve_formulation(mesh: OracleMesh, formulation: int) -> int:
    return lib().orc_resolve_formulation(mesh.ref, int(formulation))


def lines_per_path(mesh: OracleMesh, bc: _BC, walk_len: int) -> int:
    return lib().orc_lines_per_path(mesh.ref, C.byref(bc), int(walk_len))


def trace(mesh: OracleMesh, points: np.ndarray, point_prim: Optional[np.ndarray], bc: _BC,
          walk_len: int, seed: int, item_point: np.ndarray, item_path: np.ndarray,
          problem: int = 0, n_threads: int = 0, want_pos: bool = True) -> dict:
    pts = np.ascontiguousarray(points, dtype=np.float64)
    pp = None if point_prim is None else np.ascontiguousarray(point_prim, dtype=np.int32)
    ip = np.ascontiguousarray(item_point, dtype=np.int64)
    ik = np.ascontiguousarray(item_path, dtype=np.int64)
    n = ip.shape[0]
    L = lines_per_path(mesh, bc, walk_len)
    out = {"value": np.zeros(n), "abs_sum": np.zeros(n), "graze": np.zeros(n), "err": np.zeros(n),
           "vtx_prim": np.zeros((n, L), dtype=np.int32), "vtx_m": np.zeros((n, L), dtype=np.int32)}
    if want_pos:
        out["vtx_pos"] = np.zeros((n, L, mesh.dim))
    t = _TraceOut(_ptr(out["value"]), _ptr(out["abs_sum"]), _ptr(out["graze"]),
                  _ptr(out["err"]), _ptr(out["vtx_prim"]), _ptr(out["vtx_m"]),
                  _ptr(out.get("vtx_pos")))
    rc = lib().orc_trace(mesh.ref, _ptr(pts), _ptr(pp), C.c_int64(pts.shape[0]), C.byref(bc),
                         C.c_int(walk_len), C.c_uint64(seed), C.c_uint32(problem), C.c_int64(n),
                         _ptr(ip), _ptr(ik), C.byref(t), C.c_int(n_threads))
    if rc != 0:
        raise ValueError("orc_trace rejected its arguments")
    return out


def solve(mesh: OracleMesh, points: np.ndarray, point_prim: Optional[np.ndarray], bc: _BC,
          samples: int, walk_len: int, seed: int, problem: int = 0, n_threads: int = 0):
    pts = np.ascontiguousarray(points, dtype=np.float64)
    pp = None if point_prim is None else np.ascontiguousarray(point_prim, dtype=np.int32)
    P = pts.shape[0]
    mean = np.zeros(P)
    var = np.zeros(P)
    rc = lib().orc_solve(mesh.ref, _ptr(pts), _ptr(pp), C.c_int64(P), C.byref(bc),
                         C.c_int(samples), C.c_int(walk_len), C.c_uint64(seed),
                         C.c_uint32(problem), _ptr(mean), _ptr(var), C.c_int(n_threads))
    if rc != 0:
        raise ValueError("orc_solve rejected its arguments")
    return mean, var


def _anchor_args(anchors, anchor_prim, n_points, dim):
    if anchors is None and anchor_prim is None:
        return None, None, None
    A = np.ascontiguousarray(anchors, dtype=np.float64).reshape(n_points, dim)
    AP = np.ascontiguousarray(anchor_prim, dtype=np.int32).reshape(n_points)
    return A, AP, (A, AP)


def trace_grad(mesh: OracleMesh, points: np.ndarray, bc: _BC, walk_len: int, seed: int,
               item_point: np.ndarray, item_path: np.ndarray, problem: int = 0, n_threads: int = 0,
               anchors=None, anchor_prim=None) -> dict:
    """Per-path value and gradient in x0 (points off the boundary), with the
    magnitude sums, grazing margin and rounding-error bounds (units of u) of
    each path.  anchors / anchor_prim (double layer): per point a boundary
    point and its primitive for the boundary split of the gradient."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    ip = np.ascontiguousarray(item_point, dtype=np.int64)
    ik = np.ascontiguousarray(item_path, dtype=np.int64)
    A, AP, _keep = _anchor_args(anchors, anchor_prim, pts.shape[0], mesh.dim)
    n = ip.shape[0]
    out = {"value": np.zeros(n), "grad": np.zeros((n, mesh.dim)), "abs_sum": np.zeros(n),
           "grad_abs": np.zeros(n), "graze": np.zeros(n), "err": np.zeros(n), "grad_err": np.zeros(n)}
    rc = lib().orc_trace_grad(mesh.ref, _ptr(pts), C.c_int64(pts.shape[0]), C.byref(bc), C.c_int(walk_len),
                              C.c_uint64(seed), C.c_uint32(problem), C.c_int64(n), _ptr(ip), _ptr(ik),
                              None if A is None else _ptr(A), None if AP is None else _ptr(AP),
                              _ptr(out["value"]), _ptr(out["grad"]), _ptr(out["abs_sum"]),
                              _ptr(out["grad_abs"]), _ptr(out["graze"]), _ptr(out["err"]),
                              _ptr(out["grad_err"]), C.c_int(n_threads))
    if rc != 0:
        raise ValueError("orc_trace_grad rejected its arguments")
    return out


def solve_grad(mesh: OracleMesh, points: np.ndarray, bc: _BC, samples: int, walk_len: int, seed: int,
               problem: int = 0, n_threads: int = 0, anchors=None, anchor_prim=None):
    """Mean and variance of the value and of the gradient (P, dim) over paths."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    P = pts.shape[0]
    A, AP, _keep = _anchor_args(anchors, anchor_prim, P, mesh.dim)
    mean, var = np.zeros(P), np.zeros(P)
    g, gv = np.zeros((P, mesh.dim)), np.zeros((P, mesh.dim))
    rc = lib().orc_solve_grad(mesh.ref, _ptr(pts), C.c_int64(P), C.byref(bc), C.c_int(samples),
                              C.c_int(walk_len), C.c_uint64(seed), C.c_uint32(problem),
                              None if A is None else _ptr(A), None if AP is None else _ptr(AP),
                              _ptr(mean), _ptr(var), _ptr(g), _ptr(gv), C.c_int(n_threads))
    if rc != 0:
        raise ValueError("orc_solve_grad rejected its arguments")
    return mean, var, g, gv


class _ForwardOut(C.Structure):
    _fields_ = [("vtx_pos", C.c_void_p), ("vtx_w", C.c_void_p), ("vtx_prim", C.c_void_p),
                ("vtx_m", C.c_void_p), ("graze", C.c_void_p), ("perr", C.c_void_p),
                ("werr", C.c_void_p)]


def forward_paths(mesh: OracleMesh, bc: _BC, n_paths: int, walk_len: int, seed: int,
                  start_weight: Optional[np.ndarray] = None, problem: int = 0,
                  n_threads: int = 0) -> dict:
    """Forward (adjoint) single-layer paths from the boundary (all-Neumann
    meshes): per path and vertex the position, primitive, hit count and source
    strength with the rounding-error bounds (units of u) of both; per path the
    grazing margin."""
    M = int(walk_len)
    sw = None if start_weight is None else np.ascontiguousarray(start_weight, dtype=np.float64)
    out = {"pos": np.zeros((n_paths, M, mesh.dim)), "w": np.zeros((n_paths, M)),
           "prim": np.zeros((n_paths, M), dtype=np.int32), "m": np.zeros((n_paths, M), dtype=np.int32),
           "graze": np.zeros(n_paths), "perr": np.zeros((n_paths, M)), "werr": np.zeros((n_paths, M))}
    t = _ForwardOut(_ptr(out["pos"]), _ptr(out["w"]), _ptr(out["prim"]), _ptr(out["m"]),
                    _ptr(out["graze"]), _ptr(out["perr"]), _ptr(out["werr"]))
    rc = lib().orc_forward_paths(mesh.ref, C.byref(bc), _ptr(sw), C.c_int64(n_paths), C.c_int(M),
                                 C.c_uint64(seed), C.c_uint32(problem), C.byref(t), C.c_int(n_threads))
    if rc != 0:
        raise ValueError("orc_forward_paths rejected its arguments")
    return out


def forward_gather(pos: np.ndarray, w: np.ndarray, points: np.ndarray, n_threads: int = 0):
    """Mean, variance over paths and magnitude scale of the connection of every
    point to every forward-path vertex (pos: (n_paths, M, dim), w: (n_paths, M))."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    pts = np.ascontiguousarray(points, dtype=np.float64)
    n_paths, M, dim = pos.shape
    P = pts.shape[0]
    mean, var, sabs = np.zeros(P), np.zeros(P), np.zeros(P)
    rc = lib().orc_forward_gather(C.c_int(dim), C.c_int64(n_paths), C.c_int(M), _ptr(pos), _ptr(w),
                                  _ptr(pts), C.c_int64(P), _ptr(mean), _ptr(var), _ptr(sabs),
                                  C.c_int(n_threads))
    if rc != 0:
        raise ValueError("orc_forward_gather rejected its arguments")
    return mean, var, sabs


def intersect_all(mesh: OracleMesh, orig: np.ndarray, dirs: np.ndarray,
                  exclude: Optional[np.ndarray] = None, max_hits: int = 64, n_threads: int = 0):
    o = np.ascontiguousarray(orig, dtype=np.float64)
    d = np.ascontiguousarray(dirs, dtype=np.float64)
    ex = None if exclude is None else np.ascontiguousarray(exclude, dtype=np.int32)
    n = o.shape[0]
    nh = np.zeros(n, dtype=np.int32)
    hp = np.full((n, max_hits), -1, dtype=np.int32)
    ht = np.zeros((n, max_hits))
    hm = np.zeros((n, max_hits))
    lg = np.zeros(n)
    rc = lib().orc_intersect_all(mesh.ref, _ptr(o), _ptr(d), _ptr(ex), C.c_int64(n),
                                 C.c_int(max_hits), _ptr(nh), _ptr(hp), _ptr(ht), _ptr(hm),
                                 _ptr(lg), C.c_int(n_threads))
    if rc != 0:
        raise ValueError("orc_intersect_all rejected its arguments")
    return {"n_hits": nh, "prim": hp, "t": ht, "margin": hm, "graze": lg}


def self_panel(mesh: OracleMesh, prim: int, x: np.ndarray, u0: float, u1: float):
    xx = np.zeros(3)
    xx[: mesh.dim] = x
    y = np.zeros(3)
    gp = lib().orc_self_panel(mesh.ref, int(prim), xx.ctypes.data, float(u0), float(u1), y.ctypes.data)
    return gp, y[: mesh.dim]


def boundary_datum(mesh: OracleMesh, bc: _BC, prim: int, y: np.ndarray) -> float:
    yy = np.zeros(3)
    yy[: mesh.dim] = y
    return lib().orc_boundary_datum(mesh.ref, C.byref(bc), int(prim), yy.ctypes.data)


def program_value(mesh: OracleMesh, bc: _BC, y: np.ndarray) -> float:
    yy = np.zeros(3)
    yy[: mesh.dim] = y
    return lib().orc_program_value(mesh.ref, C.byref(bc), yy.ctypes.data)


# --------------------------------------------------------------------------- control variate

def prim_potential(mesh: OracleMesh, prim: int, x: np.ndarray) -> float:
    xx = np.zeros(3)
    xx[: mesh.dim] = x
    return lib().orc_prim_potential(mesh.ref, int(prim), xx.ctypes.data)


def cv_addback(mesh: OracleMesh, g: np.ndarray, points: np.ndarray, seed: int = 0,
               randomized: bool = False, n_threads: int = 0) -> np.ndarray:
    gg = np.ascontiguousarray(g, dtype=np.float64)
    pts = np.ascontiguousarray(points, dtype=np.float64)
    out = np.zeros(pts.shape[0])
    if lib().orc_cv_addback(mesh.ref, gg.ctypes.data, pts.ctypes.data, pts.shape[0],
                            C.c_uint32(seed & 0xffffffff), int(randomized), out.ctypes.data,
                            n_threads) != 0:
        raise ValueError("orc_cv_addback rejected its arguments")
    return out


def trace_cv(mesh: OracleMesh, points, point_prim, bc: _BC, walk_len: int, seed: int, g,
             item_point, item_path, problem: int = 0, n_threads: int = 0, g0=None,
             with_scales: bool = False):
    """Corrected per-path values; g0 (line-0 table) defaults to g.  With
    with_scales, a dict of the values, their magnitude sums and rounding-error
    bounds (units of u)."""
    pts = np.ascontiguousarray(points, dtype=np.float64)
    pp = None if point_prim is None else np.ascontiguousarray(point_prim, dtype=np.int32)
    gg = np.ascontiguousarray(g, dtype=np.float64)
    g00 = None if g0 is None else np.ascontiguousarray(g0, dtype=np.float64)
    ip = np.ascontiguousarray(item_point, dtype=np.int64)
    ik = np.ascontiguousarray(item_path, dtype=np.int64)
    out = np.zeros(ip.shape[0])
    sabs, err = np.zeros(ip.shape[0]), np.zeros(ip.shape[0])
    rc = lib().orc_trace_cv(mesh.ref, _ptr(pts), _ptr(pp), pts.shape[0], C.byref(bc), int(walk_len),
                            C.c_uint64(seed), C.c_uint32(problem), _ptr(gg), _ptr(g00), ip.shape[0], _ptr(ip),
                            _ptr(ik), _ptr(out), _ptr(sabs), _ptr(err), int(n_threads))
    if rc != 0:
        raise ValueError("orc_trace_cv rejected its arguments")
    if with_scales:
        return {"value": out, "abs_sum": sabs, "err": err}
    return out


# --------------------------------------------------------------------------- MLP

def mlp_n_params(n_freq: int = 16, hidden: int = 128, layers: int = 4) -> int:
    return int(lib().orc_mlp_n_params(n_freq, hidden, layers))


def mlp_forward(params, Bmat, y, bf16: bool, n_freq=16, hidden=128, layers=4) -> np.ndarray:
    P = np.ascontiguousarray(params, dtype=np.float64)
    B = np.ascontiguousarray(Bmat, dtype=np.float64)
    Y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros(Y.shape[0])
    lib().orc_mlp_forward(P.ctypes.data, B.ctypes.data, n_freq, hidden, layers, Y.shape[1], Y.shape[0],
                          Y.ctypes.data, int(bf16), out.ctypes.data)
    return out


def mlp_forward_bound(params, Bmat, y, acc, dy=None, n_freq=16, hidden=128, layers=4) -> dict:
    """The bfloat16-rounded forward pass with, per row, the output layer's
    magnitude sum ("scale"), the first-order bound of a device evaluation's
    deviation ("bound": binary32 accumulation and bfloat16 rounding flips,
    through the exact sensitivities) and the count of activations at risk of a
    flip ("risk").  acc = (first hidden layer, other hidden layers, output):
    each layer's accumulation error bound in units of u32 times the magnitude
    sum of its terms.  dy: per row, the half-width of each input coordinate
    (an input computed on the device to within dy), or None."""
    P = np.ascontiguousarray(params, dtype=np.float64)
    B = np.ascontiguousarray(Bmat, dtype=np.float64)
    Y = np.ascontiguousarray(y, dtype=np.float64)
    n = Y.shape[0]
    out, scale, bound = np.zeros(n), np.zeros(n), np.zeros(n)
    risk = np.zeros(n, dtype=np.int32)
    DY = None if dy is None else np.ascontiguousarray(np.broadcast_to(dy, (n,)), dtype=np.float64)
    lib().orc_mlp_forward_bound(P.ctypes.data, B.ctypes.data, n_freq, hidden, layers, Y.shape[1], n,
                                Y.ctypes.data, None if DY is None else DY.ctypes.data, float(acc[0]), float(acc[1]), float(acc[2]), out.ctypes.data,
                                scale.ctypes.data, bound.ctypes.data, risk.ctypes.data)
    return {"out": out, "scale": scale, "bound": bound, "risk": risk}


def mlp_loss_grad(params, Bmat, y, target, bf16: bool, n_freq=16, hidden=128, layers=4):
    P = np.ascontiguousarray(params, dtype=np.float64)
    B = np.ascontiguousarray(Bmat, dtype=np.float64)
    Y = np.ascontiguousarray(y, dtype=np.float64)
    T = np.ascontiguousarray(target, dtype=np.float64)
    grad = np.zeros(P.shape[0])
    loss = lib().orc_mlp_loss_grad(P.ctypes.data, B.ctypes.data, n_freq, hidden, layers, Y.shape[1],
                                   Y.shape[0], Y.ctypes.data, T.ctypes.data, int(bf16), grad.ctypes.data)
    return loss, grad


def adam_step(params, m, v, grad, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(grad, dtype=np.float64)
    lib().orc_adam_step(params.ctypes.data, m.ctypes.data, v.ctypes.data, g.ctypes.data, params.shape[0],
                        int(step), lr, b1, b2, eps)


def bf16_round(x: float) -> float:
    return lib().orc_bf16_round(float(x))
