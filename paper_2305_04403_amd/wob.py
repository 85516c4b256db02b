"""Thin Python binding of libwob.so (argument marshalling only).

Every step of the walk runs in the HIP kernels of ``libwob.so``; this module
only turns torch device tensors into raw device pointers, passes torch's
current HIP stream, and checks status codes.  It raises if the library is
missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwob.so")

F32, F64 = 0, 1
AUTO, DOUBLE_LAYER, DIRECT, SINGLE_LAYER = 0, 1, 2, 3
PROG_CONST, PROG_LINEAR, PROG_QUAD, PROG_INVDIST = 0, 1, 2, 3
DATA_PROGRAM, DATA_VERTEX = 0, 1
DIRICHLET, NEUMANN, ROBIN = 0, 1, 2
SAMPLE_LINE, SAMPLE_RIS = 0, 1

EXPORTED = ("wob_build_bvh", "wob_build_bvh_ex", "wob_free", "wob_get_scene_info", "wob_lines_per_path", "wob_solve",
            "wob_solve_ordered", "wob_solve_ordered_workspace", "wob_trace", "wob_intersect_all", "wob_count_work", "wob_status_string",
            "wob_batch_create", "wob_batch_launch", "wob_batch_autotune", "wob_batch_get_tune",
            "wob_batch_free", "wob_solve_batched", "wob_solve_batched_static", "wob_mlp_n_params",
            "wob_mlp_create",
            "wob_mlp_free", "wob_mlp_get_params", "wob_mlp_set_params", "wob_mlp_get_moments",
            "wob_mlp_set_moments", "wob_mlp_forward",
            "wob_mlp_backward", "wob_mlp_adam_step", "wob_mlp_train_step", "wob_cv_table",
            "wob_solve_cv", "wob_trace_cv", "wob_cv_addback", "wob_cv_emission", "wob_sample_boundary",
            "wob_starts_create", "wob_starts_from_data", "wob_starts_free", "wob_forward_paths",
            "wob_forward_gather", "wob_solve_grad", "wob_trace_grad", "wob_last_device_status",
            "wob_gather_probe", "wob_mfma_probe")


class WobError(RuntimeError):
    pass


class _BC(C.Structure):
    _fields_ = [("domain", C.c_int32), ("formulation", C.c_int32), ("program", C.c_int32),
                ("density", C.c_int32), ("sampling", C.c_int32), ("candidates", C.c_int32),
                ("params", C.c_double * 8), ("self_panel_p", C.c_double), ("mixed_k", C.c_double),
                ("mixed_p", C.c_double), ("data_mode", C.c_int32), ("path_offset", C.c_int32),
                ("vertex_data", C.c_void_p)]


class _SceneInfo(C.Structure):
    _fields_ = [("dim", C.c_int32), ("precision", C.c_int32), ("n_prims", C.c_int64),
                ("n_nodes", C.c_int64), ("n_leaves", C.c_int64), ("depth", C.c_int32),
                ("max_leaf", C.c_int32), ("device_bytes", C.c_int64), ("node_bytes", C.c_int64),
                ("prim_bytes", C.c_int64), ("n_dirichlet", C.c_int32), ("n_neumann", C.c_int32),
                ("n_robin", C.c_int32), ("reserved", C.c_int32), ("n_verts", C.c_int64)]


class _Problem(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("points", C.c_void_p), ("point_prim", C.c_void_p),
                ("n_points", C.c_int64), ("bc", _BC), ("samples", C.c_int32),
                ("walk_len", C.c_int32), ("seed", C.c_uint64), ("stream_id", C.c_uint32),
                ("reserved", C.c_int32), ("mean_out", C.c_void_p), ("var_out", C.c_void_p)]


class _Tune(C.Structure):
    _fields_ = [("block", C.c_int32), ("blocks_per_cu", C.c_int32)]


class _TargetMap(C.Structure):
    _fields_ = [("shift", C.c_float), ("scale", C.c_float), ("clip", C.c_float)]


def _tmap(m):
    return None if m is None else C.byref(_TargetMap(float(m[0]), float(m[1]), float(m[2])))


_lib = None


def lib():
    """Load libwob.so (built by ``python -m paper_2305_04403_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise WobError(f"{LIB_PATH} is missing: build it with `python -m paper_2305_04403_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    L.wob_build_bvh.argtypes = [i32, i32, vp, i64, vp, i64, vp, vp, C.POINTER(vp)]
    L.wob_build_bvh_ex.argtypes = [i32, i32, vp, i64, vp, i64, vp, vp, i32, vp, C.POINTER(vp)]
    L.wob_free.argtypes = [vp]
    L.wob_free.restype = None
    L.wob_get_scene_info.argtypes = [vp, C.POINTER(_SceneInfo)]
    L.wob_lines_per_path.argtypes = [vp, C.POINTER(_BC), i32]
    L.wob_lines_per_path.restype = i32
    L.wob_solve.argtypes = [vp, vp, vp, i64, C.POINTER(_BC), i32, i32, u64, vp, vp, vp]
    L.wob_solve_ordered.argtypes = [vp, vp, vp, i64, C.POINTER(_BC), i32, i32, u64, vp, vp, vp, C.c_size_t, vp]
    L.wob_solve_ordered_workspace.argtypes = [vp, i64, C.POINTER(C.c_size_t)]
    L.wob_trace.argtypes = [vp, vp, vp, i64, C.POINTER(_BC), i32, i32, u64, vp, vp, vp, vp, vp]
    L.wob_count_work.argtypes = [vp, vp, vp, i64, C.POINTER(_BC), i32, i32, u64, vp, vp]
    L.wob_intersect_all.argtypes = [vp, vp, vp, vp, i64, i32, vp, vp, vp, vp]
    L.wob_batch_create.argtypes = [C.POINTER(_Problem), i32, C.POINTER(_Tune), C.POINTER(vp)]
    L.wob_batch_launch.argtypes = [vp, vp]
    L.wob_batch_autotune.argtypes = [vp, i32, C.c_char_p, C.POINTER(_Tune), vp]
    L.wob_batch_get_tune.argtypes = [vp, C.POINTER(_Tune), C.POINTER(i64)]
    L.wob_batch_free.argtypes = [vp]
    L.wob_batch_free.restype = None
    L.wob_solve_batched.argtypes = [C.POINTER(_Problem), i32, C.POINTER(_Tune), vp]
    L.wob_solve_batched_static.argtypes = [C.POINTER(_Problem), i32, C.POINTER(_Tune), vp]
    for name in ("wob_batch_create", "wob_batch_launch", "wob_batch_autotune",
                 "wob_batch_get_tune", "wob_solve_batched", "wob_solve_batched_static"):
        getattr(L, name).restype = C.c_int
    L.wob_mlp_n_params.argtypes = []
    L.wob_mlp_n_params.restype = i64
    L.wob_mlp_create.argtypes = [i32, vp, vp, i64, C.POINTER(vp)]
    L.wob_mlp_free.argtypes = [vp]
    L.wob_mlp_free.restype = None
    L.wob_mlp_get_params.argtypes = [vp, vp]
    L.wob_mlp_set_params.argtypes = [vp, vp]
    L.wob_mlp_get_moments.argtypes = [vp, vp, vp]
    L.wob_mlp_set_moments.argtypes = [vp, vp, vp]
    L.wob_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
    L.wob_mlp_backward.argtypes = [vp, vp, vp, C.POINTER(_TargetMap), i64, vp, vp, vp]
    L.wob_mlp_adam_step.argtypes = [vp, vp, i64, C.c_float, C.c_float, C.c_float, C.c_float, vp]
    L.wob_mlp_train_step.argtypes = [vp, vp, vp, C.POINTER(_TargetMap), i64, i64, C.c_float, vp, vp]
    for name in ("wob_mlp_create", "wob_mlp_get_params", "wob_mlp_set_params", "wob_mlp_get_moments",
                 "wob_mlp_set_moments", "wob_mlp_forward",
                 "wob_mlp_backward", "wob_mlp_adam_step", "wob_mlp_train_step", "wob_cv_table",
            "wob_solve_cv", "wob_trace_cv", "wob_cv_addback", "wob_sample_boundary"):
        getattr(L, name).restype = C.c_int
    L.wob_cv_table.argtypes = [vp, vp, vp, vp]
    L.wob_sample_boundary.argtypes = [vp, i64, u64, vp, vp, vp]
    L.wob_sample_boundary.restype = C.c_int
    L.wob_solve_cv.argtypes = [vp, vp, vp, i64, C.POINTER(_BC), i32, i32, u64, vp, vp, vp, vp, vp]
    L.wob_trace_cv.argtypes = [vp, vp, vp, i64, C.POINTER(_BC), i32, i32, u64, vp, vp, vp, vp]
    L.wob_cv_addback.argtypes = [vp, vp, vp, i64, u64, vp, vp]
    L.wob_cv_emission.argtypes = [vp, C.POINTER(_BC), vp, vp, vp]
    for name in ("wob_cv_table", "wob_solve_cv", "wob_trace_cv", "wob_cv_addback", "wob_cv_emission"):
        getattr(L, name).restype = C.c_int
    L.wob_gather_probe.argtypes = [vp, i64, i64, i32, C.c_uint32, vp, vp]
    L.wob_gather_probe.restype = C.c_int
    L.wob_mfma_probe.argtypes = [vp, vp, vp, vp, i64, vp]
    L.wob_mfma_probe.restype = C.c_int
    L.wob_last_device_status.argtypes = [vp, C.POINTER(C.c_uint64), vp]
    L.wob_last_device_status.restype = C.c_int
    L.wob_solve_grad.argtypes = [vp, vp, i64, C.POINTER(_BC), i32, i32, u64, vp, vp, vp, vp, vp, vp, vp]
    L.wob_solve_grad.restype = C.c_int
    L.wob_trace_grad.argtypes = [vp, vp, i64, C.POINTER(_BC), i32, i32, u64, vp, vp, vp, vp, vp]
    L.wob_trace_grad.restype = C.c_int
    L.wob_starts_create.argtypes = [vp, vp, C.POINTER(vp)]
    L.wob_starts_create.restype = C.c_int
    L.wob_starts_from_data.argtypes = [vp, C.POINTER(_BC), C.c_double, C.POINTER(vp)]
    L.wob_starts_from_data.restype = C.c_int
    L.wob_starts_free.argtypes = [vp]
    L.wob_starts_free.restype = None
    L.wob_forward_paths.argtypes = [vp, C.POINTER(_BC), vp, i64, i32, u64, vp, vp, vp, vp]
    L.wob_forward_paths.restype = C.c_int
    L.wob_forward_gather.argtypes = [vp, vp, i64, i32, vp, i64, vp, vp, vp]
    L.wob_forward_gather.restype = C.c_int
    L.wob_status_string.argtypes = [C.c_int]
    L.wob_status_string.restype = C.c_char_p
    for name in ("wob_build_bvh", "wob_build_bvh_ex", "wob_get_scene_info", "wob_solve", "wob_solve_ordered",
                 "wob_solve_ordered_workspace", "wob_trace",
                 "wob_count_work", "wob_intersect_all"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(status: int, what: str):
    if status != 0:
        msg = lib().wob_status_string(status).decode()
        raise WobError(f"{what}: {msg} (status {status})")


@dataclasses.dataclass
class BC:
    """Boundary data and formulation (mirrors ``wob_bc``)."""
    domain: int = 1               # +1 interior, -1 exterior
    formulation: int = AUTO
    program: int = PROG_CONST
    params: Sequence[float] = ()
    self_panel_p: float = 1.0 / 16.0
    density: bool = False
    sampling: int = 0             # SAMPLE_LINE or SAMPLE_RIS (single layer)
    candidates: int = 0           # RIS candidates (0 = 16)
    mixed_k: float = 0.0          # Dirichlet parts of the single layer: k (0 = 4)
    mixed_p: float = 0.0          # and p_k (0 = 2/3)
    vertex_data: object = None    # per-vertex data (device tensor of the scene's dtype,
                                  # one value per mesh vertex): replaces program/params
    path_offset: int = 0          # path k draws the random numbers of path path_offset + k

    def c(self, scene: "Scene") -> _BC:
        b = _BC()
        if self.vertex_data is not None:
            _need(self.vertex_data, "vertex_data", scene.dtype, (scene.n_verts,), scene.device)
            b.data_mode, b.vertex_data = DATA_VERTEX, self.vertex_data.data_ptr()
        b.domain, b.formulation, b.program = self.domain, self.formulation, self.program
        b.density = int(bool(self.density))
        b.sampling, b.candidates = int(self.sampling), int(self.candidates)
        b.mixed_k, b.mixed_p = float(self.mixed_k), float(self.mixed_p)
        b.path_offset = int(self.path_offset)
        for i, v in enumerate(self.params):
            b.params[i] = float(v)
        b.self_panel_p = float(self.self_panel_p)
        return b


def _torch():
    import torch
    return torch


def _dev_ptr(t) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise WobError("expected a device tensor")
    if not t.is_contiguous():
        raise WobError("expected a contiguous tensor")
    return t.data_ptr()


def _stream(stream=None) -> Optional[int]:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _need(t, name: str, dtype, shape, device: Optional[int] = None, optional: bool = False):
    """Raise WobError unless t is a tensor of `dtype` and `shape` (None entries
    match any size) on the CUDA device `device`, contiguous.  Checked before any
    call into the library: a kernel reads its arrays at the sizes the call
    states, so a mismatched tensor would be read past its end."""
    if t is None:
        if optional:
            return
        raise WobError(f"{name}: a tensor is required")
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise WobError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise WobError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if t.dim() != len(shape) or any(e is not None and int(a) != int(e) for a, e in zip(t.shape, shape)):
        want = "(" + ", ".join("*" if e is None else str(e) for e in shape) + ")"
        raise WobError(f"{name}: shape {tuple(t.shape)}, expected {want}")
    if not t.is_cuda:
        raise WobError(f"{name}: expected a device tensor")
    if device is not None and t.device.index != device:
        raise WobError(f"{name}: on cuda:{t.device.index}, the scene lives on cuda:{device}")
    if not t.is_contiguous():
        raise WobError(f"{name}: expected a contiguous tensor")


def _need_points(scene, points, name: str = "points") -> int:
    """(P, dim) points of the scene's dtype on its device; returns P."""
    torch = _torch()
    if not isinstance(points, torch.Tensor):
        raise WobError(f"{name}: expected a torch tensor")
    _need(points, name, scene.dtype, (None, scene.dim), scene.device)
    return int(points.shape[0])


class Scene:
    """A boundary mesh uploaded to the current device with its line-query BVH
    (``wob_build_bvh``; with ``stream``, ``wob_build_bvh_ex`` copying on it)."""

    def __init__(self, mesh, precision: int = F32, stream=None):
        verts = np.ascontiguousarray(mesh.verts, dtype=np.float64)
        prims = np.ascontiguousarray(mesh.prims, dtype=np.int32)
        kind = None if mesh.kind is None else np.ascontiguousarray(mesh.kind, dtype=np.uint8)
        alpha = None if mesh.alpha is None else np.ascontiguousarray(mesh.alpha, dtype=np.float64)
        if verts.ndim != 2 or verts.shape[1] != mesh.dim or prims.shape != (prims.shape[0], mesh.dim):
            raise WobError("mesh: verts (V, dim) and prims (T, dim) expected")
        for a, name in ((kind, "kind"), (alpha, "alpha")):
            if a is not None and a.shape != (prims.shape[0],):
                raise WobError(f"mesh.{name}: one entry per primitive expected")
        h = C.c_void_p()
        args = (int(mesh.dim), int(precision), verts.ctypes.data, verts.shape[0], prims.ctypes.data,
                prims.shape[0], None if kind is None else kind.ctypes.data,
                None if alpha is None else alpha.ctypes.data)
        if stream is None:
            _check(lib().wob_build_bvh(*args, C.byref(h)), "wob_build_bvh")
        else:
            _check(lib().wob_build_bvh_ex(*args, 0, _stream(stream), C.byref(h)), "wob_build_bvh_ex")
        self._adopt(h, mesh.dim, precision, prims.shape[0], verts.shape[0])

    def _adopt(self, h, dim, precision, n_prims, n_verts):
        self.handle = h
        self.dim = int(dim)
        self.precision = int(precision)
        self.n_prims = int(n_prims)
        self.n_verts = int(n_verts)
        self.device = _torch().cuda.current_device()  # the library builds on the current device

    @classmethod
    def from_device(cls, dim: int, verts, prims, kind=None, alpha=None, precision: int = F32, stream=None):
        """A scene from device-resident mesh arrays (``wob_build_bvh_ex``):
        verts (V, dim) float64, prims (T, dim) int32, kind (T,) uint8 or None,
        alpha (T,) float64 or None, all on the current device.  Waits for
        ``stream`` (the current stream if None)."""
        dev = _torch().cuda.current_device()
        _need(verts, "verts", _torch().float64, (None, dim), dev)
        _need(prims, "prims", _torch().int32, (None, dim), dev)
        T = int(prims.shape[0])
        _need(kind, "kind", _torch().uint8, (T,), dev, optional=True)
        _need(alpha, "alpha", _torch().float64, (T,), dev, optional=True)
        h = C.c_void_p()
        _check(lib().wob_build_bvh_ex(int(dim), int(precision), verts.data_ptr(), int(verts.shape[0]),
                                      prims.data_ptr(), T, None if kind is None else kind.data_ptr(),
                                      None if alpha is None else alpha.data_ptr(), 1, _stream(stream),
                                      C.byref(h)), "wob_build_bvh_ex")
        self = cls.__new__(cls)
        self._adopt(h, dim, precision, T, int(verts.shape[0]))
        return self

    @property
    def dtype(self):
        torch = _torch()
        return torch.float32 if self.precision == F32 else torch.float64

    def info(self) -> dict:
        i = _SceneInfo()
        _check(lib().wob_get_scene_info(self.handle, C.byref(i)), "wob_get_scene_info")
        return {f: getattr(i, f) for f, _ in _SceneInfo._fields_ if f != "reserved"}

    def nonfinite_paths(self, stream=None) -> int:
        """Non-finite path values left out of solves on this scene since the
        last call (``wob_last_device_status``; resets the count)."""
        v = C.c_uint64()
        _check(lib().wob_last_device_status(self.handle, C.byref(v), _stream(stream)), "wob_last_device_status")
        return int(v.value)

    def lines_per_path(self, bc: BC, walk_len: int) -> int:
        b = bc.c(self)
        n = lib().wob_lines_per_path(self.handle, C.byref(b), int(walk_len))
        if n < 0:
            raise WobError("wob_lines_per_path: invalid arguments")
        return n

    def close(self):
        if getattr(self, "handle", None):
            lib().wob_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve(scene: Scene, points, bc: BC, samples: int, walk_len: int, seed: int = 0,
          point_prim=None, want_var: bool = True, stream=None, out=None, ordered: bool = False,
          workspace=None):
    """Per-point mean (and variance) of ``samples`` WoB paths.  ``points`` is a
    contiguous (P, dim) device tensor of the scene's dtype.  ``ordered``: walk
    the points in a locality order (``wob_solve_ordered``; the same paths, the
    statistics equal to the summation's rounding), in ``workspace`` (a uint8
    device tensor of at least ``ordered_workspace_bytes`` bytes) or in one
    allocated here."""
    torch = _torch()
    P = _need_points(scene, points)
    _need(point_prim, "point_prim", torch.int32, (P,), scene.device, optional=True)
    if out is None:
        mean = torch.empty(P, dtype=scene.dtype, device=points.device)
        var = torch.empty(P, dtype=scene.dtype, device=points.device) if want_var else None
    else:
        mean, var = out
        _need(mean, "mean out", scene.dtype, (P,), scene.device)
        _need(var, "var out", scene.dtype, (P,), scene.device, optional=True)
    b = bc.c(scene)
    if ordered:
        need = ordered_workspace_bytes(scene, P)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device=points.device)
        _need(workspace, "workspace", torch.uint8, (None,), scene.device)
        st = lib().wob_solve_ordered(scene.handle, _dev_ptr(points), _dev_ptr(point_prim), P, C.byref(b),
                                     int(samples), int(walk_len), C.c_uint64(seed), _dev_ptr(mean),
                                     _dev_ptr(var), _dev_ptr(workspace), workspace.numel(), _stream(stream))
        _check(st, "wob_solve_ordered")
        return mean, var
    st = lib().wob_solve(scene.handle, _dev_ptr(points), _dev_ptr(point_prim), P, C.byref(b),
                         int(samples), int(walk_len), C.c_uint64(seed), _dev_ptr(mean),
                         _dev_ptr(var), _stream(stream))
    _check(st, "wob_solve")
    return mean, var


def ordered_workspace_bytes(scene: Scene, n_points: int) -> int:
    """Device workspace bytes of an ordered solve of ``n_points`` points
    (``wob_solve_ordered_workspace``)."""
    n = C.c_size_t(0)
    _check(lib().wob_solve_ordered_workspace(scene.handle, int(n_points), C.byref(n)),
           "wob_solve_ordered_workspace")
    return int(n.value)


class Starts:
    """Start distribution of forward paths on a scene: primitive T with
    probability weight[T] / sum(weight), uniform inside T (``wob_starts_create``),
    or weights (|q(c_T)| + floor * mean |q|) A_T from the data of ``data``
    (``wob_starts_from_data``)."""

    def __init__(self, scene: Scene, weight=None, data: Optional["BC"] = None, floor: float = 0.0):
        h = C.c_void_p()
        if data is not None:
            b = data.c(scene)
            _check(lib().wob_starts_from_data(scene.handle, C.byref(b), float(floor), C.byref(h)),
                   "wob_starts_from_data")
        else:
            w = np.ascontiguousarray(weight, dtype=np.float64)
            _check(lib().wob_starts_create(scene.handle, w.ctypes.data, C.byref(h)), "wob_starts_create")
        self.handle = h
        self.scene = scene

    def close(self):
        if self.handle:
            lib().wob_starts_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def forward_paths(scene: Scene, bc: BC, n_paths: int, walk_len: int, seed: int = 0, starts=None,
                  want_vertices: bool = False, stream=None, out=None):
    """Forward single-layer paths from the boundary (``wob_forward_paths``):
    (n_paths, walk_len, 4) records (y, strength), plus the vertices' primitives
    and line hit counts when ``want_vertices``."""
    torch = _torch()
    dev = torch.device("cuda", scene.device)
    if out is not None:
        _need(out, "out", scene.dtype, (n_paths, walk_len, 4), scene.device)
    vtx = out if out is not None else torch.empty((n_paths, walk_len, 4), dtype=scene.dtype, device=dev)
    vp = torch.empty((n_paths, walk_len), dtype=torch.int32, device=dev) if want_vertices else None
    vm = torch.empty((n_paths, walk_len), dtype=torch.int32, device=dev) if want_vertices else None
    b = bc.c(scene)
    st = lib().wob_forward_paths(scene.handle, C.byref(b), None if starts is None else starts.handle,
                                 int(n_paths), int(walk_len), C.c_uint64(seed), _dev_ptr(vtx),
                                 _dev_ptr(vp), _dev_ptr(vm), _stream(stream))
    _check(st, "wob_forward_paths")
    return vtx, vp, vm


def forward_gather(scene: Scene, vtx, points, want_var: bool = True, stream=None, out=None):
    """Connect every point to every forward-path vertex (``wob_forward_gather``):
    per-point mean and variance over the paths of ``vtx`` (n_paths, walk_len, 4)."""
    torch = _torch()
    P = _need_points(scene, points)
    _need(vtx, "vtx", scene.dtype, (None, None, 4), scene.device)
    if out is None:
        mean = torch.empty(P, dtype=scene.dtype, device=points.device)
        var = torch.empty(P, dtype=scene.dtype, device=points.device) if want_var else None
    else:
        mean, var = out
        _need(mean, "mean out", scene.dtype, (P,), scene.device)
        _need(var, "var out", scene.dtype, (P,), scene.device, optional=True)
    st = lib().wob_forward_gather(scene.handle, _dev_ptr(vtx), int(vtx.shape[0]), int(vtx.shape[1]),
                                  _dev_ptr(points), P, _dev_ptr(mean), _dev_ptr(var), _stream(stream))
    _check(st, "wob_forward_gather")
    return mean, var


def _need_anchors(scene, P, anchors, anchor_prim):
    """Boundary-split anchors: both or neither; (P, dim) of the scene's dtype
    and (P,) int32 on its device."""
    torch = _torch()
    if (anchors is None) != (anchor_prim is None):
        raise WobError("anchors and anchor_prim go together")
    _need(anchors, "anchors", scene.dtype, (P, scene.dim), scene.device, optional=True)
    _need(anchor_prim, "anchor_prim", torch.int32, (P,), scene.device, optional=True)


def solve_grad(scene: Scene, points, bc: BC, samples: int, walk_len: int, seed: int = 0,
               want_var: bool = True, stream=None, anchors=None, anchor_prim=None):
    """Per-point mean value and gradient (and variances) along the same paths
    (``wob_solve_grad``); points off the boundary.  anchors / anchor_prim
    (double layer): per point a boundary point and its primitive id (-1: none)
    for the boundary split of the gradient."""
    torch = _torch()
    P, D = _need_points(scene, points), scene.dim
    _need_anchors(scene, P, anchors, anchor_prim)
    mean = torch.empty(P, dtype=scene.dtype, device=points.device)
    grad = torch.empty((P, D), dtype=scene.dtype, device=points.device)
    var = torch.empty(P, dtype=scene.dtype, device=points.device) if want_var else None
    gvar = torch.empty((P, D), dtype=scene.dtype, device=points.device) if want_var else None
    b = bc.c(scene)
    st = lib().wob_solve_grad(scene.handle, _dev_ptr(points), P, C.byref(b), int(samples), int(walk_len),
                              C.c_uint64(seed), _dev_ptr(anchors), _dev_ptr(anchor_prim), _dev_ptr(mean),
                              _dev_ptr(var), _dev_ptr(grad), _dev_ptr(gvar), _stream(stream))
    _check(st, "wob_solve_grad")
    return mean, var, grad, gvar


def trace_grad(scene: Scene, points, bc: BC, samples: int, walk_len: int, seed: int = 0, stream=None,
               anchors=None, anchor_prim=None):
    """Per-path values (P, samples) and gradients (P, samples, dim) (``wob_trace_grad``)."""
    torch = _torch()
    P, D = _need_points(scene, points), scene.dim
    _need_anchors(scene, P, anchors, anchor_prim)
    path = torch.empty((P, samples), dtype=scene.dtype, device=points.device)
    pg = torch.empty((P, samples, D), dtype=scene.dtype, device=points.device)
    b = bc.c(scene)
    st = lib().wob_trace_grad(scene.handle, _dev_ptr(points), P, C.byref(b), int(samples), int(walk_len),
                              C.c_uint64(seed), _dev_ptr(anchors), _dev_ptr(anchor_prim), _dev_ptr(path),
                              _dev_ptr(pg), _stream(stream))
    _check(st, "wob_trace_grad")
    return path, pg


def mfma_probe(a, b, c, stream=None):
    """D = A B + C per tile on the network's bfloat16 matrix instruction
    (``wob_mfma_probe``): a (T, 16, 32) and b (T, 32, 16) bfloat16, c
    (T, 16, 16) float32, all on one device; returns d like c."""
    torch = _torch()
    if not isinstance(a, torch.Tensor):
        raise WobError("a: expected a torch tensor")
    T = int(a.shape[0]) if a.dim() == 3 else -1
    dev = a.device.index if a.is_cuda else None
    _need(a, "a", torch.bfloat16, (T, 16, 32), dev)
    _need(b, "b", torch.bfloat16, (T, 32, 16), dev)
    _need(c, "c", torch.float32, (T, 16, 16), dev)
    d = torch.empty_like(c)
    _check(lib().wob_mfma_probe(a.data_ptr(), b.data_ptr(), c.data_ptr(), d.data_ptr(), T, _stream(stream)),
           "wob_mfma_probe")
    return d


def gather_probe(buf, lanes: int, reads: int, seed: int = 0, out=None, stream=None):
    """Random 32-byte gathers from the device buffer ``buf`` (``wob_gather_probe``):
    returns one float per lane (the sum of all eight floats of each record
    read)."""
    torch = _torch()
    if not isinstance(buf, torch.Tensor) or not buf.is_cuda or not buf.is_contiguous():
        raise WobError("buf: expected a contiguous device tensor")
    if out is None:
        out = torch.empty(lanes, dtype=torch.float32, device=buf.device)
    _need(out, "out", torch.float32, (lanes,), buf.device.index)
    st = lib().wob_gather_probe(_dev_ptr(buf), buf.numel() * buf.element_size(), int(lanes), int(reads),
                                C.c_uint32(seed), _dev_ptr(out), _stream(stream))
    _check(st, "wob_gather_probe")
    return out


def trace(scene: Scene, points, bc: BC, samples: int, walk_len: int, seed: int = 0,
          point_prim=None, want_vertices: bool = True, point_ids=None, stream=None):
    """Per-path values (P, samples) plus, optionally, the primitive picked and the
    hit count of every line.  ``point_ids`` (uint32 stored in an int32 tensor)
    replaces the point index used in the random-number counter."""
    torch = _torch()
    P = _need_points(scene, points)
    _need(point_prim, "point_prim", torch.int32, (P,), scene.device, optional=True)
    _need(point_ids, "point_ids", torch.int32, (P,), scene.device, optional=True)
    L = scene.lines_per_path(bc, walk_len)
    path = torch.empty((P, samples), dtype=scene.dtype, device=points.device)
    vp = torch.empty((P, samples, L), dtype=torch.int32, device=points.device) if want_vertices else None
    vm = torch.empty((P, samples, L), dtype=torch.int32, device=points.device) if want_vertices else None
    b = bc.c(scene)
    st = lib().wob_trace(scene.handle, _dev_ptr(points), _dev_ptr(point_prim), P, C.byref(b),
                         int(samples), int(walk_len), C.c_uint64(seed), _dev_ptr(point_ids),
                         _dev_ptr(path), _dev_ptr(vp), _dev_ptr(vm), _stream(stream))
    _check(st, "wob_trace")
    return path, vp, vm


def count_work(scene: Scene, points, bc: BC, samples: int, walk_len: int, seed: int = 0,
               point_prim=None, stream=None):
    torch = _torch()
    P = _need_points(scene, points)
    _need(point_prim, "point_prim", torch.int32, (P,), scene.device, optional=True)
    c = torch.zeros(4, dtype=torch.int64, device=points.device)
    b = bc.c(scene)
    st = lib().wob_count_work(scene.handle, _dev_ptr(points), _dev_ptr(point_prim), points.shape[0],
                              C.byref(b), int(samples), int(walk_len), C.c_uint64(seed),
                              _dev_ptr(c), _stream(stream))
    _check(st, "wob_count_work")
    v = c.cpu().numpy()
    return {"lines": int(v[0]), "nodes": int(v[1]), "prims": int(v[2]), "hits": int(v[3])}


def intersect_all(scene: Scene, orig, dirs, exclude=None, max_hits: int = 64, stream=None):
    torch = _torch()
    n = _need_points(scene, orig, "orig")
    _need(dirs, "dirs", scene.dtype, (n, scene.dim), scene.device)
    _need(exclude, "exclude", torch.int32, (n,), scene.device, optional=True)
    nh = torch.empty(n, dtype=torch.int32, device=orig.device)
    hp = torch.full((n, max_hits), -1, dtype=torch.int32, device=orig.device)
    ht = torch.zeros((n, max_hits), dtype=scene.dtype, device=orig.device)
    st = lib().wob_intersect_all(scene.handle, _dev_ptr(orig), _dev_ptr(dirs), _dev_ptr(exclude), n,
                                 int(max_hits), _dev_ptr(nh), _dev_ptr(hp), _dev_ptr(ht),
                                 _stream(stream))
    _check(st, "wob_intersect_all")
    return nh, hp, ht


class Batch:
    """Many problems solved by one persistent launch replayed from a hipGraph.

    ``problems``: list of dicts with keys scene, points, bc, samples, walk_len and
    optionally point_prim, seed, stream_id, want_var.  Output tensors are
    allocated here; the batch keeps every tensor alive."""

    def __init__(self, problems, tune=None):
        torch = _torch()
        self._keep = []
        self.outputs = []
        arr = (_Problem * len(problems))()
        for i, p in enumerate(problems):
            scene, pts = p["scene"], p["points"]
            P = _need_points(scene, pts, f"problem {i} points")
            _need(p.get("point_prim"), f"problem {i} point_prim", torch.int32, (P,), scene.device, optional=True)
            mean = torch.empty(P, dtype=scene.dtype, device=pts.device)
            var = torch.empty(P, dtype=scene.dtype, device=pts.device) if p.get("want_var", True) else None
            pp = p.get("point_prim")
            self._keep += [scene, pts, pp, mean, var]
            self.outputs.append((mean, var))
            arr[i].scene = scene.handle
            arr[i].points = _dev_ptr(pts)
            arr[i].point_prim = _dev_ptr(pp)
            arr[i].n_points = P
            arr[i].bc = p["bc"].c(scene)
            arr[i].samples = int(p["samples"])
            arr[i].walk_len = int(p["walk_len"])
            arr[i].seed = int(p.get("seed", 0))
            arr[i].stream_id = int(p.get("stream_id", 0))
            arr[i].reserved = 0
            arr[i].mean_out = _dev_ptr(mean)
            arr[i].var_out = _dev_ptr(var)
        t = None if tune is None else _Tune(*tune)
        h = C.c_void_p()
        _check(lib().wob_batch_create(arr, len(problems), None if t is None else C.byref(t), C.byref(h)),
               "wob_batch_create")
        self.handle = h

    def launch(self, stream=None):
        _check(lib().wob_batch_launch(self.handle, _stream(stream)), "wob_batch_launch")
        return self.outputs

    def autotune(self, sample_stride: int = 16, cache_path: Optional[str] = None, stream=None):
        t = _Tune()
        path = None if cache_path is None else cache_path.encode()
        _check(lib().wob_batch_autotune(self.handle, int(sample_stride), path, C.byref(t), _stream(stream)),
               "wob_batch_autotune")
        return (t.block, t.blocks_per_cu)

    def tune(self):
        t = _Tune()
        n = C.c_int64()
        _check(lib().wob_batch_get_tune(self.handle, C.byref(t), C.byref(n)), "wob_batch_get_tune")
        return (t.block, t.blocks_per_cu), n.value

    def close(self):
        if getattr(self, "handle", None):
            lib().wob_batch_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _problem_table(problems):
    """ctypes problem array for the batched entry points (outputs: the dicts'
    "mean_out" / "var_out" tensors, allocated here when absent)."""
    torch = _torch()
    arr = (_Problem * len(problems))()
    outs, keep = [], []
    for i, p in enumerate(problems):
        scene, pts = p["scene"], p["points"]
        P = _need_points(scene, pts, f"problem {i} points")
        pp = p.get("point_prim")
        _need(pp, f"problem {i} point_prim", torch.int32, (P,), scene.device, optional=True)
        mean = p.get("mean_out")
        var = p.get("var_out")
        if mean is None:
            mean = torch.empty(P, dtype=scene.dtype, device=pts.device)
            if var is None and p.get("want_var", True):
                var = torch.empty(P, dtype=scene.dtype, device=pts.device)
        _need(mean, f"problem {i} mean_out", scene.dtype, (P,), scene.device)
        _need(var, f"problem {i} var_out", scene.dtype, (P,), scene.device, optional=True)
        keep += [scene, pts, pp, mean, var]
        outs.append((mean, var))
        arr[i].scene = scene.handle
        arr[i].points = _dev_ptr(pts)
        arr[i].point_prim = _dev_ptr(pp)
        arr[i].n_points = P
        arr[i].bc = p["bc"].c(scene)
        arr[i].samples = int(p["samples"])
        arr[i].walk_len = int(p["walk_len"])
        arr[i].seed = int(p.get("seed", 0))
        arr[i].stream_id = int(p.get("stream_id", 0))
        arr[i].reserved = 0
        arr[i].mean_out = _dev_ptr(mean)
        arr[i].var_out = _dev_ptr(var)
    return arr, outs, keep


def solve_batched(problems, tune=None, stream=None, no_alloc: bool = False):
    """One-shot batched solve (``wob_solve_batched``), or with ``no_alloc``
    ``wob_solve_batched_static``, which allocates no device memory (at most
    ``STATIC_MAX_PROBLEMS`` problems).  Problems as for :class:`Batch`, plus
    optional caller-owned "mean_out" / "var_out" tensors.  Returns the
    per-problem (mean, var) outputs; waits for the stream."""
    arr, outs, _keep = _problem_table(problems)
    t = None if tune is None else C.byref(_Tune(*tune))
    fn = lib().wob_solve_batched_static if no_alloc else lib().wob_solve_batched
    _check(fn(arr, len(problems), t, _stream(stream)),
           "wob_solve_batched_static" if no_alloc else "wob_solve_batched")
    return outs


STATIC_MAX_PROBLEMS = 256


class MLP:
    """The control-variate network on the device (parameters owned by the library)."""

    def __init__(self, dim: int, fourier: np.ndarray, params: np.ndarray, max_batch: int = 0):
        f = np.ascontiguousarray(fourier, dtype=np.float32)
        p = np.ascontiguousarray(params, dtype=np.float32)
        n = lib().wob_mlp_n_params()
        if p.shape != (n,) or f.shape != (16, dim):
            raise WobError("MLP: wrong parameter or Fourier-matrix shape")
        h = C.c_void_p()
        _check(lib().wob_mlp_create(int(dim), f.ctypes.data, p.ctypes.data, int(max_batch), C.byref(h)),
               "wob_mlp_create")
        self.handle = h
        self.dim = dim
        self.n_params = n
        self.max_batch = max_batch

    def _need_batch(self, y, target):
        torch = _torch()
        _need(y, "y", torch.float32, (None, self.dim))
        _need(target, "target", torch.float32, (y.shape[0],), y.device.index)

    def params(self) -> np.ndarray:
        out = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().wob_mlp_get_params(self.handle, out.ctypes.data), "wob_mlp_get_params")
        return out

    def set_params(self, params: np.ndarray):
        p = np.ascontiguousarray(params, dtype=np.float32)
        _check(lib().wob_mlp_set_params(self.handle, p.ctypes.data), "wob_mlp_set_params")

    def moments(self):
        """The Adam moments (m, v): with params() the training state."""
        m = np.zeros(self.n_params, dtype=np.float32)
        v = np.zeros(self.n_params, dtype=np.float32)
        _check(lib().wob_mlp_get_moments(self.handle, m.ctypes.data, v.ctypes.data), "wob_mlp_get_moments")
        return m, v

    def set_moments(self, m: np.ndarray, v: np.ndarray):
        m = np.ascontiguousarray(m, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        if m.shape != (self.n_params,) or v.shape != (self.n_params,):
            raise WobError("MLP: wrong moment shape")
        _check(lib().wob_mlp_set_moments(self.handle, m.ctypes.data, v.ctypes.data), "wob_mlp_set_moments")

    def forward(self, y, out=None, stream=None):
        torch = _torch()
        _need(y, "y", torch.float32, (None, self.dim))
        if out is None:
            out = torch.empty(y.shape[0], dtype=torch.float32, device=y.device)
        _need(out, "out", torch.float32, (y.shape[0],), y.device.index)
        _check(lib().wob_mlp_forward(self.handle, _dev_ptr(y), y.shape[0], _dev_ptr(out), _stream(stream)),
               "wob_mlp_forward")
        return out

    def backward(self, y, target, target_map=None, stream=None):
        """target_map: (shift, scale, clip) applied to the targets inside the loss."""
        torch = _torch()
        self._need_batch(y, target)
        grad = torch.empty(self.n_params, dtype=torch.float32, device=y.device)
        loss = torch.empty(1, dtype=torch.float32, device=y.device)
        _check(lib().wob_mlp_backward(self.handle, _dev_ptr(y), _dev_ptr(target), _tmap(target_map),
                                      y.shape[0], _dev_ptr(grad), _dev_ptr(loss), _stream(stream)),
               "wob_mlp_backward")
        return loss, grad

    def adam_step(self, grad, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        _need(grad, "grad", _torch().float32, (self.n_params,))
        _check(lib().wob_mlp_adam_step(self.handle, _dev_ptr(grad), int(step), lr, b1, b2, eps,
                                       _stream(stream)), "wob_mlp_adam_step")

    def train_step(self, y, target, step: int, lr: float, loss=None, target_map=None, stream=None):
        self._need_batch(y, target)
        _need(loss, "loss", _torch().float32, (1,), y.device.index, optional=True)
        _check(lib().wob_mlp_train_step(self.handle, _dev_ptr(y), _dev_ptr(target), _tmap(target_map),
                                        y.shape[0], int(step), lr, _dev_ptr(loss), _stream(stream)),
               "wob_mlp_train_step")

    def close(self):
        if getattr(self, "handle", None):
            lib().wob_mlp_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------- control variate

def sample_boundary(scene: Scene, n: int, seed: int = 0, stream=None):
    """n area-uniform boundary points and their primitive ids (device tensors)."""
    torch = _torch()
    dev = torch.device("cuda", scene.device)
    pts = torch.empty((n, scene.dim), dtype=scene.dtype, device=dev)
    prim = torch.empty(n, dtype=torch.int32, device=dev)
    _check(lib().wob_sample_boundary(scene.handle, int(n), C.c_uint64(seed), _dev_ptr(pts), _dev_ptr(prim),
                                     _stream(stream)), "wob_sample_boundary")
    return pts, prim


def cv_table(scene: Scene, net: "MLP", stream=None):
    torch = _torch()
    g = torch.empty(scene.n_prims, dtype=torch.float32, device=torch.device("cuda", scene.device))
    _check(lib().wob_cv_table(scene.handle, net.handle, _dev_ptr(g), _stream(stream)), "wob_cv_table")
    return g


def cv_emission(scene: Scene, bc: BC, g=None, stream=None):
    """Line-0 table g0 = g + 2 phi s(centroid) (g None = 0)."""
    torch = _torch()
    _need(g, "g", torch.float32, (scene.n_prims,), scene.device, optional=True)
    g0 = torch.empty(scene.n_prims, dtype=torch.float32, device=torch.device("cuda", scene.device))
    b = bc.c(scene)
    _check(lib().wob_cv_emission(scene.handle, C.byref(b), _dev_ptr(g), _dev_ptr(g0), _stream(stream)),
           "wob_cv_emission")
    return g0


def solve_cv(scene: Scene, points, bc: BC, samples: int, walk_len: int, g, seed: int = 0,
             point_prim=None, want_var: bool = True, stream=None, out=None, g0=None):
    torch = _torch()
    P = _need_points(scene, points)
    _need(point_prim, "point_prim", torch.int32, (P,), scene.device, optional=True)
    _need(g, "g", torch.float32, (scene.n_prims,), scene.device)
    _need(g0, "g0", torch.float32, (scene.n_prims,), scene.device, optional=True)
    if out is None:
        mean = torch.empty(P, dtype=scene.dtype, device=points.device)
        var = torch.empty(P, dtype=scene.dtype, device=points.device) if want_var else None
    else:
        mean, var = out
        _need(mean, "mean out", scene.dtype, (P,), scene.device)
        _need(var, "var out", scene.dtype, (P,), scene.device, optional=True)
    b = bc.c(scene)
    _check(lib().wob_solve_cv(scene.handle, _dev_ptr(points), _dev_ptr(point_prim), P, C.byref(b),
                              int(samples), int(walk_len), C.c_uint64(seed), _dev_ptr(g), _dev_ptr(g0),
                              _dev_ptr(mean), _dev_ptr(var), _stream(stream)), "wob_solve_cv")
    return mean, var


def trace_cv(scene: Scene, points, bc: BC, samples: int, walk_len: int, g, seed: int = 0,
             point_prim=None, stream=None, g0=None):
    torch = _torch()
    P = _need_points(scene, points)
    _need(point_prim, "point_prim", torch.int32, (P,), scene.device, optional=True)
    _need(g, "g", torch.float32, (scene.n_prims,), scene.device)
    _need(g0, "g0", torch.float32, (scene.n_prims,), scene.device, optional=True)
    path = torch.empty((P, samples), dtype=scene.dtype, device=points.device)
    b = bc.c(scene)
    _check(lib().wob_trace_cv(scene.handle, _dev_ptr(points), _dev_ptr(point_prim), P, C.byref(b),
                              int(samples), int(walk_len), C.c_uint64(seed), _dev_ptr(g), _dev_ptr(g0),
                              _dev_ptr(path), _stream(stream)), "wob_trace_cv")
    return path


def cv_addback(scene: Scene, g, points, seed: int = 0, stream=None):
    torch = _torch()
    P = _need_points(scene, points)
    _need(g, "g", torch.float32, (scene.n_prims,), scene.device)
    out = torch.empty(P, dtype=scene.dtype, device=points.device)
    _check(lib().wob_cv_addback(scene.handle, _dev_ptr(g), _dev_ptr(points), points.shape[0],
                                C.c_uint64(seed), _dev_ptr(out), _stream(stream)),
           "wob_cv_addback")
    return out
