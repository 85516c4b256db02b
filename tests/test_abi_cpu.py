"""The C-ABI library loads, exports every entry point its header declares, and
rejects bad arguments on the host before touching a device (CPU only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2305_04403_amd import wob

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "wob.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(wob_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = wob.lib()
    names = declared()
    assert "wob_solve" in names and "wob_build_bvh" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(wob.EXPORTED) <= set(names)


def test_status_strings():
    L = wob.lib()
    assert L.wob_status_string(0) == b"ok"
    assert L.wob_status_string(1) == b"invalid argument"
    assert L.wob_status_string(99) == b"unknown status"


def _build(dim, prec, verts, prims, kind=None, alpha=None):
    L = wob.lib()
    v = np.ascontiguousarray(verts, np.float64)
    p = np.ascontiguousarray(prims, np.int32)
    k = None if kind is None else np.ascontiguousarray(kind, np.uint8)
    a = None if alpha is None else np.ascontiguousarray(alpha, np.float64)
    h = C.c_void_p()
    st = L.wob_build_bvh(dim, prec, v.ctypes.data, v.shape[0], p.ctypes.data, p.shape[0],
                         None if k is None else k.ctypes.data, None if a is None else a.ctypes.data,
                         C.byref(h))
    return st, h


def test_build_rejects_bad_meshes_on_host():
    tri = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0.0]])
    assert _build(4, 0, tri, [[0, 1, 2]])[0] == 1          # dim
    assert _build(3, 7, tri, [[0, 1, 2]])[0] == 1          # precision
    assert _build(3, 0, tri, [[0, 1, 3]])[0] == 4          # index out of range
    assert _build(3, 0, tri, [[0, 1, 1]])[0] == 4          # zero area
    assert _build(3, 0, np.array([[0, 0, 0], [1, 0, np.nan], [0, 1, 0.0]]), [[0, 1, 2]])[0] == 4
    assert _build(2, 0, np.array([[0, 0], [0, 0.0]]), [[0, 1]])[0] == 4  # zero length
    assert _build(3, 0, tri, [[0, 1, 2]], kind=[5])[0] == 1  # unknown kind
    # float32 rounding can make a tiny triangle degenerate
    tiny = np.array([[0, 0, 0], [1e-12, 0, 0], [0, 1e-12, 0.0]]) + 1.0
    assert _build(3, 0, tiny, [[0, 1, 2]])[0] == 4


def test_entry_points_reject_null_scene():
    L = wob.lib()
    bc = wob.BC().c(_StandInScene())
    assert L.wob_lines_per_path(None, C.byref(bc), 4) == -1
    assert L.wob_solve(None, None, None, 0, C.byref(bc), 4, 4, 0, None, None, None) == 1
    assert L.wob_trace(None, None, None, 0, C.byref(bc), 4, 4, 0, None, None, None, None, None) == 1
    assert L.wob_intersect_all(None, None, None, None, 1, 4, None, None, None, None) == 1
    assert L.wob_get_scene_info(None, None) == 1
    L.wob_free(None)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(wob, "_lib", None)
    monkeypatch.setattr(wob, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(wob.WobError):
        wob.lib()


class _StandInScene:
    """Attributes the binding validates against (no device scene behind it)."""
    dim, n_prims, n_verts, device, handle = 3, 10, 7, 0, None

    @property
    def dtype(self):
        import torch
        return torch.float32


@pytest.mark.parametrize("case", ["float64 points", "2-column points", "1-D points", "int64 point_prim",
                                  "short point_prim", "short mean out", "float64 table", "short table",
                                  "host tensor"])
def test_binding_rejects_mismatched_tensors_before_any_call(case):
    """Every entry point checks dtype, shape and device of its tensors against
    the scene before it calls into the library (a kernel would read a
    mismatched array past its end): WobError, and no library call."""
    torch = pytest.importorskip("torch")
    sc = _StandInScene()
    bc = wob.BC(1, wob.AUTO, wob.PROG_CONST, (1.0,))
    P = 5
    pts = torch.zeros((P, 3), dtype=torch.float32)
    calls = {
        "float64 points": lambda: wob.solve(sc, pts.double(), bc, 8, 2),
        "2-column points": lambda: wob.trace(sc, pts[:, :2].contiguous(), bc, 8, 2),
        "1-D points": lambda: wob.solve_grad(sc, pts.reshape(-1), bc, 8, 2),
        "int64 point_prim": lambda: wob.solve(sc, pts, bc, 8, 2, point_prim=torch.zeros(P, dtype=torch.int64)),
        "short point_prim": lambda: wob.count_work(sc, pts, bc, 8, 2, point_prim=torch.zeros(P - 1, dtype=torch.int32)),
        "short mean out": lambda: wob.solve(sc, pts, bc, 8, 2, out=(torch.zeros(P - 1), None)),
        "float64 table": lambda: wob.solve_cv(sc, pts, bc, 8, 2, g=torch.zeros(10, dtype=torch.float64)),
        "short table": lambda: wob.cv_addback(sc, torch.zeros(9), pts),
        "host tensor": lambda: wob.solve(sc, pts, bc, 8, 2),
    }
    with pytest.raises(wob.WobError):
        calls[case]()


@pytest.mark.parametrize("case,match", [("float64", "dtype"), ("short", "shape"), ("2-D", "shape"),
                                        ("host", "device tensor")])
def test_vertex_data_is_checked_against_the_scene(case, match):
    """Per-vertex data must be one value per scene vertex, of the scene's dtype,
    on its device: the kernels index it by vertex id."""
    import torch
    vd = {"float64": torch.zeros(7, dtype=torch.float64), "short": torch.zeros(6),
          "2-D": torch.zeros((7, 1)), "host": torch.zeros(7)}[case]
    with pytest.raises(wob.WobError, match=match):
        wob.BC(1, wob.AUTO, vertex_data=vd).c(_StandInScene())


_STRUCTS = [("wob_bc", "_BC"), ("wob_scene_info", "_SceneInfo"), ("wob_problem", "_Problem"),
            ("wob_tune", "_Tune"), ("wob_target_map", "_TargetMap")]


def test_binding_structs_match_the_header(tmp_path):
    """Every ctypes mirror of a header struct has the C layout: each field's
    offset and the total size, as a C compiler lays out include/wob.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    lines = ["#include <stddef.h>", "#include <stdio.h>", '#include "wob.h"', "int main(void) {"]
    want = {}
    for cname, pyname in _STRUCTS:
        st = getattr(wob, pyname)
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        want[f"{cname} size"] = C.sizeof(st)
        for f, _ in st._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
            want[f"{cname} {f}"] = getattr(st, f).offset
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    got = {ln.rsplit(" ", 1)[0]: int(ln.rsplit(" ", 1)[1]) for ln in out.splitlines()}
    assert got == want
