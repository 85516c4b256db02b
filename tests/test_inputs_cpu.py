"""Synthetic-input generators that decide which points a workload holds (CPU)."""
import numpy as np

from paper_2305_04403_amd import inputs as I


def winding_number(verts, prims, p):
    """Sum of the signed solid angles of the triangles seen from p over 4 pi
    (Van Oosterom-Strackee), by brute force."""
    A, B, C = (verts[prims[:, k]] - p for k in range(3))
    a, b, c = (np.linalg.norm(X, axis=1) for X in (A, B, C))
    num = np.einsum("ij,ij->i", A, np.cross(B, C))
    den = (a * b * c + np.einsum("ij,ij->i", A, B) * c + np.einsum("ij,ij->i", A, C) * b +
           np.einsum("ij,ij->i", B, C) * a)
    return np.sum(2.0 * np.arctan2(num, den)) / (4.0 * np.pi)


def test_inside_star_mesh_equals_winding_number():
    mesh = I.perturb_radial(I.icosphere(8), 0.1, 3, 4).as_float32_geometry()
    rng = np.random.default_rng(4)
    # points in a shell around the surface, where the decision is close
    d = rng.standard_normal((1500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    pts = d * rng.uniform(0.8, 1.2, (1500, 1))
    ins = I.inside_star_mesh(mesh, pts)
    wn = np.array([winding_number(mesh.verts, mesh.prims, p) for p in pts])
    assert np.all(np.abs(wn - np.round(wn)) < 1e-9)
    np.testing.assert_array_equal(ins, np.round(wn) == 1)
    assert 0.2 < ins.mean() < 0.8


def test_icosphere_slice_keeps_every_inside_cell():
    w = I.config_icosphere_slice(res=64)
    grid = I.slice_grid(64, 1.1).astype(np.float32).astype(np.float64)
    wn = np.array([winding_number(w.mesh.verts, w.mesh.prims, p) for p in grid])
    np.testing.assert_array_equal(np.sort(np.nonzero(np.round(wn) == 1)[0]).size, w.points.shape[0])
