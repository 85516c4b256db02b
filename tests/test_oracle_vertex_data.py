"""Pins of the oracle's per-vertex boundary data (eq. PoissonBC's g, q, g_R
given at mesh vertices and interpolated linearly on each primitive), against
closed forms and against the analytic programs where the two coincide."""
import numpy as np
import pytest

import oracle
from paper_2305_04403_amd import inputs as I


def _paths(om, pts, bc, N, M, seed, pp=None):
    P = pts.shape[0]
    return oracle.trace(om, pts, pp, bc, M, seed, np.repeat(np.arange(P), N), np.tile(np.arange(N), P),
                        want_pos=False)


@pytest.mark.parametrize("M", [1, 3, 6])
def test_linear_vertex_data_equals_the_linear_program_path_for_path(M):
    """A linear function restricted to a flat triangle is linear, so its P1
    interpolant from the vertex values is the function itself: every path of
    the double-layer walk (interior Dirichlet, perturbed icosphere) equals the
    path with the analytic linear program, to rounding."""
    mesh = I.perturb_radial(I.icosphere(6), 0.1, 3, 4)
    om = oracle.OracleMesh(mesh)
    a, b = np.array([0.3, -1.1, 0.7]), 0.25
    vd = mesh.verts @ a + b
    pts = I.ball_points(20, 0.8, 2)
    ref = _paths(om, pts, oracle.make_bc(1, oracle.DOUBLE_LAYER, oracle.PROG_LINEAR, (*a, b)), 32, M, 7)
    got = _paths(om, pts, oracle.make_bc(1, oracle.DOUBLE_LAYER, oracle.PROG_LINEAR, (*a, b), vertex_data=vd),
                 32, M, 7)
    np.testing.assert_array_equal(got["vtx_prim"], ref["vtx_prim"])
    assert np.all(np.abs(got["value"] - ref["value"]) <= 1e-12 * ref["abs_sum"])
    # and a boundary point returns the interpolated value (Table 1, Dirichlet)
    on, onp = I.mesh_surface_points(mesh, 5, 3)
    g = _paths(om, on, oracle.make_bc(1, oracle.DOUBLE_LAYER, oracle.PROG_CONST, (0.0,), vertex_data=vd),
               2, M, 1, pp=onp)
    np.testing.assert_allclose(g["value"], np.repeat(on @ a + b, 2), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("name,kind,alpha,datum,form", [
    ("direct Neumann", 1, 0.0, -1.0, oracle.DIRECT),
    ("single-layer Neumann", 1, 0.0, -1.0, oracle.SINGLE_LAYER),
    ("single-layer Robin", 2, 0.5, -0.5, oracle.SINGLE_LAYER),
])
def test_constant_vertex_data_on_the_exterior_sphere(name, kind, alpha, datum, form):
    """Exterior sphere with the flux of u = 1/|x| given at the vertices: q = -1
    (Neumann) or q + u/2 = -1/2 (Robin, alpha = 1/2).  The l = 0 recursion
    eigenvalue is -1 (Neumann) or 0 (Robin), so M = 3 is exact for the monopole;
    the polyhedral problem's flux is the mesh area A, so the mean must sit within
    4 SE of A / (4 pi |x|) plus the O(h^2) of the higher moments."""
    s = I.icosphere(8)
    mesh = I.Mesh(3, s.verts, s.prims, np.full(s.n_prims, kind, np.uint8), np.full(s.n_prims, alpha))
    om = oracle.OracleMesh(mesh)
    vd = np.full(mesh.verts.shape[0], datum)
    pts = I.ball_points(24, 2.5, 3, r_min=1.5)
    bc = oracle.make_bc(-1, form, oracle.PROG_CONST, (0.0,), vertex_data=vd)
    N = 3000
    mean, var = oracle.solve(om, pts, None, bc, N, 3, 5)
    tri = mesh.verts[mesh.prims]
    area = 0.5 * np.linalg.norm(np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0]), axis=1).sum()
    exact = area / (4 * np.pi) / np.linalg.norm(pts, axis=1)
    w = N / var
    est = np.sum(w * mean / exact) / np.sum(w)
    se = 1.0 / np.sqrt(np.sum(w * exact ** 2))
    assert abs(est - 1.0) < 4 * se + 0.01, (name, est, se)


def test_quadratic_vertex_data_on_the_circle_converges():
    """2D interior Dirichlet on the 256-gon with x^2 - y^2 given at the vertices
    (its linear interpolant on each segment differs by O(h^2) = 6e-4): the mean
    is within 4 SE + 2e-3 of the analytic solution, as with the program."""
    mesh = I.circle_polygon(256)
    om = oracle.OracleMesh(mesh)
    vd = mesh.verts[:, 0] ** 2 - mesh.verts[:, 1] ** 2
    pts = I.disk_points(40, 0.8, 4)
    bc = oracle.make_bc(1, oracle.DOUBLE_LAYER, oracle.PROG_QUAD, (), vertex_data=vd)
    N = 4000
    mean, var = oracle.solve(om, pts, None, bc, N, 4, 2)
    exact = pts[:, 0] ** 2 - pts[:, 1] ** 2
    z = np.abs(mean - exact) / np.sqrt(var / N + 1e-30)
    assert np.all(np.abs(mean - exact) < 4 * np.sqrt(var / N) + 2e-3), (z.max(), np.abs(mean - exact).max())


def test_vertex_data_requires_the_array():
    mesh = I.icosphere(2)
    om = oracle.OracleMesh(mesh)
    bc = oracle.make_bc(1, oracle.DOUBLE_LAYER, oracle.PROG_CONST, (1.0,))
    bc.data_mode = 1
    with pytest.raises(ValueError):
        oracle.solve(om, I.ball_points(2, 0.5, 1), None, bc, 4, 2, 0)
