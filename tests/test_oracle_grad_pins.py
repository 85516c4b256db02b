"""Pins of the oracle's gradient estimators (Sec. 4.1.3: the gradient is
estimated with the same paths, the kernel of the first step replaced by its
gradient in the evaluation point) against closed forms.

On a sphere or circle the gradient of each harmonic degree comes out with the
same truncation factor tau_M as the value, so a wrong derivative kernel (a sign,
a missing n_y term, a factor D) or a derivative that leaks into later steps
moves a target.  CPU only.
"""
import numpy as np
import pytest

import oracle
from paper_2305_04403_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _build(oracle_lib):
    return oracle_lib


def _fit(g, gv, ref, N):
    w = N / np.maximum(gv, 1e-300)
    est = np.sum(w * g * ref) / np.sum(w * ref * ref)
    return est, 1.0 / np.sqrt(np.sum(w * ref * ref))


def test_double_layer_gradient_sphere_truncation_factors():
    """Interior Dirichlet on the unit sphere with u = z: the gradient estimate
    is tau_M e_z with tau_1 = 2/3, tau_2 = 10/9, tau_4 = 82/81 (the value's
    factors, Sec. 4.1.2), through the hypersingular kernel grad dG/dn_y."""
    om = oracle.OracleMesh(I.icosphere(6))
    pts = I.ball_points(16, 0.5, 9)
    bc = oracle.make_bc(1, oracle.DOUBLE_LAYER, oracle.PROG_LINEAR, (0.0, 0.0, 1.0, 0.0))
    ref = np.tile([0.0, 0.0, 1.0], (16, 1))
    for M, tau in ((1, 2 / 3), (2, 10 / 9), (4, 82 / 81)):
        N = 4000
        _, _, g, gv = oracle.solve_grad(om, pts, bc, N, M, 3 + M)
        est, se = _fit(g, gv, ref, N)
        assert abs(est - tau) < 4 * se + 0.01, (M, est, tau, se)
        # the other components vanish
        assert np.all(np.abs(g[:, :2]) < 4.5 * np.sqrt(gv[:, :2] / N) + 0.01)


def test_double_layer_gradient_circle():
    """Interior Dirichlet on the 256-gon with u = x^2 - y^2: grad u = (2x, -2y)
    scaled by tau_1 = 1/2 and tau_M = 1 for M >= 2 (the double-layer kernel is
    constant on a circle)."""
    om = oracle.OracleMesh(I.circle_polygon(256))
    pts = I.disk_points(16, 0.7, 4)
    bc = oracle.make_bc(1, oracle.DOUBLE_LAYER, oracle.PROG_QUAD, ())
    ref = np.stack([2 * pts[:, 0], -2 * pts[:, 1]], axis=1)
    for M, tau in ((1, 0.5), (3, 1.0)):
        N = 4000
        _, _, g, gv = oracle.solve_grad(om, pts, bc, N, M, 7)
        est, se = _fit(g, gv, ref, N)
        assert abs(est - tau) < 4 * se + 0.01, (M, est, tau, se)


@pytest.mark.parametrize("name,form,sampling,N", [
    ("single layer, lines", oracle.SINGLE_LAYER, oracle.SAMPLE_LINE, 20000),
    ("single layer, RIS", oracle.SINGLE_LAYER, oracle.SAMPLE_RIS, 6000),
    ("direct BIE", oracle.DIRECT, oracle.SAMPLE_LINE, 6000),
])
def test_neumann_gradient_exterior_monopole(name, form, sampling, N):
    """Exterior Neumann, u = 1/|x| on a sphere (lambda_0 = -1: exact for every
    M): grad u = -x / |x|^3 per point and component within 4.5 SE (the single
    layer's first weight has an infinite-variance tail, hence more paths)."""
    s = I.icosphere(6)
    mesh = I.Mesh(3, s.verts, s.prims, np.full(s.n_prims, 1, np.uint8))
    om = oracle.OracleMesh(mesh)
    pts = I.ball_points(12, 2.5, 3, r_min=1.5)
    bc = oracle.make_bc(-1, form, oracle.PROG_INVDIST, (0.0, 0.0, 0.0), sampling=sampling)
    _, _, g, gv = oracle.solve_grad(om, pts, bc, N, 3, 6)
    exact = -pts / np.linalg.norm(pts, axis=1)[:, None] ** 3
    z = (g - exact) / np.sqrt(gv / N)
    assert np.max(np.abs(z)) < 4.5, (name, z)
    assert abs(np.sum(g * exact) / np.sum(exact * exact) - 1.0) < 0.03, name


def test_gradient_matches_finite_differences():
    """A perturbed sphere, interior Dirichlet with off-centre data, M = 3: the
    mean gradient equals the central difference (h = 0.02) of the mean value
    along each axis, the two sides of the difference sharing their paths."""
    mesh = I.perturb_radial(I.icosphere(6), 0.1, 2, 3)
    om = oracle.OracleMesh(mesh)
    bc = oracle.make_bc(1, oracle.DOUBLE_LAYER, oracle.PROG_INVDIST, (2.0, 0.5, 0.0))
    x0 = np.array([[0.2, -0.1, 0.15], [-0.3, 0.25, -0.1]])
    N, M, h = 20000, 3, 0.02
    _, _, g, gv = oracle.solve_grad(om, x0, bc, N, M, 9)
    for p in range(2):
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            pts = np.stack([x0[p] + e, x0[p] - e])
            items = np.arange(N)
            vp = oracle.trace(om, pts, None, bc, M, 9, np.zeros(N, np.int64), items, want_pos=False)["value"]
            vm = oracle.trace(om, pts, None, bc, M, 9, np.ones(N, np.int64), items, want_pos=False)["value"]
            d = (vp - vm) / (2 * h)
            fd, fd_se = d.mean(), d.std(ddof=1) / np.sqrt(N)
            z = (g[p, a] - fd) / np.sqrt(gv[p, a] / N + fd_se ** 2)
            assert abs(z) < 4.5, (p, a, g[p, a], fd, z)


def test_gradient_paths_keep_their_values():
    """The value of every path is unchanged by the gradient bookkeeping, and
    the per-path records agree with the solve's statistics."""
    mesh = I.perturb_radial(I.icosphere(5), 0.1, 2, 3)
    om = oracle.OracleMesh(mesh)
    pts = I.ball_points(5, 0.6, 2)
    for form, prog, dom, params in ((oracle.DOUBLE_LAYER, oracle.PROG_INVDIST, 1, (2.0, 0.5, 0.0)),):
        bc = oracle.make_bc(dom, form, prog, params)
        N, M = 64, 3
        ip = np.repeat(np.arange(5), N)
        ik = np.tile(np.arange(N), 5)
        t = oracle.trace(om, pts, None, bc, M, 4, ip, ik, want_pos=False)
        tg = oracle.trace_grad(om, pts, bc, M, 4, ip, ik)
        assert np.array_equal(t["value"], tg["value"])
        mean, var, g, gv = oracle.solve_grad(om, pts, bc, N, M, 4)
        assert np.allclose(g, tg["grad"].reshape(5, N, 3).mean(axis=1), rtol=1e-12, atol=1e-14)
        assert np.allclose(mean, t["value"].reshape(5, N).mean(axis=1), rtol=1e-12, atol=1e-14)


def test_gradient_rejects_density_mode():
    om = oracle.OracleMesh(I.icosphere(2))
    bc = oracle.make_bc(1, oracle.DOUBLE_LAYER, oracle.PROG_CONST, (1.0,), density=True)
    with pytest.raises(ValueError):
        oracle.solve_grad(om, np.zeros((1, 3)), bc, 4, 2, 1)


def _inward_points(mesh, n, depth, seed):
    """Points at distance `depth` inside a closed triangle mesh: area-uniform
    boundary points moved along the inward normal of their triangle."""
    on, prim = I.mesh_surface_points(mesh, n, seed)
    v, t = mesh.verts, mesh.prims[prim]
    nrm = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    return on - depth * nrm


def test_boundary_split_is_exact_for_constant_data_on_a_convex_body():
    """Constant Dirichlet data on a convex polyhedron: every line from a
    boundary point meets it once more, with weight -1, so the walk's density
    estimate is the same number from every start; the coupled walk from the
    anchor then cancels the first step's hypersingular weight exactly and
    every split gradient sample is 0 (the gradient of a constant), while the
    plain samples are not."""
    s = I.icosphere(6)
    om = oracle.OracleMesh(s)
    pts = np.concatenate([_inward_points(s, 12, 0.01, 1), I.ball_points(8, 0.5, 2)])
    A, AP = I.nearest_boundary_points(s, pts, inset=1e-3)
    bc = oracle.make_bc(1, oracle.DOUBLE_LAYER, oracle.PROG_CONST, (1.3,))
    N = 32
    ip, ik = np.repeat(np.arange(len(pts)), N), np.tile(np.arange(N), len(pts))
    r = oracle.trace_grad(om, pts, bc, 3, 5, ip, ik, anchors=A, anchor_prim=AP)
    r0 = oracle.trace_grad(om, pts, bc, 3, 5, ip, ik)
    assert np.all(np.abs(r["grad"]) <= 1e-12 * r["grad_abs"][:, None])
    assert np.median(np.abs(r0["grad"])) > 0.1
    np.testing.assert_array_equal(r["value"], r0["value"])


@pytest.mark.parametrize("anchor_kind", ["nearest", "random"])
def test_boundary_split_is_unbiased(anchor_kind):
    """u = z on the unit sphere, M = 2: the split gradient keeps the plain
    estimator's mean tau_2 e_z (10/9) whatever boundary point anchors it (the
    first step's derivative weight has mean zero); points with anchor -1 keep
    their plain samples."""
    s = I.icosphere(6)
    om = oracle.OracleMesh(s)
    pts = np.concatenate([_inward_points(s, 10, 0.05, 3), I.ball_points(6, 0.5, 4)])
    if anchor_kind == "nearest":
        A, AP = I.nearest_boundary_points(s, pts, inset=1e-3)
    else:
        A, AP = I.mesh_surface_points(s, len(pts), 5)
    AP = AP.astype(np.int32)
    AP[-1] = -1
    bc = oracle.make_bc(1, oracle.DOUBLE_LAYER, oracle.PROG_LINEAR, (0.0, 0.0, 1.0, 0.0))
    N = 4000
    _, _, g, gv = oracle.solve_grad(om, pts, bc, N, 2, 6, anchors=A, anchor_prim=AP)
    ref = np.tile([0.0, 0.0, 1.0], (len(pts), 1))
    est, se = _fit(g, gv, ref, N)
    assert abs(est - 10 / 9) < 4 * se + 0.01, (est, se)
    _, _, g0, gv0 = oracle.solve_grad(om, pts, bc, N, 2, 6)
    np.testing.assert_array_equal(g[-1], g0[-1])


def test_boundary_split_lowers_the_variance_near_the_boundary():
    """Interior Dirichlet on the perturbed icosphere (g = 1/|x - x0|), points
    0.003 inside the boundary, M = 4: with the split at the nearest boundary
    point the gradient's variance falls well below the plain estimator's (the
    hypersingular first step no longer multiplies the whole density estimate,
    only its difference from the coupled walk's)."""
    m = I.perturb_radial(I.icosphere(10), 0.1, 3, 4)
    om = oracle.OracleMesh(m)
    pts = _inward_points(m, 16, 0.003, 7)
    A, AP = I.nearest_boundary_points(m, pts, inset=1e-3)
    bc = oracle.make_bc(1, oracle.DOUBLE_LAYER, oracle.PROG_INVDIST, (2.0, 0.5, 0.0))
    _, _, g0, gv0 = oracle.solve_grad(om, pts, bc, 1000, 4, 9)
    _, _, g1, gv1 = oracle.solve_grad(om, pts, bc, 1000, 4, 9, anchors=A, anchor_prim=AP)
    ratio = gv1.sum(1) / gv0.sum(1)
    print("variance ratio per point", np.round(ratio, 3))
    assert np.median(ratio) < 0.3
