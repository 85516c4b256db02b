"""Pins of the oracle's forward (adjoint) single-layer estimator (Sec. 4.4
"Forward estimator") against closed forms and independent computations.

The forward walk samples the same truncated series as the backward walk
(Sec. 4.1.2), so on a sphere or circle each harmonic degree l comes out scaled
by tau_M = (1 - lambda) sum_{j<M} c_j lambda^j with c = (1, .., 1, 1/2) and the
recursion eigenvalue lambda_l of the Neumann row.  A dropped 1/2, a wrong sign
of the adjoint kernel, a start density without its P_T / A_T or a missing
factor 2 phi in the first weight each move one of these targets.  CPU only.
"""
import numpy as np
import pytest

import oracle
from paper_2305_04403_amd import inputs as I


@pytest.fixture(scope="module", autouse=True)
def _build(oracle_lib):
    return oracle_lib


def _neumann(mesh):
    return I.Mesh(mesh.dim, mesh.verts, mesh.prims, np.full(mesh.n_prims, 1, np.uint8))


def _fit_ratio(mean, var, ref, N):
    """Weighted least-squares factor tau in mean = tau * ref, and its SE."""
    w = N / np.maximum(var, 1e-300)
    est = np.sum(w * mean * ref) / np.sum(w * ref * ref)
    return est, 1.0 / np.sqrt(np.sum(w * ref * ref))


def _forward(om, bc, N, M, seed, points, weights=None):
    f = oracle.forward_paths(om, bc, N, M, seed, start_weight=weights)
    mean, var, _ = oracle.forward_gather(f["pos"], f["w"], points)
    return mean, var, f


def test_forward_sphere_truncation_factors():
    """Interior Neumann on the unit sphere with u = z (l = 1).  The single-layer
    Neumann row has lambda_1 = 1/(2l+1) = 1/3 there, so tau_1 = 1/3,
    tau_2 = 7/9, tau_3 = 25/27.  Without the halved last term tau_1 = 2/3 and
    tau_2 = 8/9; with the adjoint kernel's sign flipped tau_2 = 5/9."""
    om = oracle.OracleMesh(_neumann(I.icosphere(6)))
    pts = I.ball_points(16, 0.5, 9)
    bc = oracle.make_bc(1, oracle.SINGLE_LAYER, oracle.PROG_LINEAR, (0.0, 0.0, 1.0, 0.0))
    for M, tau in ((1, 1 / 3), (2, 7 / 9), (3, 25 / 27)):
        N = 30000
        mean, var, _ = _forward(om, bc, N, M, 3 + M, pts)
        est, se = _fit_ratio(mean, var, pts[:, 2], N)
        assert abs(est - tau) < 4 * se + 0.01, (M, est, tau, se)


def test_forward_circle_truncation_factors():
    """Interior Neumann on the unit circle with u = y: the Neumann row's kernel
    is constant on a circle, so lambda_l = 0 for l >= 1: tau_1 = 1/2 (the
    halved single term) and tau_M = 1 for M >= 2."""
    c = I.circle_polygon(128)
    om = oracle.OracleMesh(_neumann(c))
    pts = I.disk_points(16, 0.6, 4)
    bc = oracle.make_bc(1, oracle.SINGLE_LAYER, oracle.PROG_LINEAR, (0.0, 1.0, 0.0, 0.0))
    for M, tau in ((1, 0.5), (2, 1.0), (3, 1.0)):
        N = 30000
        mean, var, _ = _forward(om, bc, N, M, 3 + M, pts)
        est, se = _fit_ratio(mean, var, pts[:, 1], N)
        assert abs(est - tau) < 4 * se + 0.005, (M, est, tau, se)


def test_forward_exterior_sphere_monopole():
    """Exterior Neumann, u = 1/|x| on a sphere: lambda_0 = -1, the truncated
    series reproduces the l = 0 solution for every M (1/2, 1 - 1/2, ...)."""
    om = oracle.OracleMesh(_neumann(I.icosphere(6)))
    pts = I.ball_points(24, 2.5, 3, r_min=1.5)
    bc = oracle.make_bc(-1, oracle.SINGLE_LAYER, oracle.PROG_INVDIST, (0.0, 0.0, 0.0))
    exact = 1.0 / np.linalg.norm(pts, axis=1)
    for M in (1, 2, 3):
        N = 20000
        mean, var, _ = _forward(om, bc, N, M, 30 + M, pts)
        est, se = _fit_ratio(mean, var, exact, N)
        assert abs(est - 1.0) < 4 * se + 0.01, (M, est, se)


def _subdivided_centroids(verts, prims, levels):
    """Centroids and areas of each triangle split 4^levels times (midpoint rule)."""
    tri = verts[prims]  # (T, 3, 3)
    for _ in range(levels):
        a, b, c = tri[:, 0], tri[:, 1], tri[:, 2]
        ab, bc_, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
        tri = np.concatenate([np.stack(t, axis=1) for t in
                              ((a, ab, ca), (ab, b, bc_), (ca, bc_, c), (ab, bc_, ca))])
    cen = tri.mean(axis=1)
    area = 0.5 * np.linalg.norm(np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0]), axis=1)
    return cen, area, tri


@pytest.mark.parametrize("start", ["area", "abs_q", "random"])
def test_forward_first_term_is_the_single_layer_of_the_data(start):
    """M = 1: the estimate is (1/2) <G(x, .), 2 phi q> = phi int G q dA, for any
    start density.  The integral comes from a subdivided midpoint rule on the
    mesh (independent of the oracle); starts uniform by area, proportional to
    |q| A_T at the centroids, and proportional to arbitrary positive weights."""
    mesh = _neumann(I.perturb_radial(I.icosphere(5), 0.1, 2, 3))
    om = oracle.OracleMesh(mesh)
    c0 = np.array([0.2, -0.1, 0.05])
    bc = oracle.make_bc(-1, oracle.SINGLE_LAYER, oracle.PROG_INVDIST, tuple(c0))
    pts = I.ball_points(8, 2.5, 5, r_min=1.6)
    normals = om.normals()
    cen, area, tri = _subdivided_centroids(mesh.verts, mesh.prims, 3)
    parent = np.tile(np.arange(mesh.n_prims), 4 ** 3)
    r = cen - c0
    q = np.einsum("ij,ij->i", -r / np.linalg.norm(r, axis=1)[:, None] ** 3, normals[parent])
    G = 1.0 / (4 * np.pi * np.linalg.norm(pts[:, None, :] - cen[None], axis=2))
    exact = -1.0 * (G * (q * area)[None]).sum(axis=1)  # phi = -1
    weights = None
    if start == "abs_q":
        tc = mesh.verts[mesh.prims].mean(axis=1) - c0
        qc = np.einsum("ij,ij->i", -tc / np.linalg.norm(tc, axis=1)[:, None] ** 3, normals)
        a_t = 0.5 * np.linalg.norm(np.cross(mesh.verts[mesh.prims[:, 1]] - mesh.verts[mesh.prims[:, 0]],
                                            mesh.verts[mesh.prims[:, 2]] - mesh.verts[mesh.prims[:, 0]]), axis=1)
        weights = np.abs(qc) * a_t
    elif start == "random":
        weights = np.random.default_rng(2).uniform(0.1, 3.0, mesh.n_prims)
    N = 200000
    mean, var, _ = _forward(om, bc, N, 1, 77, pts, weights)
    z = (mean - exact) / np.sqrt(var / N)
    assert np.max(np.abs(z)) < 4.5, (start, z)


@pytest.mark.parametrize("dim", [2, 3])
def test_forward_matches_backward(dim):
    """Three terms of the series with no symmetry to lean on (a perturbed sphere,
    exterior, off-centre monopole; a perturbed circle, interior, quadratic data):
    the forward mean equals the backward single-layer mean of the same
    truncated series (pinned by its own closed forms) within 4.5 SE."""
    if dim == 3:
        mesh = _neumann(I.perturb_radial(I.icosphere(5), 0.1, 2, 3))
        bc = oracle.make_bc(-1, oracle.SINGLE_LAYER, oracle.PROG_INVDIST, (0.2, -0.1, 0.05))
        pts = I.ball_points(4, 2.2, 8, r_min=1.4)
    else:
        c = I.circle_polygon(96)
        ang = np.arctan2(c.verts[:, 1], c.verts[:, 0])
        v = c.verts * (1 + 0.1 * np.cos(3 * ang))[:, None]
        mesh = _neumann(I.Mesh(2, v, c.prims))
        bc = oracle.make_bc(1, oracle.SINGLE_LAYER, oracle.PROG_QUAD, ())
        pts = I.disk_points(4, 0.6, 8)
    om = oracle.OracleMesh(mesh)
    M, Nf, Nb = 3, 40000, 6000
    mf, vf, _ = _forward(om, bc, Nf, M, 11, pts)
    mb, vb = oracle.solve(om, pts, None, bc, Nb, M, 12)
    z = (mf - mb) / np.sqrt(vf / Nf + vb / Nb)
    assert np.max(np.abs(z)) < 4.5, z


def test_forward_weights_are_signed_hit_counts():
    """The adjoint kernel over the line density: W_{k+1} / W_k = phi m sgn(cos)
    with cos the angle at the new vertex between y_{k+1} - y_k and its normal,
    m the hits of the line; the last vertex carries half.  A path whose line
    finds no hit ends: zero strength and primitive -1 from there on."""
    mesh = _neumann(I.perturb_radial(I.icosphere(5), 0.1, 2, 3))
    om = oracle.OracleMesh(mesh)
    n = om.normals()
    for phi in (1, -1):
        bc = oracle.make_bc(phi, oracle.SINGLE_LAYER, oracle.PROG_INVDIST, (0.2, -0.1, 0.05))
        M = 4
        f = oracle.forward_paths(om, bc, 400, M, 5)
        c = np.array([1.0] * (M - 1) + [0.5])
        W = f["w"] / c
        for j in range(400):
            for k in range(1, M):
                if f["m"][j, k] == 0:
                    assert np.all(f["w"][j, k:] == 0) and np.all(f["prim"][j, k:] == -1)
                    break
                d = f["pos"][j, k] - f["pos"][j, k - 1]
                s = np.sign(d @ n[f["prim"][j, k]])
                assert W[j, k] / W[j, k - 1] == pytest.approx(phi * f["m"][j, k] * s, rel=1e-9)
    # an open surface (the upper half of a sphere): lines can miss it
    s = I.icosphere(4)
    keep = s.verts[s.prims].mean(axis=1)[:, 2] > 0
    om = oracle.OracleMesh(_neumann(I.Mesh(3, s.verts, s.prims[keep])))
    bc = oracle.make_bc(-1, oracle.SINGLE_LAYER, oracle.PROG_INVDIST, (0.2, -0.1, 0.05))
    f = oracle.forward_paths(om, bc, 400, 3, 5)
    assert np.all(f["w"][:, 0] != 0)
    ended = f["m"][:, 1] == 0
    assert ended.any() and (~ended).any()
    assert np.all(f["w"][ended, 1:] == 0) and np.all(f["prim"][ended, 1:] == -1)


def test_forward_starts_follow_the_weights():
    """Start primitives are drawn with probability w_T / sum w (chi-square over
    the primitives; zero weights never start a path) and uniformly inside the
    triangle (the barycentric coordinates of the start are uniform on the
    simplex)."""
    mesh = _neumann(I.icosphere(3))
    om = oracle.OracleMesh(mesh)
    T = mesh.n_prims
    w = np.random.default_rng(1).uniform(0.5, 2.0, T)
    w[::7] = 0.0
    bc = oracle.make_bc(1, oracle.SINGLE_LAYER, oracle.PROG_CONST, (1.0,))
    N = 200000
    f = oracle.forward_paths(om, bc, N, 1, 3, start_weight=w)
    cnt = np.bincount(f["prim"][:, 0], minlength=T)
    assert np.all(cnt[w == 0] == 0)
    e = N * w / w.sum()
    k = w > 0
    chi2 = np.sum((cnt[k] - e[k]) ** 2 / e[k])
    dof = int(k.sum()) - 1
    assert abs(chi2 - dof) < 5 * np.sqrt(2 * dof), (chi2, dof)
    # barycentric coordinates of the start point in its primitive
    v = mesh.verts[mesh.prims[f["prim"][:, 0]]]
    A = np.stack([v[:, 1] - v[:, 0], v[:, 2] - v[:, 0]], axis=2)
    ab = np.linalg.lstsq(A[0], (f["pos"][0, 0] - v[0, 0]), rcond=None)[0]
    assert ab.min() >= -1e-12 and ab.sum() <= 1 + 1e-12
    sol = np.einsum("nij,nj->ni", np.linalg.pinv(A), f["pos"][:, 0] - v[:, 0])
    a, b = sol[:, 0], sol[:, 1]
    assert a.min() > -1e-9 and b.min() > -1e-9 and (a + b).max() < 1 + 1e-9
    # uniform on the simplex: P(a < 1/2) = 3/4, E[a] = 1/3
    assert abs(np.mean(a < 0.5) - 0.75) < 5 * np.sqrt(0.75 * 0.25 / N)
    assert abs(np.mean(a) - 1 / 3) < 5 * np.sqrt(1 / 18 / N)


def test_forward_rejects_bad_arguments():
    mesh = I.icosphere(2)
    bc = oracle.make_bc(1, oracle.SINGLE_LAYER, oracle.PROG_CONST, (1.0,))
    with pytest.raises(ValueError):  # Dirichlet mesh
        oracle.forward_paths(oracle.OracleMesh(mesh), bc, 4, 2, 1)
    om = oracle.OracleMesh(_neumann(mesh))
    with pytest.raises(ValueError):
        oracle.forward_paths(om, bc, 4, 2, 1, start_weight=np.full(mesh.n_prims, -1.0))
    with pytest.raises(ValueError):
        oracle.forward_paths(om, bc, 4, 2, 1, start_weight=np.zeros(mesh.n_prims))
