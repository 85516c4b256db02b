"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Per-path values and the primitive picked by every line must agree for every
non-grazing path (see tests/parity.py for the grazing class and tolerances);
hit lists of single lines must agree as sets.  Inputs are seeded and synthetic.
"""
import numpy as np
import pytest

import oracle
from paper_2305_04403_amd import inputs as I
from tests import parity as PT

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def W():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_04403_amd import wob
    wob.lib()
    return wob


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def obc(bc: dict, self_p=1.0 / 16.0):
    return oracle.make_bc(bc["domain"], bc["formulation"], bc["program"], bc["params"], self_p,
                          sampling=bc.get("sampling", 0), candidates=bc.get("candidates", 0) or 16)


def wbc(W, bc: dict, self_p=1.0 / 16.0):
    return W.BC(bc["domain"], bc["formulation"], bc["program"], tuple(bc["params"]), self_p,
                sampling=bc.get("sampling", 0), candidates=bc.get("candidates", 0))


def run_trace_parity(W, mesh, pts, pp, bc, N, M, seed, precision):
    scene = W.Scene(mesh, W.F32 if precision == "f32" else W.F64)
    dt = torch.float32 if precision == "f32" else torch.float64
    tp = dev(pts, dt)
    tpp = None if pp is None else dev(pp, torch.int32)
    val, vprim, vm = W.trace(scene, tp, wbc(W, bc), N, M, seed, point_prim=tpp)
    torch.cuda.synchronize()
    om = oracle.OracleMesh(mesh)
    orc = PT.oracle_all_paths(om, pts, pp, obc(bc), N, M, seed)
    L = orc["vtx_prim"].shape[1]
    res = PT.compare_paths(orc, val.cpu().double().numpy().reshape(-1),
                           vprim.cpu().numpy().reshape(-1, L), vm.cpu().numpy().reshape(-1, L),
                           PT.RTOL_F32 if precision == "f32" else PT.RTOL_F64)
    print(res.summary(), flush=True)
    res.assert_exact()
    scene.close()
    return res


# ------------------------------------------------------------------- hit lists

@pytest.mark.parametrize("shape", ["sphere-f32", "tori-f32", "circle-f64", "circle-f32"])
def test_intersect_all_matches_brute_force(W, shape):
    rng = np.random.default_rng(3)
    if shape == "sphere-f32":
        mesh = PT.f32_mesh(I.perturb_radial(I.icosphere(10), 0.1, 3, 4))
        prec, dt = W.F32, torch.float32
    elif shape == "tori-f32":
        mesh = PT.f32_mesh(I.torus_union(grid_n=24, seed=2)[0])
        prec, dt = W.F32, torch.float32
    elif shape == "circle-f64":
        mesh = I.circle_polygon(256)
        prec, dt = W.F64, torch.float64
    else:
        mesh = PT.f32_mesh(I.circle_polygon(256))
        prec, dt = W.F32, torch.float32
    dim = mesh.dim
    n = 3000
    orig = rng.uniform(-1.5, 1.5, (n, dim))
    # a third of the lines start on the boundary and exclude their own primitive
    bp = rng.integers(0, mesh.n_prims, n // 3)
    v = mesh.verts[mesh.prims[bp]]
    w = rng.dirichlet(np.ones(dim), n // 3)
    orig[: n // 3] = np.einsum("nk,nkd->nd", w, v)
    excl = np.full(n, -1, np.int32)
    excl[: n // 3] = bp
    d = rng.standard_normal((n, dim))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    if prec == W.F32:
        orig, d = PT.f32(orig), PT.f32(d)
    scene = W.Scene(mesh, prec)
    nh, hp, ht = W.intersect_all(scene, dev(orig, dt), dev(d, dt), dev(excl, torch.int32), max_hits=32)
    torch.cuda.synchronize()
    nh, hp, ht = nh.cpu().numpy(), hp.cpu().numpy(), ht.cpu().double().numpy()
    om = oracle.OracleMesh(mesh)
    o = oracle.intersect_all(om, orig, d, excl, max_hits=32)
    rtol = PT.RTOL_F32 if prec == W.F32 else PT.RTOL_F64
    ok = o["graze"] >= PT.graze_for(rtol)
    assert ok.mean() > 0.99
    assert np.all(o["n_hits"] <= 32)
    np.testing.assert_array_equal(nh[ok], o["n_hits"][ok])
    normals = om.normals()
    for l in np.nonzero(ok)[0]:
        k = nh[l]
        gi = np.argsort(hp[l, :k])
        oi = np.argsort(o["prim"][l, :k])
        assert np.array_equal(hp[l, :k][gi], o["prim"][l, :k][oi]), l
        # t from the primitive's plane: rounding of a few units of |x| + |t|
        # (and the vertex) over the incidence |d . n|
        to = o["t"][l, :k][oi]
        c = np.abs(normals[o["prim"][l, :k][oi]] @ d[l])
        xn = np.linalg.norm(orig[l])
        tol = PT.tolerance(1.0 + np.abs(to), (2.0 * xn + 2.0 * np.abs(to)) / c, rtol)
        assert np.all(np.abs(ht[l, :k][gi] - to) <= tol), l
    scene.close()


def staircase_mesh(n=300, r=0.75):
    """n triangles, copies of one triangle scaled by r^i toward the origin: a
    binned SAH tree deeper than 32 levels (the builder's median splits take
    over there), every stack level of the traversal in use."""
    tri = np.array([[1.0, 0.0, 0.0], [1.5, 0.5, 0.0], [1.2, 0.0, 0.5]])
    s = r ** np.arange(n, dtype=np.float64)
    verts = (s[:, None, None] * tri[None]).reshape(-1, 3)
    return I.Mesh(3, verts, np.arange(3 * n, dtype=np.int32).reshape(n, 3))


def square_mesh():
    """Two triangles: the whole tree is one leaf (the root entry is a leaf)."""
    verts = np.array([[-1.0, -1.0, 0.0], [1.0, -1.0, 0.0], [1.0, 1.0, 0.0], [-1.0, 1.0, 0.0]])
    return I.Mesh(3, verts, np.array([[0, 1, 2], [0, 2, 3]], np.int32))


@pytest.mark.parametrize("shape", ["one-leaf-f32", "staircase-f64", "staircase-f32"])
def test_intersect_all_tree_shapes(W, shape):
    """Hit lists against the oracle on a scene whose tree is a single leaf and
    on one deeper than 32 levels (lines through the region where the small
    triangles nest, so that the traversal goes down the deep branches)."""
    rng = np.random.default_rng(8)
    mesh = square_mesh() if shape.startswith("one-leaf") else staircase_mesh()
    f32 = shape.endswith("f32")
    if f32:
        mesh = PT.f32_mesh(mesh)
    scene = W.Scene(mesh, W.F32 if f32 else W.F64)
    info = scene.info()
    if shape.startswith("one-leaf"):
        assert info["n_leaves"] == 1
    else:
        assert info["depth"] > 32
    n = 4000
    orig = rng.uniform(-1.5, 1.5, (n, 3))
    if not shape.startswith("one-leaf"):
        orig[: n // 2] = rng.uniform(-1.0, 1.0, (n // 2, 3)) * (10.0 ** rng.uniform(-6, 0, (n // 2, 1)))
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    dt = torch.float32 if f32 else torch.float64
    if f32:
        orig, d = PT.f32(orig), PT.f32(d)
    excl = np.full(n, -1, np.int32)
    nh, hp, ht = W.intersect_all(scene, dev(orig, dt), dev(d, dt), dev(excl, torch.int32), max_hits=64)
    torch.cuda.synchronize()
    nh, hp = nh.cpu().numpy(), hp.cpu().numpy()
    o = oracle.intersect_all(oracle.OracleMesh(mesh), orig, d, excl, max_hits=64)
    ok = o["graze"] >= PT.graze_for(PT.RTOL_F32 if f32 else PT.RTOL_F64)
    assert ok.mean() > 0.98
    assert o["n_hits"][ok].sum() > 100
    if f32 and not shape.startswith("one-leaf"):
        # binary32 cannot resolve triangles below about 1e-7 of the distance
        # to the line's origin: compare the hits of the larger ones (>= 1e-5)
        big = np.arange(mesh.n_prims) < 40
        for l in np.nonzero(ok)[0]:
            g = np.sort(hp[l, :nh[l]])
            r = np.sort(o["prim"][l, :o["n_hits"][l]])
            assert np.array_equal(g[big[g]], r[big[r]]), l
    else:
        np.testing.assert_array_equal(nh[ok], o["n_hits"][ok])
        for l in np.nonzero(ok)[0]:
            assert np.array_equal(np.sort(hp[l, :nh[l]]), np.sort(o["prim"][l, :o["n_hits"][l]])), l
    scene.close()


@pytest.mark.parametrize("shape", ["one-leaf-f32", "staircase-f64"])
def test_trace_parity_tree_shapes(W, shape):
    """Per-path parity of a double-layer walk on the one-leaf and the deep
    scene (the walk kernel's root-leaf start and its full stack)."""
    mesh = square_mesh() if shape.startswith("one-leaf") else staircase_mesh()
    prec = "f32" if shape.endswith("f32") else "f64"
    if prec == "f32":
        mesh = PT.f32_mesh(mesh)
    pts = np.random.default_rng(9).uniform(-0.9, 0.9, (40, 3))
    pts[:, 2] = np.where(np.abs(pts[:, 2]) < 0.05, 0.05, pts[:, 2])
    if prec == "f32":
        pts = PT.f32(pts)
    bc = dict(domain=1, formulation=1, program=oracle.PROG_INVDIST, params=(2.0, 0.5, 0.0))
    run_trace_parity(W, mesh, pts, None, bc, 64, 4, 21, prec)


# ------------------------------------------------------------------- per-path parity

def test_trace_parity_dirichlet_2d_f32(W):
    """2D interior Dirichlet on a perturbed 300-gon in FP32 (binary16 box
    words of the 2D records), ragged sizes."""
    c = I.circle_polygon(300)
    ang = np.arctan2(c.verts[:, 1], c.verts[:, 0])
    verts = c.verts * (1.0 + 0.1 * np.sin(3 * ang))[:, None]
    mesh = PT.f32_mesh(I.Mesh(2, verts, c.prims))
    pts = PT.f32(I.disk_points(45, 0.8, 6))
    bc = dict(domain=1, formulation=1, program=oracle.PROG_QUAD, params=())
    run_trace_parity(W, mesh, pts, None, bc, 70, 5, 23, "f32")


def test_trace_parity_circle_fp64_full_config(W):
    """2D interior Dirichlet on the 256-gon, FP64, at its full size
    (1024 points x 64 paths, M = 4)."""
    w = I.config_circle()
    res = run_trace_parity(W, w.mesh, w.points, None, w.bc, w.samples, w.walk_len, 0, "f64")
    assert res.n_checked == res.n - res.n_graze


def test_trace_parity_dirichlet_3d_f32(W):
    """3D interior Dirichlet, perturbed icosphere, FP32, M = 6, ragged sizes
    (P not a multiple of the points per block, N = 100 not a multiple of 64)."""
    mesh = PT.f32_mesh(I.perturb_radial(I.icosphere(12), 0.1, 3, 4))
    pts = PT.f32(I.ball_points(77, 0.8, 5))
    bc = dict(domain=1, formulation=1, program=3, params=(2.0, 0.5, 0.0))
    run_trace_parity(W, mesh, pts, None, bc, 100, 6, 11, "f32")


def test_trace_parity_direct_neumann_exterior(W):
    """3D exterior Neumann, direct BIE (M + 1 lines, all-hits source), with
    points both off and on the boundary."""
    s = I.icosphere(8)
    mesh = PT.f32_mesh(I.Mesh(3, s.verts, s.prims, np.full(s.n_prims, 1, np.uint8), None))
    off = I.ball_points(40, 2.5, 1, r_min=1.2)
    on, onp = I.mesh_surface_points(mesh, 24, 2)
    pts = PT.f32(np.concatenate([off, on]))
    pp = np.concatenate([np.full(40, -1), onp]).astype(np.int32)
    bc = dict(domain=-1, formulation=2, program=3, params=(0.2, -0.1, 0.1))
    run_trace_parity(W, mesh, pts, pp, bc, 64, 4, 3, "f32")


def test_trace_parity_single_layer_mixed_tori(W):
    """3D exterior Neumann / Robin (alpha = 1) single layer on the tori union,
    with boundary points (self-panel mixture at step 0 and at Robin vertices)."""
    w = I.config_tori(grid_n=24, n_points=96, samples=64, walk_len=4)
    run_trace_parity(W, w.mesh, w.points, w.point_prim, w.bc, 64, 4, 5, "f32")


def test_trace_parity_interior_single_layer_2d_f64(W):
    """2D interior Robin single layer in FP64 (segment self-panel, log kernels)."""
    m = I.circle_polygon(96)
    mesh = I.Mesh(2, m.verts, m.prims, np.full(96, 2, np.uint8), np.full(96, 0.5))
    pts = I.disk_points(40, 0.8, 9)
    s = np.random.default_rng(1).random(10)
    bp = np.arange(10, dtype=np.int32) * 7
    on = m.verts[m.prims[bp, 0]] + s[:, None] * (m.verts[m.prims[bp, 1]] - m.verts[m.prims[bp, 0]])
    pts = np.concatenate([pts, on])
    pp = np.concatenate([np.full(40, -1), bp]).astype(np.int32)
    bc = dict(domain=1, formulation=3, program=2, params=())
    run_trace_parity(W, mesh, pts, pp, bc, 64, 3, 2, "f64")


def test_trace_parity_single_layer_ris_tori(W):
    """Single layer with resampled importance sampling (16 area-uniform
    candidates) on the tori union, Neumann / Robin, points off and on the
    boundary: the kept candidate of every vertex and the path values."""
    w = I.config_tori(grid_n=20, n_points=80, boundary_frac=0.25, samples=64, walk_len=4)
    bc = dict(w.bc, sampling=1, candidates=16)
    run_trace_parity(W, w.mesh, w.points, w.point_prim, bc, 64, 4, 13, "f32")


def test_trace_parity_single_layer_ris_2d_f64(W):
    """2D interior Robin single layer with RIS (8 candidates) in FP64."""
    m = I.circle_polygon(96)
    mesh = I.Mesh(2, m.verts, m.prims, np.full(96, 2, np.uint8), np.full(96, 0.5))
    pts = I.disk_points(40, 0.8, 9)
    bc = dict(domain=1, formulation=3, program=2, params=(), sampling=1, candidates=8)
    run_trace_parity(W, mesh, pts, None, bc, 64, 3, 2, "f64")


@pytest.mark.parametrize("shape", ["tetrahedron-f32", "square-f64"])
def test_trace_parity_ris_equal_areas(W, shape):
    """RIS picks through the area-CDF guide table where every bucket edge b / K
    falls on a CDF value (primitives of equal area: a regular tetrahedron,
    K = 4, CDF 1/4, 1/2, 3/4, 1; a square in 2D), so the strict comparison at
    the bucket edges decides; exterior Robin single layer, against the
    oracle path by path."""
    if shape == "tetrahedron-f32":
        v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], np.float64)
        f = np.array([[0, 1, 2], [0, 3, 1], [0, 2, 3], [1, 3, 2]], np.int32)  # outward
        mesh = PT.f32_mesh(I.Mesh(3, v, f, np.full(4, 2, np.uint8), np.full(4, 0.5)))
        pts = PT.f32(I.ball_points(30, 4.0, 3, r_min=2.0))
        prec, M = "f32", 4
    else:
        v = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], np.float64)
        f = np.array([[0, 1], [1, 2], [2, 3], [3, 0]], np.int32)
        mesh = I.Mesh(2, v, f, np.full(4, 2, np.uint8), np.full(4, 0.5))
        pts = I.disk_points(30, 4.0, 3)
        pts = pts[np.abs(pts).max(axis=1) > 1.2]
        prec, M = "f64", 3
    bc = dict(domain=-1, formulation=3, program=3, params=(0.1, 0.2, 0.05), sampling=1, candidates=16)
    run_trace_parity(W, mesh, pts, None, bc, 64, M, 7, prec)


@pytest.mark.parametrize("sampling", [0, 1])
def test_trace_parity_mixed_tori(W, sampling):
    """Mixed problem on the tori union: every triangle Dirichlet, Neumann or
    Robin (alpha = 1) at random, single layer with the transformed first-kind
    rows on the Dirichlet parts (k = 4, p_k = 2/3), points off and on the
    boundary; line sampling and RIS."""
    w = I.config_tori(grid_n=20, n_points=80, boundary_frac=0.25, samples=64, walk_len=4)
    kind = np.random.default_rng(5).integers(0, 3, w.mesh.n_prims).astype(np.uint8)
    mesh = I.Mesh(3, w.mesh.verts, w.mesh.prims, kind, np.full(w.mesh.n_prims, 1.0))
    bc = dict(w.bc, formulation=0, sampling=sampling, candidates=16)
    run_trace_parity(W, mesh, w.points, w.point_prim, bc, 64, 4, 19, "f32")


def test_trace_parity_mixed_2d_f64(W):
    """2D interior mixed problem (random Dirichlet / Neumann / Robin segments) in FP64."""
    c = I.circle_polygon(128)
    kind = np.random.default_rng(1).integers(0, 3, 128).astype(np.uint8)
    mesh = I.Mesh(2, c.verts, c.prims, kind, np.full(128, 1.0))
    pts = I.disk_points(40, 0.8, 4)
    bc = dict(domain=1, formulation=0, program=2, params=())
    run_trace_parity(W, mesh, pts, None, bc, 64, 4, 8, "f64")


def test_ris_arguments(W):
    mesh = PT.f32_mesh(I.icosphere(4))
    scene = W.Scene(mesh, W.F32)
    pts = dev(PT.f32(I.ball_points(5, 0.5, 1)), torch.float32)
    # RIS is a single-layer sampling: the double layer rejects it
    with pytest.raises(W.WobError):
        W.solve(scene, pts, W.BC(1, W.AUTO, W.PROG_CONST, (1.0,), sampling=W.SAMPLE_RIS), 8, 2)
    neu = I.Mesh(3, mesh.verts, mesh.prims, np.full(mesh.n_prims, 1, np.uint8), None)
    s2 = W.Scene(neu, W.F32)
    for c in (-1, 65):
        with pytest.raises(W.WobError):
            W.solve(s2, pts, W.BC(-1, W.SINGLE_LAYER, W.PROG_CONST, (1.0,), sampling=W.SAMPLE_RIS,
                                  candidates=c), 8, 2)
    with pytest.raises(W.WobError):
        W.solve(s2, pts, W.BC(-1, W.SINGLE_LAYER, W.PROG_CONST, (1.0,), sampling=2), 8, 2)
    # the corrected (control-variate) walk takes RIS sampling too, but not an
    # invalid candidate count
    g = torch.zeros(mesh.n_prims, dtype=torch.float32, device="cuda")
    m, _ = W.solve_cv(s2, pts, W.BC(-1, W.SINGLE_LAYER, W.PROG_CONST, (1.0,), sampling=W.SAMPLE_RIS), 8, 2, g)
    torch.cuda.synchronize()
    assert torch.isfinite(m).all()
    with pytest.raises(W.WobError):
        W.solve_cv(s2, pts, W.BC(-1, W.SINGLE_LAYER, W.PROG_CONST, (1.0,), sampling=W.SAMPLE_RIS, candidates=65),
                   8, 2, g)
    s2.close()
    scene.close()


@pytest.mark.parametrize("N", [1, 3, 5, 7, 130])
def test_trace_parity_paths_not_a_multiple_of_lanes(W, N):
    """A lane runs several paths back to back and a wavefront may hold several
    points: path counts that leave lanes partly used, and a point count that
    leaves the last workgroup ragged, against the oracle path by path."""
    mesh = PT.f32_mesh(I.perturb_radial(I.icosphere(6), 0.1, 2, 3))
    pts = PT.f32(I.ball_points(13, 0.8, 21))
    bc = dict(domain=1, formulation=1, program=3, params=(2.0, 0.5, 0.0))
    run_trace_parity(W, mesh, pts, None, bc, N, 3, 17, "f32")


# ------------------------------------------------------------------- solve

def test_solve_mean_var_equal_trace_statistics(W):
    mesh = PT.f32_mesh(I.perturb_radial(I.icosphere(8), 0.1, 3, 4))
    pts = PT.f32(I.ball_points(133, 0.8, 5))
    bc = dict(domain=1, formulation=1, program=3, params=(2.0, 0.5, 0.0))
    scene = W.Scene(mesh, W.F32)
    tp = dev(pts, torch.float32)
    for N in (1, 63, 64, 100, 256, 300):
        mean, var = W.solve(scene, tp, wbc(W, bc), N, 5, 7, want_var=N > 1)
        val, _, _ = W.trace(scene, tp, wbc(W, bc), N, 5, 7, want_vertices=False)
        torch.cuda.synchronize()
        v = val.cpu().double().numpy()
        np.testing.assert_allclose(mean.cpu().numpy(), v.mean(axis=1), rtol=2e-6, atol=2e-6)
        if N > 1:
            np.testing.assert_allclose(var.cpu().numpy(), v.var(axis=1, ddof=1), rtol=2e-5, atol=1e-6)
    scene.close()


def test_solve_and_batch_statistics_equal_trace_with_paths_ending_at_start(W):
    """The lanes of a point take the next free path index as their paths end
    (a counter per lane group in LDS).  RIS paths on a mixed Robin / Neumann /
    Dirichlet tori scene end inside their first step more often than not, so
    a lane takes several indices in one pass; the solve's and the batch's
    per-point mean and variance must still be those of the traced paths (each
    path once), also where plain single-layer and direct-BIE solves pool two
    points per lane group: an odd point count leaves the last group one point,
    and N = 700 gives 22 paths per lane."""
    w = I.config_tori(grid_n=12, n_points=91, boundary_frac=0.25, samples=64, walk_len=4)
    kind = np.random.default_rng(3).integers(0, 3, w.mesh.n_prims).astype(np.uint8)
    mixed = PT.f32_mesh(I.Mesh(3, w.mesh.verts, w.mesh.prims, kind, np.full(w.mesh.n_prims, 1.0)))
    scene = W.Scene(mixed, W.F32)
    pts = dev(PT.f32(w.points), torch.float32)
    pp = dev(w.point_prim, torch.int32)
    for sampling in (W.SAMPLE_RIS, W.SAMPLE_LINE):
        bc = W.BC(-1, 0, W.PROG_INVDIST, (0.2, -0.1, 0.05), sampling=sampling, candidates=8)
        for N in (1, 37, 96, 100, 700):
            print(f"sampling {sampling} N {N}", flush=True)
            val = W.trace(scene, pts, bc, N, 3, 21, point_prim=pp, want_vertices=False)[0]
            mean, var = W.solve(scene, pts, bc, N, 3, 21, point_prim=pp, want_var=N > 1)
            b = W.Batch([dict(scene=scene, points=pts, point_prim=pp, bc=bc, samples=N, walk_len=3, seed=21,
                              want_var=N > 1)], tune=(256, 1))
            bm, bv = b.launch()[0]
            torch.cuda.synchronize()
            v = val.cpu().double().numpy()
            scale = np.abs(v).mean(axis=1) + 1e-30
            for m, s2 in ((mean, var), (bm, bv)):
                np.testing.assert_array_less(np.abs(m.cpu().double().numpy() - v.mean(axis=1)), 2e-6 * scale)
                if N > 1:
                    ref = v.var(axis=1, ddof=1)
                    np.testing.assert_array_less(np.abs(s2.cpu().double().numpy() - ref), 2e-5 * ref + 1e-30)
            b.close()
    scene.close()
    # the direct BIE pools two points too: exterior Neumann on a sphere, points
    # off and on the boundary
    sph = I.icosphere(8)
    neu = PT.f32_mesh(I.Mesh(3, sph.verts, sph.prims, np.full(sph.n_prims, 1, np.uint8), None))
    scene = W.Scene(neu, W.F32)
    on, onp = I.mesh_surface_points(neu, 20, 4)
    pts = dev(PT.f32(np.concatenate([I.ball_points(71, 2.5, 3, r_min=1.2), on])), torch.float32)
    pp = dev(np.concatenate([np.full(71, -1), onp]).astype(np.int32), torch.int32)
    bc = W.BC(-1, W.DIRECT, W.PROG_INVDIST, (0.2, -0.1, 0.05))
    for N in (1, 37, 100, 700):
        print(f"direct N {N}", flush=True)
        val = W.trace(scene, pts, bc, N, 3, 23, point_prim=pp, want_vertices=False)[0]
        mean, var = W.solve(scene, pts, bc, N, 3, 23, point_prim=pp, want_var=N > 1)
        torch.cuda.synchronize()
        v = val.cpu().double().numpy()
        scale = np.abs(v).mean(axis=1) + 1e-30
        np.testing.assert_array_less(np.abs(mean.cpu().double().numpy() - v.mean(axis=1)), 2e-6 * scale)
        if N > 1:
            ref = v.var(axis=1, ddof=1)
            np.testing.assert_array_less(np.abs(var.cpu().double().numpy() - ref), 2e-5 * ref + 1e-30)
    scene.close()


@pytest.mark.parametrize("N", [256, 37, 2])
def test_solve_matches_oracle_mean(W, N):
    """FP64 per-point mean and variance against the oracle's two-pass values,
    including path counts that leave lanes partly used."""
    w = I.config_circle(n_points=129, samples=N)
    scene = W.Scene(w.mesh, W.F64)
    mean, var = W.solve(scene, dev(w.points, torch.float64), wbc(W, w.bc), N, 4, 0)
    torch.cuda.synchronize()
    om = oracle.OracleMesh(w.mesh)
    m_o, v_o = oracle.solve(om, w.points, None, obc(w.bc), N, 4, 0)
    np.testing.assert_allclose(mean.cpu().numpy(), m_o, rtol=0, atol=1e-11)
    np.testing.assert_allclose(var.cpu().numpy(), v_o, rtol=1e-9, atol=1e-11)
    scene.close()


def test_full_size_icosphere_slice_sampled(W):
    """The full 3D Dirichlet workload (20,480 triangles, ~168k slice points,
    256 paths, M = 6) in the benchmark's launch configuration; at 12 sampled
    points the paths are re-traced with their original random-number indices
    and compared path by path with the oracle, and the solve's mean there must
    equal the traced paths' mean."""
    w = I.config_icosphere_slice()
    scene = W.Scene(w.mesh, W.F32)
    tp = dev(w.points, torch.float32)
    mean, var = W.solve(scene, tp, wbc(W, w.bc), w.samples, w.walk_len, w.seed)
    torch.cuda.synchronize()
    assert torch.isfinite(mean).all() and torch.isfinite(var).all()
    rng = np.random.default_rng(0)
    ids = np.sort(rng.choice(w.points.shape[0], 12, replace=False)).astype(np.int64)
    sub = w.points[ids]
    val, vprim, vm = W.trace(scene, dev(sub, torch.float32), wbc(W, w.bc), w.samples, w.walk_len,
                             w.seed, point_ids=dev(ids.astype(np.int32), torch.int32))
    torch.cuda.synchronize()
    v = val.cpu().double().numpy()
    np.testing.assert_allclose(mean.cpu().numpy()[ids], v.mean(axis=1), rtol=2e-6, atol=2e-6)
    om = oracle.OracleMesh(w.mesh)
    orc = PT.oracle_all_paths(om, sub, None, obc(w.bc), w.samples, w.walk_len, w.seed, point_ids=ids)
    L = orc["vtx_prim"].shape[1]
    res = PT.compare_paths(orc, v.reshape(-1), vprim.cpu().numpy().reshape(-1, L),
                           vm.cpu().numpy().reshape(-1, L), PT.RTOL_F32)
    print(res.summary(), flush=True)
    res.assert_exact()
    # and the estimate itself: within 5 SE + 1% of the analytic solution on average
    se = np.sqrt(var.cpu().double().numpy() / w.samples)
    z = (mean.cpu().double().numpy() - w.exact) / np.maximum(se, 1e-12)
    assert abs(np.mean(z)) < 0.2
    scene.close()


def test_full_size_tori_sampled(W):
    """The headline workload at full size (three tori, 200,992 triangles, 1M
    points with 10 % on the boundary, 512 paths, M = 4, single layer: two
    points pooled per lane group) in the benchmark's launch configuration; at
    8 sampled points (6 off and 2 on the boundary) the paths are re-traced
    with their original random-number indices and compared path by path with
    the oracle, and the solve's mean and variance there must equal the traced
    paths' (each of the 512 paths counted once)."""
    w = I.config_tori()
    scene = W.Scene(w.mesh, W.F32)
    tp = dev(w.points, torch.float32)
    pp = dev(w.point_prim, torch.int32)
    mean, var = W.solve(scene, tp, wbc(W, w.bc), w.samples, w.walk_len, w.seed, point_prim=pp)
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    on = np.flatnonzero(w.point_prim >= 0)
    off = np.flatnonzero(w.point_prim < 0)
    ids = np.sort(np.concatenate([rng.choice(off, 6, replace=False), rng.choice(on, 2, replace=False)]))
    sub, subp = w.points[ids], w.point_prim[ids]
    print(f"sampled points {ids.tolist()}", flush=True)
    val, vprim, vm = W.trace(scene, dev(sub, torch.float32), wbc(W, w.bc), w.samples, w.walk_len, w.seed,
                             point_prim=dev(subp, torch.int32), point_ids=dev(ids.astype(np.int32), torch.int32))
    torch.cuda.synchronize()
    v = val.cpu().double().numpy()
    scale = np.abs(v).mean(axis=1) + 1e-30
    np.testing.assert_array_less(np.abs(mean.cpu().double().numpy()[ids] - v.mean(axis=1)), 2e-6 * scale)
    ref_var = v.var(axis=1, ddof=1)
    np.testing.assert_array_less(np.abs(var.cpu().double().numpy()[ids] - ref_var), 2e-5 * ref_var + 1e-30)
    om = oracle.OracleMesh(w.mesh)
    orc = PT.oracle_all_paths(om, sub, subp, obc(w.bc), w.samples, w.walk_len, w.seed, point_ids=ids)
    L = orc["vtx_prim"].shape[1]
    res = PT.compare_paths(orc, v.reshape(-1), vprim.cpu().numpy().reshape(-1, L),
                           vm.cpu().numpy().reshape(-1, L), PT.RTOL_F32)
    print(res.summary(), flush=True)
    res.assert_exact()
    scene.close()


# ------------------------------------------------------------------- edge cases

def test_edge_cases(W):
    mesh = PT.f32_mesh(I.icosphere(4))
    scene = W.Scene(mesh, W.F32)
    bc = W.BC(1, W.AUTO, W.PROG_CONST, (1.0,))
    empty = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    m, v = W.solve(scene, empty, bc, 8, 3)
    assert m.numel() == 0
    pts = dev(PT.f32(I.ball_points(5, 0.5, 1)), torch.float32)
    # constant data: the double layer reproduces it exactly on every path (lambda_0 = -1)
    for M in (1, 2, 3, 7):
        m, v = W.solve(scene, pts, bc, 64, M)
        torch.cuda.synchronize()
        np.testing.assert_allclose(m.cpu().numpy(), 1.0, atol=1e-5)
        np.testing.assert_allclose(v.cpu().numpy(), 0.0, atol=1e-8)
    # variance with one sample is an argument error
    with pytest.raises(W.WobError):
        W.solve(scene, pts, bc, 1, 3)
    # out-of-range boundary ids give NaN, not a fault
    bad = dev(np.array([0, -1, 10 ** 6, -5, 3], np.int32), torch.int32)
    m, _ = W.solve(scene, pts, bc, 8, 2, point_prim=bad, want_var=False)
    torch.cuda.synchronize()
    mm = m.cpu().numpy()
    assert np.isnan(mm[2]) and np.isnan(mm[3]) and np.isfinite(mm[1])
    # Dirichlet mixed with Neumann: the single layer (AUTO) solves it, the double
    # layer and the direct BIE do not
    mixed = I.Mesh(3, mesh.verts, mesh.prims, np.array([0, 1] * (mesh.n_prims // 2), np.uint8))
    s2 = W.Scene(mixed, W.F32)
    m, _ = W.solve(s2, pts, bc, 8, 2)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(m.cpu().numpy()))
    for f in (W.DOUBLE_LAYER, W.DIRECT):
        with pytest.raises(W.WobError):
            W.solve(s2, pts, W.BC(1, f, W.PROG_CONST, (1.0,)), 8, 2)
    s2.close()
    scene.close()


def test_deterministic_and_seeded(W):
    mesh = PT.f32_mesh(I.perturb_radial(I.icosphere(6), 0.1, 3, 4))
    scene = W.Scene(mesh, W.F32)
    pts = dev(PT.f32(I.ball_points(64, 0.7, 3)), torch.float32)
    bc = W.BC(1, W.AUTO, W.PROG_LINEAR, (1.0, 0.0, 0.0, 0.0))
    a = W.solve(scene, pts, bc, 128, 4, seed=5)[0].cpu()
    b = W.solve(scene, pts, bc, 128, 4, seed=5)[0].cpu()
    c = W.solve(scene, pts, bc, 128, 4, seed=6)[0].cpu()
    assert torch.equal(a, b)
    assert not torch.equal(a, c)
    scene.close()


def test_work_counters(W):
    mesh = PT.f32_mesh(I.perturb_radial(I.icosphere(8), 0.1, 3, 4))
    scene = W.Scene(mesh, W.F32)
    pts = dev(PT.f32(I.ball_points(50, 0.7, 3)), torch.float32)
    bc = W.BC(1, W.AUTO, W.PROG_CONST, (1.0,))
    c = W.count_work(scene, pts, bc, 64, 4)
    # a closed surface meets every line through an interior or boundary point
    assert c["lines"] == 50 * 64 * 4
    assert c["hits"] >= c["lines"]
    assert c["nodes"] > c["lines"] and c["prims"] >= c["hits"]
    scene.close()


def test_nonfinite_paths_counted_and_left_out(W):
    """A boundary point where the data are singular and a point with an
    invalid primitive id have no finite path: their means are NaN, the other
    points match the oracle's finite-path statistics, and the scene's device
    status counts every left-out path once (reset on read); the same through
    a batched launch."""
    mesh = PT.f32_mesh(I.icosphere(6))
    j = 7
    c = PT.f32(mesh.verts[mesh.prims[j]].mean(axis=0))
    pts = PT.f32(np.stack([c, 0.3 * c, -0.2 * c, 0.1 * c]))
    pp = np.array([j, -1, -1, mesh.n_prims + 3], np.int32)
    scene = W.Scene(mesh, W.F32)
    assert scene.nonfinite_paths() == 0
    bc = W.BC(1, 1, W.PROG_INVDIST, tuple(c))
    tp, tpp = dev(pts, torch.float32), dev(pp, torch.int32)
    N = 64
    mean, var = W.solve(scene, tp, bc, N, 3, 4, point_prim=tpp)
    torch.cuda.synchronize()
    m = mean.cpu().double().numpy()
    assert np.isnan(m[0]) and np.isnan(m[3]) and np.all(np.isfinite(m[1:3]))
    assert scene.nonfinite_paths() == 2 * N
    assert scene.nonfinite_paths() == 0
    om, ov = oracle.solve(oracle.OracleMesh(mesh), pts[:3], pp[:3],
                          oracle.make_bc(1, oracle.DOUBLE_LAYER, oracle.PROG_INVDIST, tuple(c)), N, 3, 4)
    assert np.isnan(om[0])
    assert np.allclose(m[1:3], om[1:3], rtol=1e-5)
    b = W.Batch([dict(scene=scene, points=tp, point_prim=tpp, bc=bc, samples=N, walk_len=3, seed=4)],
                tune=(256, 1))
    (bm, _), = b.launch()
    torch.cuda.synchronize()
    assert torch.equal(bm.isnan(), mean.isnan())
    assert scene.nonfinite_paths() == 2 * N
    b.close()
    scene.close()


def test_gather_probe(W):
    """The bandwidth probe reads whole 32-byte records inside the buffer: on a
    buffer of ones every lane returns 8 per read; bad sizes are rejected."""
    buf = torch.ones((1 << 20) // 4, dtype=torch.float32, device="cuda")
    out = W.gather_probe(buf, 1000, 7, seed=3)
    torch.cuda.synchronize()
    assert torch.all(out == 56.0)
    with pytest.raises(W.WobError):
        W.gather_probe(buf[:3], 10, 1)  # 12 bytes: not a whole record
    with pytest.raises(W.WobError):
        W.gather_probe(buf[1:9], 10, 1)  # not 16-byte aligned
