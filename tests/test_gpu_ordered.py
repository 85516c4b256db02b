"""The ordered solve (wob_solve_ordered): the points walked in Morton order of
their bounding box, each keeping its own random-number index, the results
written back in the caller's order.  Its per-point mean and variance must be
those of the point's own traced paths (each path once), as for wob_solve;
equal calls give equal bits; the workspace is checked before anything runs."""
import numpy as np
import pytest

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


def check_stats(mean, var, val, tol_mean, tol_var):
    """mean / var of a solve against the traced path values (P x N)."""
    v = val.cpu().double().numpy()
    scale = np.abs(v).mean(axis=1) + 1e-300
    np.testing.assert_array_less(np.abs(mean.cpu().double().numpy() - v.mean(axis=1)), tol_mean * scale)
    if var is not None:
        ref = v.var(axis=1, ddof=1)
        np.testing.assert_array_less(np.abs(var.cpu().double().numpy() - ref), tol_var * ref + 1e-300)


def cases(W):
    """(name, scene mesh, precision, points, point_prim, BC, M): single layer on
    mixed tori (lines and RIS: two points pooled per lane group), direct BIE
    with boundary points, double layer on a slice plane (one axis of zero
    extent), the 2D circle in FP64."""
    w = I.config_tori(grid_n=12, n_points=333, boundary_frac=0.25, samples=64, walk_len=4)
    kind = np.random.default_rng(3).integers(0, 3, w.mesh.n_prims).astype(np.uint8)
    mixed = PT.f32_mesh(I.Mesh(3, w.mesh.verts, w.mesh.prims, kind, np.full(w.mesh.n_prims, 1.0)))
    sph = I.icosphere(8)
    neu = PT.f32_mesh(I.Mesh(3, sph.verts, sph.prims, np.full(sph.n_prims, 1, np.uint8), None))
    on, onp = I.mesh_surface_points(neu, 40, 4)
    dpts = np.concatenate([I.ball_points(161, 2.5, 3, r_min=1.2), on])
    dpp = np.concatenate([np.full(161, -1), onp]).astype(np.int32)
    g = I.slice_grid(24, 0.9)
    plane = g[np.linalg.norm(g, axis=1) < 0.85]
    c = I.config_circle(n_points=300)
    return [
        ("tori lines", mixed, W.F32, PT.f32(w.points), w.point_prim,
         W.BC(-1, 0, W.PROG_INVDIST, (0.2, -0.1, 0.05)), 3),
        ("tori RIS", mixed, W.F32, PT.f32(w.points), w.point_prim,
         W.BC(-1, 0, W.PROG_INVDIST, (0.2, -0.1, 0.05), sampling=W.SAMPLE_RIS, candidates=8), 3),
        ("direct", neu, W.F32, PT.f32(dpts), dpp, W.BC(-1, W.DIRECT, W.PROG_INVDIST, (0.2, -0.1, 0.05)), 3),
        ("double layer plane", PT.f32_mesh(sph), W.F32, PT.f32(plane), None,
         W.BC(1, W.DOUBLE_LAYER, W.PROG_INVDIST, (2.0, 0.5, 0.0)), 4),
        ("circle f64", c.mesh, W.F64, c.points, None, W.BC(1, W.DOUBLE_LAYER, W.PROG_QUAD, ()), 4),
    ]


@pytest.mark.parametrize("N", [1, 37, 128, 700])
def test_ordered_solve_statistics_equal_traced_paths(W, N):
    """Every case, path counts that leave lanes partly used (37, 700) and one
    path: the ordered solve's mean and variance equal the statistics of each
    point's own traced paths, as the plain solve's do."""
    for name, mesh, prec, pts, pp, bc, M in cases(W):
        print(f"{name} N {N} P {len(pts)}", flush=True)
        scene = W.Scene(mesh, prec)
        dt = torch.float32 if prec == W.F32 else torch.float64
        tp = dev(pts, dt)
        tpp = None if pp is None else dev(pp, torch.int32)
        val = W.trace(scene, tp, bc, N, M, 17, point_prim=tpp, want_vertices=False)[0]
        mo, vo = W.solve(scene, tp, bc, N, M, 17, point_prim=tpp, want_var=N > 1, ordered=True)
        mp, vp = W.solve(scene, tp, bc, N, M, 17, point_prim=tpp, want_var=N > 1)
        torch.cuda.synchronize()
        tm, tv = (2e-6, 2e-5) if prec == W.F32 else (1e-13, 1e-12)
        check_stats(mo, vo, val, tm, tv)
        check_stats(mp, vp, val, tm, tv)
        scene.close()


def test_ordered_solve_is_deterministic(W):
    """Equal calls give equal bits, with one workspace reused and with a fresh
    one (the sort is stable; every kernel of the call is deterministic)."""
    name, mesh, prec, pts, pp, bc, M = cases(W)[0]
    scene = W.Scene(mesh, prec)
    tp, tpp = dev(pts, torch.float32), dev(pp, torch.int32)
    ws = torch.empty(W.ordered_workspace_bytes(scene, len(pts)), dtype=torch.uint8, device="cuda")
    a = W.solve(scene, tp, bc, 96, M, 5, point_prim=tpp, ordered=True, workspace=ws)
    b = W.solve(scene, tp, bc, 96, M, 5, point_prim=tpp, ordered=True, workspace=ws)
    c = W.solve(scene, tp, bc, 96, M, 5, point_prim=tpp, ordered=True)
    torch.cuda.synchronize()
    for x, y in ((a, b), (a, c)):
        assert torch.equal(x[0], y[0]) and torch.equal(x[1], y[1])
    scene.close()


def test_ordered_solve_degenerate_point_sets(W):
    """One point; 50 copies of one point (a bounding box of zero extent: every
    key 0, the stable sort keeps the input order); the copies' paths differ
    (each copy has its own random-number index)."""
    mesh = PT.f32_mesh(I.icosphere(6))
    scene = W.Scene(mesh, W.F32)
    bc = W.BC(1, W.DOUBLE_LAYER, W.PROG_INVDIST, (2.0, 0.5, 0.0))
    for pts in (PT.f32(I.ball_points(1, 0.5, 2)), np.repeat(PT.f32(I.ball_points(1, 0.5, 3)), 50, axis=0)):
        tp = dev(pts, torch.float32)
        val = W.trace(scene, tp, bc, 64, 3, 9, want_vertices=False)[0]
        mo, vo = W.solve(scene, tp, bc, 64, 3, 9, ordered=True)
        torch.cuda.synchronize()
        check_stats(mo, vo, val, 2e-6, 2e-5)
        if len(pts) > 1:
            assert len(np.unique(mo.cpu().numpy())) > 1
    scene.close()


def test_ordered_solve_arguments(W):
    mesh = PT.f32_mesh(I.icosphere(4))
    scene = W.Scene(mesh, W.F32)
    bc = W.BC(1, W.DOUBLE_LAYER, W.PROG_CONST, (1.0,))
    pts = dev(PT.f32(I.ball_points(40, 0.5, 1)), torch.float32)
    need = W.ordered_workspace_bytes(scene, 40)
    assert need >= 40 * (4 * 4 + 12 + 4 + 8)
    with pytest.raises(W.WobError):  # too small
        W.solve(scene, pts, bc, 8, 2, ordered=True,
                workspace=torch.empty(need - 1, dtype=torch.uint8, device="cuda"))
    big = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(W.WobError):  # not 256-byte aligned
        W.solve(scene, pts, bc, 8, 2, ordered=True, workspace=big[1:])
    with pytest.raises(W.WobError):  # a variance needs two paths
        W.solve(scene, pts, bc, 1, 2, ordered=True)
    with pytest.raises(W.WobError):
        W.ordered_workspace_bytes(scene, -1)
    with pytest.raises(W.WobError):
        W.ordered_workspace_bytes(scene, 2 ** 31)
    m, v = W.solve(scene, pts[:0].contiguous(), bc, 8, 2, ordered=True)
    assert m.numel() == 0
    m, _ = W.solve(scene, pts, bc, 8, 2, ordered=True, workspace=big[:need])
    torch.cuda.synchronize()
    np.testing.assert_allclose(m.cpu().numpy(), 1.0, atol=1e-5)  # constant data, any paths
    scene.close()


def test_full_size_tori_ordered_all_points(W):
    """The headline workload at full size (three tori, 200,992 triangles, 1M
    points, 10 % on the boundary, 512 paths, M = 4) through the ordered solve in
    the benchmark's launch configuration: at every point the mean and variance
    equal those of the point's 512 traced paths (the traced paths themselves are
    compared with the oracle path by path at sampled points by the parity
    tests)."""
    w = I.config_tori()
    scene = W.Scene(w.mesh, W.F32)
    bc = W.BC(w.bc["domain"], w.bc["formulation"], w.bc["program"], tuple(w.bc["params"]))
    tp = dev(w.points, torch.float32)
    pp = dev(w.point_prim, torch.int32)
    mo, vo = W.solve(scene, tp, bc, w.samples, w.walk_len, w.seed, point_prim=pp, ordered=True)
    val = W.trace(scene, tp, bc, w.samples, w.walk_len, w.seed, point_prim=pp, want_vertices=False)[0]
    torch.cuda.synchronize()
    P, chunk, worst_m, worst_v = len(w.points), 1 << 17, 0.0, 0.0
    for c in range(0, P, chunk):
        v = val[c:c + chunk].double()
        assert bool(torch.isfinite(v).all())
        scale = v.abs().mean(1) + 1e-300
        ref = v.var(1, unbiased=True)
        em = ((mo[c:c + chunk].double() - v.mean(1)).abs() / scale).max().item()
        ev = ((vo[c:c + chunk].double() - ref).abs() / (ref + 1e-300)).max().item()
        worst_m, worst_v = max(worst_m, em), max(worst_v, ev)
    print(f"max mean error / mean |v| {worst_m:.2e}, max relative variance error {worst_v:.2e}", flush=True)
    assert worst_m < 2e-6 and worst_v < 2e-5
    scene.close()
