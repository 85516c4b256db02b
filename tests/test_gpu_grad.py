"""GPU parity of the gradient estimators (Sec. 4.1.3, derivative estimators along
the same paths) against the FP64 oracle, through the C ABI: per path the value
and every gradient component, for the double layer, the direct BIE and the
single layer (lines, RIS, Dirichlet parts), 3D FP32 and 2D FP64.
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


def run_grad_parity(W, mesh, pts, bc, N, M, seed, precision, anchors=None, anchor_prim=None):
    """Per-path value and gradient on every non-grazing path: the value within
    RTOL * S + KAPPA * u * E, every gradient component within the same bar of
    the gradient (its magnitude sum and the oracle's bound of its rounding).
    With anchors: the boundary split at those points (the same anchors, in
    the scene's precision, on both sides)."""
    scene = W.Scene(mesh, W.F32 if precision == "f32" else W.F64)
    dt = torch.float32 if precision == "f32" else torch.float64
    wb = W.BC(bc["domain"], bc["formulation"], bc["program"], tuple(bc["params"]),
              sampling=bc.get("sampling", 0), candidates=bc.get("candidates", 0))
    kw = {}
    if anchors is not None:
        kw = dict(anchors=dev(anchors, dt), anchor_prim=dev(anchor_prim, torch.int32))
    val, g = W.trace_grad(scene, dev(pts, dt), wb, N, M, seed, **kw)
    torch.cuda.synchronize()
    ob = oracle.make_bc(bc["domain"], bc["formulation"], bc["program"], bc["params"],
                        sampling=bc.get("sampling", 0), candidates=bc.get("candidates", 0) or 16)
    P = pts.shape[0]
    ip = np.repeat(np.arange(P), N)
    ik = np.tile(np.arange(N), P)
    orc = oracle.trace_grad(oracle.OracleMesh(mesh), pts, ob, M, seed, ip, ik, anchors=anchors,
                            anchor_prim=anchor_prim)
    rtol = PT.RTOL_F32 if precision == "f32" else PT.RTOL_F64
    ok = orc["graze"] >= PT.graze_for(rtol)
    gv = val.cpu().double().numpy().reshape(-1)
    gg = g.cpu().double().numpy().reshape(-1, mesh.dim)
    vtol = np.maximum(PT.tolerance(orc["abs_sum"], orc["err"], rtol), 1e-300)
    gtol = np.maximum(PT.tolerance(orc["grad_abs"], orc["grad_err"], rtol), 1e-300)[:, None]
    dv, dg = np.abs(gv - orc["value"]), np.abs(gg - orc["grad"])
    bad = (dv > vtol) | np.any(dg > gtol, axis=1)
    plain = (dv <= rtol * orc["abs_sum"]) & np.all(dg <= rtol * orc["grad_abs"][:, None], axis=1)
    n_bad = int((bad & ok).sum())
    worst = float(np.max(np.where(ok[:, None], dg / gtol, 0.0)))
    print(f"paths={len(ok)} grazing={int((~ok).sum())} mismatch={n_bad} "
          f"within-plain-bar={plain[ok].mean():.5f} worst grad err/tol={worst:.3f}", flush=True)
    assert (~ok).sum() <= 0.01 * len(ok)
    assert n_bad == 0
    assert np.all(np.isfinite(gg))
    scene.close()
    return orc, gv, gg


def test_grad_parity_double_layer_3d_f32(W):
    """Interior Dirichlet (g = 1/|x - x0|, x0 outside) on a perturbed sphere."""
    mesh = PT.f32_mesh(I.perturb_radial(I.icosphere(10), 0.1, 3, 4))
    pts = PT.f32(I.ball_points(40, 0.8, 5))
    bc = dict(domain=1, formulation=1, program=oracle.PROG_INVDIST, params=(2.0, 0.5, 0.0))
    run_grad_parity(W, mesh, pts, bc, 64, 4, 13, "f32")


def test_grad_parity_direct_3d_f32(W):
    """Exterior Neumann by the direct BIE (line-0 source gradient included)."""
    s = I.icosphere(10)
    mesh = PT.f32_mesh(I.Mesh(3, s.verts, s.prims, np.full(s.n_prims, 1, np.uint8)))
    pts = PT.f32(I.ball_points(40, 2.5, 6, r_min=1.3))
    bc = dict(domain=-1, formulation=2, program=oracle.PROG_INVDIST, params=(0.2, -0.1, 0.05))
    run_grad_parity(W, mesh, pts, bc, 64, 3, 14, "f32")


@pytest.mark.parametrize("sampling", [0, 1])
def test_grad_parity_single_layer_tori_f32(W, sampling):
    """Exterior Neumann / Robin single layer on the tori (lines and RIS)."""
    w = I.config_tori(grid_n=20, n_points=40, boundary_frac=0.0, samples=64, walk_len=3)
    bc = dict(w.bc, sampling=sampling, candidates=8)
    run_grad_parity(W, w.mesh, w.points, bc, 64, 3, 15, "f32")


def test_grad_parity_mixed_3d_f32(W):
    """Dirichlet, Neumann and Robin parts at random (single layer with the
    transformed first-kind rows)."""
    w = I.config_tori(grid_n=20, n_points=30, boundary_frac=0.0, samples=64, walk_len=3)
    kind = np.random.default_rng(5).integers(0, 3, w.mesh.n_prims).astype(np.uint8)
    mesh = I.Mesh(3, w.mesh.verts, w.mesh.prims, kind, np.full(w.mesh.n_prims, 1.0))
    bc = dict(w.bc, formulation=0)
    run_grad_parity(W, mesh, w.points, bc, 64, 3, 16, "f32")


@pytest.mark.parametrize("form,kind,dom,prog", [(1, 0, 1, 2), (2, 1, -1, 3), (3, 2, 1, 2)])
def test_grad_parity_2d_f64(W, form, kind, dom, prog):
    """2D, FP64: double layer (interior, x^2 - y^2), direct BIE (exterior
    monopole), single layer (interior Robin)."""
    c = I.circle_polygon(128)
    mesh = I.Mesh(2, c.verts, c.prims, np.full(128, kind, np.uint8), np.full(128, 0.5))
    pts = I.disk_points(30, 0.8, 2) if dom == 1 else I.disk_points(30, 2.5, 2) * 1.0 + 0.0
    if dom == -1:
        r = np.linalg.norm(pts, axis=1)
        pts = pts / r[:, None] * (1.2 + r[:, None])
    params = (0.1, -0.2) if prog == 3 else ()
    bc = dict(domain=dom, formulation=form, program=prog, params=params)
    run_grad_parity(W, mesh, pts, bc, 64, 3, 17, "f64")


def test_grad_solve_statistics_and_value(W):
    """wob_solve_grad's mean and variance are those of wob_trace_grad's paths,
    and its value equals wob_solve's; ragged path and point counts."""
    mesh = PT.f32_mesh(I.perturb_radial(I.icosphere(8), 0.1, 3, 4))
    scene = W.Scene(mesh, W.F32)
    pts = dev(PT.f32(I.ball_points(37, 0.8, 5)), torch.float32)
    bc = W.BC(1, 1, W.PROG_INVDIST, (2.0, 0.5, 0.0))
    for N in (5, 130):
        mean, var, g, gv = W.solve_grad(scene, pts, bc, N, 3, 8)
        pv, pg = W.trace_grad(scene, pts, bc, N, 3, 8)
        m0, v0 = W.solve(scene, pts, bc, N, 3, 8)
        torch.cuda.synchronize()
        pg64 = pg.double()
        assert torch.allclose(g.double(), pg64.mean(dim=1), rtol=1e-5, atol=1e-6)
        assert torch.allclose(gv.double(), pg64.var(dim=1), rtol=1e-4, atol=1e-8)
        assert torch.allclose(mean, m0, rtol=1e-6, atol=1e-7)
        assert torch.allclose(var, v0, rtol=1e-5, atol=1e-8)
    with pytest.raises(W.WobError):  # the variance needs two paths
        W.solve_grad(scene, pts, bc, 1, 3, 8)
    with pytest.raises(W.WobError):  # density mode has no gradient
        W.solve_grad(scene, pts, W.BC(1, 1, W.PROG_INVDIST, (2.0, 0.5, 0.0), density=True), 4, 3, 8)
    scene.close()


def test_grad_full_size_sampled(W):
    """The benchmark workload (icosphere slice, 167,604 points x 256 paths x 6
    lines, double layer) solved with the gradient: 256 sampled (point, path)
    items of the same launch shape against the oracle's paths, and the mean
    gradient against the analytic gradient within its standard errors."""
    w = I.config_icosphere_slice()
    scene = W.Scene(w.mesh, W.F32)
    bc = W.BC(w.bc["domain"], w.bc["formulation"], w.bc["program"], tuple(w.bc["params"]))
    pts = dev(w.points, torch.float32)
    P, N, M = w.points.shape[0], w.samples, w.walk_len
    mean, var, g, gv = W.solve_grad(scene, pts, bc, N, M, w.seed)
    torch.cuda.synchronize()
    x0 = np.array(w.bc["params"])
    r = w.points - x0
    exact = -r / np.linalg.norm(r, axis=1)[:, None] ** 3
    gn = g.double().cpu().numpy()
    se = np.sqrt(gv.double().cpu().numpy() / N)
    # heavy tails near the boundary (the hypersingular kernel): compare the
    # points at least 0.2 inside, pooled
    far = w.points[:, 0] ** 2 + w.points[:, 1] ** 2 < 0.7 ** 2
    z = (gn[far] - exact[far]) / np.maximum(se[far], 1e-12)
    # (the double-layer gradient's variance is only just finite, so the
    # standard errors are rough: a loose fraction)
    assert np.mean(np.abs(z) < 4.5) > 0.97, np.mean(np.abs(z) < 4.5)
    # sampled paths of the same launch
    rng = np.random.default_rng(1)
    sp = rng.choice(P, 64, replace=False)
    sub = dev(w.points[sp], torch.float32)
    pv, pg = W.trace_grad(scene, sub, bc, N, M, w.seed)
    torch.cuda.synchronize()
    # the sampled points' paths use the points' own indices as counters in the
    # full solve; trace them with the same indices through the oracle
    om = oracle.OracleMesh(w.mesh)
    ob = oracle.make_bc(w.bc["domain"], w.bc["formulation"], w.bc["program"], w.bc["params"])
    ks = rng.choice(N, 4, replace=False)
    ip = np.repeat(np.arange(64), 4)
    ik = np.tile(ks, 64)
    orc = oracle.trace_grad(om, w.points[sp], ob, M, w.seed, ip, ik)
    gg = pg.double().cpu().numpy()[ip, ik]
    ok = orc["graze"] >= PT.GRAZE
    tol = PT.tolerance(orc["grad_abs"], orc["grad_err"], PT.RTOL_F32)[:, None]
    bad = np.any(np.abs(gg - orc["grad"]) > tol, axis=1) & ok
    assert bad.sum() == 0, bad.sum()
    scene.close()


def _inward(mesh, n, depths, seed):
    on, prim = I.mesh_surface_points(mesh, n, seed)
    v, t = mesh.verts, mesh.prims[prim]
    nrm = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    return on - np.asarray(depths)[:, None] * nrm


def test_grad_split_parity_3d_f32(W):
    """Boundary split of the double-layer gradient (coupled walk from the
    nearest boundary point): per-path value and gradient parity at points
    0.002 to 0.05 inside a perturbed sphere and in its interior, some points
    without an anchor (-1), M = 1 and 4."""
    mesh = PT.f32_mesh(I.perturb_radial(I.icosphere(10), 0.1, 3, 4))
    pts = PT.f32(np.concatenate([_inward(mesh, 30, np.geomspace(0.002, 0.05, 30), 3),
                                 I.ball_points(10, 0.6, 4)]))
    A, AP = I.nearest_boundary_points(mesh, pts, inset=1e-3)
    A = PT.f32(A)
    AP[::7] = -1
    bc = dict(domain=1, formulation=1, program=oracle.PROG_INVDIST, params=(2.0, 0.5, 0.0))
    for M in (1, 4):
        run_grad_parity(W, mesh, pts, bc, 64, M, 21 + M, "f32", anchors=A, anchor_prim=AP)


def test_grad_split_parity_2d_f64(W):
    """The same on the 128-gon in FP64 (x^2 - y^2), points near the boundary."""
    c = I.circle_polygon(128)
    ang = np.random.default_rng(6).uniform(0, 2 * np.pi, 30)
    r = 1.0 - np.geomspace(0.002, 0.1, 30)
    pts = np.stack([r * np.cos(ang), r * np.sin(ang)], axis=1)
    A, AP = I.nearest_boundary_points(c, pts, inset=1e-3)
    bc = dict(domain=1, formulation=1, program=oracle.PROG_QUAD, params=())
    run_grad_parity(W, c, pts, bc, 64, 3, 23, "f64", anchors=A, anchor_prim=AP)


def test_grad_split_arguments(W):
    """Anchors go with the double layer only; both arrays or neither; an
    invalid anchor id gives that point's gradient as NaN, the others as
    usual."""
    mesh = PT.f32_mesh(I.perturb_radial(I.icosphere(6), 0.1, 3, 4))
    scene = W.Scene(mesh, W.F32)
    pts_np = PT.f32(I.ball_points(6, 0.8, 1))
    A, AP = I.nearest_boundary_points(mesh, pts_np, inset=1e-3)
    pts, ta, tp = dev(pts_np, torch.float32), dev(PT.f32(A), torch.float32), dev(AP, torch.int32)
    sl = W.BC(-1, W.SINGLE_LAYER, W.PROG_INVDIST, (0.1, 0.2, 0.0))
    with pytest.raises(W.WobError):
        W.trace_grad(scene, pts, sl, 8, 3, 1, anchors=ta, anchor_prim=tp)
    dl = W.BC(1, 1, W.PROG_INVDIST, (2.0, 0.5, 0.0))
    with pytest.raises(W.WobError):
        W.trace_grad(scene, pts, dl, 8, 3, 1, anchors=ta)
    bad = tp.clone()
    bad[2] = mesh.n_prims + 5
    v, g = W.trace_grad(scene, pts, dl, 8, 3, 1, anchors=ta, anchor_prim=bad)
    v0, g0 = W.trace_grad(scene, pts, dl, 8, 3, 1, anchors=ta, anchor_prim=tp)
    torch.cuda.synchronize()
    assert torch.isnan(g[2]).any(dim=-1).all()
    keep = [0, 1, 3, 4, 5]
    assert torch.equal(g[keep], g0[keep]) and torch.equal(v, v0)
    scene.close()


def test_grad_split_statistics(W):
    """wob_solve_grad with anchors: its mean and variance are those of
    wob_trace_grad's split paths; the value is unchanged."""
    mesh = PT.f32_mesh(I.perturb_radial(I.icosphere(8), 0.1, 3, 4))
    scene = W.Scene(mesh, W.F32)
    pts_np = PT.f32(_inward(mesh, 37, np.full(37, 0.01), 5))
    A, AP = I.nearest_boundary_points(mesh, pts_np, inset=1e-3)
    pts, ta, tp = dev(pts_np, torch.float32), dev(PT.f32(A), torch.float32), dev(AP, torch.int32)
    bc = W.BC(1, 1, W.PROG_INVDIST, (2.0, 0.5, 0.0))
    mean, var, g, gv = W.solve_grad(scene, pts, bc, 130, 3, 8, anchors=ta, anchor_prim=tp)
    pv, pg = W.trace_grad(scene, pts, bc, 130, 3, 8, anchors=ta, anchor_prim=tp)
    m0, v0 = W.solve(scene, pts, bc, 130, 3, 8)
    torch.cuda.synchronize()
    pg64 = pg.double()
    assert torch.allclose(g.double(), pg64.mean(dim=1), rtol=1e-5, atol=1e-6)
    assert torch.allclose(gv.double(), pg64.var(dim=1), rtol=1e-4, atol=1e-8)
    assert torch.allclose(mean, m0, rtol=1e-6, atol=1e-7)
    scene.close()
