"""Learned control variate on the GPU against the FP64 oracle: closed-form
add-back, per-path corrected values, density-mode targets, the table from the
network, and unbiasedness of the corrected solve."""
import numpy as np
import pytest

import oracle
from paper_2305_04403_amd import inputs as I
from tests import parity as PT
from tests.test_oracle_cv_pins import MLP_ACC, rand_net

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def W():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_04403_amd import wob
    wob.lib()
    return wob


@pytest.fixture(scope="module")
def tori():
    return I.config_tori(grid_n=16, n_points=60, boundary_frac=0.25, samples=64, walk_len=4)


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def bcs(W, w, **kw):
    b = w.bc
    return (W.BC(b["domain"], b["formulation"], b["program"], tuple(b["params"]), **kw),
            oracle.make_bc(b["domain"], b["formulation"], b["program"], b["params"], **kw))


def test_addback_matches_oracle(W, tori):
    rng = np.random.default_rng(1)
    g = PT.f32(rng.standard_normal(tori.mesh.n_prims) + 0.5)
    scene = W.Scene(tori.mesh, W.F32)
    out = W.cv_addback(scene, dev(g), dev(tori.points), seed=9)
    torch.cuda.synchronize()
    om = oracle.OracleMesh(tori.mesh)
    ref = oracle.cv_addback(om, g, tori.points, seed=9, randomized=True)
    exact = oracle.cv_addback(om, g, tori.points)
    scale = oracle.cv_addback(om, np.abs(g), tori.points)
    err = np.abs(out.cpu().double().numpy() - ref) / scale
    print(f"add-back max error / sum |g| potential: {err.max():.2e}; "
          f"randomized vs closed form {np.max(np.abs(ref - exact) / scale):.2e}")
    assert err.max() < 2e-5
    scene.close()


def test_addback_zero_and_sparse_tables(W, tori):
    """The add-back skips the tiles of 256 triangles whose g values are all
    zero: a zero table gives exact zeros, and a table with three non-zero
    triangles (6,552 triangles in 26 tiles: at least 23 tiles skipped) matches
    the oracle at the dense table's bar."""
    scene = W.Scene(tori.mesh, W.F32)
    pts = dev(tori.points)
    zero = W.cv_addback(scene, dev(np.zeros(tori.mesh.n_prims, np.float32)), pts, seed=9)
    g = np.zeros(tori.mesh.n_prims, np.float32)
    g[np.random.default_rng(3).choice(tori.mesh.n_prims, 3, replace=False)] = (1.5, -0.75, 2.0)
    out = W.cv_addback(scene, dev(g), pts, seed=9)
    torch.cuda.synchronize()
    assert bool((zero == 0).all())
    om = oracle.OracleMesh(tori.mesh)
    ref = oracle.cv_addback(om, g, tori.points, seed=9, randomized=True)
    scale = oracle.cv_addback(om, np.abs(g), tori.points)
    err = np.abs(out.cpu().double().numpy() - ref) / scale
    print(f"sparse table: max error / sum |g| potential {err.max():.2e}")
    assert err.max() < 2e-5
    scene.close()


@pytest.mark.parametrize("separate_g0,sampling", [(False, 0), (True, 0), (True, 1)])
def test_trace_cv_matches_oracle(W, tori, separate_g0, sampling):
    """Per-path corrected values against the oracle; with RIS (sampling 1, 16
    candidates) the correction sums over the candidates."""
    rng = np.random.default_rng(2)
    g = PT.f32(rng.standard_normal(tori.mesh.n_prims))
    g0 = PT.f32(rng.standard_normal(tori.mesh.n_prims) * 2.0 + 1.0) if separate_g0 else None
    scene = W.Scene(tori.mesh, W.F32)
    wb, ob = bcs(W, tori, sampling=sampling, candidates=16)
    P, N, M = tori.points.shape[0], 64, 4
    val = W.trace_cv(scene, dev(tori.points), wb, N, M, g=dev(g), seed=3,
                     point_prim=dev(tori.point_prim, torch.int32), g0=None if g0 is None else dev(g0))
    torch.cuda.synchronize()
    ip, ik = np.repeat(np.arange(P), N), np.tile(np.arange(N), P)
    cv = oracle.trace_cv(oracle.OracleMesh(tori.mesh), tori.points, tori.point_prim, ob, M, 3, g, ip, ik,
                         g0=g0, with_scales=True)
    ref = cv["value"]
    plain = oracle.trace(oracle.OracleMesh(tori.mesh), tori.points, tori.point_prim, ob, M, 3, ip, ik,
                         want_pos=False)
    v = val.cpu().double().numpy().reshape(-1)
    ok = plain["graze"] >= PT.GRAZE
    # the corrected path's own magnitude sum (every emission, table value and
    # all-hits term) and rounding-error bound: the plain path's bar
    err = np.abs(v - ref)
    tol = PT.tolerance(cv["abs_sum"], cv["err"], PT.RTOL_F32)
    bad = ok & (err > tol)
    plain_bar = ok & (err <= PT.RTOL_F32 * cv["abs_sum"])
    print(f"cv paths {len(v)}, grazing {int((~ok).sum())}, over the bar {int(bad.sum())}, "
          f"within-plain-bar {plain_bar.sum() / max(ok.sum(), 1):.5f}, "
          f"median rel {np.median((err / np.maximum(cv['abs_sum'], 1e-300))[ok]):.2e}")
    assert (~ok).mean() < 0.01
    assert bad.sum() == 0
    scene.close()


def test_density_mode_paths_match_oracle(W, tori):
    """Training targets: the boundary unknown at boundary points, without its emission."""
    scene = W.Scene(tori.mesh, W.F32)
    wb, ob = bcs(W, tori, density=True)
    pts, prim = I.mesh_surface_points(tori.mesh, 48, 7)
    pts = PT.f32(pts)
    val, vprim, vm = W.trace(scene, dev(pts), wb, 32, 3, 9, point_prim=dev(prim, torch.int32))
    torch.cuda.synchronize()
    orc = PT.oracle_all_paths(oracle.OracleMesh(tori.mesh), pts, prim, ob, 32, 3, 9)
    res = PT.compare_paths(orc, val.cpu().double().numpy().reshape(-1), vprim.cpu().numpy().reshape(-1, 3),
                           vm.cpu().numpy().reshape(-1, 3), PT.RTOL_F32)
    print(res.summary())
    res.assert_exact()
    scene.close()


def test_cv_table_is_network_at_centroids(W, tori):
    params, B = rand_net(21)
    params, B = PT.f32(params), PT.f32(B)
    scene = W.Scene(tori.mesh, W.F32)
    net = W.MLP(3, B, params)
    g = W.cv_table(scene, net).cpu().double().numpy()
    v = tori.mesh.verts[tori.mesh.prims]
    cen = PT.f32(v.mean(axis=1))
    # the device forms the centroid in binary32 (v0 + (e1 + e2) / 3 from the
    # stored binary32 edges): within 4 u32 (|v0| + |e1| + |e2|) per coordinate
    e = np.abs(v[:, 0]) + np.abs(v[:, 1] - v[:, 0]) + np.abs(v[:, 2] - v[:, 0])
    res = oracle.mlp_forward_bound(params, B, cen, MLP_ACC, dy=4 * 2.0 ** -24 * e.max(axis=1))
    d = np.abs(g - res["out"])
    print(f"table: within 1e-5 S {np.mean(d <= 1e-5 * res['scale']):.4f}, max d/bound {np.max(d / res['bound']):.3f}")
    assert np.mean(d <= 1e-5 * res["scale"]) >= 0.99
    assert np.all(d <= res["bound"])
    net.close()
    scene.close()


def test_emission_table_matches_oracle(W, tori):
    """g0 = g + 2 phi s(centroid) with the triangle's own kind (Neumann or Robin)."""
    rng = np.random.default_rng(8)
    g = PT.f32(rng.standard_normal(tori.mesh.n_prims))
    scene = W.Scene(tori.mesh, W.F32)
    wb, ob = bcs(W, tori)
    g0 = W.cv_emission(scene, wb, dev(g)).cpu().double().numpy()
    e0 = W.cv_emission(scene, wb).cpu().double().numpy()
    torch.cuda.synchronize()
    om = oracle.OracleMesh(tori.mesh)
    cen = tori.mesh.verts[tori.mesh.prims].mean(axis=1)
    ref = np.array([2.0 * ob.domain * oracle.boundary_datum(om, ob, j, cen[j]) for j in range(tori.mesh.n_prims)])
    scale = np.abs(ref) + np.median(np.abs(ref))
    assert np.max(np.abs(e0 - ref) / scale) < 1e-5
    assert np.max(np.abs(g0 - (g + ref)) / (scale + np.abs(g))) < 1e-5
    with pytest.raises(W.WobError):  # not a single-layer problem
        W.cv_emission(scene, W.BC(1, W.DOUBLE_LAYER, W.PROG_CONST, (1.0,)))
    scene.close()


@pytest.mark.parametrize("sampling", [0, 1])
def test_solve_cv_is_unbiased_on_gpu(W, tori, sampling):
    """Corrected and plain solves on the same points: the per-point difference of
    the means is within 4.5 standard errors of zero, for an arbitrary table
    (lines and RIS)."""
    rng = np.random.default_rng(5)
    g = PT.f32(rng.standard_normal(tori.mesh.n_prims) * 2.0)
    scene = W.Scene(tori.mesh, W.F32)
    wb, _ = bcs(W, tori, sampling=sampling, candidates=16)
    pts = dev(tori.points)
    pp = dev(tori.point_prim, torch.int32)
    N = 16384
    mp, vp = W.solve(scene, pts, wb, N, 4, seed=1, point_prim=pp)
    g0 = W.cv_emission(scene, wb, dev(g))
    mc, vc = W.solve_cv(scene, pts, wb, N, 4, g=dev(g), seed=2, point_prim=pp, g0=g0)
    torch.cuda.synchronize()
    d = mc.double().cpu().numpy() - mp.double().cpu().numpy()
    se = np.sqrt((vp.double().cpu().numpy() + vc.double().cpu().numpy()) / N)
    z = d / se
    print(f"max |z| = {np.abs(z).max():.2f}")
    assert np.abs(z).max() < 4.5
    # the mean of traced corrected paths plus the add-back is the solve's mean
    val = W.trace_cv(scene, pts, wb, 256, 4, g=dev(g), seed=7, point_prim=pp, g0=g0)
    add = W.cv_addback(scene, g0, pts, seed=7)
    m2, _ = W.solve_cv(scene, pts, wb, 256, 4, g=dev(g), seed=7, point_prim=pp, g0=g0)
    torch.cuda.synchronize()
    np.testing.assert_allclose(m2.cpu().numpy(), val.double().mean(dim=1).cpu().numpy() + add.cpu().numpy(),
                               rtol=1e-5, atol=1e-5)
    scene.close()


@pytest.mark.parametrize("kinds", ["neumann", "mixed"])
def test_trained_table_lowers_variance_against_g0(W, kinds):
    """What the trained network gains over the method without it: on an
    exterior sphere (every line meets it once, so the single-layer weights stay
    bounded and walk estimates of the density carry signal), the pipeline of
    cv.py (density targets from the walk, training on the matrix cores, table
    at the centroids, line-0 emission table) against g = g0 = 0, on the same
    paths (same seed), per point: the paired mean log variance ratio is below
    -0.15 and more than 10 standard errors from 0."""
    import math
    from paper_2305_04403_amd import cv as CV
    s = I.icosphere(16)
    T = s.n_prims
    kk = (np.full(T, 1, np.uint8) if kinds == "neumann"
          else np.random.default_rng(1).integers(1, 3, T).astype(np.uint8))
    mesh = I.Mesh(3, s.verts, s.prims, kk, np.where(kk == 2, 1.0, 0.0)).as_float32_geometry()
    scene = W.Scene(mesh, W.F32)
    bc = W.BC(-1, W.SINGLE_LAYER, W.PROG_INVDIST, (0.5, 0.2, 0.0))
    pts = dev(PT.f32(I.ball_points(20_000, 2.5, 3, r_min=1.1)))
    N, M = 128, 4
    zero = torch.zeros(T, dtype=torch.float32, device="cuda")
    v0 = W.solve_cv(scene, pts, bc, N, M, zero, seed=5, g0=zero)[1].double().cpu().numpy()
    lcv = CV.LearnedControlVariate(scene, bc, M, CV.CVConfig(n_train=1 << 18))
    lcv.fit()
    v1 = lcv.solve(pts, N, seed=5)[1].double().cpu().numpy()
    torch.cuda.synchronize()
    lr = np.log(v1 / v0)
    se = lr.std() / math.sqrt(len(lr))
    print(f"{kinds}: paired mean log(var learned / var g=0) {lr.mean():+.4f} +- {se:.4f}, "
          f"median var ratio {np.median(v1) / np.median(v0):.3f}")
    assert np.all(np.isfinite(lr))
    assert lr.mean() < -0.15 and lr.mean() < -10 * se
    lcv.close()
    scene.close()


def test_density_mode_off_the_boundary_is_nan(W, tori):
    """Density mode at points off the boundary (no boundary unknown there): the
    paths are NaN, on both sides, and counted by the scene's status."""
    scene = W.Scene(tori.mesh, W.F32)
    dbc, od = bcs(W, tori, density=True)
    pts = PT.f32(I.ball_points(5, 0.2, 1) + np.array([3.0, 0.0, 0.0]))
    scene.nonfinite_paths()
    v = W.trace(scene, dev(pts), dbc, 8, 3, 1)[0]
    m, _ = W.solve(scene, dev(pts), dbc, 8, 3, 1)
    torch.cuda.synchronize()
    assert torch.isnan(v).all()
    assert scene.nonfinite_paths() == 5 * 8
    o = oracle.trace(oracle.OracleMesh(tori.mesh), pts, None, od, 3, 1, np.repeat(np.arange(5), 2),
                     np.tile(np.arange(2), 5), want_pos=False)
    assert np.isnan(o["value"]).all()
    scene.close()


def test_non_finite_network_switches_the_control_variate_off(W, tori):
    """A fit that diverges (a learning rate of 1e38, forced from the host: the
    parameters overflow) leaves non-finite parameters: the control variate is
    switched off, says why, and solve() runs plain WoB (the same values as
    wob.solve with the same seed).  Non-finite learning rates and parameters
    are argument errors of the library itself."""
    from paper_2305_04403_amd import cv as CV
    scene = W.Scene(tori.mesh, W.F32)
    wb, _ = bcs(W, tori)
    for bad in (float("nan"), float("inf")):
        with pytest.raises(W.WobError):
            CV.LearnedControlVariate(scene, wb, 4, CV.CVConfig(n_train=32768, lr=bad)).fit()
    lcv = CV.LearnedControlVariate(scene, wb, 4, CV.CVConfig(n_train=32768, lr=1e38))
    info = lcv.fit()
    assert lcv.disabled and info["cv_disabled"] == lcv.disabled
    pts, pp = dev(tori.points), dev(tori.point_prim, torch.int32)
    m, v = lcv.solve(pts, 64, seed=3, point_prim=pp)
    m0, v0 = W.solve(scene, pts, wb, 64, 4, seed=3, point_prim=pp)
    torch.cuda.synchronize()
    assert torch.isfinite(m).all()
    assert torch.equal(m, m0) and torch.equal(v, v0)
    lcv.close()
    scene.close()


def test_training_state_checkpoint_and_resume(W):
    """Parameters and Adam moments saved after 5 training steps and restored
    into a new network: 3 more steps there give the parameters of 3 more
    steps of the uninterrupted network, bit for bit."""
    from tests.test_oracle_cv_pins import rand_net
    params, B = rand_net(21)
    params, B = PT.f32(params), PT.f32(B)
    rng = np.random.default_rng(4)
    y = dev(PT.f32(rng.uniform(-1.2, 1.2, (1024, 3))))
    t = dev(PT.f32(rng.standard_normal(1024)))
    a = W.MLP(3, B, params, max_batch=1024)
    for step in range(1, 6):
        a.train_step(y, t, step, 2e-3)
    torch.cuda.synchronize()
    p5, (m5, v5) = a.params(), a.moments()
    assert np.abs(m5).max() > 0 and np.abs(v5).max() > 0
    b = W.MLP(3, B, params, max_batch=1024)
    b.set_params(p5)
    b.set_moments(m5, v5)
    for step in range(6, 9):
        a.train_step(y, t, step, 2e-3)
        b.train_step(y, t, step, 2e-3)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a.params(), b.params())
    ma, va = a.moments()
    mb, vb = b.moments()
    np.testing.assert_array_equal(ma, mb)
    np.testing.assert_array_equal(va, vb)
    a.close()
    b.close()
