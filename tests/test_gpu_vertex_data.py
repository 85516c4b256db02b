"""GPU parity with boundary data given per mesh vertex (interpolated linearly on
each primitive; the datum of the primitive's own kind, eq. PoissonBC) against
the FP64 oracle through the C ABI: per-path picks and values for the double
layer, the direct BIE and the single layer (lines, RIS, mixed kinds), 3D FP32
and 2D FP64, the gradient estimator, the batched solve, and scenes built from
device-resident mesh arrays on a stream (wob_build_bvh_ex).
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


def vertex_values(verts: np.ndarray, seed: int) -> np.ndarray:
    """A smooth field plus independent noise per vertex (data that no analytic
    program reproduces), seeded."""
    rng = np.random.default_rng(seed)
    x = np.zeros((verts.shape[0], 3))
    x[:, :verts.shape[1]] = verts
    return np.sin(2 * x[:, 0]) + np.cos(3 * x[:, 1]) * (1 + x[:, 2]) + 0.1 * rng.standard_normal(verts.shape[0])


def run_vertex_parity(W, mesh, pts, pp, bc, vd, N, M, seed, precision):
    prec, dt = (W.F32, torch.float32) if precision == "f32" else (W.F64, torch.float64)
    rtol = PT.RTOL_F32 if precision == "f32" else PT.RTOL_F64
    vd = PT.f32(vd) if precision == "f32" else np.asarray(vd, dtype=np.float64)
    scene = W.Scene(mesh, prec)
    assert scene.info()["n_verts"] == mesh.verts.shape[0]
    wb = W.BC(bc["domain"], bc["formulation"], oracle.PROG_CONST, (), sampling=bc.get("sampling", 0),
              candidates=bc.get("candidates", 0), vertex_data=dev(vd, dt))
    tpp = None if pp is None else dev(pp, torch.int32)
    val, vprim, vm = W.trace(scene, dev(pts, dt), wb, N, M, seed, point_prim=tpp)
    torch.cuda.synchronize()
    ob = oracle.make_bc(bc["domain"], bc["formulation"], oracle.PROG_CONST, (0.0,),
                        sampling=bc.get("sampling", 0), candidates=bc.get("candidates", 0) or 16,
                        vertex_data=vd)
    orc = PT.oracle_all_paths(oracle.OracleMesh(mesh), pts, pp, ob, N, M, seed)
    L = orc["vtx_prim"].shape[1]
    res = PT.compare_paths(orc, val.cpu().double().numpy().reshape(-1),
                           vprim.cpu().numpy().reshape(-1, L), vm.cpu().numpy().reshape(-1, L), rtol)
    print(res.summary(), flush=True)
    res.assert_exact()
    scene.close()
    return res


def test_vertex_data_double_layer_3d_f32(W):
    """Interior Dirichlet on a perturbed icosphere, FP32, M = 5, ragged sizes."""
    mesh = PT.f32_mesh(I.perturb_radial(I.icosphere(10), 0.1, 3, 4))
    pts = PT.f32(I.ball_points(45, 0.8, 5))
    bc = dict(domain=1, formulation=1)
    run_vertex_parity(W, mesh, pts, None, bc, vertex_values(mesh.verts, 1), 70, 5, 31, "f32")


def test_vertex_data_direct_neumann_exterior_3d_f32(W):
    """Exterior Neumann by the direct BIE (the all-hits source term reads the
    data at every hit), points off and on the boundary."""
    s = I.icosphere(8)
    mesh = PT.f32_mesh(I.Mesh(3, s.verts, s.prims, np.full(s.n_prims, 1, np.uint8), None))
    off = I.ball_points(40, 2.5, 1, r_min=1.2)
    on, onp = I.mesh_surface_points(mesh, 24, 2)
    pts = PT.f32(np.concatenate([off, on]))
    pp = np.concatenate([np.full(40, -1), onp]).astype(np.int32)
    bc = dict(domain=-1, formulation=2)
    run_vertex_parity(W, mesh, pts, pp, bc, vertex_values(mesh.verts, 2), 64, 4, 3, "f32")


@pytest.mark.parametrize("sampling", [0, 1])
def test_vertex_data_mixed_tori_f32(W, sampling):
    """Tori union with random Dirichlet / Neumann / Robin triangles (alpha = 1),
    single layer with the transformed first-kind rows, lines and RIS, points
    off and on the boundary."""
    w = I.config_tori(grid_n=20, n_points=80, boundary_frac=0.25, samples=64, walk_len=4)
    kind = np.random.default_rng(5).integers(0, 3, w.mesh.n_prims).astype(np.uint8)
    mesh = I.Mesh(3, w.mesh.verts, w.mesh.prims, kind, np.full(w.mesh.n_prims, 1.0))
    bc = dict(domain=-1, formulation=0, sampling=sampling, candidates=16)
    run_vertex_parity(W, mesh, w.points, w.point_prim, bc, vertex_values(mesh.verts, 3), 64, 4, 19, "f32")


def test_vertex_data_mixed_2d_f64(W):
    """2D interior mixed problem in FP64, points off and on the boundary."""
    c = I.circle_polygon(128)
    kind = np.random.default_rng(1).integers(0, 3, 128).astype(np.uint8)
    mesh = I.Mesh(2, c.verts, c.prims, kind, np.full(128, 1.0))
    pts = I.disk_points(40, 0.8, 4)
    s = np.random.default_rng(2).random(8)
    bp = np.arange(8, dtype=np.int32) * 13
    on = c.verts[c.prims[bp, 0]] + s[:, None] * (c.verts[c.prims[bp, 1]] - c.verts[c.prims[bp, 0]])
    pp = np.concatenate([np.full(40, -1), bp]).astype(np.int32)
    bc = dict(domain=1, formulation=0)
    run_vertex_parity(W, mesh, np.concatenate([pts, on]), pp, bc, vertex_values(mesh.verts, 4), 64, 4, 8,
                      "f64")


def test_vertex_data_gradient_3d_f32(W):
    """The gradient estimator (Sec. 4.1.3) with per-vertex Dirichlet data: the
    value and every component within the per-path bar."""
    mesh = PT.f32_mesh(I.perturb_radial(I.icosphere(10), 0.1, 3, 4))
    pts = PT.f32(I.ball_points(40, 0.8, 5))
    vd = PT.f32(vertex_values(mesh.verts, 5))
    scene = W.Scene(mesh, W.F32)
    wb = W.BC(1, 1, vertex_data=dev(vd, torch.float32))
    N, M, seed = 64, 4, 13
    val, g = W.trace_grad(scene, dev(pts, torch.float32), wb, N, M, seed)
    torch.cuda.synchronize()
    ob = oracle.make_bc(1, 1, oracle.PROG_CONST, (0.0,), vertex_data=vd)
    P = pts.shape[0]
    orc = oracle.trace_grad(oracle.OracleMesh(mesh), pts, ob, M, seed, np.repeat(np.arange(P), N),
                            np.tile(np.arange(N), P))
    ok = orc["graze"] >= PT.GRAZE
    gv = val.cpu().double().numpy().reshape(-1)
    gg = g.cpu().double().numpy().reshape(-1, 3)
    vtol = np.maximum(PT.tolerance(orc["abs_sum"], orc["err"], PT.RTOL_F32), 1e-300)
    gtol = np.maximum(PT.tolerance(orc["grad_abs"], orc["grad_err"], PT.RTOL_F32), 1e-300)[:, None]
    bad = (np.abs(gv - orc["value"]) > vtol) | np.any(np.abs(gg - orc["grad"]) > gtol, axis=1)
    print(f"paths={len(ok)} grazing={int((~ok).sum())} mismatch={int((bad & ok).sum())}", flush=True)
    assert (~ok).sum() <= 0.01 * len(ok)
    assert int((bad & ok).sum()) == 0
    scene.close()


def test_vertex_data_batched_equals_single(W):
    """A batch mixing a per-vertex-data problem with an analytic-program one on
    the same scene: each problem's mean equals its single-problem solve's
    (same paths, same order of the sums)."""
    mesh = PT.f32_mesh(I.perturb_radial(I.icosphere(8), 0.1, 3, 4))
    scene = W.Scene(mesh, W.F32)
    vd = dev(PT.f32(vertex_values(mesh.verts, 6)), torch.float32)
    pts = dev(PT.f32(I.ball_points(300, 0.8, 7)), torch.float32)
    bv = W.BC(1, 1, vertex_data=vd)
    bp = W.BC(1, 1, oracle.PROG_LINEAR, (0.3, -1.1, 0.7, 0.25))
    probs = [dict(scene=scene, points=pts, bc=bv, samples=64, walk_len=4, seed=3),
             dict(scene=scene, points=pts, bc=bp, samples=64, walk_len=4, seed=4)]
    outs = W.solve_batched(probs)
    torch.cuda.synchronize()
    for p, (mean, var) in zip(probs, outs):
        m1, v1 = W.solve(scene, pts, p["bc"], 64, 4, p["seed"])
        torch.cuda.synchronize()
        np.testing.assert_allclose(mean.cpu().numpy(), m1.cpu().numpy(), rtol=1e-6, atol=1e-6)
    scene.close()


def test_vertex_data_rejected_when_mismatched(W):
    mesh = PT.f32_mesh(I.icosphere(4))
    scene = W.Scene(mesh, W.F32)
    pts = dev(PT.f32(I.ball_points(8, 0.5, 1)), torch.float32)
    n = mesh.verts.shape[0]
    for bad in (torch.zeros(n - 1, device="cuda"), torch.zeros(n, dtype=torch.float64, device="cuda")):
        with pytest.raises(W.WobError):
            W.solve(scene, pts, W.BC(1, 1, vertex_data=bad), 8, 2)
    scene.close()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_build_from_device_arrays_on_a_stream(W, precision):
    """wob_build_bvh_ex with device-resident mesh arrays on a side stream builds
    the same scene as wob_build_bvh from host arrays: equal scene info and
    bit-identical traced paths."""
    w = I.config_tori(grid_n=16, n_points=64, boundary_frac=0.25, samples=32, walk_len=4)
    kind = np.random.default_rng(5).integers(0, 3, w.mesh.n_prims).astype(np.uint8)
    mesh = I.Mesh(3, w.mesh.verts, w.mesh.prims, kind, np.linspace(0.5, 1.5, w.mesh.n_prims))
    prec, dt = (W.F32, torch.float32) if precision == "f32" else (W.F64, torch.float64)
    host = W.Scene(mesh, prec)
    side = torch.cuda.Stream()
    d = dict(verts=dev(mesh.verts, torch.float64), prims=dev(mesh.prims, torch.int32),
             kind=dev(mesh.kind, torch.uint8), alpha=dev(mesh.alpha, torch.float64))
    torch.cuda.synchronize()
    built = W.Scene.from_device(3, d["verts"], d["prims"], d["kind"], d["alpha"], prec, stream=side)
    assert built.info() == host.info()
    pts = dev(w.points if precision == "f64" else PT.f32(w.points), dt)
    pp = dev(w.point_prim, torch.int32)
    bc = W.BC(-1, 0, oracle.PROG_LINEAR, (0.3, -1.1, 0.7, 0.25))
    a = W.trace(host, pts, bc, 32, 4, 9, point_prim=pp)
    b = W.trace(built, pts, bc, 32, 4, 9, point_prim=pp)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    # host arrays through the stream form: the same again
    h2 = W.Scene(mesh, prec, stream=side)
    assert h2.info() == host.info()
    for s in (host, built, h2):
        s.close()
