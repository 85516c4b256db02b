"""GPU parity of the forward (adjoint) single-layer estimator (Sec. 4.4.3,
forward estimator) against the FP64 oracle, through the C ABI.

Paths: every vertex's primitive and hit count must agree for non-grazing
paths; positions and strengths within the rounding of the start weight (the
line steps multiply it by exact integers and signs).  Connection step: GPU and
oracle on the same seeded synthetic records.
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


def _neumann(mesh):
    return I.Mesh(mesh.dim, mesh.verts, mesh.prims, np.full(mesh.n_prims, 1, np.uint8))


def compare_forward(orc, vtx, vp, vm, precision):
    """Per-path comparison; returns (n, n_graze, n_checked, n_mismatch, worst ratio).
    Every vertex's primitive and line hit count identical; its position within
    RTOL (1 + |y|) + KAPPA u P and its strength within RTOL |w| + KAPPA u E_w,
    P and E_w the oracle's rounding-error bounds of the vertex (its position
    error propagated along the path; the strength's first factor 2 phi q A / P
    carries the rounding of q, the steps multiply by the exact +-m)."""
    rtol = PT.RTOL_F32 if precision == "f32" else PT.RTOL_F64
    n, M = orc["w"].shape
    dim = orc["pos"].shape[2]
    g_pos = vtx[:, :, :dim]
    g_w = vtx[:, :, 3]
    graze = orc["graze"] < PT.graze_for(rtol)
    ok = ~graze
    vmis = np.any(orc["prim"] != vp, axis=1) | np.any(orc["m"] != vm, axis=1)
    werr = np.abs(g_w - orc["w"])
    wtol = np.maximum(PT.tolerance(np.abs(orc["w"]), orc["werr"], rtol), 1e-300)
    # positions of live vertices (an ended path's records sit at 1e18 on the GPU)
    perr = np.where(orc["prim"] >= 0, np.linalg.norm(g_pos - orc["pos"], axis=2), 0.0)
    ptol = PT.tolerance(1.0 + np.linalg.norm(orc["pos"], axis=2), orc["perr"], rtol)
    bad = vmis | np.any(werr > wtol, axis=1) | np.any(perr > ptol, axis=1)
    ratio = np.where(ok[:, None], np.maximum(werr / wtol, perr / ptol), 0.0)
    return n, int(graze.sum()), int(ok.sum()), int((bad & ok).sum()), float(ratio.max())


def run_paths_parity(W, mesh, bc, n_paths, M, seed, precision, weights=None):
    scene = W.Scene(mesh, W.F32 if precision == "f32" else W.F64)
    starts = None if weights is None else W.Starts(scene, weights)
    wb = W.BC(bc["domain"], 3, bc["program"], tuple(bc["params"]))
    vtx, vp, vm = W.forward_paths(scene, wb, n_paths, M, seed, starts=starts, want_vertices=True)
    torch.cuda.synchronize()
    ob = oracle.make_bc(bc["domain"], oracle.SINGLE_LAYER, bc["program"], bc["params"])
    orc = oracle.forward_paths(oracle.OracleMesh(mesh), ob, n_paths, M, seed, start_weight=weights)
    n, ng, nc, nm, worst = compare_forward(orc, vtx.cpu().double().numpy(), vp.cpu().numpy(),
                                           vm.cpu().numpy(), precision)
    print(f"paths={n} grazing={ng} checked={nc} mismatch={nm} worst err/tol={worst:.3f}", flush=True)
    assert ng <= 0.01 * n
    assert nm == 0
    if starts is not None:
        starts.close()
    scene.close()
    return orc, vtx


@pytest.mark.parametrize("start", ["area", "weights"])
def test_forward_paths_parity_3d_f32(W, start):
    """Exterior Neumann (off-centre monopole) on a perturbed sphere, 1,027 paths
    (a ragged last lane group and workgroup), M = 4; starts uniform by area or
    from arbitrary weights with zeros."""
    mesh = _neumann(PT.f32_mesh(I.perturb_radial(I.icosphere(10), 0.1, 3, 4)))
    bc = dict(domain=-1, program=oracle.PROG_INVDIST, params=(0.2, -0.1, 0.05))
    w = None
    if start == "weights":
        w = np.random.default_rng(4).uniform(0.0, 2.0, mesh.n_prims)
        w[::5] = 0.0
    orc, vtx = run_paths_parity(W, mesh, bc, 1027, 4, 17, "f32", weights=w)
    if w is not None:
        assert np.all(w[orc["prim"][:, 0]] > 0)


def test_forward_paths_parity_tori_f32(W):
    """Exterior Neumann on the union of three tori (lines with many hits)."""
    wl = I.config_tori(grid_n=20, n_points=8, samples=8, walk_len=4)
    mesh = _neumann(wl.mesh)
    bc = dict(domain=-1, program=oracle.PROG_INVDIST, params=(0.1, 0.2, -0.1))
    run_paths_parity(W, mesh, bc, 2000, 5, 23, "f32")


def test_forward_paths_parity_2d_f64(W):
    """Interior Neumann with quadratic data on a perturbed circle, FP64."""
    c = I.circle_polygon(200)
    ang = np.arctan2(c.verts[:, 1], c.verts[:, 0])
    mesh = _neumann(I.Mesh(2, c.verts * (1 + 0.1 * np.cos(3 * ang))[:, None], c.prims))
    bc = dict(domain=1, program=oracle.PROG_QUAD, params=())
    run_paths_parity(W, mesh, bc, 1501, 4, 5, "f64")


def test_forward_single_vertex_paths(W):
    """M = 1: no line at all; every record is the start with half its strength."""
    mesh = _neumann(PT.f32_mesh(I.icosphere(6)))
    bc = dict(domain=1, program=oracle.PROG_LINEAR, params=(0.0, 0.0, 1.0, 0.0))
    orc, vtx = run_paths_parity(W, mesh, bc, 5, 1, 3, "f32")
    assert np.all(orc["m"] == 0)


def test_forward_starts_from_data(W):
    """Data-proportional starts built on the device (|q(c_T)| A_T plus a floor
    times the area-weighted mean) pick the same start primitives as a table
    built from the same weights formed with the oracle's boundary datum."""
    mesh = _neumann(PT.f32_mesh(I.perturb_radial(I.icosphere(10), 0.1, 3, 4)))
    c0 = (0.8, 0.1, 0.0)  # close to the surface: the data are concentrated
    scene = W.Scene(mesh, W.F32)
    om = oracle.OracleMesh(mesh)
    ob = oracle.make_bc(-1, oracle.SINGLE_LAYER, oracle.PROG_INVDIST, c0)
    tri = mesh.verts[mesh.prims]
    cen = tri.mean(axis=1)
    area = 0.5 * np.linalg.norm(np.cross(tri[:, 1] - tri[:, 0], tri[:, 2] - tri[:, 0]), axis=1)
    q = np.array([oracle.boundary_datum(om, ob, j, cen[j]) for j in range(mesh.n_prims)])
    bc = W.BC(-1, 3, oracle.PROG_INVDIST, c0)
    for floor in (0.0, 0.1):
        w = (np.abs(q) + floor * np.sum(np.abs(q) * area) / area.sum()) * area
        s1 = W.Starts(scene, data=bc, floor=floor)
        s2 = W.Starts(scene, w)
        _, p1, _ = W.forward_paths(scene, bc, 20000, 1, 5, starts=s1, want_vertices=True)
        _, p2, _ = W.forward_paths(scene, bc, 20000, 1, 5, starts=s2, want_vertices=True)
        same = (p1 == p2).float().mean().item()
        assert same > 0.999, (floor, same)
        s1.close()
        s2.close()
    scene.close()


@pytest.mark.parametrize("dim,precision", [(3, "f32"), (2, "f32"), (3, "f64"), (2, "f64")])
def test_forward_gather_parity(W, dim, precision):
    """Connection of 300 points (two partial workgroups) to 777 synthetic paths
    of 3 vertices (a tenth ending early), points inside and outside the unit
    sphere: mean within the rounding scale, variance within 1e-3 relative."""
    pos, w = I.forward_records(777, 3, dim, 9)
    pts = I.ball_points(300, 2.2, 3, r_min=1.3)[:, :dim]
    pts[::3] *= 0.3
    if precision == "f32":
        pos, w, pts = PT.f32(pos), PT.f32(w), PT.f32(pts)
    mesh = _neumann(I.icosphere(2) if dim == 3 else I.circle_polygon(8))
    scene = W.Scene(mesh, W.F32 if precision == "f32" else W.F64)
    dt = torch.float32 if precision == "f32" else torch.float64
    rec = np.zeros((777, 3, 4))
    rec[:, :, :dim] = pos
    rec[:, :, 3] = w
    mean, var = W.forward_gather(scene, dev(rec, dt), dev(pts, dt))
    torch.cuda.synchronize()
    om, ov, oa = oracle.forward_gather(pos, w, pts)
    rtol = 2e-5 if precision == "f32" else 1e-12
    err = np.abs(mean.cpu().double().numpy() - om)
    assert np.all(err <= rtol * oa), (err / oa).max()
    verr = np.abs(var.cpu().double().numpy() - ov) / ov
    assert verr.max() < (1e-3 if precision == "f32" else 1e-9), verr.max()
    scene.close()


def test_forward_gather_edge_cases(W):
    """No points; one path without variance; a point 1e-6 from a vertex; the
    records of an ended path (strength 0 at 1e18) add nothing, also for a point
    at the origin."""
    mesh = _neumann(I.icosphere(2))
    scene = W.Scene(mesh, W.F64)
    pos, w = I.forward_records(1, 2, 3, 1, end_frac=0.0)
    rec = np.zeros((1, 2, 4))
    rec[:, :, :3] = pos
    rec[:, :, 3] = w
    t = dev(rec, torch.float64)
    m, v = W.forward_gather(scene, t, torch.zeros((0, 3), dtype=torch.float64, device="cuda"))
    assert m.numel() == 0
    pts = np.stack([pos[0, 0] + 1e-6, np.array([0.1, 0.2, 0.3])])
    m, v = W.forward_gather(scene, t, dev(pts, torch.float64), want_var=False)
    om, _, _ = oracle.forward_gather(pos, w, pts)
    assert np.all(np.isfinite(m.cpu().numpy()))
    assert np.allclose(m.cpu().numpy(), om, rtol=1e-12, atol=0)
    with pytest.raises(W.WobError):
        W.forward_gather(scene, t, dev(pts, torch.float64), want_var=True)  # one path: no variance
    ended = rec.copy()
    ended[0, 1] = (1e18, 1e18, 1e18, 0.0)
    p0 = np.array([[0.0, 0.0, 0.0], [0.3, -0.2, 0.1]])
    m, _ = W.forward_gather(scene, dev(ended, torch.float64), dev(p0, torch.float64), want_var=False)
    om, _, _ = oracle.forward_gather(pos[:, :1], w[:, :1], p0)
    assert np.allclose(m.cpu().numpy(), om, rtol=1e-12, atol=0)
    scene.close()


def test_forward_rejects_bad_arguments(W):
    mesh = I.icosphere(3)
    bc = W.BC(1, 3, W.PROG_LINEAR, (0.0, 0.0, 1.0, 0.0))
    sd = W.Scene(mesh, W.F32)  # all Dirichlet
    with pytest.raises(W.WobError):
        W.forward_paths(sd, bc, 8, 2)
    sn = W.Scene(_neumann(mesh), W.F32)
    with pytest.raises(W.WobError):  # RIS is a backward sampling
        W.forward_paths(sn, W.BC(1, 3, 1, (0.0, 0.0, 1.0, 0.0), sampling=W.SAMPLE_RIS), 8, 2)
    with pytest.raises(W.WobError):  # the double layer has no forward form here
        W.forward_paths(sn, W.BC(1, 1, 1, (0.0, 0.0, 1.0, 0.0)), 8, 2)
    with pytest.raises(W.WobError):
        W.Starts(sn, -np.ones(mesh.n_prims))
    with pytest.raises(W.WobError):
        W.Starts(sn, np.zeros(mesh.n_prims))
    st = W.Starts(sd, np.ones(mesh.n_prims))
    with pytest.raises(W.WobError):  # a table of another scene
        W.forward_paths(sn, bc, 8, 2, starts=st)
    buf = torch.zeros(8 * 2 * 4 + 1, dtype=torch.float32, device="cuda")
    with pytest.raises(W.WobError):  # records not 16-byte aligned
        W.forward_paths(sn, bc, 8, 2, out=buf[1:].view(8, 2, 4))
    st.close()
    sd.close()
    sn.close()


def test_forward_full_size_sampled(W):
    """The benchmark's forward workload (exterior Neumann on the three-tori
    union, 200,992 triangles, 2^20 paths of 4 vertices, |q|-proportional
    starts): its first 2,000 paths against the oracle's, and the connection of
    16 sampled points against the oracle's connection to the same GPU-independent
    synthetic records at the full path count."""
    wl = I.config_tori()
    mesh = _neumann(wl.mesh)
    scene = W.Scene(mesh, W.F32)
    c0 = (0.1, 0.2, -0.1)
    cen = mesh.verts[mesh.prims].mean(axis=1)
    om = oracle.OracleMesh(mesh)
    n = om.normals()
    r = cen - np.array(c0)
    q = -np.einsum("ij,ij->i", r, n) / np.linalg.norm(r, axis=1) ** 3
    e1 = mesh.verts[mesh.prims[:, 1]] - mesh.verts[mesh.prims[:, 0]]
    e2 = mesh.verts[mesh.prims[:, 2]] - mesh.verts[mesh.prims[:, 0]]
    wts = np.abs(q) * 0.5 * np.linalg.norm(np.cross(e1, e2), axis=1)
    starts = W.Starts(scene, wts)
    bc = W.BC(-1, 3, oracle.PROG_INVDIST, c0)
    n_paths, M = 1 << 20, 4
    vtx, vp, vm = W.forward_paths(scene, bc, n_paths, M, 99, starts=starts, want_vertices=True)
    torch.cuda.synchronize()
    ob = oracle.make_bc(-1, oracle.SINGLE_LAYER, oracle.PROG_INVDIST, c0)
    K = 2000
    orc = oracle.forward_paths(om, ob, K, M, 99, start_weight=wts)
    res = compare_forward(orc, vtx[:K].cpu().double().numpy(), vp[:K].cpu().numpy(), vm[:K].cpu().numpy(), "f32")
    print("full-size paths", res, flush=True)
    # 200,992 triangles: lines crossing many small, distant primitives take more
    # ill-conditioned hit decisions (grazing up to 2 %)
    assert res[1] <= 0.02 * K and res[3] == 0
    assert bool(torch.isfinite(vtx).all())
    # connection at full path count on synthetic records, 16 sampled points
    pos, w = I.forward_records(n_paths, M, 3, 5)
    pos, w = PT.f32(pos), PT.f32(w)
    rec = np.zeros((n_paths, M, 4), np.float32)
    rec[:, :, :3] = pos
    rec[:, :, 3] = w
    pts = PT.f32(I.ball_points(16, 2.0, 8, r_min=1.2))
    mean, var = W.forward_gather(scene, dev(rec, torch.float32), dev(pts, torch.float32))
    torch.cuda.synchronize()
    om_, ov, oa = oracle.forward_gather(pos, w, pts)
    err = np.abs(mean.cpu().double().numpy() - om_)
    assert np.all(err <= 2e-5 * oa), (err / oa).max()
    assert np.max(np.abs(var.cpu().double().numpy() - ov) / ov) < 1e-3
    starts.close()
    scene.close()
