"""Batched persistent solve (one launch, hipGraph replay, autotuned shape)
against single-problem solves and the oracle."""
import os

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


def small_problems(W):
    """Uneven problems: interior Dirichlet and exterior Neumann, N from 64 to 512."""
    specs = [
        (I.perturb_radial(I.icosphere(8), 0.1, 3, 4), None, 1, 1, I.ball_points(301, 0.8, 1), 64, 4),
        (I.perturb_radial(I.icosphere(12), 0.05, 2, 5), None, 1, 1, I.ball_points(77, 0.8, 2), 100, 6),
        (I.icosphere(10), 1, -1, 2, I.ball_points(150, 2.0, 3, r_min=1.2), 256, 3),
        (I.perturb_radial(I.icosphere(6), 0.12, 1, 1), None, 1, 1, I.ball_points(33, 0.7, 4), 512, 3),
        (I.icosphere(5), 1, -1, 2, I.ball_points(1000, 2.0, 5, r_min=1.3), 128, 2),
    ]
    out = []
    for k, (mesh, kind, dom, form, pts, N, M) in enumerate(specs):
        if kind is not None:
            mesh = I.Mesh(3, mesh.verts, mesh.prims, np.full(mesh.n_prims, kind, np.uint8))
        mesh = PT.f32_mesh(mesh)
        pts = PT.f32(pts)
        c = (2.0, 0.5, 0.0) if dom == 1 else (0.2, -0.1, 0.05)
        out.append(dict(mesh=mesh, scene=W.Scene(mesh, W.F32), points=dev(pts, torch.float32), pts=pts,
                        bc=W.BC(dom, form, W.PROG_INVDIST, c), samples=N, walk_len=M, seed=11 + k,
                        obc=oracle.make_bc(dom, form, oracle.PROG_INVDIST, c)))
    return out


def test_batch_equals_single_solves_and_replays(W):
    probs = small_problems(W)
    ref = [W.solve(p["scene"], p["points"], p["bc"], p["samples"], p["walk_len"], p["seed"]) for p in probs]
    torch.cuda.synchronize()
    for tune in ((256, 4), (128, 2), (512, 1), (64, 16)):
        b = W.Batch(probs, tune=tune)
        for rep in range(3):
            outs = b.launch()
            torch.cuda.synchronize()
            for (m, v), (mr, vr) in zip(outs, ref):
                assert torch.equal(m, mr), (tune, rep)
                assert torch.equal(v, vr), (tune, rep)
            # unrelated eager work between replays
            _ = (torch.randn(1000, device="cuda") * 2).sum().item()
            for o in outs:
                o[0].fill_(float("nan"))
        b.close()


def test_batch_trees_of_different_depth(W):
    """Problems whose trees differ in depth share one persistent launch (the
    workgroup's LDS stacks are sized for the deepest): a one-leaf tree, the
    37-level staircase and a sphere, each equal to its single solve."""
    from tests.test_gpu_parity import square_mesh, staircase_mesh
    meshes = [square_mesh(), staircase_mesh(), I.perturb_radial(I.icosphere(8), 0.1, 3, 4)]
    rng = np.random.default_rng(12)
    probs = []
    for k, mesh in enumerate(meshes):
        mesh = PT.f32_mesh(mesh)
        pts = PT.f32(rng.uniform(-0.7, 0.7, (90 + 37 * k, 3)))
        pts[:, 2] = np.where(np.abs(pts[:, 2]) < 0.05, 0.05, pts[:, 2])
        probs.append(dict(scene=W.Scene(mesh, W.F32), points=dev(pts, torch.float32),
                          bc=W.BC(1, 1, W.PROG_INVDIST, (2.0, 0.5, 0.0)), samples=96, walk_len=4, seed=31 + k))
    assert probs[1]["scene"].info()["depth"] > 32 and probs[0]["scene"].info()["n_leaves"] == 1
    ref = [W.solve(p["scene"], p["points"], p["bc"], p["samples"], p["walk_len"], p["seed"]) for p in probs]
    torch.cuda.synchronize()
    b = W.Batch(probs, tune=(128, 2))
    for rep in range(2):
        outs = b.launch()
        torch.cuda.synchronize()
        for (m, v), (mr, vr) in zip(outs, ref):
            # bitwise equal (a point whose paths all miss the open meshes has no
            # finite path and a NaN mean on both sides)
            for x, xr in ((m, mr), (v, vr)):
                assert torch.equal(x.isnan(), xr.isnan()), rep
                assert torch.equal(x[~x.isnan()], xr[~xr.isnan()]), rep
    b.close()
    for p in probs:
        p["scene"].close()


def test_batch_single_layer_forms_equal_single_solves(W):
    """A batch holding every kernel form (double layer, direct BIE, single
    layer with line sampling and with RIS, on a mixed Dirichlet / Neumann /
    Robin mesh, points off and on the boundary) equals the single solves."""
    w = I.config_tori(grid_n=12, n_points=200, boundary_frac=0.25, samples=64, walk_len=4)
    kind = np.random.default_rng(3).integers(0, 3, w.mesh.n_prims).astype(np.uint8)
    mixed = PT.f32_mesh(I.Mesh(3, w.mesh.verts, w.mesh.prims, kind, np.full(w.mesh.n_prims, 1.0)))
    sm = W.Scene(mixed, W.F32)
    pm = dev(PT.f32(w.points), torch.float32)
    pp = torch.as_tensor(w.point_prim, dtype=torch.int32, device="cuda")
    base = small_problems(W)
    probs = [base[0], base[2]]
    for k, (sampling, N) in enumerate(((W.SAMPLE_LINE, 64), (W.SAMPLE_RIS, 96))):
        bc = W.BC(-1, 0, W.PROG_INVDIST, (0.2, -0.1, 0.05), sampling=sampling, candidates=8)
        probs.append(dict(scene=sm, points=pm, point_prim=pp, bc=bc, samples=N, walk_len=3, seed=40 + k))
    ref = [W.solve(p["scene"], p["points"], p["bc"], p["samples"], p["walk_len"], p["seed"],
                   point_prim=p.get("point_prim")) for p in probs]
    torch.cuda.synchronize()
    for tune in ((128, 2), (256, 1)):
        b = W.Batch(probs, tune=tune)
        for rep in range(2):
            outs = b.launch()
            torch.cuda.synchronize()
            for i, ((m, v), (mr, vr)) in enumerate(zip(outs, ref)):
                assert torch.isfinite(mr).all(), i
                assert torch.equal(m, mr), (tune, rep, i)
                assert torch.equal(v, vr), (tune, rep, i)
            for o in outs:
                o[0].fill_(float("nan"))
        b.close()


def test_batch_stream_id_follows_oracle(W):
    """A problem with stream_id q draws the counter field 'problem' = q: its mean
    equals the oracle's mean over the same paths (FP32 vs FP64)."""
    p = small_problems(W)[0]
    b = W.Batch([dict(p, stream_id=7)])
    (m, v), = b.launch()
    torch.cuda.synchronize()
    om = oracle.OracleMesh(p["mesh"])
    P, N = p["pts"].shape[0], p["samples"]
    tr = oracle.trace(om, p["pts"], None, p["obc"], p["walk_len"], p["seed"],
                      np.repeat(np.arange(P), N), np.tile(np.arange(N), P), problem=7, want_pos=False)
    mo = tr["value"].reshape(P, N).mean(axis=1)
    # the mean of N paths is within the mean of their bars (plus the binary32
    # rounding of the mean itself)
    tol = PT.tolerance(tr["abs_sum"], tr["err"], PT.RTOL_F32).reshape(P, N).mean(axis=1)
    # points none of whose paths takes a grazing decision (a point holds N of them)
    ok = (tr["graze"].reshape(P, N) >= PT.GRAZE).all(axis=1)
    assert ok.mean() > 0.9
    err = np.abs(m.cpu().double().numpy() - mo)
    assert np.all(err[ok] <= tol[ok] + PT.U_F32 * np.abs(mo[ok]))
    # and it differs from stream 0
    m0, _ = W.solve(p["scene"], p["points"], p["bc"], p["samples"], p["walk_len"], p["seed"])
    assert not torch.equal(m, m0)
    b.close()


def test_batch_autotune_cache(W, tmp_path):
    probs = small_problems(W)
    ref = [W.solve(p["scene"], p["points"], p["bc"], p["samples"], p["walk_len"], p["seed"])[0] for p in probs]
    cache = str(tmp_path / "tune.txt")
    b = W.Batch(probs)
    t1 = b.autotune(sample_stride=2, cache_path=cache)
    assert t1[0] in (64, 128, 256, 512) and 1 <= t1[1] <= 24 and t1[0] // 64 * t1[1] <= 24
    lines = open(cache).read().split("\n")
    assert len([l for l in lines if l.strip()]) == 1
    t2 = b.autotune(sample_stride=2, cache_path=cache)  # served from the cache
    assert t2 == t1
    assert len([l for l in open(cache).read().split("\n") if l.strip()]) == 1
    outs = b.launch()
    torch.cuda.synchronize()
    for (m, _), mr in zip(outs, ref):
        assert torch.equal(m, mr)
    b.close()


def test_batch_rejects_mixed_precision(W):
    probs = small_problems(W)[:1]
    s64 = W.Scene(I.icosphere(3), W.F64)
    bad = dict(probs[0], scene=s64, points=dev(probs[0]["pts"], torch.float64))
    with pytest.raises(W.WobError):
        W.Batch([probs[0], bad])
    with pytest.raises(W.WobError):
        W.Batch([dict(probs[0], stream_id=256)])


def test_full_size_batched_sampled(W):
    """The full 64-problem batched workload in one persistent launch; at sampled
    points of four problems the paths are re-traced with their original
    random-number indices: the batch mean equals the traced paths' mean and the
    traced paths match the oracle path by path."""
    ws = I.config_batched()
    scenes = [W.Scene(w.mesh, W.F32) for w in ws]
    probs = []
    for w, s in zip(ws, scenes):
        probs.append(dict(scene=s, points=dev(w.points, torch.float32),
                          bc=W.BC(w.bc["domain"], w.bc["formulation"], w.bc["program"], w.bc["params"]),
                          samples=w.samples, walk_len=w.walk_len, seed=w.seed))
    b = W.Batch(probs)
    outs = b.launch()
    torch.cuda.synchronize()
    rng = np.random.default_rng(1)
    checked = 0
    for k in (0, 1, 17, 63):
        w, s, (m, v) = ws[k], scenes[k], outs[k]
        assert torch.isfinite(m).all()
        ids = np.sort(rng.choice(w.points.shape[0], 3, replace=False))
        sub = w.points[ids]
        val, vprim, vm = W.trace(s, dev(sub, torch.float32), probs[k]["bc"], w.samples, w.walk_len,
                                 w.seed, point_ids=dev(ids.astype(np.int32), torch.int32))
        torch.cuda.synchronize()
        vv = val.cpu().double().numpy()
        np.testing.assert_allclose(m.cpu().numpy()[ids], vv.mean(axis=1), rtol=2e-6, atol=2e-6)
        om = oracle.OracleMesh(w.mesh)
        ob = oracle.make_bc(w.bc["domain"], w.bc["formulation"], w.bc["program"], w.bc["params"])
        orc = PT.oracle_all_paths(om, sub, None, ob, w.samples, w.walk_len, w.seed, point_ids=ids)
        L = orc["vtx_prim"].shape[1]
        res = PT.compare_paths(orc, vv.reshape(-1), vprim.cpu().numpy().reshape(-1, L),
                               vm.cpu().numpy().reshape(-1, L), PT.RTOL_F32)
        print(w.name, res.summary(), flush=True)
        # meshes of up to 200k triangles: lines that cross many small, distant
        # primitives take more ill-conditioned hit decisions
        res.assert_exact(max_graze_frac=0.02)
        checked += res.n_checked
    assert checked > 1000
    b.close()
