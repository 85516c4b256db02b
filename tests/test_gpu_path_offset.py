"""Path ranges (wob_bc.path_offset): path k of a solve draws the random numbers
of path path_offset + k, so a solve split into ranges of paths holds the
paths of the whole, and the ranges' per-point statistics merge (Chan's
formula) into those of the whole solve: resuming a solve, or sharing its paths
among devices.  Checked against the full range of the same kernel bit for bit,
against the FP64 oracle path by path, and by merging."""
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


def cases(W):
    """(scene mesh, points, point_prim, wob.BC kwargs, M): double layer inside a
    perturbed sphere, single layer (lines, RIS) and direct BIE on the tori."""
    sph = PT.f32_mesh(I.perturb_radial(I.icosphere(8), 0.1, 3, 4))
    w = I.config_tori(grid_n=16, n_points=41, boundary_frac=0.25, samples=64, walk_len=4)
    neu = PT.f32_mesh(I.Mesh(3, w.mesh.verts, w.mesh.prims, np.full(w.mesh.n_prims, 1, np.uint8), None))
    off = w.point_prim < 0
    return [
        ("double layer", sph, PT.f32(I.ball_points(37, 0.8, 5)), None,
         dict(domain=1, formulation=W.DOUBLE_LAYER, program=W.PROG_INVDIST, params=(2.0, 0.5, 0.0)), 5),
        ("single layer", w.mesh, w.points, w.point_prim,
         dict(domain=-1, formulation=W.SINGLE_LAYER, program=w.bc["program"], params=tuple(w.bc["params"])), 4),
        ("single layer RIS", w.mesh, w.points, w.point_prim,
         dict(domain=-1, formulation=W.SINGLE_LAYER, program=w.bc["program"], params=tuple(w.bc["params"]),
              sampling=W.SAMPLE_RIS, candidates=16), 4),
        ("direct", neu, w.points[off], None,
         dict(domain=-1, formulation=W.DIRECT, program=w.bc["program"], params=tuple(w.bc["params"])), 3),
    ]


def test_offset_paths_are_the_full_ranges_columns(W):
    """Paths o .. o + n - 1 of a point, traced with path_offset o, equal (bit for
    bit: values, picks, hit counts) columns o .. o + n - 1 of the trace of
    paths 0 .. o + n - 1."""
    for name, mesh, pts, pp, kw, M in cases(W):
        scene = W.Scene(mesh, W.F32)
        tp = dev(pts, torch.float32)
        tpp = None if pp is None else dev(pp, torch.int32)
        full = W.trace(scene, tp, W.BC(**kw), 160, M, 5, point_prim=tpp)
        part = W.trace(scene, tp, W.BC(**kw, path_offset=100), 60, M, 5, point_prim=tpp)
        torch.cuda.synchronize()
        for a, b in zip(full, part):
            assert torch.equal(a[:, 100:160], b), name
        scene.close()


def test_offset_paths_match_oracle(W):
    """Paths 1000 .. 1063 (path_offset 1000) against the oracle's paths of the
    same ids, per path (picks exact outside the grazing class, values within
    the per-path bar)."""
    name, mesh, pts, pp, kw, M = cases(W)[1]
    scene = W.Scene(mesh, W.F32)
    N, seed, o = 64, 9, 1000
    val, vprim, vm = W.trace(scene, dev(pts, torch.float32), W.BC(**kw, path_offset=o), N, M, seed,
                             point_prim=dev(pp, torch.int32))
    torch.cuda.synchronize()
    P = pts.shape[0]
    ob = oracle.make_bc(kw["domain"], kw["formulation"], kw["program"], kw["params"])
    orc = oracle.trace(oracle.OracleMesh(mesh), pts, pp, ob, M, seed, np.repeat(np.arange(P), N),
                       np.tile(np.arange(N), P) + o, want_pos=False)
    L = orc["vtx_prim"].shape[1]
    res = PT.compare_paths(orc, val.cpu().double().numpy().reshape(-1), vprim.cpu().numpy().reshape(-1, L),
                           vm.cpu().numpy().reshape(-1, L), PT.RTOL_F32)
    print(name, res.summary(), flush=True)
    res.assert_exact()
    scene.close()


def test_resume_by_path_ranges_merges_into_the_whole(W):
    """A solve of 256 paths split into ranges of 100 and 156 (the second with
    path_offset 100): Chan's merge of the two ranges' (n, mean, M2) equals the
    whole solve's mean and variance to the binary32 rounding of the outputs."""
    for name, mesh, pts, pp, kw, M in cases(W):
        scene = W.Scene(mesh, W.F32)
        tp = dev(pts, torch.float32)
        tpp = None if pp is None else dev(pp, torch.int32)
        m, v = W.solve(scene, tp, W.BC(**kw), 256, M, 3, point_prim=tpp)
        m1, v1 = W.solve(scene, tp, W.BC(**kw), 100, M, 3, point_prim=tpp)
        m2, v2 = W.solve(scene, tp, W.BC(**kw, path_offset=100), 156, M, 3, point_prim=tpp)
        torch.cuda.synchronize()
        m, v, m1, v1, m2, v2 = (x.cpu().double().numpy() for x in (m, v, m1, v1, m2, v2))
        n1, n2 = 100.0, 156.0
        n = n1 + n2
        d = m2 - m1
        mm = m1 + d * n2 / n
        vv = ((n1 - 1) * v1 + (n2 - 1) * v2 + d * d * n1 * n2 / n) / (n - 1)
        scale = np.abs(m) + np.sqrt(v / n) + 1e-30
        err = np.abs(mm - m) / scale
        print(f"{name}: merged mean max rel {err.max():.2e}", flush=True)
        assert err.max() < 2e-6, name
        np.testing.assert_allclose(vv, v, rtol=2e-5, atol=1e-12)
        scene.close()


def test_path_offset_arguments(W):
    mesh = PT.f32_mesh(I.icosphere(4))
    scene = W.Scene(mesh, W.F32)
    pts = dev(PT.f32(I.ball_points(8, 0.5, 1)), torch.float32)
    for o, n in ((-1, 8), (2 ** 31 - 8, 8), (2 ** 31 - 1, 1)):
        with pytest.raises(W.WobError):
            W.solve(scene, pts, W.BC(1, W.DOUBLE_LAYER, W.PROG_CONST, (1.0,), path_offset=o), n, 2,
                    want_var=n > 1)
    m, _ = W.solve(scene, pts, W.BC(1, W.DOUBLE_LAYER, W.PROG_CONST, (1.0,), path_offset=2 ** 31 - 9), 8, 2)
    torch.cuda.synchronize()
    np.testing.assert_allclose(m.cpu().numpy(), 1.0, atol=1e-5)  # constant data, any paths
    scene.close()
    # the forward estimator's paths have ids of their own: no offset
    neu = I.Mesh(3, mesh.verts, mesh.prims, np.full(mesh.n_prims, 1, np.uint8), None)
    s2 = W.Scene(neu, W.F32)
    with pytest.raises(W.WobError):
        W.forward_paths(s2, W.BC(-1, W.SINGLE_LAYER, W.PROG_INVDIST, (0.2, 0.1, 0.0), path_offset=4), 64, 3)
    s2.close()
