"""Every oracle entry point on tiny inputs (test infrastructure): run under the
sanitized oracle build, where any out-of-bounds access or undefined behaviour
aborts.  Covers 2D and 3D, every formulation, line sampling and RIS, mixed
kinds, density mode, boundary starts, per-vertex data, gradients with and
without the boundary split, the corrected walk, forward paths and their
connection, the network's reference passes, and rejected arguments."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

import oracle  # noqa: E402
from paper_2305_04403_amd import inputs as I  # noqa: E402


def items(P, N):
    return np.repeat(np.arange(P), N), np.tile(np.arange(N), P)


def main():
    sph = I.perturb_radial(I.icosphere(4), 0.1, 3, 4)
    tor = I.config_tori(grid_n=8, n_points=12, boundary_frac=0.25, samples=8, walk_len=3)
    kinds = np.random.default_rng(1).integers(0, 3, tor.mesh.n_prims).astype(np.uint8)
    mixed = I.Mesh(3, tor.mesh.verts, tor.mesh.prims, kinds, np.full(tor.mesh.n_prims, 1.0))
    circ = I.circle_polygon(32)
    c2 = I.Mesh(2, circ.verts, circ.prims, np.random.default_rng(2).integers(0, 3, 32).astype(np.uint8),
                np.full(32, 0.5))
    for mesh in (sph, tor.mesh, mixed, circ, c2):
        om = oracle.OracleMesh(mesh)
        dim = mesh.dim
        pts = I.ball_points(6, 0.5, 1) if dim == 3 else I.disk_points(6, 0.5, 1)
        on, onp = I.mesh_surface_points(mesh, 3, 2) if dim == 3 else (None, None)
        if on is None:
            onp = np.array([1, 5, 9], dtype=np.int32)
            on = 0.5 * (mesh.verts[mesh.prims[onp, 0]] + mesh.verts[mesh.prims[onp, 1]])
        P = np.concatenate([pts, on])
        pp = np.concatenate([np.full(len(pts), -1), onp]).astype(np.int32)
        ip, ik = items(len(P), 4)
        prog = (oracle.PROG_INVDIST, (2.0, 0.5, 0.0)) if dim == 3 else (oracle.PROG_QUAD, ())
        vd = np.sin(mesh.verts[:, 0])
        for form in (oracle.AUTO, oracle.DOUBLE_LAYER, oracle.DIRECT, oracle.SINGLE_LAYER):
            for sampling in (oracle.SAMPLE_LINE, oracle.SAMPLE_RIS):
                for data in (None, vd):
                    for dom in (1, -1):
                        bc = oracle.make_bc(dom, form, prog[0], prog[1], sampling=sampling, candidates=4,
                                            vertex_data=data)
                        try:
                            oracle.trace(om, P, pp, bc, 3, 7, ip, ik, want_pos=True)
                            oracle.solve(om, P, pp, bc, 4, 3, 7)
                            oracle.solve(om, P, pp, oracle.make_bc(dom, form, prog[0], prog[1], density=True,
                                                                   sampling=sampling, candidates=4),
                                         4, 2, 7)
                        except ValueError:
                            pass  # a combination this boundary does not allow
                        try:
                            a, ap = I.nearest_boundary_points(mesh, pts, inset=1e-3)
                            ap[0] = -1
                            oracle.trace_grad(om, pts, bc, 3, 9, *items(len(pts), 4), anchors=a, anchor_prim=ap)
                            oracle.solve_grad(om, pts, bc, 4, 3, 9, anchors=a, anchor_prim=ap)
                        except ValueError:
                            pass
                        try:
                            oracle.trace_grad(om, pts, bc, 3, 9, *items(len(pts), 4))
                            oracle.solve_grad(om, pts, bc, 4, 3, 9)
                        except ValueError:
                            pass
        orig = P
        dirs = np.random.default_rng(3).standard_normal(P.shape)
        oracle.intersect_all(om, orig, dirs, exclude=pp)
        if dim == 3:
            g = np.random.default_rng(4).standard_normal(mesh.n_prims)
            oracle.cv_addback(om, g, pts)
            oracle.cv_addback(om, g, pts, randomized=True)
            bc = oracle.make_bc(-1, oracle.SINGLE_LAYER, prog[0], prog[1])
            try:
                oracle.trace_cv(om, P, pp, bc, 3, 5, g, ip, ik, g0=g, with_scales=True)
            except ValueError:
                pass
    # forward paths and their connection (all-Neumann)
    neu = I.Mesh(3, sph.verts, sph.prims, np.full(sph.n_prims, 1, np.uint8))
    om = oracle.OracleMesh(neu)
    for sw in (None, np.linspace(0.1, 1.0, neu.n_prims)):
        f = oracle.forward_paths(om, oracle.make_bc(-1, oracle.SINGLE_LAYER, oracle.PROG_INVDIST, (0.1, 0.0, 0.0)),
                                 16, 3, 5, start_weight=sw)
        oracle.forward_gather(f["pos"], f["w"], I.ball_points(5, 2.0, 3, r_min=1.3))
    # the network's reference passes
    n = oracle.mlp_n_params()
    rng = np.random.default_rng(6)
    params = rng.standard_normal(n) * 0.05
    B = rng.standard_normal((16, 3))
    y = rng.uniform(-1, 1, (9, 3))
    oracle.mlp_forward(params, B, y, bf16=True)
    oracle.mlp_forward_bound(params, B, y, (7.0, 25.0, 35.0), dy=np.full(9, 1e-7))
    t = rng.standard_normal(9)
    t[3] = np.nan
    _, gr = oracle.mlp_loss_grad(params, B, y, t, bf16=True)
    oracle.adam_step(params.copy(), np.zeros(n), np.zeros(n), gr, 1, 1e-3)
    # rejected arguments
    for bad in (dict(walk_len=0), dict(anchor=True)):
        try:
            om = oracle.OracleMesh(sph)
            if "anchor" in bad:
                oracle.trace_grad(om, pts3 := I.ball_points(2, 0.5, 1),
                                  oracle.make_bc(-1, oracle.SINGLE_LAYER, oracle.PROG_CONST, (1.0,)), 2, 1,
                                  *items(2, 2), anchors=pts3, anchor_prim=np.zeros(2, np.int32))
            else:
                oracle.solve(om, I.ball_points(2, 0.5, 1), None, oracle.make_bc(), 2, 0, 1)
            raise SystemExit("an invalid call was accepted")
        except ValueError:
            pass
    print("ok")


if __name__ == "__main__":
    main()
