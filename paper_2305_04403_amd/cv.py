"""Learned control variate for the single-layer walk (not in the paper).

The network learns, from estimates that WoB itself produces, the boundary
unknown mu(y) minus its own emission 2 phi s(y) (the part of mu that the rest
of a path carries).  Its values at the primitive centroids form the table g of
``wob_solve_cv``, whose estimator is unbiased for every g, so the network only
has to be good enough to cut variance.

Steps, each a call into libwob.so (this module only sequences them):
  1. ``wob_sample_boundary``: n area-uniform boundary points;
  2. ``wob_solve`` in density mode (walk length M - 1, a few paths each):
     one noisy estimate of the target per point;
  3. ``wob_mlp_train_step`` (matrix-core forward / backward + Adam) over the
     points, cosine learning-rate decay, on targets standardised and clipped
     inside the loss (median and interquartile range of a 64k subsample read
     back to the host; clipping only shapes the fit: the estimator stays exact
     for any g);
  4. the output layer is rescaled to the raw targets, ``wob_cv_table``
     evaluates the network at every centroid (g) and ``wob_cv_emission`` adds
     the line-0 emission at the centroid (g0 = g + 2 phi s).
If training leaves non-finite parameters, or the tables hold non-finite
values, the control variate is switched off (``disabled`` names why) and
``solve`` runs plain WoB, which needs no table.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Optional

import numpy as np

from . import wob

N_FREQ, HIDDEN, LAYERS = 16, 128, 4


@dataclasses.dataclass
class CVConfig:
    n_train: int = 2_000_000   # boundary points with one target each
    target_paths: int = 4      # WoB paths averaged per target
    epochs: int = 1
    batch: int = 16384
    lr: float = 2e-3
    sigma: float = 1.5         # scale of the Fourier frequencies
    clip: float = 5.0          # targets clipped to median +- clip * (robust std) for the fit
    seed: int = 12345


def init_params(dim: int, sigma: float, seed: int):
    """He-initialised parameters and a Gaussian Fourier matrix (binary32)."""
    rng = np.random.default_rng(seed)
    n = wob.lib().wob_mlp_n_params()
    p = np.zeros(n, dtype=np.float32)
    o, n_in = 0, 2 * N_FREQ
    for l in range(LAYERS + 1):
        out = 1 if l == LAYERS else HIDDEN
        p[o:o + out * n_in] = rng.standard_normal(out * n_in) * math.sqrt(2.0 / n_in)
        o += out * n_in + out
        n_in = HIDDEN
    B = (rng.standard_normal((N_FREQ, dim)) * sigma).astype(np.float32)
    return p, B


class LearnedControlVariate:
    def __init__(self, scene: wob.Scene, bc: wob.BC, walk_len: int, cfg: Optional[CVConfig] = None):
        if walk_len < 2:
            raise wob.WobError("the learned control variate needs walk_len >= 2")
        self.scene, self.bc, self.walk_len = scene, bc, walk_len
        self.cfg = cfg or CVConfig()
        self.net = None
        self.g = None
        self.g0 = None
        self.timings = {}
        self.history = []
        self.disabled = None  # why the control variate is off, if it is

    def fit(self, stream=None) -> dict:
        import torch
        cfg = self.cfg
        sync = torch.cuda.synchronize
        t0 = time.perf_counter()
        pts, prim = wob.sample_boundary(self.scene, cfg.n_train, cfg.seed, stream=stream)
        dbc = dataclasses.replace(self.bc, density=True)
        target, _ = wob.solve(self.scene, pts, dbc, cfg.target_paths, self.walk_len - 1,
                              seed=cfg.seed + 1, point_prim=prim, want_var=False, stream=stream)
        sub = target[: min(cfg.n_train, 1 << 16)].cpu().numpy().astype(np.float64)
        t1 = time.perf_counter()
        sub = sub[np.isfinite(sub)]
        med = float(np.median(sub)) if sub.size else 0.0
        q25, q75 = np.quantile(sub, [0.25, 0.75]) if sub.size else (0.0, 1.0)
        scale = float(max((q75 - q25) / 1.349, 1e-12))
        tmap = (med, scale, cfg.clip)
        p0, B = init_params(self.scene.dim, cfg.sigma, cfg.seed + 2)
        self.net = wob.MLP(self.scene.dim, B, p0, max_batch=cfg.batch)
        steps_per_epoch = max(1, cfg.n_train // cfg.batch)
        total = steps_per_epoch * cfg.epochs
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        step = 0
        for ep in range(cfg.epochs):
            for k in range(steps_per_epoch):
                step += 1
                lr = cfg.lr * 0.5 * (1.0 + math.cos(math.pi * (step - 1) / total))
                sl = slice(k * cfg.batch, (k + 1) * cfg.batch)
                self.net.train_step(pts[sl], target[sl], step, lr, loss=loss, target_map=tmap, stream=stream)
                if k == steps_per_epoch - 1:
                    self.history.append(float(loss.item()))
        sync()
        t2 = time.perf_counter()
        # back to raw targets: f = scale * f_n + median
        p = self.net.params()
        self.disabled = None
        if not np.isfinite(p).all():
            self.disabled = "the trained network's parameters are not finite"
            self.g = self.g0 = None
        else:
            o = p.shape[0] - HIDDEN - 1
            p[o:o + HIDDEN] *= scale
            p[-1] = p[-1] * scale + med
            self.net.set_params(p)
            self.g = wob.cv_table(self.scene, self.net, stream=stream)
            self.g0 = wob.cv_emission(self.scene, self.bc, self.g, stream=stream)
            if not (np.isfinite(self.g.cpu().numpy()).all() and np.isfinite(self.g0.cpu().numpy()).all()):
                self.disabled = "the network's tables are not finite"
                self.g = self.g0 = None
        sync()
        t3 = time.perf_counter()
        self.timings = {"targets_s": t1 - t0, "train_s": t2 - t1, "table_s": t3 - t2, "fit_s": t3 - t0,
                        "train_steps": total, "final_loss": self.history[-1] if self.history else None,
                        "target_median": med, "target_scale": scale, "cv_disabled": self.disabled}
        return self.timings

    def solve(self, points, samples: int, seed: int = 0, point_prim=None, want_var=True, stream=None):
        if self.disabled:  # plain WoB: the same estimator without the control variate
            return wob.solve(self.scene, points, self.bc, samples, self.walk_len, seed=seed,
                             point_prim=point_prim, want_var=want_var, stream=stream)
        if self.g is None:
            raise wob.WobError("fit() first")
        return wob.solve_cv(self.scene, points, self.bc, samples, self.walk_len, self.g, seed=seed,
                            point_prim=point_prim, want_var=want_var, stream=stream, g0=self.g0)

    def close(self):
        if self.net is not None:
            self.net.close()
            self.net = None
