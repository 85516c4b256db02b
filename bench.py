"""Walk-on-boundary throughput on one MI355X.

Headline workload (the largest single-GPU configuration): 3D exterior mixed
Neumann / Robin problem (Robin coefficient 1) on the 200,992-triangle union of
three tori (R = 1, r = 0.3, random rotations), data from a point source inside
the tori; 1,000,000 evaluation points, 10 % of them on the boundary; 512 paths
per point, path length 4; single-layer formulation with line sampling, FP32.

One step = one wob_solve over every point (direction sampling, all-hits BVH
traversal, hit selection, weights, emission and the per-point mean / variance
reduction, all in one kernel).  The scene (BVH) is built once before timing, as
a model's weights would be; inputs are resident in device memory.

Prints one JSON line: path samples/s (value), lines/s, the roofline record of
the walk kernel (vector-ALU and vector-memory roofs, HBM traffic) and the FP64
oracle timed on a bounded sample on host cores.  More legs in the same line,
each with its own timing and roofline record:
  slice     - 3D interior Dirichlet, 20,480-triangle perturbed icosphere,
              every cell of a 512 x 512 slice inside it, 256 paths, M = 6;
  circle    - 2D interior Dirichlet, 256-segment circle, 1,024 points, 64
              paths, M = 4, FP64;
  batched   - 64 problems of uneven size (2k-200k triangles, 1k-256k points,
              128-1024 paths, Dirichlet and exterior Neumann) in one persistent
              launch replayed from a hipGraph, launch shape autotuned;
  cv        - the headline workload: RMSE against the analytic solution at
              equal wall time, plain WoB with 512 paths against the learned
              control variate (fit + corrected solve) and RIS;
  forward   - exterior Neumann data concentrated near one spot of the same
              tori: the forward (adjoint) estimator with every point connected
              to every path vertex against the backward walks at equal wall
              time, and the throughput of its two kernels;
  grad      - value and gradient along the same paths on the slice workload:
              cost relative to the value alone, gradient error.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published vector peaks (256 CUs at 2.4 GHz; an FMA counts as two
# operations; the fp32 figure includes packed math, which this build does not
# use, so one half of it is the attainable issue rate)
FP32_PEAK_TFLOPS = 157.3
FP64_PEAK_TFLOPS = 78.6
CU_CLOCKS_PER_S = 256 * 2.4e9
# algorithmic operations of the traversal: a visited interior record tests the
# boxes of its four children (4-wide records), each slab test (near / far sides
# ordered by the direction's signs, fixed per line) 6 FMA (12), 2 three-way
# max / min (4) and one compare = 17; a tested triangle (numerator form of
# Moller-Trumbore, a miss) is two cross products (18), three dots (15), x - v0
# (3), three sign products and four compares = 43
BOX_TESTS_PER_NODE = 4
NODE_FLOP, TRI_FLOP = BOX_TESTS_PER_NODE * 17, 43
# algorithmic bytes: an interior record is its children's boxes (4 x 6 binary16
# values, 48 B) and entries (4 x 4 B); a tested triangle is v0, e1, e2
# (9 x 4 B); a hit also reads id, kind and alpha (12 B)
NODE_BYTES, TRI_BYTES, HIT_BYTES = 64, 36, 12
# bytes the kernel loads through the vector memory path: an interior record is
# 64 B (four 16-byte loads), a tested triangle 48 B of its 64-byte record (three
# loads), and each line's path step re-reads the kept hit's triangle and normal
# (48 + 16 B)
NODE_LOAD_BYTES, TRI_LOAD_BYTES, STEP_LOAD_BYTES = 64, 48, 64

KERNEL_SOURCES = ("paper_2305_04403_amd/csrc/device.hpp", "paper_2305_04403_amd/csrc/walk.hpp",
                  "paper_2305_04403_amd/csrc/internal.hpp", "paper_2305_04403_amd/csrc/wob.hip")
# committed counter summaries of each leg's kernel and the sources they were
# taken from: their figures are reported only while those sources are unchanged
PROFILES = {
    # the headline solve walks its points in Morton order: the ordering code
    # shapes the walk kernel's counters too
    "tori": ("profiles/walk_kernel_tori200992_1M_points.md",
             KERNEL_SOURCES + ("paper_2305_04403_amd/csrc/order.hip",)),
    "slice": ("profiles/walk_kernel_icosphere20480_slice512_dirichlet.md", KERNEL_SOURCES),
    "batched": ("profiles/batch_kernel_64_problems.md",
                KERNEL_SOURCES + ("paper_2305_04403_amd/csrc/batch.hip",)),
}


def kernel_source_hash(sources) -> str:
    """SHA-256 of the kernel sources' code: the files concatenated in order,
    each with its comments removed and its whitespace runs collapsed to one
    space (a change of comments or layout leaves the kernels, and so the
    counters taken from them, as they were)."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f)) as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()


def measured_profile(leg: str):
    """From the committed counter summary of a leg's kernel: HBM bytes per
    launch (FETCH + WRITE, calibrated), and where present the per-level
    memory fractions and the VALU busy / utilization figures; None when the
    kernel code changed since the counters were taken."""
    try:
        path, sources = PROFILES[leg]
        with open(os.path.join(ROOT, path)) as fh:
            text = fh.read()
    except (OSError, KeyError):
        return None
    keys = ("source-sha256-prefix:", "traffic-bytes-per-launch:", "memory-levels:", "valu:")
    rec = dict(line.strip().split(": ", 1) for line in text.splitlines() if line.strip().startswith(keys))
    prefix = rec.get("source-sha256-prefix", "")
    if not prefix or not kernel_source_hash(sources).startswith(prefix):
        return None
    fetch, write = (int(v) for v in rec["traffic-bytes-per-launch"].split())
    out = {"traffic": fetch + write, "profile": path}
    for k in ("memory-levels", "valu"):
        if k in rec:
            out[k] = {a: float(b) for a, b in (kv.split("=") for kv in rec[k].split())}
    return out


def walk_roofline(cnt, kern_s, cal, fp64=False, prof=None):
    """Roofline record of one walk kernel from its work counters and average
    launch time.  roofline: algorithmic vector-ALU operations per second
    against the published vector peak (the traversal is not a contraction: no
    MFMA).  vector_memory: the bytes the kernel loads per second (node and
    triangle records, path-step re-reads) against the rate at which the CUs'
    vector memory path serves random 32-byte records held in L1 (the library's
    gather probe, 32 KiB working set, same run): the ceiling of record loads
    whatever level holds the scene.  hbm: the measured HBM traffic (committed
    counter summary) over the launch time, against 8 TB/s.  memory_roof: the
    per-level request rates of the same summary, each over the gather probe's
    rate into that level (L1: 32 KiB set, L2: 2 MiB, L2 misses: 20 MiB), the
    largest being the roof."""
    traffic = prof["traffic"] if prof else None
    lines, nodes, prims, hits = cnt["lines"], cnt["nodes"], cnt["prims"], cnt["hits"]
    alg_flop = nodes * NODE_FLOP + prims * TRI_FLOP
    alg_bytes = nodes * NODE_BYTES + prims * TRI_BYTES + hits * HIT_BYTES
    peak = FP64_PEAK_TFLOPS if fp64 else FP32_PEAK_TFLOPS
    achieved = alg_flop / kern_s / 1e12
    loads = nodes * NODE_LOAD_BYTES + prims * TRI_LOAD_BYTES + lines * STEP_LOAD_BYTES
    vm = loads / kern_s / 1e9
    out = {
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic},
        "vector_memory": {"achieved": vm, "peak": cal["32KiB"], "unit": "GB/s", "frac": vm / cal["32KiB"],
                          "bytes_per_line": loads / lines,
                          "records_per_clk_per_cu": (nodes + prims + lines) / kern_s / CU_CLOCKS_PER_S,
                          "ceiling": "random 32-byte records from an L1-resident buffer (gather probe, 32 KiB)"},
        "work_per_line": {"interior_records": nodes / lines, "box_tests": BOX_TESTS_PER_NODE * nodes / lines,
                          "triangles": prims / lines, "hits": hits / lines},
        "algorithmic_flop_per_launch": alg_flop,
        "algorithmic_bytes_per_launch": alg_bytes,
        "algorithmic_GB/s": alg_bytes / kern_s / 1e9,
    }
    if traffic is not None:
        out["hbm"] = {"achieved": traffic / kern_s / 1e9, "peak": 8000.0, "unit": "GB/s",
                      "frac": traffic / kern_s / 8e12}
    if prof and "memory-levels" in prof:
        lv = prof["memory-levels"]
        top = max(lv, key=lv.get)
        out["memory_roof"] = {"levels": lv, "frac": lv[top], "level": top, "source": prof["profile"]}
    if prof and "valu" in prof:
        out["valu"] = dict(prof["valu"], source=prof["profile"])
    return out


def time_solve(torch, wob, scene, pts, pp, bc, N, M, seed, steps, warmup, ordered=False):
    """Warm-up, then `steps` solves bracketed by HIP events on the stream the
    kernel runs on; returns (wall seconds per step, average kernel seconds,
    mean, var).  ``ordered``: the ordered solve (Morton order of the points,
    sort and write-back inside the timed call), its workspace allocated once
    beforehand like the outputs."""
    P = pts.shape[0]
    mean = torch.empty(P, dtype=scene.dtype, device="cuda")
    var = torch.empty(P, dtype=scene.dtype, device="cuda")
    kw = {}
    if ordered:
        kw = dict(ordered=True, workspace=torch.empty(wob.ordered_workspace_bytes(scene, P), dtype=torch.uint8,
                                                      device="cuda"))
    for _ in range(warmup):
        wob.solve(scene, pts, bc, N, M, seed, point_prim=pp, out=(mean, var), **kw)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[2 * k].record(stream)
        wob.solve(scene, pts, bc, N, M, seed, point_prim=pp, out=(mean, var), **kw)
        ev[2 * k + 1].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    kern = 1e-3 * float(np.mean([ev[2 * k].elapsed_time(ev[2 * k + 1]) for k in range(steps)]))
    return wall, kern, mean, var


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--cpu-sample-points", type=int, default=16)
    p.add_argument("--skip-cpu-baseline", action="store_true")
    p.add_argument("--legs", default="main,slice,circle,batched,cv,forward,grad",
                   help="comma-separated subset of main, slice, circle, batched, cv, forward, grad, "
                        "cv_decomposition, truncation (the last two not in the default set)")
    p.add_argument("--copy-probe-mib", type=int, default=0,
                   help="after timing, copy this many MiB device-to-device once (a kernel of known "
                        "traffic that calibrates hardware byte counters)")
    return p.parse_args()


def cpu_baseline(w, n_points):
    import oracle
    om = oracle.OracleMesh(w.mesh)
    bc = oracle.make_bc(w.bc["domain"], w.bc["formulation"], w.bc["program"], w.bc["params"])
    idx = np.linspace(0, w.points.shape[0] - 1, n_points).astype(np.int64)
    pp = None if w.point_prim is None else w.point_prim[idx]
    threads = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    oracle.solve(om, w.points[idx], pp, bc, w.samples, w.walk_len, w.seed, n_threads=threads)
    dt = time.perf_counter() - t0
    paths = n_points * w.samples
    return {"value": paths / dt, "unit": "path samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_points} evenly spaced points of the same workload ("
                      f"{0 if pp is None else int((pp >= 0).sum())} on the boundary) x {w.samples} paths x "
                      f"{w.walk_len} lines, brute force over all {w.mesh.n_prims} primitives, FP64; "
                      f"{dt:.1f} s"}


def timed_leg(torch, wob, w, steps, warmup, cal, leg=None, fp64=False, ordered=False):
    """A single-problem workload: solve timing (``ordered``: the ordered
    solve), work counters of exactly the timed paths (the order of the points
    changes no path), roofline record, RMSE against the analytic solution."""
    scene = wob.Scene(w.mesh, wob.F64 if fp64 else wob.F32)
    info = scene.info()
    bc = wob.BC(w.bc["domain"], w.bc["formulation"], w.bc["program"], tuple(w.bc["params"]))
    dt = torch.float64 if fp64 else torch.float32
    pts = torch.as_tensor(w.points, dtype=dt, device="cuda")
    pp = None if w.point_prim is None else torch.as_tensor(w.point_prim, dtype=torch.int32, device="cuda")
    P, N, M = pts.shape[0], w.samples, w.walk_len
    cnt = wob.count_work(scene, pts, bc, N, M, w.seed, point_prim=pp)
    wall, kern, mean, var = time_solve(torch, wob, scene, pts, pp, bc, N, M, w.seed, steps, warmup, ordered)
    m = mean.double().cpu().numpy()
    ok = np.isfinite(m)
    out = {"workload": w.name, "points": P, "paths_per_point": N, "walk_len": M,
           "primitives": w.mesh.n_prims, "value": P * N / wall, "unit": "path samples/s",
           "point_order": "Morton order, sorted inside the timed call" if ordered else "as given",
           "ms_per_step": 1e3 * wall, "kernel_ms": 1e3 * kern, "steps": steps,
           "lines_per_s": cnt["lines"] / wall,
           "rmse_vs_analytic": float(np.sqrt(np.mean((m[ok] - w.exact[ok]) ** 2))),
           "median_abs_err": float(np.median(np.abs(m[ok] - w.exact[ok]))),
           "mean_se": float(np.mean(np.sqrt(var.double().cpu().numpy()[ok] / N))),
           "nonfinite_points": int((~ok).sum()),
           "scene": {k: info[k] for k in ("n_nodes", "n_leaves", "depth", "device_bytes")}}
    out.update(walk_roofline(cnt, kern, cal, fp64=fp64,
                             prof=measured_profile(leg) if leg else None))
    scene.close()
    return out


def batched_leg(torch, wob, I, cal, steps=2):
    from concurrent.futures import ThreadPoolExecutor
    ws = I.config_batched()
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=min(16, len(os.sched_getaffinity(0)))) as ex:
        scenes = list(ex.map(lambda w: wob.Scene(w.mesh, wob.F32), ws))
    t_build = time.perf_counter() - t0
    probs = [dict(scene=s, points=torch.as_tensor(w.points, dtype=torch.float32, device="cuda"),
                  bc=wob.BC(w.bc["domain"], w.bc["formulation"], w.bc["program"], tuple(w.bc["params"])),
                  samples=w.samples, walk_len=w.walk_len, seed=w.seed) for w, s in zip(ws, scenes)]
    b = wob.Batch(probs)
    t0 = time.perf_counter()
    tune = b.autotune(sample_stride=16)
    t_tune = time.perf_counter() - t0
    b.launch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        outs = b.launch()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    paths = sum(w.points.shape[0] * w.samples for w in ws)
    lines = sum(w.points.shape[0] * w.samples * (w.walk_len + (1 if w.bc["formulation"] == 2 else 0))
                for w in ws)
    rel = []
    for w, (m, v) in zip(ws, outs):
        mm = m.double().cpu().numpy()
        rel.append(float(np.sqrt(np.mean((mm - w.exact) ** 2)) / np.sqrt(np.mean(w.exact ** 2))))
    (blk, bpc), n_tiles = b.tune()
    b.close()
    # work per line of every problem (its points with 8 paths each: the same
    # line statistics), scaled to the problem's lines
    cnt = {"lines": 0, "nodes": 0.0, "prims": 0.0, "hits": 0.0}
    for w, p in zip(ws, probs):
        c = wob.count_work(p["scene"], p["points"], p["bc"], 8, w.walk_len, w.seed)
        n_lines = w.points.shape[0] * w.samples * (w.walk_len + (1 if w.bc["formulation"] == 2 else 0))
        cnt["lines"] += n_lines
        for k in ("nodes", "prims", "hits"):
            cnt[k] += c[k] * n_lines / c["lines"]
    roof = walk_roofline(cnt, dt, cal, prof=measured_profile("batched"))
    for s in scenes:
        s.close()
    return {"workload": "64 perturbed spheres, 2k-200k triangles (sum %d), %d points, 128-1024 paths, M=4, "
                        "Dirichlet interior + Neumann exterior, FP32" % (sum(w.mesh.n_prims for w in ws),
                                                                         sum(w.points.shape[0] for w in ws)),
            "value": paths / dt, "unit": "path samples/s", "ms_per_launch": 1e3 * dt, "lines_per_s": lines / dt,
            "paths": paths, "tiles": n_tiles, "launch": "persistent, hipGraph replay",
            "autotuned": {"block": blk, "blocks_per_cu": bpc, "tune_s": t_tune},
            "bvh_build_s": t_build, "median_relative_rmse_vs_analytic": float(np.median(rel)), **roof}


def _boot_ratio(mse_a, mse_b, med_a, med_b, reps=4000, seed=0):
    """Paired bootstrap over seeds of sqrt(mean mse_a / mean mse_b) and of the
    ratio of mean median errors: the point estimates and 95 % intervals."""
    import math
    mse_a, mse_b, med_a, med_b = (np.asarray(v, dtype=np.float64) for v in (mse_a, mse_b, med_a, med_b))
    rng = np.random.default_rng(seed)
    k = len(mse_a)
    idx = rng.integers(0, k, (reps, k))
    r = np.sqrt(mse_a[idx].mean(1) / mse_b[idx].mean(1))
    q = med_a[idx].mean(1) / med_b[idx].mean(1)
    return {"rmse_ratio": math.sqrt(mse_a.mean() / mse_b.mean()),
            "rmse_ratio_95": [float(np.quantile(r, 0.025)), float(np.quantile(r, 0.975))],
            # the median seed's RMSE ratio: what a typical run sees, where the
            # pooled ratio is set by the rare seed that draws an extreme path
            "rmse_ratio_median_seed": math.sqrt(float(np.median(mse_a)) / float(np.median(mse_b))),
            "median_err_ratio": float(med_a.mean() / med_b.mean()),
            "median_err_ratio_95": [float(np.quantile(q, 0.025)), float(np.quantile(q, 0.975))]}


def _tail_shares(vals):
    """Share of the sum of squared per-path deviations (from each point's mean)
    carried by the most extreme 0.01 %, 0.1 % and 1 % of paths."""
    v = vals.double().cpu().numpy()
    sq = np.sort(((v - v.mean(axis=1, keepdims=True)) ** 2).ravel())[::-1]
    tot = max(sq.sum(), 1e-300)
    return {f"top_{q * 100:g}%": float(sq[: max(1, int(q * sq.size))].sum() / tot) for q in (1e-4, 1e-3, 1e-2)}


def cv_leg(torch, wob, I, n_seeds=10):
    """Equal wall time on the 1M points: plain WoB at 512 paths against the
    corrected estimator with (a) g = g0 = 0 (hit-selection Rao-Blackwellisation
    only), (b) the learned network (fit included in its time) and (c) the same
    without the fit time; and plain resampled importance sampling (4, 16 and
    32 area candidates) in place of line sampling, and the corrected walk on
    RIS-16 and RIS-32 (g = g0 = 0, and learned).  Every variant runs with
    `n_seeds` seeds; RMSE ratios pool the per-seed squared errors and carry a
    paired bootstrap 95 % interval over the seeds.  Also the per-point
    variance of each variant (paired log ratio against (a) on the same seeds)
    and the share of the squared path deviations that the most extreme paths
    carry (2000 points x 512 paths)."""
    import dataclasses
    import math
    from paper_2305_04403_amd import cv as CV
    w = I.config_tori()
    scene = wob.Scene(w.mesh, wob.F32)
    bc = wob.BC(w.bc["domain"], w.bc["formulation"], w.bc["program"], tuple(w.bc["params"]))
    pts = torch.as_tensor(w.points, dtype=torch.float32, device="cuda")
    pp = torch.as_tensor(w.point_prim, dtype=torch.int32, device="cuda")
    N, M = w.samples, w.walk_len
    sync = torch.cuda.synchronize
    ex = w.exact
    zero = torch.zeros(scene.n_prims, dtype=torch.float32, device="cuda")

    # first launches load code objects: warm every kernel of both pipelines on small inputs
    wob.solve(scene, pts[:4096].contiguous(), bc, 64, M, point_prim=pp[:4096].contiguous())
    warm = CV.LearnedControlVariate(scene, bc, M, CV.CVConfig(n_train=32768))
    warm.fit()
    warm.solve(pts[:4096].contiguous(), 64, point_prim=pp[:4096].contiguous())
    warm.close()
    sync()

    seeds = tuple(range(11, 11 + n_seeds))

    def slope(fn, lo=64, hi=320):
        """Cost per path and the fixed rest (add-back, launch overheads): the
        slope between `lo` and `hi` paths on the full point set, fastest of two
        runs each, after a full-size warm-up (a one-off stall in a probe would
        otherwise skew the slope)."""
        fn(lo)
        sync()
        tt = []
        for n_probe in (lo, hi):
            best = float("inf")
            for _ in range(2):
                t0 = time.perf_counter()
                fn(n_probe)
                sync()
                best = min(best, time.perf_counter() - t0)
            tt.append(best)
        per = max((tt[1] - tt[0]) / (hi - lo), 1e-9)
        return per, max(tt[0] - lo * per, 0.0)

    def record(runs, times, extra_s=0.0):
        a = [m.double().cpu().numpy() for m, _ in runs]
        mse = [float(np.mean((x - ex) ** 2)) for x in a]
        med = [float(np.median(np.abs(x - ex))) for x in a]
        var = np.mean([v.double().cpu().numpy() for _, v in runs], axis=0)
        return {"seconds": extra_s + float(np.mean(times)), "rmse": math.sqrt(float(np.mean(mse))),
                "rmse_per_seed": [math.sqrt(x) for x in mse], "median_abs_err": float(np.mean(med)),
                "mean_var": float(var.mean()), "median_var": float(np.median(var)),
                "_mse": mse, "_med": med, "_var": var}

    def timed(fn):
        runs, times = [], []
        for sd in seeds:
            t0 = time.perf_counter()
            runs.append(fn(sd))
            sync()
            times.append(time.perf_counter() - t0)
        return runs, times

    out = {"workload": w.name + ", 1M points (10% on the boundary), M=4", "seeds": len(seeds)}
    runs, times = timed(lambda sd: wob.solve(scene, pts, bc, N, M, seed=sd, point_prim=pp))
    plain = record(runs, times)
    plain["paths"] = N
    t_plain = plain["seconds"]

    lcv = CV.LearnedControlVariate(scene, bc, M, CV.CVConfig())
    fit = lcv.fit()
    # the network on the matrix cores: forward over 2^20 points (106,752 FLOP each)
    yq = torch.rand((1 << 20, 3), dtype=torch.float32, device="cuda") * 4.0 - 2.0
    fq = torch.empty(1 << 20, dtype=torch.float32, device="cuda")
    lcv.net.forward(yq, out=fq)
    st_ = torch.cuda.current_stream()
    q0, q1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    q0.record(st_)
    for _ in range(5):
        lcv.net.forward(yq, out=fq)
    q1.record(st_)
    sync()
    t_mlp = 1e-3 * q0.elapsed_time(q1) / 5
    mlp_tflops = (1 << 20) * 106752 / t_mlp / 1e12
    t0 = time.perf_counter()
    wob.cv_addback(scene, lcv.g0, pts)
    sync()
    t_add = time.perf_counter() - t0
    ris16 = dataclasses.replace(bc, sampling=wob.SAMPLE_RIS, candidates=16)
    ris32 = dataclasses.replace(bc, sampling=wob.SAMPLE_RIS, candidates=32)

    # cost per path and fixed cost of each corrected walk with its own tables
    # (the add-back skips the triangles with g0 = 0: all of them for g0 = 0)
    costs = {}

    def cost(b, g, g0):
        key = (id(b), g is zero)
        if key not in costs:
            costs[key] = slope(lambda n: wob.solve_cv(scene, pts, b, n, M, g, seed=2, point_prim=pp, g0=g0))
        return costs[key]

    variants = {"plain": plain}

    def run_cv(name, g, g0, fixed_s, seed0, b=bc):
        per_path, base = cost(b, g, g0)
        n = int(max(8, (t_plain - fixed_s - base) / per_path // 8 * 8))  # lanes take paths one by one: any N
        runs, times = timed(lambda sd: wob.solve_cv(scene, pts, b, n, M, g, seed=sd + 100 * seed0,
                                                    point_prim=pp, g0=g0))
        variants[name] = record(runs, times, fixed_s)
        variants[name]["paths"] = n
        variants[name]["path_cost_vs_line"] = per_path / (t_plain / N)

    run_cv("rb_only", zero, zero, 0.0, 3)
    run_cv("learned", lcv.g, lcv.g0, fit["fit_s"], 5)
    variants["learned"].update({"fit_s": fit["fit_s"], "targets_s": fit["targets_s"], "train_s": fit["train_s"],
                                "train_steps": fit["train_steps"]})
    run_cv("learned_inference_only", lcv.g, lcv.g0, 0.0, 6)
    # the paper's sampling for Robin / mixed problems: RIS over area-uniform
    # candidates (16 in the paper; 4 is cheaper than a traced line)
    for C in (4, 16, 32):
        b = dataclasses.replace(bc, sampling=wob.SAMPLE_RIS, candidates=C)
        pp_cost, rest = slope(lambda n: wob.solve(scene, pts, b, n, M, seed=2, point_prim=pp))
        n = int(max(8, (t_plain - rest) / pp_cost // 8 * 8))
        runs, times = timed(lambda sd: wob.solve(scene, pts, b, n, M, seed=sd + 700 + C, point_prim=pp))
        variants[f"ris_{C}"] = record(runs, times)
        variants[f"ris_{C}"].update({"paths": n, "path_cost_vs_line": pp_cost / (t_plain / N)})
    # the corrected walk on RIS (16 candidates): the pick's mean over the
    # candidates replaces the pick, with g = g0 = 0 and with the learned tables
    run_cv("ris_16_rb_only", zero, zero, 0.0, 8, b=ris16)
    run_cv("ris_16_learned", lcv.g, lcv.g0, fit["fit_s"], 9, b=ris16)
    # 32 candidates (the paper takes 16): the cheaper pick made more candidates
    # affordable, and they thin the tail further
    run_cv("ris_32_rb_only", zero, zero, 0.0, 10, b=ris32)
    run_cv("ris_32_learned", lcv.g, lcv.g0, fit["fit_s"], 11, b=ris32)

    # the same-paths variance comparison (N paths, seed 11): every variant's
    # per-point variance against the Rao-Blackwellised one, paired by point
    v_rb = wob.solve_cv(scene, pts, bc, N, M, zero, seed=11, point_prim=pp, g0=zero)[1].double().cpu().numpy()
    v_ln = wob.solve_cv(scene, pts, bc, N, M, lcv.g, seed=11, point_prim=pp, g0=lcv.g0)[1].double().cpu().numpy()
    v_rr = wob.solve_cv(scene, pts, ris16, N, M, zero, seed=11, point_prim=pp, g0=zero)[1].double().cpu().numpy()
    v_rl = wob.solve_cv(scene, pts, ris16, N, M, lcv.g, seed=11, point_prim=pp,
                        g0=lcv.g0)[1].double().cpu().numpy()

    def paired(a, b):
        lr = np.log(np.maximum(a, 1e-30) / np.maximum(b, 1e-30))
        lr = lr[np.isfinite(lr)]
        return {"mean_log_var_ratio": float(lr.mean()), "se": float(lr.std() / math.sqrt(max(len(lr), 1))),
                "median_log_var_ratio": float(np.median(lr))}

    out["learned_vs_rb_same_paths"] = paired(v_ln, v_rb)
    out["ris_16_learned_vs_ris_16_rb_same_paths"] = paired(v_rl, v_rr)
    sub = slice(0, 2000)
    ps, pps = pts[sub].contiguous(), pp[sub].contiguous()
    out["tail_share_of_squared_deviation"] = {
        "plain": _tail_shares(wob.trace(scene, ps, bc, N, M, seed=11, point_prim=pps)[0]),
        "rb_only": _tail_shares(wob.trace_cv(scene, ps, bc, N, M, zero, seed=11, point_prim=pps, g0=zero)),
        "ris_16": _tail_shares(wob.trace(scene, ps, dataclasses.replace(bc, sampling=wob.SAMPLE_RIS,
                                                                         candidates=16),
                                         N, M, seed=11, point_prim=pps)[0]),
        "ris_16_rb_only": _tail_shares(wob.trace_cv(scene, ps, ris16, N, M, zero, seed=11, point_prim=pps,
                                                    g0=zero))}
    for name, r in variants.items():
        if name != "plain":
            r.update(_boot_ratio(plain["_mse"], r["_mse"], plain["_med"], r["_med"]))
    for name, r in variants.items():
        for k in ("_mse", "_med", "_var"):
            r.pop(k)
        out[name] = r
    out["mlp_forward"] = {"points": 1 << 20, "ms": 1e3 * t_mlp, "TFLOP/s": mlp_tflops, "peak_bf16_TFLOP/s": 2500.0,
                          "frac": mlp_tflops / 2500.0}
    out["addback_s"] = t_add
    out["corrected_path_cost_vs_plain"] = costs[(id(bc), False)][0] / (t_plain / N)
    out["fixed_cost_s"] = {"learned_tables": costs[(id(bc), False)][1], "zero_tables": costs[(id(bc), True)][1]}
    out["rmse_ratio_equal_time"] = out["learned"]["rmse_ratio"]
    out["rmse_ratio_equal_time_95"] = out["learned"]["rmse_ratio_95"]
    out["median_err_ratio_equal_time"] = out["learned"]["median_err_ratio"]
    lcv.close()
    scene.close()
    return out


def cv_decomposition_leg(torch, wob, I):
    """Why the density control variate cannot reach large gains on the
    three-tori problem (not in the default legs; ~1 minute): per-triangle
    density tables estimated at the centroids by the walk itself with 64,
    1024 and 16384 paths each (two independent tables at 16384, their
    correlation), used as the control variate's table on 100k of the points
    against g = 0 on the same paths."""
    import math
    w = I.config_tori()
    scene = wob.Scene(w.mesh, wob.F32)
    bc = wob.BC(w.bc["domain"], w.bc["formulation"], w.bc["program"], tuple(w.bc["params"]))
    idx = np.random.default_rng(0).choice(len(w.points), 100_000, replace=False)
    pts = torch.as_tensor(w.points[idx], dtype=torch.float32, device="cuda")
    pp = torch.as_tensor(w.point_prim[idx], dtype=torch.int32, device="cuda")
    ex = w.exact[idx]
    N, M = w.samples, w.walk_len
    sync = torch.cuda.synchronize
    zero = torch.zeros(scene.n_prims, dtype=torch.float32, device="cuda")
    v_rb = wob.solve_cv(scene, pts, bc, N, M, zero, seed=11, point_prim=pp, g0=zero)[1].double().cpu().numpy()
    cen = torch.as_tensor(w.mesh.verts[w.mesh.prims].mean(axis=1), dtype=torch.float32, device="cuda")
    ids = torch.arange(scene.n_prims, dtype=torch.int32, device="cuda")
    dbc = wob.BC(bc.domain, bc.formulation, bc.program, bc.params, density=True)
    out = {"workload": w.name + ", 100k of the points, 512 paths, M=4"}
    tables = {}
    for n_t, sd in ((64, 99), (1024, 99), (16384, 99), (16384, 100)):
        t0 = time.perf_counter()
        g, gv = wob.solve(scene, cen, dbc, n_t, M - 1, seed=sd, point_prim=ids)
        sync()
        key = f"table_{n_t}" + ("_b" if sd == 100 else "")
        tables[key] = g.float().contiguous()
        g0 = wob.cv_emission(scene, bc, tables[key])
        add = wob.cv_addback(scene, g0, pts).double().cpu().numpy()
        m, v = wob.solve_cv(scene, pts, bc, N, M, tables[key], seed=11, point_prim=pp, g0=g0)
        sync()
        v = v.double().cpu().numpy()
        lr = np.log(np.maximum(v, 1e-30) / np.maximum(v_rb, 1e-30))
        out[key] = {"paths_per_triangle": n_t, "seconds": time.perf_counter() - t0,
                    "median_var_per_path": float(gv.median()), "median_abs_g": float(g.abs().median()),
                    "mean_var_ratio_vs_rb": float(v.mean() / v_rb.mean()),
                    "mean_log_var_ratio_vs_rb": float(lr.mean()),
                    "rmse": float(np.sqrt(np.mean((m.double().cpu().numpy() + add - ex) ** 2)))}
    a, b = tables["table_16384"].cpu().numpy(), tables["table_16384_b"].cpu().numpy()
    out["independent_16384_tables"] = {"correlation": float(np.corrcoef(a, b)[0, 1]),
                                       "median_abs_difference": float(np.median(np.abs(a - b))),
                                       "median_abs_value": float(np.median(np.abs(a)))}
    scene.close()
    return out


def truncation_leg(torch, wob, I, grid_n=28, n_points=1000, launches=2, paths=1 << 18):
    """Truncation bias of the single layer on the three-tori union at about 20k
    triangles (not in the default legs): for M = 2..6 and three boundary
    conditions (the benchmark's random Neumann / Robin triangles with Robin
    coefficient 1; the same with 0.1; every triangle Neumann), the mean over
    `launches` x `paths` paths at each of `n_points` points off the boundary,
    the same seeds for every M, so that a path at M + 1 extends the path at M
    (line i's random numbers depend on i only) and consecutive estimates are
    paired.  Reports per M the signed error against the analytic solution
    (median relative, mean with its standard error over the points), the
    median per-point standard error, and the paired increment from M - 1."""
    import dataclasses
    import math
    w = I.config_tori(grid_n=grid_n, n_points=n_points, boundary_frac=0.0)
    xs = tuple(w.bc["params"])
    pts = torch.as_tensor(w.points, dtype=torch.float32, device="cuda")
    ex = w.exact
    out = {"workload": f"three tori, {w.mesh.n_prims} triangles, {n_points} points off the boundary, "
                       f"{launches} x {paths} paths per point per M", "problems": {}}
    kinds = w.mesh.kind
    for label, kind, alpha in (("mixed_robin_alpha_1", None, 1.0), ("mixed_robin_alpha_0.1", None, 0.1),
                               ("neumann", I.NEUMANN, 0.0)):
        k = kinds if kind is None else np.full(w.mesh.n_prims, kind, np.uint8)
        mesh = dataclasses.replace(w.mesh, kind=k, alpha=np.where(k == I.ROBIN, alpha, 0.0))
        scene = wob.Scene(mesh, wob.F32)
        bc = wob.BC(-1, wob.SINGLE_LAYER, wob.PROG_INVDIST, xs)
        rows, prev = {}, None
        for M in range(2, 7):
            ms, vs = [], []
            for j in range(launches):
                m, v = wob.solve(scene, pts, bc, paths, M, seed=1000 + j)
                ms.append(m.double().cpu().numpy())
                vs.append(v.double().cpu().numpy())
            mean = np.mean(ms, axis=0)
            se = np.sqrt(np.mean(vs, axis=0) / (launches * paths))
            e = mean - ex
            rec = {"median_relative_error": float(np.median(e / ex)), "mean_error": float(e.mean()),
                   "mean_error_se": float(e.std() / math.sqrt(len(e))), "median_point_se": float(np.median(se))}
            if prev is not None:
                d = mean - prev
                rec["increment_mean"] = float(d.mean())
                rec["increment_se"] = float(d.std() / math.sqrt(len(d)))
            rows[str(M)] = rec
            prev = mean
            print(f"[bench] truncation {label} M={M}: median relative error {rec['median_relative_error']:+.4f}, "
                  f"median point SE {rec['median_point_se']:.4f}", file=sys.stderr, flush=True)
        out["problems"][label] = rows
        scene.close()
    return out


# connection of a point to a forward-path vertex: 3 differences, 3 products and
# 2 sums for rho^2, one reciprocal square root, one multiply-add = 11
GATHER_PAIR_FLOP = 11


def gather_calibration(torch, wob, sizes=(("32KiB", 32 << 10), ("2MiB", 2 << 20), ("20MiB", 20 << 20),
                                          ("256MiB", 256 << 20)), reads=64, reps=5):
    """Random 32-byte gather rate (GB/s) at each working-set size, measured with
    the library's probe kernel: the bandwidth roof of the memory level that
    holds a working set of that size (32 KiB: the CU's L1; 2 MiB: L2; 20 MiB
    and 256 MiB: MALL / HBM)."""
    lanes = 256 * 2048  # 8 waves on each SIMD of 256 CUs
    out = torch.empty(lanes, dtype=torch.float32, device="cuda")
    res = {}
    for name, nb in sizes:
        buf = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        for _ in range(2):
            wob.gather_probe(buf, lanes, reads, 1, out=out)
        st = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for r in range(reps):
            wob.gather_probe(buf, lanes, reads, 2 + r, out=out)
        e1.record(st)
        torch.cuda.synchronize()
        t = 1e-3 * e0.elapsed_time(e1) / reps
        res[name] = lanes * reads * 32 / t / 1e9
        del buf
    return res


def forward_leg(torch, wob, I):
    """Forward (adjoint) single-layer estimator with path reuse against the
    backward walks, exterior Neumann data concentrated near one spot of the
    three-tori union (source 0.05 below the surface), 1M points off the
    boundary, M = 4, FP32: RMSE against the analytic solution at equal wall
    time (3 seeds pooled), the backward direct BIE at 512 paths per point
    setting the time; forward paths started uniformly by area and by the
    magnitude of the data; plus the throughput of the forward path kernel and
    of the connection kernel."""
    import math
    w = I.config_tori_neumann()
    scene = wob.Scene(w.mesh, wob.F32)
    xs = tuple(w.bc["params"])
    bc_direct = wob.BC(-1, wob.AUTO, wob.PROG_INVDIST, xs)
    bc_sl = wob.BC(-1, wob.SINGLE_LAYER, wob.PROG_INVDIST, xs)
    pts = torch.as_tensor(w.points, dtype=torch.float32, device="cuda")
    M, N = w.walk_len, w.samples
    ex = w.exact
    sync = torch.cuda.synchronize
    seeds = (21, 22, 23)
    starts_q = wob.Starts(scene, data=bc_sl, floor=0.05)
    # warm every kernel on small inputs
    wob.solve(scene, pts[:4096].contiguous(), bc_direct, 16, M)
    wob.solve(scene, pts[:4096].contiguous(), bc_sl, 16, M)
    v, _, _ = wob.forward_paths(scene, bc_sl, 4096, M, 1)
    wob.forward_gather(scene, v, pts[:4096].contiguous())
    sync()

    def pooled(ms):
        mse = [np.mean((m.double().cpu().numpy() - ex) ** 2) for m in ms]
        med = [np.median(np.abs(m.double().cpu().numpy() - ex)) for m in ms]
        return math.sqrt(float(np.mean(mse))), float(np.mean(med)), [math.sqrt(float(x)) for x in mse]

    out = {"workload": w.name + ", 1M points off the boundary, M=4", "seeds": len(seeds)}
    t_ref = None
    for name, bc in (("backward_direct", bc_direct), ("backward_single_layer", bc_sl)):
        ms, tm = [], []
        for sd in seeds:
            t0 = time.perf_counter()
            m, _ = wob.solve(scene, pts, bc, N, M, seed=sd, want_var=False)
            sync()
            tm.append(time.perf_counter() - t0)
            ms.append(m)
        r, e, ps = pooled(ms)
        out[name] = {"paths": N, "seconds": float(np.mean(tm)), "rmse": r, "rmse_per_seed": ps,
                     "median_abs_err": e}
        if t_ref is None:
            t_ref = float(np.mean(tm))

    # kernel throughput: 2^20 forward paths, and the connection of every point
    n_probe = 1 << 20
    vtx = torch.empty((n_probe, M, 4), dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record(st)
    wob.forward_paths(scene, bc_sl, n_probe, M, 7, starts=starts_q, out=vtx)
    e[1].record(st)
    n_g = 1 << 16
    mean = torch.empty(pts.shape[0], dtype=torch.float32, device="cuda")
    var = torch.empty_like(mean)
    e[2].record(st)
    wob.forward_gather(scene, vtx[:n_g], pts, out=(mean, var))
    e[3].record(st)
    sync()
    t_paths = 1e-3 * e[0].elapsed_time(e[1])
    t_gather = 1e-3 * e[2].elapsed_time(e[3])
    pairs = pts.shape[0] * n_g * M
    out["paths_kernel"] = {"paths": n_probe, "ms": 1e3 * t_paths, "path_samples_per_s": n_probe / t_paths,
                           "lines_per_s": n_probe * (M - 1) / t_paths}
    gf = pairs * GATHER_PAIR_FLOP / t_gather / 1e12
    out["gather_kernel"] = {"points": int(pts.shape[0]), "paths": n_g, "vertices": n_g * M, "ms": 1e3 * t_gather,
                            "pairs_per_s": pairs / t_gather,
                            "roofline": {"bound": "alu", "achieved": gf, "peak": FP32_PEAK_TFLOPS,
                                         "unit": "TFLOP/s", "frac": gf / FP32_PEAK_TFLOPS,
                                         "flop_per_pair": GATHER_PAIR_FLOP}}
    per_path = t_gather / n_g + t_paths / n_probe
    n_eq = int(max(1024, t_ref / per_path // 1024 * 1024))
    del vtx
    for name, starts in (("forward_area_starts", None), ("forward_data_starts", starts_q)):
        ms, tm = [], []
        for sd in seeds:
            t0 = time.perf_counter()
            v, _, _ = wob.forward_paths(scene, bc_sl, n_eq, M, sd + 50, starts=starts)
            m, _ = wob.forward_gather(scene, v, pts, want_var=False)
            sync()
            tm.append(time.perf_counter() - t0)
            ms.append(m)
            del v
        r, e2, ps = pooled(ms)
        ref = out["backward_direct"]
        out[name] = {"paths_shared_by_all_points": n_eq, "seconds": float(np.mean(tm)), "rmse": r,
                     "rmse_per_seed": ps, "median_abs_err": e2, "rmse_ratio_vs_backward_direct": ref["rmse"] / r,
                     "median_err_ratio_vs_backward_direct": ref["median_abs_err"] / e2}
    starts_q.close()
    scene.close()
    return out


def grad_leg(torch, wob, I, near=0.05):
    """Value and gradient along the same paths on the benchmark workload
    (icosphere slice, every inside cell x 256 paths x 6 lines): the time of
    wob_solve_grad against wob_solve, and the gradient error against the
    analytic gradient of g = 1/|x - x0|; then the boundary split of the
    gradient (anchors at the nearest boundary point for the points closer
    than `near` to the boundary) at equal time, with the error split into the
    component along the normal at the nearest boundary point and the
    tangential rest, near the boundary and away from it."""
    import math
    w = I.config_icosphere_slice()
    scene = wob.Scene(w.mesh, wob.F32)
    bc = wob.BC(w.bc["domain"], w.bc["formulation"], w.bc["program"], tuple(w.bc["params"]))
    pts = torch.as_tensor(w.points, dtype=torch.float32, device="cuda")
    N, M = w.samples, w.walk_len
    A, AP = I.nearest_boundary_points(w.mesh, w.points, inset=1e-3)
    dist = np.linalg.norm(w.points - A, axis=1)
    is_near = dist < near
    AP_on = np.where(is_near, AP, -1).astype(np.int32)
    ta = torch.as_tensor(A, dtype=torch.float32, device="cuda")
    tp = torch.as_tensor(AP_on, dtype=torch.int32, device="cuda")
    v, t = w.mesh.verts, w.mesh.prims[AP]
    nrm = np.cross(v[t[:, 1]] - v[t[:, 0]], v[t[:, 2]] - v[t[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    wob.solve_grad(scene, pts[:4096].contiguous(), bc, 16, M)
    wob.solve_grad(scene, pts[:4096].contiguous(), bc, 16, M, anchors=ta[:4096].contiguous(),
                   anchor_prim=tp[:4096].contiguous())
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        out = fn()
        e1.record(st)
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1)

    (m0, _), t_val = timed(lambda: wob.solve(scene, pts, bc, N, M, w.seed))
    (mean, var, g, gv), t_grad = timed(lambda: wob.solve_grad(scene, pts, bc, N, M, w.seed))
    x0 = np.array(w.bc["params"])
    r = w.points - x0
    exact = -r / np.linalg.norm(r, axis=1)[:, None] ** 3

    def errors(gr):
        e = gr.double().cpu().numpy() - exact
        en = np.einsum("ij,ij->i", e, nrm)
        et = np.linalg.norm(e - en[:, None] * nrm, axis=1)
        tot = np.linalg.norm(e, axis=1)
        rm = lambda x, msk: float(np.sqrt(np.mean(x[msk] ** 2))) if msk.any() else None
        every = np.ones(len(e), bool)
        return {"rmse": rm(tot, every), "median_err": float(np.median(tot)),
                "rmse_near": rm(tot, is_near), "rmse_far": rm(tot, ~is_near),
                "rmse_normal_near": rm(en, is_near), "rmse_tangential_near": rm(et, is_near),
                "rmse_normal_far": rm(en, ~is_near), "rmse_tangential_far": rm(et, ~is_near)}

    plain = errors(g)
    # the split at about the same time: scale the paths by the measured cost
    _, t_probe = timed(lambda: wob.solve_grad(scene, pts, bc, N, M, w.seed, anchors=ta, anchor_prim=tp))
    n_split = max(8, int(N * t_grad / t_probe) // 8 * 8)
    (_, _, gs, _), t_split = timed(lambda: wob.solve_grad(scene, pts, bc, n_split, M, w.seed, anchors=ta,
                                                          anchor_prim=tp))
    split = errors(gs)
    scene.close()
    return {"workload": w.name, "solve_ms": t_val, "solve_grad_ms": t_grad, "cost_ratio": t_grad / t_val,
            "grad_rmse": plain["rmse"], "grad_median_err": plain["median_err"],
            "grad_rms_exact": float(np.sqrt(np.mean(np.sum(exact ** 2, axis=1)))),
            "value_rmse": float(np.sqrt(np.mean((mean.double().cpu().numpy() - w.exact) ** 2))),
            "plain": dict(plain, paths=N, ms=t_grad),
            "boundary_split": dict(split, paths=n_split, ms=t_split, near_distance=near,
                                   points_near=int(is_near.sum()),
                                   rmse_ratio_equal_time=plain["rmse"] / split["rmse"])}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2305_04403_amd import inputs as I
    from paper_2305_04403_amd import wob

    torch.cuda.set_device(0)
    legs = set(args.legs.split(","))
    cal = gather_calibration(torch, wob)
    extra = {}

    def leg(name, key, fn):
        if name in legs:
            t0 = time.perf_counter()
            extra[key] = fn()
            print(f"[bench] {name} leg done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    leg("slice", "slice", lambda: timed_leg(torch, wob, I.config_icosphere_slice(), max(3, args.steps // 4), 1,
                                            cal, leg="slice"))
    leg("circle", "circle", lambda: timed_leg(torch, wob, I.config_circle(), 20, 3, cal, fp64=True))
    leg("batched", "batched", lambda: batched_leg(torch, wob, I, cal))
    leg("cv", "cv_equal_time", lambda: cv_leg(torch, wob, I))
    leg("cv_decomposition", "cv_decomposition", lambda: cv_decomposition_leg(torch, wob, I))
    leg("truncation", "truncation", lambda: truncation_leg(torch, wob, I))
    leg("forward", "forward_equal_time", lambda: forward_leg(torch, wob, I))
    leg("grad", "gradient", lambda: grad_leg(torch, wob, I))

    # the headline: the three-tori workload
    w = I.config_tori()
    main_rec = (timed_leg(torch, wob, w, args.steps, args.warmup, cal, leg="tori", ordered=True)
                if "main" in legs else None)
    if main_rec is None:
        print(json.dumps({"legs": extra, "gather_calibration_GB/s": cal}))
        return
    print(f"[bench] main done: {main_rec['value'] / 1e6:.1f} M path samples/s", file=sys.stderr, flush=True)
    rec = {
        "metric": "WoB path samples/s at 1 GPU",
        "value": main_rec["value"],
        "unit": "path samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_rec["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "points": main_rec["points"],
                   "boundary_points": int((w.point_prim >= 0).sum()),
                   "paths_per_point": w.samples, "walk_len": w.walk_len, "triangles": w.mesh.n_prims,
                   "formulation": "single layer, line sampling (exterior Neumann / Robin)",
                   "point_order": main_rec["point_order"],
                   "parallelism": "none (1 GPU)"},
    }
    for k in ("lines_per_s", "kernel_ms", "roofline", "vector_memory", "hbm", "memory_roof", "valu", "work_per_line",
              "algorithmic_flop_per_launch", "algorithmic_bytes_per_launch", "algorithmic_GB/s",
              "rmse_vs_analytic", "median_abs_err", "mean_se", "nonfinite_points", "scene"):
        if k in main_rec:
            rec[k] = main_rec[k]
    rec["gather_calibration_GB/s"] = cal
    rec.update(extra)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        rec["copy_probe_bytes"] = 4 * n
    if not args.skip_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_points)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
