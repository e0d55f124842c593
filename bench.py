#!/usr/bin/env python3
"""Benchmark of the batched Monte-Carlo RayCast on one MI355X.

Workload (default): the d=10 Gaussian-mixture cloud, N = 100 000 generators
(8 isotropic components, sigma 0.05, centres uniform in [0.2, 0.8]^10, rows
outside the unit cube redrawn), 1024 uniform directions per cell, i.e.
1.024e8 rays.  One step = the whole hot path on that batch: the MFMA candidate
scan with its fused top-2 epilogue, cube clip and winner re-evaluation, the
FP64 recheck of uncertain rays, the per-cell volume / second-moment / facet
accumulation, and the adjoint of the volume, second moment and facet areas
with respect to all generator positions.  Inputs are resident in HBM before
the timed region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|bf16x3]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_MFMA_PEAK = 157.3e12   # MI355X dense FP32 matrix, FLOP/s
BF16_MFMA_PEAK = 2.5e15     # MI355X dense BF16 matrix, FLOP/s


def directions_threaded(cells, R, d, seed, workers=8):
    """Same draws as workloads.mc_directions, generated on a thread pool."""
    import concurrent.futures as cf

    import workloads as W

    cells = np.asarray(cells)
    out = np.empty((cells.size, R, d), dtype=np.float32)
    chunks = np.array_split(np.arange(cells.size), max(1, workers * 8))

    def work(ix):
        if ix.size:
            out[ix] = W.mc_directions(cells[ix], R, d, seed=seed)

    with cf.ThreadPoolExecutor(workers) as ex:
        list(ex.map(work, chunks))
    return out


def measured_traffic(name, n, R):
    """HBM bytes per launch of the scan kernel from the committed counter
    summary, or None when the kernel source changed since it was taken (or
    the workload differs)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", name)
    try:
        doc = json.load(open(path))
        h = hashlib.sha256()
        for f in doc["kernel_sources"]:
            h.update(open(os.path.join(ROOT, f), "rb").read())
    except (OSError, ValueError, KeyError):
        return None
    if h.hexdigest() != doc["kernel_sources_sha256"]:
        return None
    if n != 100_000 or R != 1024:
        return None
    return float(doc["hbm_bytes_per_launch"])


def cpu_baseline(X, cells, Ds, single=None, dirs_single=None):
    """The FP64 oracle on a bounded sample of the same workload (all host
    threads): RayCast of the sampled cells' rays over all nodes plus their
    Monte-Carlo sums.  ``Ds`` holds the sampled cells' directions.  With
    ``single`` (a smaller sample of cells and their directions) the same is
    timed on one thread."""
    import oracle

    oracle.build()
    cores = oracle.num_threads()
    t0 = time.perf_counter()
    oracle.mc_volume_area(X, cells, Ds)
    dt = time.perf_counter() - t0
    rays = cells.size * Ds.shape[1]
    out = dict(value=rays / dt, unit="rays/s", cores=cores, kind="oracle",
               sample=f"{cells.size} random cells x {Ds.shape[1]} rays of the same workload "
                      f"({rays} rays, each over all {X.shape[0]} nodes; {dt:.1f} s)")
    if single is not None:
        oracle.set_threads(1)
        t0 = time.perf_counter()
        oracle.mc_volume_area(X, single, dirs_single)
        dt1 = time.perf_counter() - t0
        oracle.set_threads(cores)
        r1 = single.size * dirs_single.shape[1]
        out["single_thread"] = dict(value=r1 / dt1, unit="rays/s", cores=1,
                                    sample=f"{single.size} of those cells ({r1} rays; {dt1:.1f} s)")
    return out


def _timed(stream, fn, steps):
    import torch

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def bench_uneven(args):
    """64 uniform clouds, d in {3,4,6,8,12,16}, N log-uniform in [1e3, 2e5],
    256 rays per cell, one graph launch per step (a tuned exact single-cloud
    scan per cloud on parallel branches, then one batched FP64 recheck); also
    timed as 64 separate single-cloud calls."""
    import torch

    import paper_2405_10050_amd as vg
    import workloads as W

    dev = torch.device("cuda", 0)
    spec = W.uneven_batch_spec(64, seed=0)
    R = 256
    probs = []
    for c, (dc, nc, sc) in enumerate(spec):
        X = torch.from_numpy(W.uniform_cloud(nc, dc, seed=sc)).to(dev)
        D = W.mc_directions_device(nc, R, dc, seed=5000 + c, device=dev)
        probs.append((X, D))
    print("[bench] uneven batch ready", file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream(dev)
    outs = vg.raycast_cells_batched(probs)  # tunes, captures
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        vg.raycast_cells_batched(probs, out=outs)
    ms = _timed(stream, lambda: vg.raycast_cells_batched(probs, out=outs), args.steps)
    st = vg.stats()
    ms_sep = _timed(stream, lambda: [vg.raycast_cells(X, D) for X, D in probs], 1)
    rays = sum(nc * R for _, nc, _ in spec)
    flops = sum(2.0 * dc * nc * nc * R + 2.0 * dc * nc * nc for dc, nc, _ in spec)
    return {
        "metric": "rays/sec batched uneven RayCast (64 clouds, d in {3..16}, N in [1e3, 2e5])",
        "value": rays / (ms / 1e3), "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "uneven64: 64 uniform clouds, 256 MC rays per cell, one graph of "
                               "per-cloud scans on 4 branches + batched FP64 recheck",
                   "clouds": len(spec), "cells": sum(nc for _, nc, _ in spec), "rays": rays,
                   "flagged_rays_per_step": st["flagged"],
                   "separate_launches_ms": ms_sep, "speedup_vs_separate": ms_sep / ms},
        "roofline": {"bound": "mfma", "achieved": flops / (ms / 1e3) / 1e12, "peak": 157.3,
                     "unit": "TFLOP/s", "frac": flops / (ms / 1e3) / FP32_MFMA_PEAK,
                     "traffic": None, "note": "weighted over clouds: sum 2 d N (N R + N) / time"},
    }


def bench_grad(args):
    """d=4, N=50 000 uniform, 512 rays per cell: forward (volume, second
    moment, facets) and forward + adjoint of the centroidal energy."""
    import torch

    import paper_2405_10050_amd as vg
    import workloads as W

    d, n, R = 4, 50_000, 512
    dev = torch.device("cuda", 0)
    X = torch.from_numpy(W.uniform_cloud(n, d, seed=0)).to(dev)
    D = torch.from_numpy(directions_threaded(np.arange(n), R, d, seed=1)).to(dev)
    stream = torch.cuda.current_stream(dev)
    res = vg.mc_volume_area(X, D)
    ones = torch.ones(n, device=dev)
    fwd = lambda: vg.mc_volume_area(X, D, out=res)
    both = lambda: (vg.mc_volume_area(X, D, out=res), vg.mc_backward(X, D, res, None, ones, None))
    for _ in range(args.warmup):
        both()
    ms_f = _timed(stream, fwd, args.steps)
    ms_b = _timed(stream, both, args.steps)
    return {
        "metric": "MC volume+grad cells/s (d=4, N=50k, 512 rays/cell, centroidal energy)",
        "value": n / (ms_b / 1e3), "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_b, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "uniform d=4 N=50000, 512 MC rays per cell, loss = sum of second moments",
                   "forward_ms": ms_f, "forward_cells_per_s": n / (ms_f / 1e3),
                   "adjoint_over_forward": (ms_b - ms_f) / ms_f, "rays": n * R},
    }


def bench_nbr(args):
    """Neighbour-restricted Monte-Carlo after the exhaustive search (the
    remark closing Sec. 3.1): uniform d=4 N=50 000 (or d=6 N=10 000), 512 rays
    per cell.  The search and the adjacency build are timed once; a step is
    the estimators over each cell's neighbour list plus the adjoint of the
    centroidal energy.  The same step over all nodes is timed beside it."""
    import torch

    import paper_2405_10050_amd as vg
    import workloads as W

    d, n = (4, 50_000) if args.workload == "nbr_d4_n50000" else (6, 10_000)
    R = 512
    dev = torch.device("cuda", 0)
    X = torch.from_numpy(W.uniform_cloud(n, d, seed=0)).to(dev)
    D = torch.from_numpy(directions_threaded(np.arange(n), R, d, seed=1)).to(dev)
    t0 = time.perf_counter()
    mesh = vg.explore(X, W.descent_draws(d))
    t_explore = time.perf_counter() - t0
    print(f"[bench] explore: {mesh['sigma'].shape[0]} vertices in {t_explore:.1f} s", file=sys.stderr,
          flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nb = vg.tuple_neighbors(torch.from_numpy(mesh["sigma"]).to(dev), n)
    torch.cuda.synchronize()
    t_nbr = time.perf_counter() - t0
    stream = torch.cuda.current_stream(dev)
    ones = torch.ones(n, device=dev)
    res = vg.mc_volume_area(X, D, neighbors=nb)
    full = vg.mc_volume_area(X, D)
    step = lambda: (vg.mc_volume_area(X, D, neighbors=nb, out=res),  # noqa: E731
                    vg.mc_backward(X, D, res, None, ones, None))
    step_full = lambda: (vg.mc_volume_area(X, D, out=full),  # noqa: E731
                         vg.mc_backward(X, D, full, None, ones, None))
    for _ in range(args.warmup):
        step()
    ms = _timed(stream, step, args.steps)
    st = vg.stats()
    ms_full = _timed(stream, step_full, 1)
    agree = float((res.idx == full.idx).float().mean().item())
    nnz = int(nb[1].numel())
    return {
        "metric": f"MC volume+grad cells/s over neighbour lists (d={d}, N={n}, 512 rays/cell)",
        "value": n / (ms / 1e3), "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"uniform d={d} N={n}, 512 MC rays per cell, scan over each cell's "
                               "neighbours from the exhaustive search, loss = sum of second moments",
                   "explore_s": t_explore, "vertices": int(mesh["sigma"].shape[0]),
                   "neighbors_s": t_nbr, "neighbor_entries": nnz, "neighbors_per_cell": nnz / n,
                   "rays": n * R, "flagged_rays_per_step": st["flagged"],
                   "full_scan_ms_per_step": ms_full, "speedup_vs_full_scan": ms_full / ms,
                   "argmin_agreement_with_full_scan": agree},
    }


def bench_incircle(args):
    """Monte-Carlo estimators with the rays cast by the incircle RayCast of
    Algorithm 1 over a uniform-grid index (low dimension, large N): uniform
    d=3 N=1 000 000 with 64 rays per cell, or d=4 N=50 000 with 512.  A step
    is the estimators' forward pass (volumes, second moments, facet areas).
    The same step with the dense scan over all nodes is timed once beside it."""
    import torch

    import paper_2405_10050_amd as vg
    import workloads as W

    d, n, R = (3, 1_000_000, 64) if args.workload == "incircle_d3_n1000000" else (4, 50_000, 512)
    dev = torch.device("cuda", 0)
    X = torch.from_numpy(W.uniform_cloud(n, d, seed=0)).to(dev)
    D = W.mc_directions_device(n, R, d, seed=1, device=dev)
    stream = torch.cuda.current_stream(dev)
    res = vg.mc_volume_area(X, D, incircle=True)
    step = lambda: vg.mc_volume_area(X, D, incircle=True, out=res)  # noqa: E731
    for _ in range(args.warmup):
        step()
    ms = _timed(stream, step, args.steps)
    st = vg.stats()
    print(f"[bench] incircle: {ms:.1f} ms/step, dense scan next", file=sys.stderr, flush=True)
    full = vg.mc_volume_area(X, D)
    ms_full = _timed(stream, lambda: vg.mc_volume_area(X, D, out=full), 1)
    agree = float((res.idx == full.idx).float().mean().item())
    vol_rel = float(((res.volume - full.volume).abs() / full.volume).max().item())
    rays = n * R
    return {
        "metric": f"MC rays/s, incircle RayCast with a grid index (d={d}, N={n}, {R} rays/cell)",
        "value": rays / (ms / 1e3), "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"uniform d={d} N={n}, {R} MC rays per cell, volumes + second "
                               "moments + facet areas",
                   "rays": rays, "nn_calls_per_ray": st["nn_calls"] / rays,
                   "grid_nn_calls_per_ray": st["nn_grid_calls"] / rays,
                   "flagged_rays_per_step": st["flagged"],
                   "dense_scan_ms_per_step": ms_full, "speedup_vs_dense_scan": ms_full / ms,
                   "argmin_agreement_with_dense_scan": agree,
                   "max_rel_volume_diff_vs_dense_scan": vol_rel},
    }


def bench_hmc(args):
    """Integrals of f(x) = |x - 1/2|^2 over every cell, d=5, N=10 000, 1000
    rays per cell (the sizes of the paper's comparison of the integrators in
    Sec. 4): the clipped vertex search once, then per step the Monte-Carlo
    forward pass (areas) and the heuristic integrals of Sec. 3.3 from the
    vertices.  The Monte-Carlo integrals of Algorithm 3 with m = 2 draws are
    timed beside them.  The integral over the cube is d/12 exactly."""
    import torch

    import paper_2405_10050_amd as vg
    import workloads as W

    d, n, R, m = 5, 10_000, 1000, 2
    dev = torch.device("cuda", 0)
    X = torch.from_numpy(W.uniform_cloud(n, d, seed=0)).to(dev)
    D = W.mc_directions_device(n, R, d, seed=1, device=dev)
    T = torch.rand((n, R, m), generator=torch.Generator(device=dev).manual_seed(2), device=dev)
    T.clamp_(min=1e-7, max=1 - 1e-7)
    f = lambda p: ((p - 0.5) ** 2).sum(dim=1)  # noqa: E731
    t0 = time.perf_counter()
    mesh = vg.explore(X, clip=True)
    t_explore = time.perf_counter() - t0
    stream = torch.cuda.current_stream(dev)
    res = vg.mc_volume_area(X, D)

    def step():
        vg.mc_volume_area(X, D, out=res)
        return vg.hmc_integrals(X, mesh, res, f)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    t0 = time.perf_counter()
    vg.mc_volume_area(X, D, out=res)
    mci = vg.mc_integrals(X, D, res, f, T)
    torch.cuda.synchronize()
    ms_mc = (time.perf_counter() - t0) * 1e3
    exact = d / 12.0
    return {
        "metric": "cells/s heuristic Monte-Carlo integrals (d=5, N=10000, 1000 rays/cell)",
        "value": n / (ms / 1e3), "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "uniform d=5 N=10000, 1000 MC rays per cell, f = |x - 1/2|^2, clipped diagram",
                   "explore_s": t_explore, "vertices": int(mesh["sigma"].shape[0]),
                   "mc_integrals_ms_per_step": ms_mc,
                   "hmc_total_rel_err": float(out.cell.double().sum().item()) / exact - 1.0,
                   "mc_total_rel_err": float(mci.volume.double().sum().item()) / exact - 1.0,
                   "hmc_volume_sum": float(out.volume.double().sum().item())},
    }


def bench_explore_incircle(args):
    """Exhaustive search of a uniform cloud (d=3, N = 100 000, or d=2,
    N = 300 000, the largest 2-D size of the paper's timings) with the edge
    rays cast by Algorithm 1 (grid index, InitialHeuristic); the same search
    with the dense scan is timed beside it and must return the same
    vertices."""
    import torch

    import paper_2405_10050_amd as vg
    import workloads as W

    d, n = {"explore_incircle_d3_n100000": (3, 100_000), "explore_incircle_d3_n1000000": (3, 1_000_000),
            "explore_incircle_d2_n300000": (2, 300_000)}[args.workload]
    print(f"[bench] explore d={d} N={n} with Algorithm 1 (warm-up, then timed)", file=sys.stderr, flush=True)
    X = torch.from_numpy(W.uniform_cloud(n, d, seed=0)).cuda()
    draws = W.descent_draws(d)
    if args.warmup:
        vg.explore(X, draws, incircle=True, heuristic=True)
    t0 = time.perf_counter()
    m = vg.explore(X, draws, incircle=True, heuristic=True)
    dt = time.perf_counter() - t0
    print(f"[bench] explore with Algorithm 1: {dt:.2f} s; dense scan next", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    ref = vg.explore(X, draws)
    dt_scan = time.perf_counter() - t0
    same = bool(np.array_equal(np.unique(m["sigma"], axis=0), np.unique(ref["sigma"], axis=0)))
    nv = m["sigma"].shape[0]
    return {
        "metric": "vertices/sec exhaustive Voronoi vertex search",
        "value": nv / dt, "unit": "vertices/s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"uniform d={d} N={n}, unbounded diagram, edge rays by Algorithm 1 "
                               "with a grid index and InitialHeuristic",
                   "vertices": nv, "raycasts": m["raycasts"],
                   "nn_calls_per_raycast": m["nn_calls"] / m["raycasts"],
                   "dense_scan_s": dt_scan, "speedup_vs_dense_scan": dt_scan / dt,
                   "same_vertex_set_as_dense_scan": same},
    }


# Vertices and neighbours per cell with periodic boundary conditions as Table
# empscaling prints them (d = 2..6), for the comparison in the JSON line.
EMPSCALING_TABLE = {2: (6.6, 6.6), 3: (29.2, 16.6), 4: (191, 43), 5: (1250, 95), 6: (9720, 210)}


def bench_periodic(args):
    """Exhaustive search of the periodic diagram (the torus) of uniform
    clouds for d = 2..6: vertices and neighbours per cell, the quantities of
    Table empscaling, with the search's vertex rate over all five."""
    import torch

    import paper_2405_10050_amd as vg
    import workloads as W

    sizes = {2: 100_000, 3: 100_000, 4: 20_000, 5: 2000, 6: 1000}
    rows, total_v, total_t = [], 0, 0.0
    for d, n in sizes.items():
        X = torch.from_numpy(W.uniform_cloud(n, d, seed=0)).cuda()
        draws = W.descent_draws(d)
        if args.warmup:
            vg.explore(X, draws, periodic=True)
        t0 = time.perf_counter()
        m = vg.explore(X, draws, periodic=True)
        dt = time.perf_counter() - t0
        ids, sh = m["sigma"].astype(np.int64), m["shift"].astype(np.int64)
        pairs = []
        for a in range(d + 1):
            for b in range(a + 1, d + 1):
                rel = np.zeros(ids.shape[0], dtype=np.int64)
                for q in range(d):
                    rel += (sh[:, b, q] - sh[:, a, q] + 1) * 3 ** q
                pairs.append((ids[:, a] * n + ids[:, b]) * 3 ** d + rel)
        facets = np.unique(np.concatenate(pairs)).size
        nv = ids.shape[0]
        total_v += nv
        total_t += dt
        row = {"d": d, "N": n, "vertices": nv, "seconds": dt, "raycasts": m["raycasts"],
               "vertices_per_cell": (d + 1) * nv / n, "neighbours_per_cell": 2 * facets / n,
               "table_empscaling": EMPSCALING_TABLE[d]}
        rows.append(row)
        print(f"[bench] periodic d={d} N={n}: {nv} vertices in {dt:.2f} s, "
              f"{row['vertices_per_cell']:.1f} vertices and {row['neighbours_per_cell']:.1f} neighbours per cell",
              file=sys.stderr, flush=True)
    return {
        "metric": "vertices/sec exhaustive Voronoi vertex search",
        "value": total_v / total_t, "unit": "vertices/s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
        "ms_per_step": total_t * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "periodic diagram (torus) of uniform clouds, d=2..6 "
                               "(N = 1e5, 1e5, 2e4, 2000, 1000)", "per_dimension": rows},
    }


def bench_explore(args):
    """Exhaustive vertex search (Algorithm 2) of a uniform cloud: the
    unbounded diagram, or (clipped_*) the diagram clipped to the unit cube."""
    import torch

    import paper_2405_10050_amd as vg
    import workloads as W

    n, d = (1000, 2) if args.workload.endswith("d2_n1000") else (10_000, 6)
    clip = args.workload.startswith("clipped")
    X = torch.from_numpy(W.uniform_cloud(n, d, seed=0)).cuda()
    draws = None if clip else W.descent_draws(d)
    if args.warmup:
        vg.explore(X, draws, clip=clip)
    t0 = time.perf_counter()
    m = vg.explore(X, draws, clip=clip)
    dt = time.perf_counter() - t0
    nv = m["sigma"].shape[0]
    kind = "diagram clipped to the unit cube (faces as vertex constraints)" if clip else "unbounded diagram"
    return {
        "metric": "vertices/sec exhaustive Voronoi vertex search",
        "value": nv / dt, "unit": "vertices/s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": f"uniform d={d} N={n}, {kind}", "vertices": nv,
                   "unbounded_edges": int(m["b_sigma"].shape[0]), "raycasts": m["raycasts"]},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--workload", default="gmm8_d10_n100000",
                    choices=["gmm8_d10_n100000", "uneven64", "uniform_d4_n50000",
                             "uniform_d2_n1000", "uniform_d6_n10000", "nbr_d4_n50000",
                             "nbr_d6_n10000", "incircle_d3_n1000000", "incircle_d4_n50000",
                             "clipped_d2_n1000", "clipped_d6_n10000", "hmc_d5_n10000",
                             "explore_incircle_d3_n100000", "explore_incircle_d2_n300000",
                             "explore_incircle_d3_n1000000", "periodic_d2to6"])
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--rays", type=int, default=1024)
    ap.add_argument("--cpu-cells", type=int, default=256, help="oracle sample size (0: skip)")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (calibrates the "
                         "FETCH_SIZE / WRITE_SIZE counters of a profiler run)")
    ap.add_argument("--compare-bf16", type=int, default=1,
                    help="also time the split-BF16x3 form of the step (extra field)")
    ap.add_argument("--dirs", default="device", choices=["device", "input"],
                    help="directions drawn on the device from the seed (default) or read from HBM")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): it measures one GPU's "
              "share of the work; the Monte-Carlo path shards over cells with no exchange",
              file=sys.stderr)
        sys.exit(1)

    import torch

    import paper_2405_10050_amd as vg
    import workloads as W

    if args.workload != "gmm8_d10_n100000":
        other = {"uneven64": bench_uneven, "uniform_d4_n50000": bench_grad,
                 "uniform_d2_n1000": bench_explore, "uniform_d6_n10000": bench_explore,
                 "nbr_d4_n50000": bench_nbr, "nbr_d6_n10000": bench_nbr,
                 "incircle_d3_n1000000": bench_incircle, "incircle_d4_n50000": bench_incircle,
                 "clipped_d2_n1000": bench_explore, "clipped_d6_n10000": bench_explore,
                 "hmc_d5_n10000": bench_hmc, "explore_incircle_d3_n100000": bench_explore_incircle,
                 "explore_incircle_d2_n300000": bench_explore_incircle,
                 "explore_incircle_d3_n1000000": bench_explore_incircle, "periodic_d2to6": bench_periodic}
        print(json.dumps(other[args.workload](args)), flush=True)
        return

    d, n, R = 10, args.n, args.rays
    seed = 1  # direction seed of the workload
    t_setup = time.perf_counter()
    X = W.gaussian_mixture_cloud(n=n, d=d, seed=0)
    dev = torch.device("cuda", 0)
    nodes = torch.from_numpy(X).to(dev)
    dirs = None
    if args.dirs == "input":
        dirs = torch.from_numpy(directions_threaded(np.arange(n), R, d, seed=seed)).to(dev)
    print(f"[bench] inputs ready in {time.perf_counter() - t_setup:.1f} s", file=sys.stderr, flush=True)
    if args.copy_probe_mib > 0:
        src = torch.empty(args.copy_probe_mib << 18, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # every launch of a step goes to one (default-priority) stream, which is
    # also the stream the step is captured on
    stream = torch.cuda.Stream(dev)
    g_vol = torch.ones(n, device=dev)
    g_en = torch.ones(n, device=dev)
    g_fa = torch.ones((n, R), device=dev)
    grad = torch.empty((n, d), device=dev)

    def make_step(precision):
        res = vg.mc_volume_area(nodes, dirs, precision=precision, seed=seed, rays_per_cell=R)

        def step():
            vg.mc_volume_area(nodes, dirs, precision=precision, seed=seed, rays_per_cell=R, out=res)
            if not args.no_backward:
                vg.mc_backward(nodes, dirs, res, g_vol, g_en, g_fa, out=grad)

        return res, step

    def run(precision, steps, warmup):
        """Warm-up steps (eager), then the step captured into a hipGraph and
        replayed `steps` times, each replay bracketed by HIP events on the
        capture stream; then 3 eager steps with the library's HIP events
        around each candidate-scan launch.  Returns the result buffers, the
        replay durations, the scan duration and the counters of a step."""
        with torch.cuda.stream(stream):
            res, step = make_step(precision)
            warmup = max(1, warmup)  # the capture needs the scratch already grown
            for w in range(warmup):
                step()
                torch.cuda.synchronize()
                print(f"[bench] {precision} warmup {w + 1}/{warmup} done", file=sys.stderr, flush=True)
            st = vg.stats()
            eager = [res.t.clone(), res.idx.clone(), res.volume.clone(), grad.clone()]
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=stream):
                step()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
            torch.cuda.synchronize()
            ev[0].record(stream)
            for k in range(steps):
                graph.replay()
                ev[k + 1].record(stream)
            torch.cuda.synchronize()
            replay_ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
            # the replays reproduce the eager step bit for bit
            same = all(torch.equal(a.view(torch.int32) if a.is_floating_point() else a,
                                   b.view(torch.int32) if b.is_floating_point() else b)
                       for a, b in zip(eager, [res.t, res.idx, res.volume, grad]))
            vg.set_profiling(True)
            for _ in range(3):
                step()
            st_p = vg.stats()
            vg.set_profiling(False)
            del graph
        print(f"[bench] {precision}: {steps} replays, median {np.median(replay_ms):.1f} ms",
              file=sys.stderr, flush=True)
        return res, replay_ms, st_p["scan_ms"] / max(1, st_p["scan_launches"]), st, same

    res, replay_ms, scan_ms, st, same = run(args.precision, args.steps, args.warmup)
    ms_step = float(np.median(replay_ms))
    rays = n * R
    value = rays / (ms_step / 1e3)
    flops = 2.0 * d * n * rays + 2.0 * d * n * n  # U.R~^T per ray + X.R^T per cell
    peaks = vg.peak_rates()
    if args.precision == "bf16x3":
        achieved = 3.0 * flops / (scan_ms / 1e3)
        peak, peak_meas = BF16_MFMA_PEAK, peaks["bf16_mfma"]
    else:
        achieved = flops / (scan_ms / 1e3)
        peak, peak_meas = FP32_MFMA_PEAK, peaks["fp32_mfma"]

    traffic = None
    if args.precision == "fp32" and args.dirs == "device":
        traffic = measured_traffic("cell_scan_fp32_gmm8_d10_n100000_traffic.json", n, R)
    out = {
        "metric": "rays/sec batched RayCast (d=10,N=100k) at 1e-5 rel err; MC volume+grad cells/s",
        "value": value,
        "unit": "rays/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {
            "workload": f"gaussian-mixture d={d} N={n}, {R} MC rays per cell, directions drawn on the device "
                        "(RayCast + FP64 recheck + volume/area/second moment + adjoint)"
                        if args.dirs == "device" else
                        f"gaussian-mixture d={d} N={n}, {R} MC rays per cell, directions read from HBM "
                        "(RayCast + FP64 recheck + volume/area/second moment + adjoint)",
            "d": d, "n_nodes": n, "rays_per_cell": R, "rays": rays,
            "directions": "Philox4x32-10 + Box-Muller on the device, seed 1" if args.dirs == "device"
                          else "host PCG64 draw, resident in HBM",
            "cells_per_s": n / (ms_step / 1e3),
            "flagged_rays_per_step": st["flagged"],
            "backward": not args.no_backward,
            "timing": f"median of {args.steps} hipGraph replays of the captured step (HIP events per replay)",
            "replay_ms_min_median_max": [float(np.min(replay_ms)), ms_step, float(np.max(replay_ms))],
            "mean_ms_per_step": float(np.mean(replay_ms)),
            "replays_equal_eager_step": same,
        },
        "roofline": {
            "bound": "mfma",
            "kernel": f"cell_scan_{args.precision}",
            "achieved": achieved / 1e12,
            "peak": peak / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "peak_measured": peak_meas / 1e12,
            "frac_of_measured_peak": achieved / peak_meas,
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (FETCH_SIZE, WRITE_SIZE, copy-calibrated)",
            "algorithmic_bytes": float(n * d * 4 + rays * 9 + (rays * d * 4 if args.dirs == "input" else 0)),
            "scan_ms": scan_ms,
            "scan_timing": "HIP events around each scan launch on its stream, 3 eager steps after the replays",
            "node_order": "scan (Morton order, exact block and chunk skipping)"
                          if d <= (10 if args.precision == "bf16x3" else 12) else "index",
            "evaluated_pair_fraction": st["scan_pairs"] / (float(n) * rays),
            "executed": (3.0 if args.precision == "bf16x3" else 1.0) * 2.0 * d * st["scan_pairs"] / (scan_ms / 1e3)
                        / 1e12,
            "executed_frac": (3.0 if args.precision == "bf16x3" else 1.0) * 2.0 * d * st["scan_pairs"]
                             / (scan_ms / 1e3) / peak,
            "note": "achieved/frac count the dense scan's 2 d N (N R + N) flops; the scan in scan order "
                    "evaluates only the ray-node pairs it cannot rule out (evaluated_pair_fraction), so "
                    "frac can exceed 1; executed/executed_frac are the MFMA flops actually run",
        },
        "measured_peaks_tflops": {k: v / 1e12 for k, v in peaks.items()},
    }
    if args.compare_bf16 and args.precision == "fp32":
        # the split-precision form of the same step, timed the same way
        res_b, rep_b, scan_b, sb, same_b = run("bf16x3", args.steps, 1)
        ms_b = float(np.median(rep_b))
        agree = float((res_b.idx == res.idx).float().mean().item())
        rel_t = float(((res_b.t - res.t).abs() / res.t).max().item())
        out["bf16x3"] = {
            "ms_per_step": ms_b, "rays_per_s": rays / (ms_b / 1e3), "speedup_vs_fp32": ms_step / ms_b,
            "scan_ms": scan_b, "flagged_rays_per_step": sb["flagged"],
            "evaluated_pair_fraction": sb["scan_pairs"] / (float(n) * rays),
            "executed_frac_bf16_peak": 3.0 * 2.0 * d * sb["scan_pairs"] / (scan_b / 1e3) / BF16_MFMA_PEAK,
            "roofline_frac_bf16_peak": 3.0 * flops / (scan_b / 1e3) / BF16_MFMA_PEAK,
            "roofline_frac_measured_bf16_peak": 3.0 * flops / (scan_b / 1e3) / peaks["bf16_mfma"],
            "fp32_equivalent_tflops": flops / (scan_b / 1e3) / 1e12,
            "argmin_agreement_with_fp32": agree, "max_rel_t_diff_vs_fp32": rel_t,
            "replays_equal_eager_step": same_b,
        }
    if args.cpu_cells > 0:
        rng = np.random.default_rng(123)
        sample = np.sort(rng.choice(n, args.cpu_cells, replace=False))
        dir_fn = (lambda c: W.philox_directions(c, R, d, seed=seed)) if args.dirs == "device" else \
                 (lambda c: directions_threaded(c, R, d, seed=seed))
        out["cpu_baseline"] = cpu_baseline(X, sample, dir_fn(sample), single=sample[:8], dirs_single=dir_fn(sample[:8]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
