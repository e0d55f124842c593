"""Adjoint at the full size of the differentiation workload: d=4, N=50 000
uniform generators, 512 Monte-Carlo rays per cell, loss = sum of the cells'
second moments (the centroidal energy).  The GPU gradient at 32 seeded
generators is checked against the oracle's closed form and against central
finite differences (h = 1e-6) of the FP64 estimator with frozen directions.

Only rays of the generator's own cell and of its Voronoi neighbours' cells
depend on x_m (the neighbours come from the oracle's star of m).  For a
neighbour cell's ray, t* = min(t_m(x_m), t_rest) with t_rest the RayCast over
all other nodes, which does not depend on x_m; so a finite difference only
recomputes t_m for those rays and the full RayCast for the rays of cell m."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu

D_, N_, R_ = 4, 50_000, 512
H = 1e-6


def _energy_terms(t, d):
    return t ** (d + 2)


def test_gradient_full_size_32_generators():
    import bench
    import paper_2405_10050_amd as vg

    X = W.uniform_cloud(N_, D_, seed=0)
    dirs = bench.directions_threaded(np.arange(N_), R_, D_, seed=1)
    dev = torch.device("cuda", 0)
    nodes = torch.from_numpy(X).to(dev)
    dd = torch.from_numpy(dirs).to(dev)
    res = vg.mc_volume_area(nodes, dd)
    grad = vg.mc_backward(nodes, dd, res, None, torch.ones(N_, device=dev), None).cpu().numpy()
    del dd

    X64 = X.astype(np.float64)
    S = oracle.sphere_area(D_)
    scale = S / ((D_ + 2) * R_)
    picks = W.fd_generators(N_, 32, seed=1)
    draws = W.descent_draws(D_, seed=11)
    g_ref = np.empty((picks.size, D_))
    g_fd = np.empty((picks.size, D_))
    kinked = np.zeros((picks.size, D_), dtype=bool)
    for a, m in enumerate(picks):
        star = oracle.star(X64, m, draws)
        nb = np.setdiff1d(np.unique(star), [m])
        cells = np.concatenate([[m], nb])
        Dc = dirs[cells]
        ref = oracle.mc_volume_area(X64, cells, Dc)
        G = oracle.mc_adjoint(X64, cells, Dc, ref["t"], ref["idx"], None, np.ones(cells.size), None)
        g_ref[a] = G[m]
        # neighbour rays: t_rest excludes m (and the ray's own generator)
        U = Dc[1:].reshape(-1, D_).astype(np.float64)
        gen = np.repeat(nb, R_).astype(np.int32)
        excl = np.sort(np.stack([gen, np.full_like(gen, m)], axis=1), axis=1).astype(np.int32)
        t_rest, _, _ = oracle.raycast(X64, X64[gen], U, gen, excl=excl, clip=True)
        for k in range(D_):
            Ls, wins = [], []
            for sgn in (+1.0, -1.0):
                Xp = X64.copy()
                Xp[m, k] += sgn * H
                o = oracle.mc_volume_area(Xp, [m], Dc[:1])
                Dl = Xp[m] - Xp[gen]
                den = (U * Dl).sum(axis=1)
                with np.errstate(divide="ignore", invalid="ignore"):
                    tm = np.where(den > 0, (Dl * Dl).sum(axis=1) / (2 * den), np.inf)
                tn = np.minimum(t_rest, tm)
                Ls.append(scale * (_energy_terms(o["t"], D_).sum() + _energy_terms(tn, D_).sum()))
                wins.append((o["idx"].copy(), tm < t_rest))
            g_fd[a, k] = (Ls[0] - Ls[1]) / (2 * H)
            # a ray whose winner differs between +h and -h puts a kink inside the
            # difference quotient: the energy is continuous there, its derivative not
            kinked[a, k] = (not np.array_equal(wins[0][0], wins[1][0])) or \
                (not np.array_equal(wins[0][1], wins[1][1]))
    # the FP64 closed form against finite differences, away from kinks
    ok = ~kinked
    print(f"finite differences: {int(kinked.sum())} of {kinked.size} components straddle a "
          "winner change", flush=True)
    assert kinked.sum() <= kinked.size // 8
    assert np.allclose(g_fd[ok], g_ref[ok], rtol=1e-5, atol=1e-6 * np.abs(g_ref).max())
    # the GPU adjoint against the FP64 closed form
    g_gpu = grad[picks]
    err = np.linalg.norm(g_gpu - g_ref) / np.linalg.norm(g_ref)
    print(f"gradient at 32 generators: GPU vs FP64 closed form {err:.2e}, "
          f"FD vs closed form {np.linalg.norm(g_fd - g_ref) / np.linalg.norm(g_ref):.2e}", flush=True)
    assert err < 1e-4
