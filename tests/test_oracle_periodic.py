"""Pins of the oracle's periodic search (Algorithm 2 on the torus R^d / Z^d):
the vertex set against qhull's Delaunay triangulation of the 3^d-tiled
cloud, the Euler relations every simple tessellation of the torus obeys,
edges seen from both ends, the empty-ball property, and Meijering's mean
vertex count of the 3-D Poisson-Voronoi cell."""
import itertools
import math

import numpy as np
import pytest

import oracle
import workloads as W


def _encode(ids, shift, d):
    """Image codes i * 3^d + c(k) of ids [..] with shifts [.., d]."""
    c = np.zeros(ids.shape, dtype=np.int64)
    for a in range(d):
        c += (shift[..., a].astype(np.int64) + 1) * 3 ** a
    return ids.astype(np.int64) * 3 ** d + c


def _canonical(ids, shift, d):
    """Sort each row by node and translate it so its first node has k = 0."""
    order = np.argsort(ids, axis=1, kind="stable")
    ids = np.take_along_axis(ids, order, axis=1)
    shift = np.take_along_axis(shift, order[..., None], axis=1)
    shift = shift - shift[:, :1, :]
    return ids, shift


def _tiled_delaunay(X):
    """Periodic vertices from qhull: circumcentres in [0,1)^d of the Delaunay
    simplices of the cloud tiled 3^d times; returns canonical codes and the
    circumcentres moved to the canonical frame."""
    from scipy.spatial import Delaunay

    n, d = X.shape
    shifts = np.array(list(itertools.product([-1, 0, 1], repeat=d)))
    P = (shifts[:, None, :] + X[None, :, :]).reshape(-1, d)
    tri = Delaunay(P)
    S = P[tri.simplices]
    A = 2 * (S[:, 1:] - S[:, :1])
    b = (S[:, 1:] ** 2).sum(-1) - (S[:, :1] ** 2).sum(-1)
    ok = np.abs(np.linalg.det(A)) > 1e-12
    simp = tri.simplices[ok]
    c = np.linalg.solve(A[ok], b[ok][..., None])[..., 0]
    inside = np.all((c >= 0) & (c < 1), axis=1)
    simp, c = simp[inside], c[inside]
    ids = simp % n
    shift = shifts[simp // n]
    order = np.argsort(ids, axis=1, kind="stable")
    k0 = np.take_along_axis(shift, order[:, :1, None], axis=1)[:, 0, :]
    ids, shift = _canonical(ids, shift, d)
    return np.sort(_encode(ids, shift, d), axis=1), c - k0


@pytest.mark.parametrize("d,n,seed", [(2, 100, 0), (2, 400, 1), (3, 200, 2), (4, 100, 3)])
def test_periodic_vertices_are_qhulls_on_the_tiled_cloud(d, n, seed):
    X = W.uniform_cloud(n, d, seed=seed).astype(np.float64)
    m = oracle.explore_periodic(X, W.descent_draws(d))
    assert m["duplicates"] == 0
    keys, cen = _tiled_delaunay(X)
    got = {tuple(r): v for r, v in zip(m["key"].astype(np.int64).tolist(), m["coord"])}
    ref = {tuple(r): v for r, v in zip(keys.tolist(), cen)}
    assert set(got) == set(ref)
    worst = max(float(np.abs(got[k] - ref[k]).max()) for k in ref)
    assert worst <= 1e-9, worst


def _counts(m, d):
    """Vertices V, distinct edges E and distinct facets F of a periodic mesh."""
    ids, sh = m["sigma"].astype(np.int64), m["shift"].astype(np.int64)
    V = ids.shape[0]
    edges = set()
    for o in range(d + 1):
        ei = np.delete(ids, o, axis=1)
        es = np.delete(sh, o, axis=1)
        es = es - es[:, :1, :]
        edges.update(map(tuple, _encode(ei, es, d).tolist()))
    facets = set()
    for a, b in itertools.combinations(range(d + 1), 2):
        rel = _encode(np.zeros(V, dtype=np.int64), sh[:, b] - sh[:, a], d)
        facets.update(zip(ids[:, a].tolist(), ids[:, b].tolist(), rel.tolist()))
    return V, len(edges), len(facets)


@pytest.mark.parametrize("d,n,seed", [(2, 300, 4), (3, 300, 5), (4, 150, 6)])
def test_periodic_euler_relations(d, n, seed):
    """On the torus (Euler characteristic 0) a simple tessellation with n
    cells has (d+1) V / 2 edges and: d=2, V = 2n; d=3, F = n + V; d=4,
    F = V/2 + 3n (cell Euler relations summed over the cells)."""
    X = W.uniform_cloud(n, d, seed=seed)
    m = oracle.explore_periodic(X, W.descent_draws(d))
    V, E, F = _counts(m, d)
    assert 2 * E == (d + 1) * V
    if d == 2:
        assert V == 2 * n and F == 3 * n
    elif d == 3:
        assert F == n + V
    else:
        assert 2 * F == V + 6 * n


@pytest.mark.parametrize("d,n,seed", [(2, 200, 7), (3, 150, 8), (5, 120, 9)])
def test_periodic_vertices_have_empty_balls(d, n, seed):
    X = W.uniform_cloud(n, d, seed=seed).astype(np.float64)
    m = oracle.explore_periodic(X, W.descent_draws(d))
    shifts = np.array(list(itertools.product([-1, 0, 1], repeat=d)))
    P = (shifts[:, None, :] + X[None, :, :]).reshape(-1, d)
    pid = np.tile(np.arange(n), len(shifts))
    psh = np.repeat(shifts, n, axis=0)
    rng = np.random.default_rng(seed)
    for v in rng.choice(m["key"].shape[0], min(200, m["key"].shape[0]), replace=False):
        p = m["coord"][v]
        gen = X[m["sigma"][v]] + m["shift"][v]
        rho = np.sqrt(((gen - p) ** 2).sum(axis=1))
        assert rho.max() - rho.min() <= 1e-9 * rho.max()
        assert rho.max() < 0.5
        dist = np.sqrt(((P - p) ** 2).sum(axis=1))
        member = np.zeros(len(P), dtype=bool)
        for i, k in zip(m["sigma"][v], m["shift"][v]):
            member |= (pid == i) & np.all(psh == k, axis=1)
        assert member.sum() == d + 1
        assert dist[~member].min() >= rho.min() * (1 - 1e-9)


def test_periodic_3d_mean_vertex_count_is_meijerings():
    """The typical 3-D Poisson-Voronoi cell has 96 pi^2 / 35 = 27.07 vertices
    on average (Meijering); 1000 uniform nodes on the torus come within 2 %
    (the per-cell count has a standard deviation near 7)."""
    d, n = 3, 1000
    m = oracle.explore_periodic(W.uniform_cloud(n, d, seed=0), W.descent_draws(d))
    per_cell = (d + 1) * m["key"].shape[0] / n
    assert per_cell == pytest.approx(96 * math.pi ** 2 / 35, rel=0.02)


def test_periodic_search_reports_balls_too_large():
    """Three nodes in 3-D: vertex balls reach radius 1/2 and beyond, outside
    what the key codes describe."""
    with pytest.raises(RuntimeError, match="radius|past the images"):
        oracle.explore_periodic(W.uniform_cloud(3, 3, seed=0), W.descent_draws(3))
