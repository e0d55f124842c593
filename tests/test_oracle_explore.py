"""Pins of the oracle's exhaustive search (Algorithm 2).

The vertex set of the unbounded diagram equals the set of (d+1)-tuples of
generators whose circumsphere is empty (incircle criterion, Sec. 2.2), i.e.
the Delaunay simplices.  Checked by brute force on tiny inputs, by the 2-D
Euler relation, by edge-incidence counts, by the volume of the hull and by
scipy's Delaunay triangulation (qhull).
"""
import itertools

import numpy as np
import pytest

import workloads as W


def _brute_force_vertices(X):
    n, d = X.shape
    out = []
    for s in itertools.combinations(range(n), d + 1):
        P = X[list(s)]
        A = 2.0 * (P[1:] - P[0])
        b = ((P[1:] - P[0]) ** 2).sum(axis=1)
        try:
            y = np.linalg.solve(A, b)
        except np.linalg.LinAlgError:
            continue
        c = P[0] + y
        r2 = ((P[0] - c) ** 2).sum()
        d2 = ((X - c) ** 2).sum(axis=1)
        if np.all(d2 >= r2 * (1 - 1e-12)):
            out.append(s)
    return np.array(out, dtype=np.int32)


def _hull_size_2d(P):
    """Andrew's monotone chain: number of strict hull vertices."""
    pts = sorted(map(tuple, P))

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    return len(lower) + len(upper) - 2


@pytest.mark.parametrize("d,n,seed", [(2, 12, 0), (2, 14, 1), (3, 11, 2), (3, 12, 3)])
def test_tiny_inputs_match_brute_force_empty_spheres(oracle_mod, d, n, seed):
    X = W.uniform_cloud(n, d, seed=seed)
    m = oracle_mod.explore(X, W.descent_draws(d, seed=seed))
    got = oracle_mod.sorted_rows(m["sigma"])
    want = oracle_mod.sorted_rows(_brute_force_vertices(X.astype(np.float64)))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n,seed", [(50, 0), (400, 1), (1000, 0)])
def test_2d_euler_relation(oracle_mod, n, seed):
    """Planar triangulation of n points with h on the hull:
    V = 2n - 2 - h triangles and h unbounded edges."""
    X = W.uniform_cloud(n, 2, seed=seed)
    m = oracle_mod.explore(X, W.descent_draws(2, seed=seed))
    h = _hull_size_2d(X.astype(np.float64))
    assert m["sigma"].shape[0] == 2 * n - 2 - h
    assert m["b_sigma"].shape[0] == h
    assert m["duplicates"] == 0


@pytest.mark.parametrize("d,n", [(2, 300), (3, 200), (4, 120)])
def test_every_edge_has_two_vertices_or_one_unbounded_ray(oracle_mod, d, n):
    X = W.uniform_cloud(n, d, seed=3)
    m = oracle_mod.explore(X, W.descent_draws(d))
    count = {}
    for s in m["sigma"]:
        for o in range(d + 1):
            e = tuple(np.delete(s, o))
            count[e] = count.get(e, 0) + 1
    unb = set()
    for s, om in zip(m["b_sigma"], m["b_omit"]):
        unb.add(tuple(s[s != om]))
    assert set(count.values()) <= {1, 2}
    ones = {e for e, c in count.items() if c == 1}
    assert ones == unb
    # coordinates are equidistant to their generators
    X64 = X.astype(np.float64)
    for s, v in zip(m["sigma"][:200], m["coord"][:200]):
        r = np.linalg.norm(X64[s] - v, axis=1)
        assert np.allclose(r, r[0], rtol=1e-9)


@pytest.mark.parametrize("d,n", [(2, 500), (3, 200)])
def test_simplex_volumes_sum_to_hull_volume(oracle_mod, d, n):
    from math import factorial

    from scipy.spatial import ConvexHull

    X = W.uniform_cloud(n, d, seed=6).astype(np.float64)
    m = oracle_mod.explore(X, W.descent_draws(d))
    vol = 0.0
    for s in m["sigma"]:
        P = X[s]
        vol += abs(np.linalg.det(P[1:] - P[0])) / factorial(d)
    assert vol == pytest.approx(ConvexHull(X).volume, rel=1e-10)


@pytest.mark.parametrize("d,n", [(2, 1000), (3, 300)])
def test_matches_scipy_delaunay(oracle_mod, d, n):
    from scipy.spatial import Delaunay

    X = W.uniform_cloud(n, d, seed=0)
    m = oracle_mod.explore(X, W.descent_draws(d))
    ref = np.sort(Delaunay(X.astype(np.float64)).simplices, axis=1).astype(np.int32)
    assert np.array_equal(oracle_mod.sorted_rows(m["sigma"]), oracle_mod.sorted_rows(ref))
    if d == 2 and n == 1000:
        assert m["sigma"].shape[0] == 1980 and m["b_sigma"].shape[0] == 18


def test_search_direction_and_circumcentre(oracle_mod):
    """SearchDirection is a unit vector orthogonal to the edge's generators'
    span and pointing away from the omitted generator; moving along it keeps
    the point equidistant to the edge's generators."""
    d = 5
    X = W.uniform_cloud(40, d, seed=9).astype(np.float64)
    s = np.arange(d + 1, dtype=np.int32) * 3
    v = oracle_mod.circumcentre(X, s)
    r = np.linalg.norm(X[s] - v, axis=1)
    assert np.allclose(r, r[0], rtol=1e-12)
    for o in range(d + 1):
        eta = np.delete(s, o)
        u = oracle_mod.search_direction(X, eta, s[o])
        assert np.linalg.norm(u) == pytest.approx(1.0, rel=1e-14)
        assert np.allclose((X[eta[1:]] - X[eta[0]]) @ u, 0.0, atol=1e-12)
        assert u @ (X[s[o]] - X[eta[0]]) < 0
        p = v + 0.37 * u
        rr = np.linalg.norm(X[eta] - p, axis=1)
        assert np.allclose(rr, rr[0], rtol=1e-12)
        assert np.linalg.norm(X[s[o]] - p) > rr[0]


@pytest.mark.parametrize("d,n,i", [(2, 300, 7), (3, 200, 11), (4, 150, 3), (4, 150, 149)])
def test_star_equals_vertices_of_full_search_containing_i(oracle_mod, d, n, i):
    X = W.uniform_cloud(n, d, seed=31)
    full = oracle_mod.explore(X, W.descent_draws(d))
    want = full["sigma"][np.any(full["sigma"] == i, axis=1)]
    got = oracle_mod.star(X, i, W.descent_draws(d, seed=9))
    assert np.array_equal(oracle_mod.sorted_rows(got), oracle_mod.sorted_rows(want))
