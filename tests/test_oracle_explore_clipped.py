"""Pins of the oracle's exhaustive search on the diagram clipped to the unit
cube (Algorithm 2 with the cube's faces as constraints).

Each check reaches the result by a route of its own: brute-force enumeration
of constraint sets, the 2-D Euler relation, half-plane clipping of the
square, convex hulls of the cells, and the unbounded diagram of the same
points."""
import itertools

import numpy as np
import pytest

import oracle
import workloads as W


def _keys(sigma):
    return {tuple(int(v) for v in row) for row in sigma}


def _brute_force(X, tol=1e-9):
    """Every point of the cube fixed by d+1 constraints -- a >= 1 generators
    at a common distance that no other generator undercuts, and d+1-a faces
    x_k = s on distinct axes -- keyed like the oracle (face code n + 2k + s)."""
    n, d = X.shape
    out = {}
    for a in range(1, d + 2):
        for A in itertools.combinations(range(n), a):
            for axes in itertools.combinations(range(d), d + 1 - a):
                for sides in itertools.product((0, 1), repeat=len(axes)):
                    M = np.zeros((d, d))
                    b = np.zeros(d)
                    xa = X[A[0]]
                    r = 0
                    for g in A[1:]:
                        M[r] = 2.0 * (X[g] - xa)
                        b[r] = X[g] @ X[g] - xa @ xa
                        r += 1
                    for k, s in zip(axes, sides):
                        M[r, k] = 1.0
                        b[r] = s
                        r += 1
                    if abs(np.linalg.det(M)) < 1e-12:
                        continue
                    v = np.linalg.solve(M, b)
                    if np.any(v < -tol) or np.any(v > 1 + tol):
                        continue
                    d2 = ((X - v) ** 2).sum(axis=1)
                    rho = d2[A[0]]
                    others = np.delete(d2, A)
                    if others.size and others.min() <= rho * (1 + 1e-9) + 1e-15:
                        continue
                    key = tuple(sorted(list(A) + [n + 2 * k + s for k, s in zip(axes, sides)]))
                    out[key] = v
    return out


@pytest.mark.parametrize("d,n,seed", [(2, 1, 0), (2, 2, 1), (2, 7, 2), (2, 12, 3), (3, 1, 0),
                                      (3, 5, 4), (3, 9, 5), (4, 6, 6)])
def test_clipped_explore_equals_brute_force(d, n, seed):
    X = W.uniform_cloud(n, d, seed=seed)
    m = oracle.explore_clipped(X)
    ref = _brute_force(X.astype(np.float64))
    assert _keys(m["sigma"]) == set(ref)
    for row, v in zip(m["sigma"], m["coord"]):
        assert np.allclose(v, ref[tuple(int(c) for c in row)], atol=1e-9)
    assert m["duplicates"] == 0


@pytest.mark.parametrize("n", [1, 2, 3, 50, 1000])
def test_clipped_explore_2d_euler(n):
    """A clipped planar diagram of n cells: corners have degree 2, every other
    vertex degree 3, so 2E = 3V - 4, and V - E + (n + 1) = 2 gives V = 2n + 2."""
    X = W.uniform_cloud(n, 2, seed=0)
    m = oracle.explore_clipped(X)
    assert m["sigma"].shape[0] == 2 * n + 2
    corners = sum(1 for row in m["sigma"] if (row >= n).sum() == 2)
    assert corners == 4


def _clip_polygon(poly, a, b):
    """Sutherland-Hodgman: the part of polygon `poly` with a.p <= b."""
    out = []
    for p, q in zip(poly, poly[1:] + poly[:1]):
        fp, fq = a @ p - b, a @ q - b
        if fp <= 0:
            out.append(p)
        if fp * fq < 0:
            out.append(p + (q - p) * (fp / (fp - fq)))
    return out


def test_clipped_explore_2d_cells_are_the_half_plane_polygons():
    n = 60
    X = W.uniform_cloud(n, 2, seed=11).astype(np.float64)
    m = oracle.explore_clipped(X)
    for i in range(n):
        poly = [np.array(c, dtype=np.float64) for c in ((0, 0), (1, 0), (1, 1), (0, 1))]
        for j in range(n):
            if j != i:
                # |p - x_i|^2 <= |p - x_j|^2  <=>  2 (x_j - x_i).p <= |x_j|^2 - |x_i|^2
                poly = _clip_polygon(poly, 2 * (X[j] - X[i]), X[j] @ X[j] - X[i] @ X[i])
        mine = m["coord"][(m["sigma"] == i).any(axis=1)]
        assert len(mine) == len(poly), i
        for p in poly:
            assert np.abs(mine - p).max(axis=1).min() < 1e-9, (i, p)


def test_clipped_explore_3d_cell_volumes_sum_to_one():
    from scipy.spatial import ConvexHull

    n = 150
    X = W.uniform_cloud(n, 3, seed=12)
    m = oracle.explore_clipped(X)
    vols = np.array([ConvexHull(m["coord"][(m["sigma"] == i).any(axis=1)]).volume for i in range(n)])
    assert vols.min() > 0
    assert vols.sum() == pytest.approx(1.0, abs=1e-9)


@pytest.mark.parametrize("d,n", [(2, 1000), (3, 300)])
def test_clipped_interior_vertices_are_the_unbounded_ones_inside(d, n):
    X = W.uniform_cloud(n, d, seed=0)
    clipped = oracle.explore_clipped(X)
    full = oracle.explore(X, W.descent_draws(d))
    inner = clipped["sigma"][(clipped["sigma"] < n).all(axis=1)]
    inside = full["sigma"][((full["coord"] > 0) & (full["coord"] < 1)).all(axis=1)]
    assert _keys(inner) == _keys(inside)


@pytest.mark.parametrize("d,n", [(2, 300), (3, 200), (4, 80)])
def test_clipped_edges_are_seen_from_both_ends(d, n):
    X = W.uniform_cloud(n, d, seed=d)
    m = oracle.explore_clipped(X)
    seen = {}
    for row in m["sigma"]:
        for o in range(d + 1):
            e = tuple(int(v) for q, v in enumerate(row) if q != o)
            if min(e) < n:  # keeps a generator: an edge, not a corner point
                seen[e] = seen.get(e, 0) + 1
    assert set(seen.values()) == {2}
