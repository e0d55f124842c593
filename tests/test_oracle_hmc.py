"""Pins of the oracle's heuristic Monte-Carlo integrals (Sec. 3.3) over the
clipped diagram: exactness where the rule must be exact, and reductions to
volumes computed by other routes."""
import numpy as np
import pytest

import oracle
import workloads as W


def _clip_polygon(poly, a, b):
    out = []
    for p, q in zip(poly, poly[1:] + poly[:1]):
        fp, fq = a @ p - b, a @ q - b
        if fp <= 0:
            out.append(p)
        if fp * fq < 0:
            out.append(p + (q - p) * (fp / (fp - fq)))
    return out


def _polygon_area_centroid(poly):
    P = np.array(poly)
    x, y = P[:, 0], P[:, 1]
    xn, yn = np.roll(x, -1), np.roll(y, -1)
    cr = x * yn - xn * y
    A = cr.sum() / 2
    return A, np.array([((x + xn) * cr).sum(), ((y + yn) * cr).sum()]) / (6 * A)


def _facet_members(sig, n):
    mem = {}
    for v, row in enumerate(sig):
        for a in row:
            if a >= n:
                continue
            for b in row:
                if b != a:
                    j = int(b) if b < n else -2 - int(b - n)
                    mem.setdefault((int(a), j), []).append(v)
    return mem


def test_hmc_2d_is_exact_for_linear_f_with_exact_lengths():
    """In 2-D a facet is a segment: the mean of its two vertices is its
    midpoint, so the interface rule integrates a linear f exactly, and so
    does the pyramid rule over each triangle (x_i, segment)."""
    n = 40
    X = W.uniform_cloud(n, 2, seed=21).astype(np.float64)
    m = oracle.explore_clipped(X)
    mem = _facet_members(m["sigma"], n)
    areas = {k: float(np.linalg.norm(m["coord"][v[0]] - m["coord"][v[1]])) for k, v in mem.items()}
    c0, c = 0.7, np.array([1.3, -2.1])
    f = lambda p: c0 + p @ c  # noqa: E731
    r = oracle.hmc_integrals(X, m["sigma"], m["coord"], areas, f)
    for (i, j), v in mem.items():
        mid = m["coord"][v].mean(axis=0)
        assert r["F"][(i, j)] == pytest.approx(areas[(i, j)] * f(mid), rel=1e-12, abs=1e-15)
    for i in range(n):
        poly = [np.array(q, dtype=np.float64) for q in ((0, 0), (1, 0), (1, 1), (0, 1))]
        for j in range(n):
            if j != i:
                poly = _clip_polygon(poly, 2 * (X[j] - X[i]), X[j] @ X[j] - X[i] @ X[i])
        A, cen = _polygon_area_centroid(poly)
        assert r["volume"][i] == pytest.approx(A, rel=1e-12)
        assert r["cell"][i] == pytest.approx(A * f(cen), rel=1e-11)


def _planar_polygon_area(P):
    """Area of a convex planar polygon given by its vertices in any order."""
    c = P.mean(axis=0)
    Q = P - c
    _, _, vt = np.linalg.svd(Q)
    uv = Q @ vt[:2].T
    order = np.argsort(np.arctan2(uv[:, 1], uv[:, 0]))
    x, y = uv[order, 0], uv[order, 1]
    return 0.5 * abs((x * np.roll(y, -1) - np.roll(x, -1) * y).sum())


def test_hmc_3d_volume_with_exact_areas_is_the_hull_volume():
    from scipy.spatial import ConvexHull

    n = 60
    X = W.uniform_cloud(n, 3, seed=22).astype(np.float64)
    m = oracle.explore_clipped(X)
    mem = _facet_members(m["sigma"], n)
    areas = {k: _planar_polygon_area(m["coord"][v]) for k, v in mem.items()}
    r = oracle.hmc_integrals(X, m["sigma"], m["coord"], areas, lambda p: np.ones(len(p)))
    for i in range(n):
        hull = ConvexHull(m["coord"][(m["sigma"] == i).any(axis=1)]).volume
        assert r["volume"][i] == pytest.approx(hull, rel=1e-10)
        assert r["cell"][i] == pytest.approx(hull, rel=1e-10)


@pytest.mark.parametrize("d,n,R", [(2, 50, 256), (3, 40, 256)])
def test_hmc_constant_f_with_mc_areas(d, n, R):
    X = W.uniform_cloud(n, d, seed=23)
    D = W.mc_directions(range(n), R, d, seed=24)
    mc = oracle.mc_volume_area(X, np.arange(n), D)
    m = oracle.explore_clipped(X)
    r = oracle.hmc_integrals(X, m["sigma"], m["coord"], mc["facets"], lambda p: np.ones(len(p)))
    for k, A in mc["facets"].items():
        assert r["F"][k] == pytest.approx(A, rel=1e-13)
    assert np.allclose(r["cell"], r["volume"], rtol=1e-13)
    # per ray h l^{d-1} / |n.u| = l^d (Sec. 3.3), so the volume from the
    # Monte-Carlo areas is the direct estimator's value
    assert np.allclose(r["volume"], mc["volume"], rtol=1e-10, atol=0)
