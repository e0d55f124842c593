"""GPU exhaustive search (Algorithm 2, batched by level) against the
oracle's sequential Algorithm 2: identical vertex and unbounded-edge sets."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    import paper_2405_10050_amd as vg
    return vg


@pytest.mark.parametrize("d,n", [(2, 1000), (2, 37), (3, 300), (4, 200), (5, 100), (6, 80)])
def test_explore_matches_oracle(vg, d, n):
    print(f"explore d={d} n={n}", flush=True)
    X = W.uniform_cloud(n, d, seed=0)
    draws = W.descent_draws(d)
    got = vg.explore(torch.from_numpy(X).cuda(), draws)
    ref = oracle.explore(X, draws)
    a = oracle.sorted_rows(got["sigma"])
    b = oracle.sorted_rows(ref["sigma"])
    assert a.shape == b.shape and np.array_equal(a, b)
    # coordinates of the same key agree (both FP64 solves)
    order_g = np.lexsort(got["sigma"].T[::-1])
    order_r = np.lexsort(ref["sigma"].T[::-1])
    cg, cr = got["coord"][order_g], ref["coord"][order_r]
    assert np.allclose(cg, cr, rtol=1e-9, atol=1e-12)
    # unbounded edges as sets of (vertex key, omitted generator)
    bg = oracle.sorted_rows(np.column_stack([got["b_sigma"], got["b_omit"]]))
    br = oracle.sorted_rows(np.column_stack([ref["b_sigma"], ref["b_omit"]]))
    assert np.array_equal(bg, br)
    if d == 2 and n == 1000:
        assert a.shape[0] == 1980 and bg.shape[0] == 18


def test_explore_d6_n1000_equals_sequential_oracle(vg):
    d, n = 6, 1000
    X = W.uniform_cloud(n, d, seed=0)
    draws = W.descent_draws(d)
    got = vg.explore(torch.from_numpy(X).cuda(), draws)
    ref = oracle.explore(X, draws)
    assert np.array_equal(oracle.sorted_rows(got["sigma"]), oracle.sorted_rows(ref["sigma"]))
    bg = oracle.sorted_rows(np.column_stack([got["b_sigma"], got["b_omit"]]))
    br = oracle.sorted_rows(np.column_stack([ref["b_sigma"], ref["b_omit"]]))
    assert np.array_equal(bg, br)


def test_explore_d6_n10000_full_size_properties(vg):
    """The d=6, N=10 000 exhaustive search at full size: the simplices of the
    vertex keys tile the convex hull (volumes sum to its volume), every hull
    facet carries exactly one unbounded edge, and sampled vertices satisfy the
    incircle criterion by brute force."""
    from math import factorial

    from scipy.spatial import ConvexHull

    d, n = 6, 10_000
    X = W.uniform_cloud(n, d, seed=0)
    X64 = X.astype(np.float64)
    got = vg.explore(torch.from_numpy(X).cuda(), W.descent_draws(d))
    sig = got["sigma"]
    print(f"d=6 N=10000: {sig.shape[0]} vertices, {got['b_sigma'].shape[0]} unbounded edges",
          flush=True)
    # no duplicate keys
    assert np.unique(sig, axis=0).shape[0] == sig.shape[0]
    P = X64[sig]
    vol = np.abs(np.linalg.det(P[:, 1:] - P[:, :1])).sum() / factorial(d)
    hull = ConvexHull(X64)
    assert vol == pytest.approx(hull.volume, rel=1e-9)
    assert got["b_sigma"].shape[0] == hull.simplices.shape[0]
    rng = np.random.default_rng(0)
    for v in rng.choice(sig.shape[0], 2000, replace=False):
        c = got["coord"][v]
        d2 = ((X64 - c) ** 2).sum(axis=1)
        r2 = d2[sig[v]]
        assert np.allclose(r2, r2[0], rtol=1e-7)
        assert d2.min() >= r2[0] * (1 - 1e-9)


@pytest.mark.parametrize("incircle", [False, True])
def test_explore_d2_n300000_is_qhulls_delaunay(vg, incircle):
    """At N = 3e5 (the FP64 recheck then splits each queued ray's nodes over
    workgroups): the vertex keys are exactly qhull's Delaunay triangles, and
    the unbounded edges its hull edges."""
    from scipy.spatial import Delaunay

    n, d = 300_000, 2
    X = W.uniform_cloud(n, d, seed=0)
    got = vg.explore(torch.from_numpy(X).cuda(), W.descent_draws(d), incircle=incircle, heuristic=incircle)
    tri = Delaunay(X.astype(np.float64))
    a = oracle.sorted_rows(got["sigma"])
    b = oracle.sorted_rows(np.sort(tri.simplices.astype(np.int32), axis=1))
    assert a.shape == b.shape and np.array_equal(a, b)
    assert got["b_sigma"].shape[0] == tri.convex_hull.shape[0]


def test_explore_d3_n300000_is_qhulls_delaunay(vg):
    """d = 3, N = 3e5: the queued edge rays of far hull vertices take the
    exact-width split of the FP64 recheck over 2^18 nodes or more; the
    vertex keys are exactly qhull's Delaunay tetrahedra."""
    from scipy.spatial import Delaunay

    n, d = 300_000, 3
    X = W.uniform_cloud(n, d, seed=0)
    got = vg.explore(torch.from_numpy(X).cuda(), W.descent_draws(d))
    print(f"explore d=3 n=3e5: {got['sigma'].shape[0]} vertices", flush=True)
    tri = Delaunay(X.astype(np.float64))
    a = oracle.sorted_rows(got["sigma"])
    b = oracle.sorted_rows(np.sort(tri.simplices.astype(np.int32), axis=1))
    assert a.shape == b.shape and np.array_equal(a, b)
    assert got["b_sigma"].shape[0] == tri.convex_hull.shape[0]


def test_explore_d6_n10000_equals_the_oracles_full_search(vg):
    """The d=6, N=10 000 workload at full size against the oracle's own
    sequential Algorithm 2 (run once by tests/golden/make_explore_d6_n10000.py):
    the same vertex keys and unbounded edges, compared by SHA-256 of the
    sorted int32 rows."""
    import hashlib
    import json
    import os

    path = os.path.join(os.path.dirname(__file__), "golden", "explore_d6_n10000.json")
    if not os.path.exists(path):
        pytest.skip("run tests/golden/make_explore_d6_n10000.py first (about an hour on one core)")
    gold = json.load(open(path))
    d, n = 6, 10_000
    X = W.uniform_cloud(n, d, seed=0)
    got = vg.explore(torch.from_numpy(X).cuda(), W.descent_draws(d))

    def digest(a):
        rows = np.ascontiguousarray(oracle.sorted_rows(np.asarray(a, dtype=np.int32)), dtype="<i4")
        return hashlib.sha256(rows.tobytes()).hexdigest()

    assert got["sigma"].shape[0] == gold["vertices"]
    assert got["b_sigma"].shape[0] == gold["unbounded_edges"]
    assert digest(got["sigma"]) == gold["sigma_sha256"]
    assert digest(np.column_stack([got["b_sigma"], got["b_omit"]])) == gold["unbounded_sha256"]
