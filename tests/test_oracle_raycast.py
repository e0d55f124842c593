"""Pins of the oracle's RayCast (definition of the first bisector hit,
Sec. 2.2 eq. (t) with the half-space restriction of Algorithm 1).

Each pin reaches the answer by a route that does not use eq. (t):
  * bisection of "g is a nearest generator of x + s u" along the ray;
  * the incircle criterion at the hit (Sec. 2.2);
  * Algorithm 1 itself (iterative nearest-neighbour projection);
  * a lone generator, whose only exit is a face of the cube.
"""
import json
import os

import numpy as np
import pytest

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _nearest(X, p):
    return np.argmin(((X - p) ** 2).sum(axis=1))


def _inside_cell(X, g, p):
    """g is a nearest generator of p (ties count as inside)."""
    d2 = ((X - p) ** 2).sum(axis=1)
    return d2[g] <= d2.min()


def test_sphere_area_golden(oracle_mod):
    gold = json.load(open(os.path.join(GOLD, "sphere_area.json")))
    for d, S in zip(gold["d"], gold["S"]):
        assert oracle_mod.sphere_area(d) == pytest.approx(S, rel=1e-14)


@pytest.mark.parametrize("d,n", [(2, 50), (3, 200), (5, 300)])
def test_mc_ray_matches_bisection_of_cell_membership(oracle_mod, d, n):
    X = W.uniform_cloud(n, d, seed=d)
    X64 = X.astype(np.float64)
    cells = np.arange(0, n, max(1, n // 12))
    D = W.mc_directions(cells, 16, d, seed=7)
    t, idx, _ = oracle_mod.raycast_cells(X, cells, D)
    D64 = D.astype(np.float64).reshape(-1, d)
    for k in range(t.size):
        i = cells[k // 16]
        x, u = X64[i], D64[k]
        # bracket: inside at 0, outside beyond the cube diagonal
        lo, hi = 0.0, 2.0 * np.sqrt(d)

        def inside(s):
            p = x + s * u
            return _inside_cell(X64, i, p) and np.all(p >= 0.0) and np.all(p <= 1.0)

        assert inside(lo) and not inside(hi)
        for _ in range(80):
            mid = 0.5 * (lo + hi)
            if inside(mid):
                lo = mid
            else:
                hi = mid
        assert t[k] == pytest.approx(lo, rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("d,n", [(2, 40), (3, 120), (4, 200)])
def test_hit_satisfies_incircle_criterion(oracle_mod, d, n):
    """At p = x + t u the sphere through g and x_j contains no generator."""
    X = W.uniform_cloud(n, d, seed=10 + d)
    X64 = X.astype(np.float64)
    cells = np.arange(n)
    D = W.mc_directions(cells, 8, d, seed=3)
    t, idx, _ = oracle_mod.raycast_cells(X, cells, D)
    D64 = D.astype(np.float64).reshape(-1, d)
    nodes_hit = 0
    for k in range(t.size):
        i = k // 8
        p = X64[i] + t[k] * D64[k]
        rad2 = ((p - X64[i]) ** 2).sum()
        d2 = ((X64 - p) ** 2).sum(axis=1)
        assert d2.min() >= rad2 * (1 - 1e-10)
        if idx[k] >= 0:
            nodes_hit += 1
            assert d2[idx[k]] == pytest.approx(rad2, rel=1e-10)
            assert idx[k] != i
        else:
            face = -2 - idx[k]
            kk, s = divmod(face, 2)
            assert p[kk] == pytest.approx(float(s), abs=1e-12)
    assert nodes_hit > t.size // 4


def test_lone_generator_exits_through_a_face(oracle_mod):
    d = 4
    X = W.uniform_cloud(1, d, seed=5)
    D = W.mc_directions([0], 256, d, seed=5)
    t, idx, t2 = oracle_mod.raycast_cells(X, [0], D)
    assert np.all(idx <= -2)
    p = X[0].astype(np.float64) + t[:, None] * D[0].astype(np.float64)
    assert np.all(p >= -1e-12) and np.all(p <= 1 + 1e-12)
    on_face = np.min(np.minimum(np.abs(p), np.abs(p - 1.0)), axis=1)
    assert np.all(on_face <= 1e-12)
    # the reported face is the one the point lies on
    faces = -2 - idx
    kk, s = faces // 2, faces % 2
    assert np.allclose(p[np.arange(256), kk], s, atol=1e-12)
    assert np.all(np.isinf(t2) | (t2 >= t))


@pytest.mark.parametrize("d,n", [(2, 300), (3, 300), (4, 300)])
@pytest.mark.parametrize("heuristic", [False, True])
def test_definition_matches_algorithm1_on_explore_rays(oracle_mod, d, n, heuristic):
    """Edge rays from Voronoi vertices: the brute-force definition and the
    paper's iterative incircle RayCast return the same generator and t."""
    X = W.uniform_cloud(n, d, seed=20 + d)
    mesh = oracle_mod.explore(X, W.descent_draws(d), mode=0)
    rng = np.random.default_rng(0)
    pick = rng.choice(mesh["sigma"].shape[0], 60, replace=False)
    O, U, E = [], [], []
    for v in pick:
        sig = mesh["sigma"][v]
        o = rng.integers(d + 1)
        eta = np.delete(sig, o)
        O.append(mesh["coord"][v])
        U.append(oracle_mod.search_direction(X, eta, sig[o]))
        E.append(eta)
    O, U, E = np.array(O), np.array(U), np.array(E, dtype=np.int32)
    t, idx, t2 = oracle_mod.raycast(X, O, U, E[:, 0], excl=E, clip=False)
    ta, ia, calls = oracle_mod.raycast_incircle(X, O, U, E, heuristic=heuristic)
    assert np.array_equal(idx, ia)
    hit = idx >= 0
    assert np.allclose(t[hit], ta[hit], rtol=1e-9, atol=1e-12)
    assert np.all(calls >= 1)


def test_excluded_and_backward_nodes_are_never_returned(oracle_mod):
    d, n = 3, 100
    X = W.uniform_cloud(n, d, seed=4).astype(np.float64)
    rng = np.random.default_rng(1)
    g = rng.integers(n, size=200)
    U = rng.standard_normal((200, d))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    t, idx, _ = oracle_mod.raycast(X, X[g], U, g, excl=g[:, None], clip=True)
    for k in range(200):
        if idx[k] >= 0:
            assert idx[k] != g[k]
            assert U[k] @ (X[idx[k]] - X[g[k]]) > 0


@pytest.mark.slow
def test_table_nncalls_soft_pin(oracle_mod):
    """Algorithm 1 inside Algorithm 2 on 1000 uniform generators needs about
    as many nn calls per vertex as Table nncalls prints (+-10 %)."""
    gold = json.load(open(os.path.join(GOLD, "nncalls_table.json")))
    for a, d in enumerate(gold["d"][:3]):
        X = W.uniform_cloud(1000, d, seed=0)
        for mode, key in ((1, "incircle"), (2, "incircle_heuristic")):
            m = oracle_mod.explore(X, W.descent_draws(d), mode=mode)
            per_vertex = m["nn_calls"] / m["sigma"].shape[0]
            assert per_vertex == pytest.approx(gold[key][a], rel=0.10), (d, key, per_vertex)
