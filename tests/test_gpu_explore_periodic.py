"""GPU exhaustive search of the periodic diagram (Algorithm 2 on the torus
R^d / Z^d, VG_PERIODIC) against the FP64 oracle: vertex keys bit-exact as
sets, FP64 coordinates to 1e-9; at larger sizes against relations that hold
for any simple tessellation of the torus, and sampled empty balls."""
import itertools
import math

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


def _explore(vg, X):
    d = X.shape[1]
    return vg.explore(torch.from_numpy(X).cuda(), W.descent_draws(d), periodic=True)


@pytest.mark.parametrize("d,n,seed", [(2, 100, 0), (2, 1000, 0), (3, 300, 1), (4, 200, 2), (5, 120, 9)])
def test_periodic_explore_matches_oracle(vg, d, n, seed):
    print(f"periodic explore d={d} n={n} seed={seed}", flush=True)
    X = W.uniform_cloud(n, d, seed=seed)
    got = _explore(vg, X)
    ref = oracle.explore_periodic(X, W.descent_draws(d))
    assert got["b_sigma"].shape[0] == 0
    g = {tuple(r): v for r, v in zip(got["key"].tolist(), got["coord"])}
    r = {tuple(k): v for k, v in zip(ref["key"].tolist(), ref["coord"])}
    assert len(g) == got["key"].shape[0]
    assert set(g) == set(r)
    worst = max(float(np.abs(g[k] - r[k]).max()) for k in r)
    assert worst <= 1e-9, worst


def _edge_count(ids, sh, d):
    """Distinct edges: each vertex key minus one entry, translated so its
    first node has k = 0, hashed to 64 bits."""
    n_codes = 3 ** d
    mult = np.random.default_rng(0).integers(1, 2**62, size=d, dtype=np.int64) | 1
    hs = []
    for o in range(d + 1):
        ei = np.delete(ids, o, axis=1).astype(np.int64)
        es = np.delete(sh, o, axis=1).astype(np.int64)
        es = es - es[:, :1, :]
        code = ei * n_codes
        for a in range(d):
            code = code + (es[..., a] + 1) * 3 ** a
        hs.append((code * mult).sum(axis=1))  # wraps mod 2^64
    return np.unique(np.concatenate(hs)).size


def _facet_count(ids, sh, n, d):
    """Distinct facets: pairs (i, j) of a key with the shift of j relative to i."""
    codes = []
    for a, b in itertools.combinations(range(d + 1), 2):
        rel = np.zeros(ids.shape[0], dtype=np.int64)
        for q in range(d):
            rel += (sh[:, b, q].astype(np.int64) - sh[:, a, q] + 1) * 3 ** q
        codes.append((ids[:, a].astype(np.int64) * n + ids[:, b]) * 3 ** d + rel)
    return np.unique(np.concatenate(codes)).size


def _sampled_empty_balls(X, m, count, seed):
    n, d = X.shape
    X64 = X.astype(np.float64)
    shifts = np.array(list(itertools.product([-1, 0, 1], repeat=d)))
    rng = np.random.default_rng(seed)
    for v in rng.choice(m["key"].shape[0], count, replace=False):
        p = m["coord"][v]
        gen = X64[m["sigma"][v]] + m["shift"][v]
        rho = np.sqrt(((gen - p) ** 2).sum(axis=1))
        assert rho.max() - rho.min() <= 1e-9 * rho.max()
        # nearest image of every node to p, and its distance
        dd = np.full(n, np.inf)
        for k in shifts:
            dd = np.minimum(dd, np.sqrt(((X64 + k - p) ** 2).sum(axis=1)))
        dd[m["sigma"][v]] = np.inf
        assert dd.min() >= rho.min() * (1 - 1e-9)


@pytest.mark.parametrize("d,n", [(2, 100_000), (3, 100_000), (4, 20_000), (5, 2000), (6, 1000)])
def test_periodic_explore_relations_at_size(vg, d, n):
    """Every simple tessellation of the torus with n cells has (d+1) V / 2
    edges, and: d=2, V = 2n; d=3, F = n + V; d=4, F = V/2 + 3n."""
    X = W.uniform_cloud(n, d, seed=0)
    m = _explore(vg, X)
    ids, sh = m["sigma"], m["shift"]
    V = ids.shape[0]
    print(f"  periodic d={d} N={n}: {V} vertices, {(d + 1) * V / n:.2f} per cell, "
          f"{m['raycasts']} raycasts", flush=True)
    assert np.unique(m["key"], axis=0).shape[0] == V
    assert 2 * _edge_count(ids, sh, d) == (d + 1) * V
    if d <= 4:
        F = _facet_count(ids, sh, n, d)
        if d == 2:
            assert V == 2 * n and F == 3 * n
        elif d == 3:
            assert F == n + V
            # Meijering: 96 pi^2 / 35 vertices per 3-D Poisson-Voronoi cell
            assert (d + 1) * V / n == pytest.approx(96 * math.pi ** 2 / 35, rel=0.005)
        else:
            assert 2 * F == V + 6 * n
    _sampled_empty_balls(X, m, 200, seed=d)


def test_periodic_explore_neighbour_growth_per_dimension(vg):
    """Neighbours per cell grow by a factor between 2.2 and 2.6 from d to d+1
    (Sec. 2.4), measured on the periodic diagram for d = 2..6."""
    sizes = {2: 20_000, 3: 20_000, 4: 5000, 5: 2000, 6: 1000}
    nbr = {}
    for d, n in sizes.items():
        m = _explore(vg, W.uniform_cloud(n, d, seed=1))
        nbr[d] = 2 * _facet_count(m["sigma"], m["shift"], n, d) / n
        print(f"  d={d} N={n}: {(d + 1) * m['key'].shape[0] / n:.1f} vertices and {nbr[d]:.1f} neighbours "
              "per cell", flush=True)
    assert nbr[2] == 6.0
    for d in range(2, 6):
        assert 2.2 <= nbr[d + 1] / nbr[d] <= 2.6, (d, nbr)


def test_periodic_explore_rejects_nodes_outside_the_unit_cube(vg):
    X = W.uniform_cloud(50, 3, seed=3)
    X[7, 1] = 1.0
    with pytest.raises(vg.VGError):
        _explore(vg, X)


def test_periodic_explore_reports_balls_of_radius_half_or_more(vg):
    """Three nodes in 3-D: vertex balls reach radius 1/2, which the key codes
    cannot describe; the search widens its layer to w = 1 and then reports
    it (the oracle fails the same way)."""
    X = W.uniform_cloud(3, 3, seed=0)
    with pytest.raises(vg.VGError, match="radius|draws"):
        _explore(vg, X)


def test_periodic_explore_argument_errors(vg):
    X = torch.from_numpy(W.uniform_cloud(200, 3, seed=4)).cuda()
    with pytest.raises(vg.VGError, match="excludes"):
        vg.explore(X, W.descent_draws(3), clip=True, periodic=True)
    with pytest.raises(vg.VGError, match="excludes"):
        vg.explore(X, W.descent_draws(3), incircle=True, periodic=True)
    with pytest.raises(vg.VGError, match="draws"):
        vg.explore(X, None, periodic=True)
    X9 = torch.from_numpy(W.uniform_cloud(50, 9, seed=4)).cuda()
    with pytest.raises(vg.VGError, match="d <= 8"):
        vg.explore(X9, W.descent_draws(9), periodic=True)
