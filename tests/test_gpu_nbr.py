"""Neighbour-restricted Monte-Carlo RayCast (the remark closing Sec. 3.1):
the cell adjacency built on the GPU from Voronoi vertex tuples, and the
Monte-Carlo estimators with each cell's scan restricted to its neighbours.

The vertex tuples come from the oracle's exhaustive search; the expected
adjacency is the set of ordered pairs inside those tuples, and the expected
estimator values are the oracle's scan over ALL nodes, so a missing
neighbour or a wrong row mapping shows up as a parity failure."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.parity import compare_rays, runner_up_cells, tie_adjusted

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    import paper_2405_10050_amd as vg
    return vg


def _pairs_csr(sigma, n):
    """Ordered pairs (a, b), a != b, inside each tuple, unique, as CSR."""
    L = sigma.shape[1]
    a = np.repeat(sigma, L, axis=1).ravel()
    b = np.tile(sigma, (1, L)).ravel()
    keep = a != b
    key = np.unique(a[keep].astype(np.int64) * (n + 1) + b[keep])
    rows, cols = key // (n + 1), key % (n + 1)
    off = np.zeros(n + 1, dtype=np.int64)
    np.add.at(off, rows + 1, 1)
    return np.cumsum(off), cols.astype(np.int32)


_MESH = {}


def _mesh(d, n, seed):
    if (d, n, seed) not in _MESH:
        X = W.uniform_cloud(n, d, seed=seed)
        _MESH[(d, n, seed)] = (X, oracle.explore(X, W.descent_draws(d)))
    return _MESH[(d, n, seed)]


@pytest.mark.parametrize("d,n", [(2, 1000), (3, 500), (4, 300), (6, 100)])
def test_tuple_neighbors_equal_the_pairs_of_the_oracle_tuples(vg, d, n):
    print(f"neighbours d={d} n={n}", flush=True)
    X, mesh = _mesh(d, n, 70 + d)
    dev = torch.device("cuda", 0)
    off, nbr = vg.tuple_neighbors(torch.from_numpy(mesh["sigma"]).to(dev), n)
    off_ref, nbr_ref = _pairs_csr(mesh["sigma"], n)
    assert np.array_equal(off.cpu().numpy(), off_ref)
    assert np.array_equal(nbr.cpu().numpy(), nbr_ref)
    # every generator of a bounded or unbounded diagram has a neighbour
    assert np.all(np.diff(off_ref) >= 1)


def _check_against_oracle(res, ref, X, D, rtol):
    n = X.shape[0]
    idx = res.idx.cpu().numpy()
    compare_rays(res.t.cpu().numpy(), idx, ref["t"], ref["idx"], ref["t2"], rtol=rtol,
                 runner_up=runner_up_cells(X, np.arange(n), D, ref["idx"]))
    assert np.allclose(res.volume.cpu().numpy(), ref["volume"], rtol=rtol, atol=0)
    assert np.allclose(res.energy2.cpu().numpy(), ref["energy2"], rtol=rtol, atol=0)
    cnt = res.facet_count.cpu().numpy()
    fj = res.facet_j.cpu().numpy()
    fa = res.facet_area.cpu().numpy()
    # every facet, with the oracle's sums on the GPU's choice among tied candidates
    adj = oracle.mc_volume_area(X, np.arange(n), D, rays=tie_adjusted(ref["t"], ref["idx"], ref["t2"], idx))
    got = {(i, int(fj[i, s])): float(fa[i, s]) for i in range(n) for s in range(cnt[i])}
    assert set(got) == set(adj["facets"])
    for key, A in adj["facets"].items():
        assert got[key] == pytest.approx(A, rel=rtol), key


@pytest.mark.parametrize("d,n,R,prec", [(2, 1000, 128, "fp32"), (3, 500, 256, "fp32"),
                                        (4, 300, 512, "fp32"), (4, 300, 512, "bf16x3"),
                                        (6, 100, 256, "fp32")])
def test_mc_over_neighbours_matches_oracle_over_all_nodes(vg, d, n, R, prec):
    print(f"mc neighbours d={d} n={n} R={R} {prec}", flush=True)
    X, mesh = _mesh(d, n, 70 + d)
    D = W.mc_directions(range(n), R, d, seed=5)
    dev = torch.device("cuda", 0)
    nodes = torch.from_numpy(X).to(dev)
    dirs = torch.from_numpy(D).to(dev)
    nb = vg.tuple_neighbors(torch.from_numpy(mesh["sigma"]).to(dev), n)
    res = vg.mc_volume_area(nodes, dirs, precision=prec, neighbors=nb)
    torch.cuda.synchronize()
    ref = oracle.mc_volume_area(X, np.arange(n), D)
    _check_against_oracle(res, ref, X, D, 1e-5)
    # the same rays through the full scan
    full = vg.mc_volume_area(nodes, dirs, precision=prec)
    compare_rays(full.t.cpu().numpy(), full.idx.cpu().numpy(), ref["t"], ref["idx"], ref["t2"], rtol=1e-5,
                 runner_up=runner_up_cells(X, np.arange(n), D, ref["idx"]))
    # and the adjoint through the neighbour result equals the full one's
    g_full = vg.mc_backward(nodes, dirs, full, torch.ones(n, device=dev), torch.ones(n, device=dev), None)
    g_nb = vg.mc_backward(nodes, dirs, res, torch.ones(n, device=dev), torch.ones(n, device=dev), None)
    assert torch.allclose(g_nb, g_full, rtol=1e-4, atol=1e-6 * float(g_full.abs().max()))


def test_superset_lists_and_invalid_entries_change_nothing(vg):
    d, n, R = 3, 500, 256
    X, mesh = _mesh(d, n, 73)
    D = W.mc_directions(range(n), R, d, seed=6)
    dev = torch.device("cuda", 0)
    nodes = torch.from_numpy(X).to(dev)
    dirs = torch.from_numpy(D).to(dev)
    off, nbr = _pairs_csr(mesh["sigma"], n)
    rng = np.random.default_rng(1)
    rows = []
    for i in range(n):
        row = list(nbr[off[i]:off[i + 1]])
        extra = rng.choice(n, 7, replace=False)
        row += [int(e) for e in extra if e != i] + [-5, n + 3, 2 ** 31 - 1]
        rng.shuffle(row)
        rows.append(np.array(row, dtype=np.int32))
    off2 = np.concatenate([[0], np.cumsum([len(r) for r in rows])]).astype(np.int64)
    nbr2 = np.concatenate(rows).astype(np.int32)
    res = vg.mc_volume_area(nodes, dirs, neighbors=(torch.from_numpy(off2).to(dev),
                                                    torch.from_numpy(nbr2).to(dev)))
    torch.cuda.synchronize()
    ref = oracle.mc_volume_area(X, np.arange(n), D)
    _check_against_oracle(res, ref, X, D, 1e-5)


def test_neighbor_argument_errors(vg):
    dev = torch.device("cuda", 0)
    sig = torch.tensor([[0, 1, 9]], dtype=torch.int32, device=dev)
    with pytest.raises(vg.VGError):
        vg.tuple_neighbors(sig, 5)  # entry 9 outside [0, 5)
    X = torch.rand(10, 3, device=dev)
    D = torch.nn.functional.normalize(torch.randn(10, 4, 3, device=dev), dim=2)
    with pytest.raises(ValueError):
        vg.mc_volume_area(X, D, neighbors=(torch.zeros(5, dtype=torch.int64, device=dev),
                                           torch.zeros(0, dtype=torch.int32, device=dev)))
