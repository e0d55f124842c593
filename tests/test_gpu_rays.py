"""GPU parity of the general RayCast (arbitrary origins, eta exclusion,
clip on/off) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.parity import compare_rays, runner_up_rays

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    import paper_2405_10050_amd as vg
    return vg


def _edge_rays(X, d, count, seed):
    """Edge rays of the oracle's Voronoi vertices (origins rounded to FP32)."""
    mesh = oracle.explore(X, W.descent_draws(d))
    rng = np.random.default_rng(seed)
    pick = rng.choice(mesh["sigma"].shape[0], min(count, mesh["sigma"].shape[0]), replace=False)
    O, U, E = [], [], []
    for v in pick:
        sig = mesh["sigma"][v]
        o = rng.integers(d + 1)
        eta = np.delete(sig, o)
        O.append(mesh["coord"][v])
        U.append(oracle.search_direction(X, eta, sig[o]))
        E.append(eta)
    return (np.array(O).astype(np.float32), np.array(U).astype(np.float32),
            np.array(E, dtype=np.int32))


@pytest.mark.parametrize("d,n", [(2, 500), (3, 400), (4, 300), (6, 200), (9, 120)])
@pytest.mark.parametrize("clip", [False, True])
def test_edge_rays_match_oracle(vg, d, n, clip):
    print(f"rays d={d} n={n} clip={clip}", flush=True)
    X = W.uniform_cloud(n, d, seed=40 + d)
    O, U, E = _edge_rays(X, d, 700, seed=d)
    dev = torch.device("cuda", 0)
    t, idx, st = vg.raycast(torch.from_numpy(X).to(dev), torch.from_numpy(O).to(dev),
                            torch.from_numpy(U).to(dev), torch.from_numpy(E[:, 0].copy()).to(dev),
                            torch.from_numpy(E).to(dev), clip=clip)
    t_ref, idx_ref, t2_ref = oracle.raycast(X, O, U, E[:, 0], excl=E, clip=clip)
    compare_rays(t.cpu().numpy(), idx.cpu().numpy(), t_ref, idx_ref, t2_ref, rtol=1e-5,
                 runner_up=runner_up_rays(X, O, U, E[:, 0], E, clip, idx_ref))


@pytest.mark.parametrize("d,n,m", [(3, 1000, 5000), (5, 777, 3000), (16, 257, 1000)])
def test_generator_rays_match_oracle(vg, d, n, m):
    X = W.uniform_cloud(n, d, seed=9)
    rng = np.random.default_rng(d)
    g = rng.integers(n, size=m).astype(np.int32)
    U = rng.standard_normal((m, d))
    U = (U / np.linalg.norm(U, axis=1, keepdims=True)).astype(np.float32)
    O = X[g]
    dev = torch.device("cuda", 0)
    t, idx, st = vg.raycast(torch.from_numpy(X).to(dev), torch.from_numpy(O).to(dev),
                            torch.from_numpy(U).to(dev), torch.from_numpy(g).to(dev),
                            torch.from_numpy(g[:, None].copy()).to(dev), clip=True)
    t_ref, idx_ref, t2_ref = oracle.raycast(X, O, U, g, excl=g[:, None], clip=True)
    compare_rays(t.cpu().numpy(), idx.cpu().numpy(), t_ref, idx_ref, t2_ref, rtol=1e-5,
                 runner_up=runner_up_rays(X, O, U, g, g[:, None], True, idx_ref))


def test_no_hit_rays(vg):
    """Rays leaving the hull of the nodes without clipping have no hit."""
    X = W.uniform_cloud(50, 2, seed=1)
    dev = torch.device("cuda", 0)
    far = np.argmax(X[:, 0])
    O = X[[far]]
    U = np.array([[1.0, 0.0]], dtype=np.float32)
    g = np.array([far], dtype=np.int32)
    t, idx, st = vg.raycast(torch.from_numpy(X).to(dev), torch.from_numpy(O).to(dev),
                            torch.from_numpy(U).to(dev), torch.from_numpy(g).to(dev),
                            torch.from_numpy(g[:, None].copy()).to(dev), clip=False)
    t_ref, idx_ref, _ = oracle.raycast(X, O, U, g, excl=g[:, None], clip=False)
    assert idx_ref[0] == -1 and idx.item() == -1
    assert not np.isfinite(t.item())
    assert st.item() & vg.ST_NO_HIT


def test_argument_errors(vg):
    dev = torch.device("cuda", 0)
    X = torch.rand(10, 17, device=dev)
    D = torch.rand(10, 4, 17, device=dev)
    with pytest.raises(vg.VGError):
        vg.raycast_cells(X, D)  # d = 17 > VG_MAX_DIM
    with pytest.raises(vg.VGError):
        vg.raycast_cells(torch.rand(10, 3), torch.rand(10, 4, 3))  # CPU tensors
    with pytest.raises(ValueError):
        vg.raycast_cells(torch.rand(10, 3, device=dev), torch.rand(9, 4, 3, device=dev))


@pytest.mark.parametrize("d", [3, 7])
def test_node_split_scan_matches_whole_range_scan(vg, d):
    """A call with few rays splits the nodes over workgroups and merges the
    partial top-2 states; the same rays inside one call large enough not to
    split give the same argmin and t*.  (Which rays the certificate queues
    may differ where the runner-up's t sits within an ulp of the division-free
    filter, so t* is compared to FP32 rounding and the status bits on all but
    a few rays.)"""
    n, m = 6000, 300_000
    rng = np.random.default_rng(60 + d)
    X = torch.from_numpy(W.uniform_cloud(n, d, seed=61)).cuda()
    g = torch.from_numpy(rng.integers(n, size=m).astype(np.int32)).cuda()
    U = rng.standard_normal((m, d))
    U = torch.from_numpy((U / np.linalg.norm(U, axis=1, keepdims=True)).astype(np.float32)).cuda()
    O = X[g.long()] + 0.01 * torch.rand(m, d, device="cuda")
    ex = g[:, None].contiguous()
    t_all, i_all, s_all = vg.raycast(X, O, U, g, ex, clip=True)
    for lo in (0, 1000, 150_000, m - 700):
        hi = min(m, lo + 700)
        t, i, s = vg.raycast(X, O[lo:hi].contiguous(), U[lo:hi].contiguous(), g[lo:hi].contiguous(),
                             ex[lo:hi].contiguous(), clip=True)
        assert torch.equal(i, i_all[lo:hi])
        assert torch.allclose(t, t_all[lo:hi], rtol=3e-7, atol=0)
        assert int((s != s_all[lo:hi]).sum()) <= 2
