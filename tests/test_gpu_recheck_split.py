"""FP64 recheck of Monte-Carlo rays over clouds of 2^18 nodes or more.  There
the queue is split over node chunks (8 queued rays per workgroup share each
node tile, the chunks' top-2 folded per ray) and the queue beyond the split's
first 8192 rays goes to one workgroup per ray.  Every ray of sampled cells
that hold a rechecked ray is compared with the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.parity import compare_rays, runner_up_cells

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    import paper_2405_10050_amd as m
    return m


def check_rechecked_cells(vg, X, D, t, idx, st, n_cells, seed):
    st = st.cpu().numpy()
    rechecked = (st & vg.ST_RECHECKED) != 0
    cells = np.nonzero(rechecked.any(axis=1))[0]
    assert cells.size > 0
    pick = np.sort(np.random.default_rng(seed).choice(cells, min(n_cells, cells.size), replace=False))
    sel = torch.from_numpy(pick).to(t.device)
    Ds = D[sel].cpu().numpy()
    tr, ir, t2r = oracle.raycast_cells(X, pick, Ds)
    compare_rays(t[sel].cpu().numpy().ravel(), idx[sel].cpu().numpy().ravel(), tr, ir, t2r, rtol=1e-5,
                 runner_up=runner_up_cells(X, pick, Ds, ir))
    # the rechecked rays themselves: FP64 argmin, t* rounded once to FP32
    rr = rechecked[pick].ravel()
    tie = oracle.near_tie(tr, t2r)
    keep = rr & ~tie
    assert np.array_equal(idx[sel].cpu().numpy().ravel()[keep], ir[keep])
    np.testing.assert_allclose(t[sel].cpu().numpy().ravel()[keep], tr[keep], rtol=2 ** -23)
    return int(rechecked.sum())


def test_split_recheck_uniform_d3(vg):
    """Uniform d = 3, N = 300 000, 16 rays per cell, the dense FP32 scan and
    the incircle path: a short queue, all of it in the split."""
    n, d, R = 300_000, 3, 16
    X = W.uniform_cloud(n, d, seed=3)
    dev = torch.device("cuda", 0)
    Xd = torch.from_numpy(X).to(dev)
    D = W.mc_directions_device(n, R, d, seed=4, device=dev)
    for incircle in (False, True):
        print(f"split recheck: uniform d={d} n={n} R={R} incircle={incircle}", flush=True)
        t, idx, st = vg.raycast_cells(Xd, D, incircle=incircle)
        torch.cuda.synchronize()
        q = check_rechecked_cells(vg, X, D, t, idx, st, 24, seed=5)
        print(f"  {q} rays rechecked", flush=True)


def test_split_recheck_queue_beyond_the_split(vg):
    """Gaussian mixture d = 10, N = 270 000, 32 rays per cell, the split-BF16
    scan: its wider certificate queues more than 8192 rays, so both the split
    and the per-ray kernel run; sampled cells of both are checked."""
    n, d, R = 270_000, 10, 32
    X = W.gaussian_mixture_cloud(n, d, seed=6)
    dev = torch.device("cuda", 0)
    D = W.mc_directions_device(n, R, d, seed=7, device=dev)
    print(f"split recheck: mixture d={d} n={n} R={R} bf16x3", flush=True)
    t, idx, st = vg.raycast_cells(torch.from_numpy(X).to(dev), D, precision="bf16x3")
    torch.cuda.synchronize()
    q = check_rechecked_cells(vg, X, D, t, idx, st, 48, seed=8)
    print(f"  {q} rays rechecked", flush=True)
    assert q > 8192


def _far_rays(X, m, seed):
    """FP64 rays from origins 3 away from the cube's centre, aimed back into
    the cloud, each with its nearest node as generator (so the origin lies in
    that node's cell): FP32 cancellation in |r - x|^2 - |g - x|^2 sends most
    of them to the FP64 recheck."""
    rng = np.random.default_rng(seed)
    n, d = X.shape
    v = rng.standard_normal((m, d))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    O = 0.5 + 3.0 * v
    U = -v + 0.2 * rng.standard_normal((m, d))
    U /= np.linalg.norm(U, axis=1, keepdims=True)
    X64 = X.astype(np.float64)
    x2 = (X64 * X64).sum(axis=1)
    g = np.empty(m, dtype=np.int32)
    for a in range(0, m, 64):
        dd = x2[None, :] - 2.0 * (O[a:a + 64] @ X64.T)
        g[a:a + 64] = np.argmin(dd, axis=1)
    return O, U, g


@pytest.mark.parametrize("d,m", [(3, 500), (3, 6000), (8, 500), (8, 6000)])
def test_split_recheck_of_fp64_origin_rays(vg, d, m):
    """General rays with FP64 origins over N = 2^18 + 1000 nodes: queues
    below and above 2048 rays take the per-ray and the tiled split recheck;
    a sample is compared with the oracle's RayCast on the same FP64 rays."""
    n = (1 << 18) + 1000
    X = W.uniform_cloud(n, d, seed=70 + d)
    O, U, g = _far_rays(X, m, seed=d)
    dev = torch.device("cuda", 0)
    print(f"fp64-origin rays d={d} n={n} m={m}", flush=True)
    t, idx, st = vg.raycast(torch.from_numpy(X).to(dev), torch.from_numpy(O).to(dev), torch.from_numpy(U).to(dev),
                            torch.from_numpy(g).to(dev), torch.from_numpy(g[:, None].copy()).to(dev), clip=False)
    s = vg.stats()
    print(f"  {s['flagged']} of {m} rays rechecked", flush=True)
    assert s["flagged"] > m // 4
    if m > 4096:
        assert s["flagged"] > 2048  # the tiled split, not the per-ray kernel
    pick = np.sort(np.random.default_rng(1).choice(m, min(m, 400), replace=False))
    tr, ir, t2r = oracle.raycast(X, O[pick], U[pick], g[pick], excl=g[pick, None], clip=False)
    from tests.parity import runner_up_rays
    compare_rays(t.cpu().numpy()[pick], idx.cpu().numpy()[pick], tr, ir, t2r, rtol=1e-5,
                 runner_up=runner_up_rays(X, O[pick], U[pick], g[pick], g[pick, None], False, ir))
