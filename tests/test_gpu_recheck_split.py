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
