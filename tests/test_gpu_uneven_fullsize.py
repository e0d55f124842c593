"""Parity at the full size of the uneven batch, in the launch configuration
the benchmark times: 64 uniform clouds (d in {3, 4, 6, 8, 12, 16}, N
log-uniform in [1e3, 2e5], 256 rays per cell, 7.8e8 rays) in one batched,
graph-captured call; two seeded cells of every cloud against the FP64
oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.parity import compare_rays, runner_up_cells

pytestmark = pytest.mark.gpu


def test_uneven64_full_size_sampled_cells(tmp_path, monkeypatch):
    import paper_2405_10050_amd as vg

    monkeypatch.setenv("VG_TUNE_CACHE", str(tmp_path / "tune.txt"))
    dev = torch.device("cuda", 0)
    spec = W.uneven_batch_spec(64, seed=0)
    R = 256
    probs, host = [], []
    for c, (dc, nc, sc) in enumerate(spec):
        X = W.uniform_cloud(nc, dc, seed=sc)
        probs.append((torch.from_numpy(X).to(dev), W.mc_directions_device(nc, R, dc, seed=5000 + c, device=dev)))
        host.append(X)
    print(f"uneven64: {sum(nc for _, nc, _ in spec)} cells ready", flush=True)
    outs = vg.raycast_cells_batched(probs)
    torch.cuda.synchronize()
    print(f"uneven64: batched call done, {vg.stats()['flagged']} rays rechecked", flush=True)
    rng = np.random.default_rng(11)
    for c, ((dc, nc, _), X, (_, D), (t, idx, _)) in enumerate(zip(spec, host, probs, outs)):
        cells = np.sort(rng.choice(nc, 2, replace=False))
        Dc = D[torch.from_numpy(cells).to(dev)].cpu().numpy()
        tr, ir, t2r = oracle.raycast_cells(X, cells, Dc)
        sel = torch.from_numpy(cells).to(dev)
        compare_rays(t[sel].cpu().numpy().ravel(), idx[sel].cpu().numpy().ravel(), tr, ir, t2r, rtol=1e-5,
                     runner_up=runner_up_cells(X, cells, Dc, ir))
    print("uneven64: 128 sampled cells match the oracle", flush=True)
