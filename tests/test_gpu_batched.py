"""Uneven batches in one persistent launch: parity with the oracle and with
the single-cloud path, hipGraph replays against eager launches, and the
tuner's cache file."""
import os

import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.parity import compare_rays, runner_up_cells

pytestmark = pytest.mark.gpu

SPEC = [(3, 1500, 256), (4, 700, 100), (6, 2000, 256), (8, 900, 64), (12, 1200, 256),
        (16, 400, 300), (2, 257, 33), (10, 3000, 256)]


@pytest.fixture(scope="module")
def vg():
    import paper_2405_10050_amd as vg
    return vg


@pytest.fixture(scope="module")
def batch():
    dev = torch.device("cuda", 0)
    clouds = []
    for c, (d, n, R) in enumerate(SPEC):
        X = W.uniform_cloud(n, d, seed=200 + c)
        D = W.mc_directions(range(n), R, d, seed=300 + c)
        clouds.append((X, D, torch.from_numpy(X).to(dev), torch.from_numpy(D).to(dev)))
    return clouds


def _run(vg, batch, prec="fp32"):
    outs = vg.raycast_cells_batched([(c[2], c[3]) for c in batch], precision=prec)
    torch.cuda.synchronize()
    return [(t.cpu().numpy(), i.cpu().numpy(), s.cpu().numpy()) for t, i, s in outs]


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_batched_matches_oracle_and_single_path(vg, batch, prec, tmp_path, monkeypatch):
    monkeypatch.setenv("VG_TUNE_CACHE", str(tmp_path / "tune.txt"))
    got = _run(vg, batch, prec)
    assert (tmp_path / "tune.txt").exists()
    rng = np.random.default_rng(5)
    for (X, D, Xd, Dd), (t, idx, st) in zip(batch, got):
        n = X.shape[0]
        cells = np.sort(rng.choice(n, min(n, 40), replace=False))
        tr, ir, t2r = oracle.raycast_cells(X, cells, D[cells])
        compare_rays(t[cells].ravel(), idx[cells].ravel(), tr, ir, t2r, rtol=1e-5,
                     runner_up=runner_up_cells(X, cells, D[cells], ir))
        t1, i1, s1 = vg.raycast_cells(Xd, Dd, precision=prec)
        assert np.array_equal(i1.cpu().numpy(), idx)
        assert np.array_equal(t1.cpu().numpy().view(np.uint32), t.view(np.uint32))


def test_graph_replays_match_eager(vg, batch, monkeypatch):
    monkeypatch.setenv("VG_NO_GRAPH", "1")
    eager = _run(vg, batch)
    monkeypatch.delenv("VG_NO_GRAPH")
    probs = [(c[2], c[3]) for c in batch]
    outs = vg.raycast_cells_batched(probs)  # capture + first launch
    for rep in range(3):
        # eager work of the program between replays
        for t, i, s in outs:
            t.zero_()
            i.fill_(-7)
        torch.cuda.synchronize()
        outs2 = vg.raycast_cells_batched(probs, out=outs)  # replay into the same buffers
        torch.cuda.synchronize()
        for (t, i, s), (te, ie, se) in zip(outs2, eager):
            assert np.array_equal(i.cpu().numpy(), ie), rep
            assert np.array_equal(t.cpu().numpy().view(np.uint32), te.view(np.uint32)), rep
            assert np.array_equal(s.cpu().numpy(), se), rep
