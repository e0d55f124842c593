"""Uneven batches in one graph launch (one exact single-cloud scan per cloud
on parallel branches, then one batched FP64 recheck): parity with the oracle
and with the single-cloud path in every tile shape, hipGraph replays against
eager launches, and the tuner's cache file."""
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


@pytest.mark.parametrize("shape", [0, 1, 2])
def test_every_tile_shape_equals_the_single_path(vg, batch, shape, monkeypatch):
    """Half, the default and twice the default rays per workgroup: the rays'
    results do not depend on the tile shape."""
    monkeypatch.setenv("VG_BATCH_SHAPE", str(shape))
    for prec in ("fp32", "bf16x3"):
        got = _run(vg, batch, prec)
        for (X, D, Xd, Dd), (t, idx, st) in zip(batch, got):
            t1, i1, s1 = vg.raycast_cells(Xd, Dd, precision=prec)
            assert np.array_equal(i1.cpu().numpy(), idx)
            assert np.array_equal(t1.cpu().numpy().view(np.uint32), t.view(np.uint32))
            assert np.array_equal(s1.cpu().numpy(), st)


def test_tuner_cache_file_format(vg, batch, tmp_path, monkeypatch):
    """One line per (K-steps, log2 N, rays per cell, precision, node order, shape) with a
    positive time per ray-node pair; a second call with the same file probes
    nothing new, so the file is left as it was."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("VG_TUNE_CACHE", str(path))
    _run(vg, batch[:3])
    text = path.read_text()
    rows = [ln.split() for ln in text.splitlines()]
    assert len(rows) >= 3
    for r in rows:
        assert len(r) == 7
        kp, log2n, R, bf16, order, shape = map(int, r[:6])
        assert 1 <= kp <= 8 and log2n >= 0 and 1 <= R <= 4096 and bf16 == 0 and 0 <= shape <= 2
        assert order == (1 if kp <= 6 else 0)  # FP32: scan order for d <= 12 by default
        assert float(r[6]) > 0
    mtime = path.stat().st_mtime_ns
    _run(vg, batch[:3])
    assert path.stat().st_mtime_ns == mtime and path.read_text() == text
