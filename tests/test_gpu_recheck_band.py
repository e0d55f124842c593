"""The targeted FP64 recheck of Monte-Carlo rays (an FP32 pass keeps the
candidates that can still win, only those are evaluated in FP64) against the
full FP64 pass over every node: the same t*, index and status on every ray,
bit for bit, including lattices whose ties overflow the kept list, and
against the oracle."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.parity import compare_rays, runner_up_cells

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    import paper_2405_10050_amd as vg
    return vg


def _both(vg, nodes, dirs, precision, monkeypatch):
    t, idx, st = vg.raycast_cells(nodes, dirs, precision=precision)
    s = vg.stats()
    monkeypatch.setenv("VG_FULL_RECHECK", "1")
    t2, idx2, st2 = vg.raycast_cells(nodes, dirs, precision=precision)
    s2 = vg.stats()
    monkeypatch.delenv("VG_FULL_RECHECK")
    return (t, idx, st, s), (t2, idx2, st2, s2)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("d,n,R", [(2, 3000, 128), (3, 2000, 256), (5, 1000, 128), (8, 1500, 128),
                                   (10, 2000, 256), (13, 500, 64), (16, 800, 64)])
def test_band_recheck_equals_full_recheck(vg, d, n, R, precision, monkeypatch):
    print(f"band recheck d={d} n={n} R={R} {precision}", flush=True)
    dev = torch.device("cuda", 0)
    X = W.gaussian_mixture_cloud(n=n, d=d, seed=d) if d >= 8 else W.uniform_cloud(n, d, seed=d)
    nodes = torch.from_numpy(X).to(dev)
    dirs = torch.from_numpy(W.mc_directions(range(n), R, d, seed=90 + d)).to(dev)
    (t, idx, st, s), (t2, idx2, st2, s2) = _both(vg, nodes, dirs, precision, monkeypatch)
    assert s["flagged"] == s2["flagged"] and s["flagged"] > 0
    assert s["fp64_ties"] == s2["fp64_ties"]
    assert torch.equal(t.view(torch.int32), t2.view(torch.int32))
    assert torch.equal(idx, idx2)
    assert torch.equal(st, st2)


@pytest.mark.parametrize("d,m", [(2, 12), (3, 8)])
def test_band_recheck_on_lattice_ties(vg, d, m, monkeypatch):
    """An exact lattice with rays along lattice directions: many rays meet
    several bisectors at once (the kept list overflows on some lanes and
    the ray falls back to the full pass); results equal the full recheck and
    the oracle (lowest index on FP64 ties)."""
    dev = torch.device("cuda", 0)
    X = W.jittered_lattice(m, d, jitter=0.0, seed=0)
    n = X.shape[0]
    e = np.stack(np.meshgrid(*[np.arange(-1, 2)] * d, indexing="ij"), -1).reshape(-1, d)
    e = e[np.any(e != 0, axis=1)].astype(np.float64)
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    D = W.mc_directions(range(n), 64, d, seed=5)
    D[:, :e.shape[0]] = e.astype(np.float32)
    nodes, dirs = torch.from_numpy(X).to(dev), torch.from_numpy(D).to(dev)
    (t, idx, st, s), (t2, idx2, st2, s2) = _both(vg, nodes, dirs, "fp32", monkeypatch)
    assert torch.equal(t.view(torch.int32), t2.view(torch.int32))
    assert torch.equal(idx, idx2)
    assert torch.equal(st, st2)
    assert s["flagged"] > 0
    t_ref, idx_ref, t2_ref = oracle.raycast_cells(X, np.arange(n), D)
    compare_rays(t.cpu().numpy(), idx.cpu().numpy(), t_ref, idx_ref, t2_ref, rtol=1e-5,
                 runner_up=runner_up_cells(X, np.arange(n), D, idx_ref))


def test_band_recheck_with_near_duplicate_nodes(vg, monkeypatch):
    """Nodes a few ulps from a generator: their u.e is at the level of its
    rounding, so the FP32 pass must keep them (or fall back); results equal
    the full recheck."""
    dev = torch.device("cuda", 0)
    d, n, R = 3, 400, 128
    X = W.uniform_cloud(n, d, seed=11)
    for i in range(0, 40, 2):
        X[i + 1] = np.nextafter(X[i], np.float32(1.0))
    nodes = torch.from_numpy(X).to(dev)
    dirs = torch.from_numpy(W.mc_directions(range(n), R, d, seed=12)).to(dev)
    (t, idx, st, s), (t2, idx2, st2, s2) = _both(vg, nodes, dirs, "fp32", monkeypatch)
    assert torch.equal(t.view(torch.int32), t2.view(torch.int32))
    assert torch.equal(idx, idx2)
    assert torch.equal(st, st2)
