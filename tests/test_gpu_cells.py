"""GPU parity of the Monte-Carlo cell RayCast (MFMA scan, FP64 recheck)
against the FP64 oracle, at sizes spanning several tiles and ragged tails."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.parity import compare_rays, runner_up_cells

pytestmark = pytest.mark.gpu

CASES = [
    # d, N, rays per cell
    (2, 1, 33),
    (2, 2, 1),
    (2, 17, 128),
    (3, 300, 64),
    (4, 1000, 256),
    (5, 257, 100),
    (6, 600, 512),
    (7, 129, 40),
    (8, 513, 128),
    (10, 700, 1024),
    (11, 200, 300),
    (12, 400, 64),
    (16, 300, 96),
]


@pytest.fixture(scope="module")
def vg():
    import paper_2405_10050_amd as vg
    return vg


def _run(vg, X, D, precision):
    dev = torch.device("cuda", 0)
    nodes = torch.from_numpy(X).to(dev)
    dirs = torch.from_numpy(D).to(dev)
    t, idx, st = vg.raycast_cells(nodes, dirs, precision=precision)
    torch.cuda.synchronize()
    return t.cpu().numpy().ravel(), idx.cpu().numpy().ravel(), st.cpu().numpy().ravel()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("d,n,R", CASES)
def test_cells_match_oracle(vg, d, n, R, precision):
    print(f"cells d={d} n={n} R={R} {precision}", flush=True)
    X = W.uniform_cloud(n, d, seed=100 + d)
    D = W.mc_directions(range(n), R, d, seed=7)
    t, idx, st = _run(vg, X, D, precision)
    t_ref, idx_ref, t2_ref = oracle.raycast_cells(X, np.arange(n), D)
    excused, worst = compare_rays(t, idx, t_ref, idx_ref, t2_ref, rtol=1e-5,
                                  runner_up=runner_up_cells(X, np.arange(n), D, idx_ref))
    assert excused <= max(2, t.size // 1000)
    if n == 1:
        assert np.all(idx <= -2)


def test_cells_gaussian_mixture_d10(vg):
    """The d=10 Gaussian-mixture workload shape (clustered, with far cells)."""
    X = W.gaussian_mixture_cloud(n=4000, d=10, seed=3)
    cells = np.arange(0, 4000, 97)
    D = W.mc_directions(range(4000), 256, 10, seed=1)
    for prec in ("fp32", "bf16x3"):
        t, idx, st = _run(vg, X, D, prec)
        t = t.reshape(4000, 256)[cells].ravel()
        idx = idx.reshape(4000, 256)[cells].ravel()
        t_ref, idx_ref, t2_ref = oracle.raycast_cells(X, cells, D[cells])
        compare_rays(t, idx, t_ref, idx_ref, t2_ref, rtol=1e-5,
                     runner_up=runner_up_cells(X, cells, D[cells], idx_ref))


def test_cells_lattice_ties_are_flagged(vg):
    """An exact lattice has exactly equal candidates; every such ray must be
    re-evaluated in FP64 and come back with the oracle's lowest-index winner."""
    m = 6
    h = 1.0 / m
    g = (np.stack(np.meshgrid(*[np.arange(m)] * 2, indexing="ij"), -1).reshape(-1, 2) + 0.5) * h
    X = g.astype(np.float32)
    n = X.shape[0]
    # directions along lattice diagonals hit two bisectors and a corner at once
    base = np.array([[1, 1], [1, -1], [-1, 1], [-1, -1], [1, 0], [0, 1], [-1, 0], [0, -1]],
                    dtype=np.float64)
    base /= np.linalg.norm(base, axis=1, keepdims=True)
    D = np.broadcast_to(base.astype(np.float32), (n, 8, 2)).copy()
    t, idx, st = _run(vg, X, D, "fp32")
    t_ref, idx_ref, t2_ref = oracle.raycast_cells(X, np.arange(n), D)
    tie = oracle.near_tie(t_ref, t2_ref)
    assert tie.sum() > 0
    assert np.all(st[tie] & vg.ST_RECHECKED)
    assert np.array_equal(idx, idx_ref)
    assert np.allclose(t, t_ref, rtol=1e-6)


def test_cells_deterministic(vg):
    X = W.uniform_cloud(500, 6, seed=1)
    D = W.mc_directions(range(500), 128, 6, seed=2)
    a = _run(vg, X, D, "fp32")
    b = _run(vg, X, D, "fp32")
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))
