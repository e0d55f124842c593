"""Edge cases of the boundary on the GPU: the largest ray count per cell,
empty batches, duplicate generators (the method's degenerate input), nodes
outside the unit cube under the grid index, and sizes past the limits."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.parity import compare_rays, runner_up_cells, runner_up_rays

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    import paper_2405_10050_amd as vg
    return vg


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_largest_ray_count_per_cell(vg, precision):
    d, n, R = 3, 40, 4096
    X = W.uniform_cloud(n, d, seed=31)
    D = W.mc_directions(range(n), R, d, seed=32)
    dev = torch.device("cuda", 0)
    t, idx, _ = vg.raycast_cells(torch.from_numpy(X).to(dev), torch.from_numpy(D).to(dev), precision=precision)
    t_ref, idx_ref, t2_ref = oracle.raycast_cells(X, np.arange(n), D)
    compare_rays(t.cpu().numpy(), idx.cpu().numpy(), t_ref, idx_ref, t2_ref, rtol=1e-5,
                 runner_up=runner_up_cells(X, np.arange(n), D, idx_ref))


def test_ray_count_past_the_limit_is_rejected(vg):
    dev = torch.device("cuda", 0)
    X = torch.rand(8, 2, device=dev)
    D = torch.nn.functional.normalize(torch.randn(8, 4097, 2, device=dev), dim=2)
    with pytest.raises(vg.VGError):
        vg.raycast_cells(X, D)


def test_empty_ray_batch(vg):
    dev = torch.device("cuda", 0)
    X = torch.rand(10, 3, device=dev)
    empty = torch.empty((0, 3), device=dev)
    g = torch.empty(0, dtype=torch.int32, device=dev)
    for incircle in (False, True):
        t, idx, st = vg.raycast(X, empty, empty, g, incircle=incircle)
        assert t.numel() == 0 and idx.numel() == 0 and st.numel() == 0


@pytest.mark.parametrize("mode", ["fp32", "bf16x3", "incircle"])
def test_duplicate_generators_match_oracle(vg, mode):
    """Two generators at the same point: neither is ever eligible from the
    other (u.(x_j - x_i) = 0), on both sides; their rays are still settled."""
    d, n, R = 2, 60, 128
    X = W.uniform_cloud(n, d, seed=33)
    X[8] = X[7]
    X[30] = X[29]
    D = W.mc_directions(range(n), R, d, seed=34)
    dev = torch.device("cuda", 0)
    nodes, dirs = torch.from_numpy(X).to(dev), torch.from_numpy(D).to(dev)
    if mode == "incircle":
        t, idx, _ = vg.raycast_cells(nodes, dirs, incircle=True)
    else:
        t, idx, _ = vg.raycast_cells(nodes, dirs, precision=mode)
    t_ref, idx_ref, t2_ref = oracle.raycast_cells(X, np.arange(n), D)
    compare_rays(t.cpu().numpy(), idx.cpu().numpy(), t_ref, idx_ref, t2_ref, rtol=1e-5,
                 runner_up=runner_up_cells(X, np.arange(n), D, idx_ref))


@pytest.mark.parametrize("heuristic", [False, True])
def test_incircle_with_nodes_outside_the_cube_defers_to_fp64(vg, heuristic):
    """The grid covers [0,1]^d; with a node outside it the ring bound does not
    hold, so every ray is settled by the FP64 recheck, and results stay
    those of the definition."""
    d, n, m = 3, 300, 2000
    rng = np.random.default_rng(35)
    X = (rng.random((n, d)) * 1.6 - 0.3).astype(np.float32)
    g = rng.integers(n, size=m).astype(np.int32)
    U = rng.standard_normal((m, d))
    U = (U / np.linalg.norm(U, axis=1, keepdims=True)).astype(np.float32)
    O = X[g]
    dev = torch.device("cuda", 0)
    t, idx, st = vg.raycast(torch.from_numpy(X).to(dev), torch.from_numpy(O).to(dev), torch.from_numpy(U).to(dev),
                            torch.from_numpy(g).to(dev), torch.from_numpy(g[:, None].copy()).to(dev), clip=False,
                            incircle=True, heuristic=heuristic)
    assert vg.stats()["flagged"] == m
    t_ref, idx_ref, t2_ref = oracle.raycast(X, O, U, g, excl=g[:, None], clip=False)
    compare_rays(t.cpu().numpy(), idx.cpu().numpy(), t_ref, idx_ref, t2_ref, rtol=1e-5,
                 runner_up=runner_up_rays(X, O, U, g, g[:, None], False, idx_ref))


def test_wide_recheck_general_rays_match_oracle(vg):
    """N = 300 000 (the FP64 recheck then takes one workgroup per queued ray):
    nodes outside the cube send every incircle ray to it."""
    d, n, m = 3, 300_000, 2000
    rng = np.random.default_rng(36)
    X = (rng.random((n, d)) * 1.2 - 0.1).astype(np.float32)
    g = rng.integers(n, size=m).astype(np.int32)
    U = rng.standard_normal((m, d))
    U = (U / np.linalg.norm(U, axis=1, keepdims=True)).astype(np.float32)
    O = X[g]
    dev = torch.device("cuda", 0)
    t, idx, st = vg.raycast(torch.from_numpy(X).to(dev), torch.from_numpy(O).to(dev), torch.from_numpy(U).to(dev),
                            torch.from_numpy(g).to(dev), torch.from_numpy(g[:, None].copy()).to(dev), clip=True,
                            incircle=True)
    assert vg.stats()["flagged"] == m
    t_ref, idx_ref, t2_ref = oracle.raycast(X, O, U, g, excl=g[:, None], clip=True)
    compare_rays(t.cpu().numpy(), idx.cpu().numpy(), t_ref, idx_ref, t2_ref, rtol=1e-5,
                 runner_up=runner_up_rays(X, O, U, g, g[:, None], True, idx_ref))


def test_wide_recheck_cells_match_oracle(vg):
    """The Monte-Carlo rays of N = 300 000 cells: the cells holding rays the
    FP32 scan flagged (settled by the wide FP64 recheck) against the oracle."""
    d, n, R = 3, 300_000, 8
    X = W.uniform_cloud(n, d, seed=37)
    dev = torch.device("cuda", 0)
    dirs = W.mc_directions_device(n, R, d, seed=38, device=dev)
    t, idx, st = vg.raycast_cells(torch.from_numpy(X).to(dev), dirs)
    rechecked = ((st & vg.ST_RECHECKED) != 0).any(dim=1).nonzero().flatten().cpu().numpy()
    assert rechecked.size > 0
    cells = rechecked[:200]
    D = dirs[torch.from_numpy(cells).to(dev)].cpu().numpy()
    t_ref, idx_ref, t2_ref = oracle.raycast_cells(X, cells, D)
    sel = torch.from_numpy(cells).to(dev)
    compare_rays(t[sel].cpu().numpy(), idx[sel].cpu().numpy(), t_ref, idx_ref, t2_ref, rtol=1e-5,
                 runner_up=runner_up_cells(X, cells, D, idx_ref))
