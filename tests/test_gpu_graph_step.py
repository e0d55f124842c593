"""The Monte-Carlo step (seeded forward estimators + adjoint) captured into a
hipGraph, as the benchmark times it: every replay, with other eager work and
synchronisations in between, reproduces the eager step bit for bit."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_captured_step_replays_match_eager(precision):
    import paper_2405_10050_amd as vg

    d, n, R = 6, 3000, 256
    dev = torch.device("cuda", 0)
    nodes = torch.from_numpy(W.uniform_cloud(n, d, seed=21)).to(dev)
    other = torch.from_numpy(W.uniform_cloud(500, 4, seed=22)).to(dev)
    gv, ge = torch.ones(n, device=dev), torch.ones(n, device=dev)
    ga = torch.ones((n, R), device=dev)
    grad = torch.empty((n, d), device=dev)
    stream = torch.cuda.Stream(dev)
    with torch.cuda.stream(stream):
        res = vg.mc_volume_area(nodes, precision=precision, seed=5, rays_per_cell=R)

        def step():
            vg.mc_volume_area(nodes, precision=precision, seed=5, rays_per_cell=R, out=res)
            vg.mc_backward(nodes, None, res, gv, ge, ga, out=grad)

        step()
        torch.cuda.synchronize()
        want = [x.clone() for x in (res.t, res.idx, res.status, res.volume, res.energy2, res.facet_count, grad)]
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            step()
        for rep in range(3):
            # scribble over the outputs and run other library work between replays
            for x in (res.t, res.volume, grad):
                x.fill_(-1.0)
            res.idx.fill_(-7)
            vg.raycast_cells(other, seed=rep, rays_per_cell=64)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            got = (res.t, res.idx, res.status, res.volume, res.energy2, res.facet_count, grad)
            for a, b in zip(want, got):
                assert torch.equal(a.view(torch.int32) if a.is_floating_point() else a,
                                   b.view(torch.int32) if b.is_floating_point() else b), f"replay {rep}"
