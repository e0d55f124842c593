"""GPU parity of the integrals of a function f over cells and facets
(Algorithm 3 with its inner loop of draws, Sec. 3.1) against the FP64 oracle.

The integrand is the same formula on both sides (numpy for the oracle, torch
for the GPU), evaluated at each side's own sample points; the draws are the
seeded inputs of ``workloads``."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.parity import compare_rays, runner_up_cells, tie_adjusted

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    import paper_2405_10050_amd as vg
    return vg


def _coeffs(d):
    rng = np.random.default_rng(100 + d)
    return rng.standard_normal(d), rng.standard_normal(d)


def _f_np(d):
    a, b = _coeffs(d)
    return lambda p: 1.0 + np.sin(3.0 * (p @ a)) + (p - 0.5) @ b + (p * p).sum(axis=1)


def _f_torch(d, dev):
    a, b = (torch.from_numpy(v).to(dev, torch.float32) for v in _coeffs(d))
    return lambda p: 1.0 + torch.sin(3.0 * (p @ a)) + (p - 0.5) @ b + (p * p).sum(dim=1)


@pytest.mark.parametrize("d,n,R,m", [(2, 500, 128, 4), (3, 300, 256, 3), (4, 200, 512, 2),
                                     (10, 150, 256, 2), (6, 100, 64, 0), (16, 60, 64, 1)])
def test_function_integrals_match_oracle(vg, d, n, R, m):
    print(f"integrals d={d} n={n} R={R} m={m}", flush=True)
    X = W.uniform_cloud(n, d, seed=60 + d)
    D = W.mc_directions(range(n), R, d, seed=8)
    T = W.mc_radial_draws(range(n), R, m, seed=9)
    dev = torch.device("cuda", 0)
    nodes = torch.from_numpy(X).to(dev)
    dirs = torch.from_numpy(D).to(dev)
    res = vg.mc_volume_area(nodes, dirs)
    out = vg.mc_integrals(nodes, dirs, res, _f_torch(d, dev), torch.from_numpy(T).to(dev) if m else None)
    torch.cuda.synchronize()
    ref0 = oracle.mc_volume_area(X, np.arange(n), D)
    idx = res.idx.cpu().numpy()
    compare_rays(res.t.cpu().numpy(), idx, ref0["t"], ref0["idx"], ref0["t2"], rtol=1e-5,
                 runner_up=runner_up_cells(X, np.arange(n), D, ref0["idx"]))
    # the oracle's integrals on the GPU's choice among tied candidates
    ref = oracle.mc_integrals(X, np.arange(n), D, T, _f_np(d),
                              rays=tie_adjusted(ref0["t"], ref0["idx"], ref0["t2"], idx))
    if m:
        assert np.allclose(out.volume.cpu().numpy(), ref["F_V"], rtol=1e-5, atol=1e-6 * np.abs(ref["F_V"]).max())
    else:
        assert out.volume is None
    # the facet rows equal the forward call's (entries past the count are unset)
    assert torch.equal(out.facet_count, res.facet_count)
    valid = torch.arange(R, device=dev)[None, :] < out.facet_count[:, None]
    assert torch.equal(out.facet_j[valid], res.facet_j[valid])
    cnt = out.facet_count.cpu().numpy()
    fj = out.facet_j.cpu().numpy()
    ff = out.facet.cpu().numpy()
    scale = max(abs(v) for v in ref["F"].values())
    got = {(i, int(fj[i, s])): float(ff[i, s]) for i in range(n) for s in range(cnt[i])}
    assert set(got) == set(ref["F"])
    for key, v in ref["F"].items():
        assert got[key] == pytest.approx(v, rel=1e-5, abs=1e-6 * scale), key


def test_constant_integrand_gives_the_areas(vg):
    d, n, R = 3, 200, 256
    X = W.uniform_cloud(n, d, seed=3)
    D = W.mc_directions(range(n), R, d, seed=4)
    dev = torch.device("cuda", 0)
    nodes = torch.from_numpy(X).to(dev)
    dirs = torch.from_numpy(D).to(dev)
    res = vg.mc_volume_area(nodes, dirs)
    T = torch.ones((n, R, 2), device=dev)
    out = vg.mc_integrals(nodes, dirs, res, lambda p: torch.ones(p.shape[0], device=p.device), T)
    # f = 1: facet integrals are the areas; t = 1: the volume integral is d times the volume
    valid = torch.arange(R, device=dev)[None, :] < res.facet_count[:, None]
    assert torch.equal(out.facet_count, res.facet_count)
    assert torch.equal(out.facet_j[valid], res.facet_j[valid])
    assert torch.allclose(out.facet[valid], res.facet_area[valid], rtol=1e-6, atol=0)
    assert torch.allclose(out.volume, d * res.volume, rtol=2e-6, atol=0)
