"""GPU parity of the Monte-Carlo estimators (volume, second moment, facet
areas) and of their adjoint against the FP64 oracle."""
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


def _gpu_facets(res, n):
    cnt = res.facet_count.cpu().numpy()
    fj = res.facet_j.cpu().numpy()
    fa = res.facet_area.cpu().numpy()
    out = {}
    for i in range(n):
        for s in range(cnt[i]):
            out[(i, int(fj[i, s]))] = float(fa[i, s])
    return out, cnt, fj


@pytest.mark.parametrize("d,n,R,prec", [(2, 1000, 128, "fp32"), (3, 400, 256, "fp32"),
                                        (4, 500, 512, "fp32"), (6, 300, 100, "fp32"),
                                        (10, 300, 1024, "fp32"), (10, 300, 1024, "bf16x3"),
                                        (16, 120, 64, "fp32"), (2, 500, 1, "fp32"), (3, 300, 16, "fp32"),
                                        (5, 200, 33, "fp32"), (3, 1000, 64, "bf16x3")])
def test_mc_volume_area_match_oracle(vg, d, n, R, prec):
    print(f"mc d={d} n={n} R={R} {prec}", flush=True)
    X = W.uniform_cloud(n, d, seed=d)
    D = W.mc_directions(range(n), R, d, seed=3)
    dev = torch.device("cuda", 0)
    res = vg.mc_volume_area(torch.from_numpy(X).to(dev), torch.from_numpy(D).to(dev), precision=prec)
    torch.cuda.synchronize()
    ref = oracle.mc_volume_area(X, np.arange(n), D)
    idx = res.idx.cpu().numpy()
    compare_rays(res.t.cpu().numpy(), idx, ref["t"], ref["idx"], ref["t2"], rtol=1e-5,
                 runner_up=runner_up_cells(X, np.arange(n), D, ref["idx"]))
    vol = res.volume.cpu().numpy()
    en = res.energy2.cpu().numpy()
    assert np.allclose(vol, ref["volume"], rtol=1e-5, atol=0)
    assert np.allclose(en, ref["energy2"], rtol=1e-5, atol=0)
    got, cnt, fj = _gpu_facets(res, n)
    # every facet, with the oracle's sums taken on the GPU's choice among
    # tied candidates (compare_rays checked it is a correct one)
    adj = oracle.mc_volume_area(X, np.arange(n), D, rays=tie_adjusted(ref["t"], ref["idx"], ref["t2"], idx))
    for key, A in adj["facets"].items():
        assert key in got, f"facet {key} missing"
        assert got[key] == pytest.approx(A, rel=1e-5), key
    assert set(got) == set(adj["facets"]), "extra facets"
    # rows are sorted by j and counts match
    for i in range(0, n, 17):
        row = fj[i, :cnt[i]]
        assert np.all(np.diff(row) > 0)


@pytest.mark.parametrize("d,n,R", [(2, 200, 64), (4, 300, 128), (10, 150, 256)])
def test_backward_matches_oracle_adjoint(vg, d, n, R):
    X = W.uniform_cloud(n, d, seed=50 + d)
    D = W.mc_directions(range(n), R, d, seed=4)
    dev = torch.device("cuda", 0)
    nodes = torch.from_numpy(X).to(dev)
    dirs = torch.from_numpy(D).to(dev)
    res = vg.mc_volume_area(nodes, dirs)
    rng = np.random.default_rng(0)
    gv = rng.standard_normal(n).astype(np.float32)
    ge = rng.standard_normal(n).astype(np.float32)
    _, cnt, fj = _gpu_facets(res, n)
    # a facet's upstream weight is a fixed function of (i, j)
    wfac = lambda i, j: np.sin(0.37 * i + 1.3 * j + 0.1)
    ga = np.zeros((n, R), dtype=np.float32)
    for i in range(n):
        for s in range(cnt[i]):
            ga[i, s] = wfac(i, fj[i, s])
    grad = vg.mc_backward(nodes, dirs, res, torch.from_numpy(gv).to(dev),
                          torch.from_numpy(ge).to(dev), torch.from_numpy(ga).to(dev)).cpu().numpy()
    t = res.t.cpu().numpy().ravel().astype(np.float64)
    idx = res.idx.cpu().numpy().ravel()
    cells = np.repeat(np.arange(n), R)
    ga_ray = np.array([wfac(i, j) for i, j in zip(cells, idx)], dtype=np.float32)
    g_ref = oracle.mc_adjoint(X, np.arange(n), D, t, idx, gv, ge, ga_ray.astype(np.float64))
    err = np.linalg.norm(grad - g_ref) / np.linalg.norm(g_ref)
    assert err < 1e-4, err
    # deterministic
    grad2 = vg.mc_backward(nodes, dirs, res, torch.from_numpy(gv).to(dev),
                           torch.from_numpy(ge).to(dev), torch.from_numpy(ga).to(dev)).cpu().numpy()
    assert np.array_equal(grad.view(np.uint32), grad2.view(np.uint32))


def test_autograd_function_centroidal_energy(vg):
    d, n, R = 4, 400, 256
    X = W.uniform_cloud(n, d, seed=2)
    D = W.mc_directions(range(n), R, d, seed=5)
    dev = torch.device("cuda", 0)
    nodes = torch.from_numpy(X).to(dev).requires_grad_(True)
    dirs = torch.from_numpy(D).to(dev)
    vol, en, area = vg.VoronoiMC.apply(nodes, dirs)
    loss = en.sum()
    loss.backward()
    res = vg.VoronoiMC.last_result
    t = res.t.detach().cpu().numpy().ravel().astype(np.float64)
    idx = res.idx.cpu().numpy().ravel()
    g_ref = oracle.mc_adjoint(X, np.arange(n), D, t, idx, None, np.ones(n), None)
    g = nodes.grad.cpu().numpy()
    assert np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref) < 1e-4


def test_backward_d4_512_rays_full_gradient(vg):
    """The d=4 / 512-rays shape of the differentiation workload at N = 2000,
    small enough for the oracle's closed-form gradient over every ray."""
    d, n, R = 4, 2000, 512
    X = W.uniform_cloud(n, d, seed=0)
    D = W.mc_directions(range(n), R, d, seed=1)
    dev = torch.device("cuda", 0)
    nodes = torch.from_numpy(X).to(dev)
    dirs = torch.from_numpy(D).to(dev)
    res = vg.mc_volume_area(nodes, dirs)
    grad = vg.mc_backward(nodes, dirs, res, None, torch.ones(n, device=dev), None).cpu().numpy()
    ref = oracle.mc_volume_area(X, np.arange(n), D)
    g_ref = oracle.mc_adjoint(X, np.arange(n), D, ref["t"], ref["idx"], None, np.ones(n), None)
    err = np.linalg.norm(grad - g_ref) / np.linalg.norm(g_ref)
    assert err < 1e-4, err
    # the 32 finite-difference generators of the workload, component-wise
    pick = W.fd_generators(n, 32, seed=1)
    scale = np.abs(g_ref).max()
    assert np.allclose(grad[pick], g_ref[pick], rtol=1e-3, atol=1e-4 * scale)
