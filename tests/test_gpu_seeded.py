"""Monte-Carlo directions drawn on the device (Philox4x32-10 + Box-Muller,
keyed by (seed, cell, ray)): the dumped directions against the host
implementation of the same generator, the seeded calls against the same calls
on the dumped directions (bit for bit), and the seeded results against the
FP64 oracle run on the host generator's directions."""
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


def _ulps(a, b):
    ia = a.view(np.int32).astype(np.int64)
    ib = b.view(np.int32).astype(np.int64)
    return np.abs(ia - ib)


@pytest.mark.parametrize("d", [2, 3, 4, 5, 8, 10, 13, 16])
def test_dumped_directions_equal_the_host_generator(vg, d):
    """Same published generator on both sides: the words are integers and
    equal; the FP64 Box-Muller may differ in a last FP64 bit between the two
    math libraries, which after rounding to FP32 almost never shows."""
    cells = np.array([0, 1, 77, 12345, 2 ** 31 - 2])
    for c in cells:
        got = vg.dump_dirs(d, 1, 300, seed=0xDEADBEEF12345, first_cell=int(c)).cpu().numpy()[0]
        want = W.philox_directions([c], 300, d, seed=0xDEADBEEF12345)[0]
        u = _ulps(got, want)
        assert u.max() <= 1
        assert np.count_nonzero(u) <= 2, f"cell {c}: {np.count_nonzero(u)} components differ"


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("d,n,R", [(2, 300, 33), (3, 500, 128), (4, 257, 64), (6, 400, 100),
                                   (10, 300, 1024), (12, 200, 96), (16, 150, 64)])
def test_seeded_scan_equals_the_scan_of_the_dumped_directions(vg, d, n, R, precision):
    print(f"seeded d={d} n={n} R={R} {precision}", flush=True)
    dev = torch.device("cuda", 0)
    X = W.uniform_cloud(n, d, seed=500 + d)
    nodes = torch.from_numpy(X).to(dev)
    t, idx, st = vg.raycast_cells(nodes, precision=precision, seed=41 + d, rays_per_cell=R)
    flagged = vg.stats()["flagged"]
    D = vg.dump_dirs(d, n, R, seed=41 + d)
    t2, idx2, st2 = vg.raycast_cells(nodes, D, precision=precision)
    assert vg.stats()["flagged"] == flagged
    assert torch.equal(t.view(torch.int32), t2.view(torch.int32))
    assert torch.equal(idx, idx2)
    assert torch.equal(st, st2)
    # and the oracle on the host generator's directions
    Dh = W.philox_directions(np.arange(n), R, d, seed=41 + d)
    same_dir = np.all(Dh == D.cpu().numpy(), axis=-1).ravel()
    t_ref, idx_ref, t2_ref = oracle.raycast_cells(X, np.arange(n), Dh)
    keep = same_dir  # a direction one FP32 ulp apart is another ray
    compare_rays(t.cpu().numpy().ravel()[keep], idx.cpu().numpy().ravel()[keep], t_ref[keep], idx_ref[keep],
                 t2_ref[keep], rtol=1e-5,
                 runner_up=lambda m: runner_up_cells(X, np.arange(n), Dh, idx_ref)(_expand(keep, m)))
    assert keep.mean() > 0.999


def _expand(keep, m):
    full = np.zeros(keep.size, dtype=bool)
    full[np.nonzero(keep)[0][m]] = True
    return full


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_seeded_estimators_and_adjoint_equal_the_dumped_ones(vg, precision):
    d, n, R = 5, 600, 256
    dev = torch.device("cuda", 0)
    X = W.uniform_cloud(n, d, seed=77)
    nodes = torch.from_numpy(X).to(dev)
    a = vg.mc_volume_area(nodes, precision=precision, seed=2024, rays_per_cell=R)
    D = vg.dump_dirs(d, n, R, seed=2024)
    b = vg.mc_volume_area(nodes, D, precision=precision)
    for f in ("volume", "energy2", "facet_count", "t", "idx", "status"):
        x, y = getattr(a, f), getattr(b, f)
        assert torch.equal(x.view(torch.int32) if x.dtype == torch.float32 else x,
                           y.view(torch.int32) if y.dtype == torch.float32 else y), f
    valid = torch.arange(R, device=dev)[None, :] < a.facet_count[:, None]
    assert torch.equal(a.facet_j[valid], b.facet_j[valid])
    assert torch.equal(a.facet_area[valid], b.facet_area[valid])
    rng = np.random.default_rng(3)
    gv = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to(dev)
    ge = torch.from_numpy(rng.standard_normal(n).astype(np.float32)).to(dev)
    ga = torch.from_numpy(rng.standard_normal((n, R)).astype(np.float32)).to(dev)
    g1 = vg.mc_backward(nodes, None, a, gv, ge, ga)
    g2 = vg.mc_backward(nodes, D, b, gv, ge, ga)
    assert torch.equal(g1, g2)
    # volumes against the oracle on the host generator's directions
    Dh = W.philox_directions(np.arange(n), R, d, seed=2024)
    ref = oracle.mc_volume_area(X, np.arange(n), Dh)
    if np.array_equal(Dh, D.cpu().numpy()):
        assert np.allclose(a.volume.cpu().numpy(), ref["volume"], rtol=1e-5, atol=0)


def test_seeded_autograd_function(vg):
    d, n, R = 3, 300, 128
    dev = torch.device("cuda", 0)
    X = torch.from_numpy(W.uniform_cloud(n, d, seed=78)).to(dev).requires_grad_(True)
    vol, en, fa = vg.VoronoiMC.apply(X, None, "fp32", 7, R)
    en.sum().backward()
    D = vg.dump_dirs(d, n, R, seed=7)
    res = vg.mc_volume_area(X.detach(), D)
    g = vg.mc_backward(X.detach(), D, res, None, torch.ones(n, device=dev), None)
    assert torch.equal(X.grad, g)


def test_seeded_argument_errors(vg):
    dev = torch.device("cuda", 0)
    X = torch.rand(10, 3, device=dev)
    with pytest.raises(ValueError):
        vg.raycast_cells(X, seed=1)  # no rays_per_cell
    with pytest.raises(vg.VGError):
        vg.raycast_cells(X, seed=1, rays_per_cell=4097)
    with pytest.raises(vg.VGError):
        vg.raycast_cells(X, seed=1, rays_per_cell=8, incircle=True)
    with pytest.raises(vg.VGError):
        vg.dump_dirs(17, 1, 8, seed=1)
