"""The Monte-Carlo cell scan in scan order (nodes sorted along a Morton
curve, each cell scanning outwards from its own place and skipping node
blocks and chunks whose bound on u.r~ is below every ray's second best)
against the scan over every node in index order: the skip is exact, so t*,
the index, the status and the flagged set agree bit for bit; and both agree
with the FP64 oracle."""
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


def _both(vg, X, D=None, precision="fp32", seed=None, R=None):
    out = []
    for order in ("scan", "index"):
        t, idx, st = vg.raycast_cells(X, D, precision=precision, seed=seed, rays_per_cell=R, order=order)
        out.append((t, idx, st, vg.stats()))
    return out


def _assert_same(a, b):
    (t, idx, st, s), (t2, idx2, st2, s2) = a, b
    assert torch.equal(t.view(torch.int32), t2.view(torch.int32))
    assert torch.equal(idx, idx2)
    assert torch.equal(st, st2)
    assert s["flagged"] == s2["flagged"]
    assert s["fp64_ties"] == s2["fp64_ties"]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("d,n,R,kind", [(2, 5000, 64, "uni"), (3, 20000, 256, "uni"), (3, 3001, 100, "gmm"),
                                        (4, 7777, 33, "uni"), (6, 9000, 256, "uni"), (8, 4000, 128, "gmm"),
                                        (10, 6000, 1024, "gmm"), (12, 2500, 64, "uni"), (16, 1500, 96, "gmm"),
                                        # 512 rays per workgroup: four column blocks x four waves up to d=6
                                        (3, 9000, 512, "uni"), (5, 6000, 400, "gmm"), (6, 5000, 512, "uni"),
                                        (8, 3000, 512, "uni")])
def test_scan_order_equals_index_order(vg, d, n, R, kind, precision):
    print(f"scan order d={d} n={n} R={R} {kind} {precision}", flush=True)
    dev = torch.device("cuda", 0)
    X = W.gaussian_mixture_cloud(n=n, d=d, seed=d) if kind == "gmm" else W.uniform_cloud(n, d, seed=d)
    nodes = torch.from_numpy(X).to(dev)
    a, b = _both(vg, nodes, precision=precision, seed=50 + d, R=R)
    _assert_same(a, b)
    pairs = float(n) * R * n
    assert b[3]["scan_pairs"] >= pairs  # index order: every node block for every ray column block
    assert 0 < a[3]["scan_pairs"] <= b[3]["scan_pairs"]
    if d <= 4 and n >= 5000:
        assert a[3]["scan_pairs"] < 0.5 * b[3]["scan_pairs"]  # low d: most blocks provably out of reach


@pytest.mark.parametrize("n", [1, 2, 31, 33, 127, 129, 513, 1025])
def test_scan_order_small_and_ragged_clouds(vg, n):
    dev = torch.device("cuda", 0)
    for d in (2, 5):
        X = W.uniform_cloud(n, d, seed=n + d)
        nodes = torch.from_numpy(X).to(dev)
        D = torch.from_numpy(W.mc_directions(range(n), 40, d, seed=7)).to(dev)
        a, b = _both(vg, nodes, D)
        _assert_same(a, b)
        t_ref, idx_ref, t2_ref = oracle.raycast_cells(X, np.arange(n), W.mc_directions(range(n), 40, d, seed=7))
        compare_rays(a[0].cpu().numpy().ravel(), a[1].cpu().numpy().ravel(), t_ref, idx_ref, t2_ref, rtol=1e-5,
                     runner_up=runner_up_cells(X, np.arange(n), W.mc_directions(range(n), 40, d, seed=7), idx_ref))


def test_scan_order_on_lattice_ties_and_near_duplicates(vg):
    """Exact lattice (many equal candidates: ties flagged, FP64 picks the
    lowest index) and nodes a few ulps apart (tiny nearest-node distance):
    the skip decisions must not change any of it."""
    dev = torch.device("cuda", 0)
    X = W.jittered_lattice(10, 3, jitter=0.0, seed=0)
    X[5] = np.nextafter(X[4], np.float32(1.0))
    n = X.shape[0]
    D = torch.from_numpy(W.mc_directions(range(n), 64, 3, seed=3)).to(dev)
    a, b = _both(vg, torch.from_numpy(X).to(dev), D)
    _assert_same(a, b)
    assert a[3]["flagged"] > 0


def test_scan_order_clustered_cloud_against_oracle(vg):
    """A tightly clustered cloud (the case the order is for): sampled cells
    against the FP64 oracle, and fewer evaluated pairs than nodes x rays."""
    dev = torch.device("cuda", 0)
    d, n, R = 10, 20000, 256
    X = W.gaussian_mixture_cloud(n=n, d=d, seed=4)
    nodes = torch.from_numpy(X).to(dev)
    t, idx, st = vg.raycast_cells(nodes, precision="fp32", seed=9, rays_per_cell=R, order="scan")
    s = vg.stats()
    assert s["scan_pairs"] < 0.9 * float(n) * R * n
    cells = np.sort(np.random.default_rng(2).choice(n, 12, replace=False))
    Dh = W.philox_directions(cells, R, d, seed=9)
    Dd = np.stack([vg.dump_dirs(d, 1, R, 9, first_cell=int(c)).cpu().numpy()[0] for c in cells])
    keep = np.all(Dh == Dd, axis=-1).ravel()
    t_ref, idx_ref, t2_ref = oracle.raycast_cells(X, cells, Dh)
    tt = t.cpu().numpy()[cells].ravel()
    ii = idx.cpu().numpy()[cells].ravel()
    full = runner_up_cells(X, cells, Dh, idx_ref)
    compare_rays(tt[keep], ii[keep], t_ref[keep], idx_ref[keep], t2_ref[keep], rtol=1e-5,
                 runner_up=lambda m: full(_expand(keep, m)))


def _expand(keep, m):
    out = np.zeros(keep.size, dtype=bool)
    out[np.nonzero(keep)[0][m]] = True
    return out


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_scan_order_estimators_equal(vg, precision):
    dev = torch.device("cuda", 0)
    d, n, R = 4, 6000, 128
    X = torch.from_numpy(W.uniform_cloud(n, d, seed=31)).to(dev)
    a = vg.mc_volume_area(X, precision=precision, seed=5, rays_per_cell=R, order="scan")
    b = vg.mc_volume_area(X, precision=precision, seed=5, rays_per_cell=R, order="index")
    for f in ("volume", "energy2", "facet_count", "t", "idx", "status"):
        x, y = getattr(a, f), getattr(b, f)
        assert torch.equal(x.view(torch.int32) if x.dtype == torch.float32 else x,
                           y.view(torch.int32) if y.dtype == torch.float32 else y), f
    valid = torch.arange(R, device=dev)[None, :] < a.facet_count[:, None]
    assert torch.equal(a.facet_j[valid], b.facet_j[valid])
    assert torch.equal(a.facet_area[valid], b.facet_area[valid])


def test_scan_order_batched(vg, tmp_path, monkeypatch):
    """The batched call sorts each cloud of d <= 12 (FP32) in its graph; forced
    index order gives the same bits."""
    monkeypatch.setenv("VG_TUNE_CACHE", str(tmp_path / "tune.txt"))
    dev = torch.device("cuda", 0)
    probs = []
    for c, (d, n, R) in enumerate([(3, 4000, 128), (6, 2500, 64), (10, 1200, 256), (14, 700, 64)]):
        X = torch.from_numpy(W.uniform_cloud(n, d, seed=600 + c)).to(dev)
        D = torch.from_numpy(W.mc_directions(range(n), R, d, seed=700 + c)).to(dev)
        probs.append((X, D))
    a = vg.raycast_cells_batched(probs, order="scan")
    b = vg.raycast_cells_batched(probs, order="index")
    torch.cuda.synchronize()
    for (t, i, s), (t2, i2, s2) in zip(a, b):
        assert torch.equal(t.view(torch.int32), t2.view(torch.int32))
        assert torch.equal(i, i2)
        assert torch.equal(s, s2)


def test_order_flags_exclude_each_other(vg):
    dev = torch.device("cuda", 0)
    X = torch.rand(50, 3, device=dev)
    import ctypes
    flags = vg.VG_SCAN_ORDER | vg.VG_INDEX_ORDER
    t = torch.empty(50 * 8, device=dev)
    i = torch.empty(50 * 8, dtype=torch.int32, device=dev)
    c = vg._ctx(dev)
    rc = vg._lib.vg_raycast_cells_seeded(c, 3, 50, vg._ptr(X), 8, 1, flags, vg._ptr(t), vg._ptr(i), None)
    assert rc == -1  # VG_EINVAL
    with pytest.raises(ValueError):
        vg.raycast_cells(X, seed=1, rays_per_cell=8, order="morton")


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_scan_order_non_unit_directions(vg, precision):
    """The skip bounds hold for unit directions only: a workgroup holding a
    longer direction skips nothing, so scan order still gives the
    index-order bits, both when every ray is scaled and when one is."""
    dev = torch.device("cuda", 0)
    d, n, R = 5, 3000, 64
    X = W.uniform_cloud(n, d, seed=77)
    D = W.mc_directions(range(n), R, d, seed=78)
    nodes = torch.from_numpy(X).to(dev)
    for scale in ("all", "one"):
        Dm = D.copy()
        if scale == "all":
            Dm *= np.float32(3.0)
        else:
            Dm[17, 5] *= np.float32(1.5)
        a, b = _both(vg, nodes, torch.from_numpy(Dm).to(dev), precision=precision)
        _assert_same(a, b)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("d,kind", [(3, "uni"), (5, "uni"), (4, "gmm")])
def test_scan_order_beyond_the_chunk_table(vg, d, kind, precision):
    """More chunks than the LDS table of sorted chunk bounds holds (2048):
    64 rays per cell run 128-node chunks, so N = 300 000 has 2344, and the
    big-cloud kernel shares each table entry among two consecutive chunks
    (keyed by the larger bound, each chunk's own bound checked inside).
    Still the index-order bits."""
    print(f"beyond table d={d} {kind} {precision}", flush=True)
    dev = torch.device("cuda", 0)
    n, R = 300_000, 64
    X = W.gaussian_mixture_cloud(n=n, d=d, seed=90 + d) if kind == "gmm" else W.uniform_cloud(n, d, seed=90 + d)
    X = torch.from_numpy(X).to(dev)
    a, b = _both(vg, X, precision=precision, seed=91, R=R)
    _assert_same(a, b)
    assert a[3]["scan_pairs"] < 0.2 * b[3]["scan_pairs"]


def _random_configs(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        d = int(rng.integers(2, 17))
        n = int(np.exp(rng.uniform(np.log(2), np.log(30000))))
        R = int(rng.choice([1, 7, 33, 64, 100, 256, 512, 1024]))
        R = max(1, min(R, int(1e7 // n)))
        out.append((d, n, R, str(rng.choice(["uni", "gmm"])), str(rng.choice(["fp32", "bf16x3"])),
                    int(rng.integers(1, 1 << 30))))
    return out


@pytest.mark.parametrize("d,n,R,kind,precision,seed", _random_configs(24, 2025))
def test_scan_order_random_configurations(vg, d, n, R, kind, precision, seed):
    """Seeded random shapes (d 2..16, N log-uniform up to 3e4, odd and even
    ray counts, uniform and clustered clouds, both precisions): every skip is
    exact, so scan order gives the index-order bits."""
    print(f"random d={d} n={n} R={R} {kind} {precision}", flush=True)
    dev = torch.device("cuda", 0)
    X = W.gaussian_mixture_cloud(n=n, d=d, seed=seed % 1000) if (kind == "gmm" and n >= 16) \
        else W.uniform_cloud(n, d, seed=seed % 1000)
    a, b = _both(vg, torch.from_numpy(X).to(dev), precision=precision, seed=seed, R=R)
    _assert_same(a, b)
