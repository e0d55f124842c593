"""The allocation-free Monte-Carlo RayCast entry point (vg_raycast_cells_noalloc)
against the allocating one (vg_raycast_cells): same kernels, so the results
must be bitwise equal, on two calls in a row (the second smaller, so that the
fixed scratch still holds the first call's queue and counters) and on a
lattice whose ties fill the FP64 recheck queue."""
import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    import paper_2405_10050_amd as vg
    return vg


def _both(vg, X, D, precision):
    dev = torch.device("cuda", 0)
    nodes = torch.from_numpy(X).to(dev)
    dirs = torch.from_numpy(D).to(dev)
    ref = vg.raycast_cells(nodes, dirs, precision=precision)
    ref_flagged = vg.stats()["flagged"]
    n, R = D.shape[:2]
    out = (torch.full((n, R), -7.0, device=dev), torch.full((n, R), -9, dtype=torch.int32, device=dev),
           torch.full((n, R), 255, dtype=torch.uint8, device=dev))
    got = vg.raycast_cells_noalloc(nodes, dirs, precision=precision, out=out)
    flagged = vg.stats()["flagged"]
    torch.cuda.synchronize()
    return [a.cpu().numpy() for a in ref], [a.cpu().numpy() for a in got], ref_flagged, flagged


def _assert_same(ref, got):
    t0, i0, s0 = ref
    t1, i1, s1 = got
    assert np.array_equal(t0.view(np.uint32), t1.view(np.uint32)), "t differs"
    assert np.array_equal(i0, i1), "idx differs"
    assert np.array_equal(s0, s1), "status differs"


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_noalloc_matches_allocating_call_twice(vg, precision):
    # first call: 1000 lattice cells x 512 rays (ties: a long recheck queue)
    print(f"noalloc lattice d=3 m=10 R=512 {precision}", flush=True)
    X = W.jittered_lattice(10, 3, jitter=0.0, seed=0)
    D = W.mc_directions(range(X.shape[0]), 512, 3, seed=11)
    # the first 26 rays of every cell run along lattice directions: they meet
    # several bisectors (or faces) at once and must go through the recheck
    e = np.stack(np.meshgrid(*[np.arange(-1, 2)] * 3, indexing="ij"), -1).reshape(-1, 3)
    e = e[np.any(e != 0, axis=1)].astype(np.float64)
    D[:, :26] = (e / np.linalg.norm(e, axis=1, keepdims=True)).astype(np.float32)
    ref, got, f_ref, f_got = _both(vg, X, D, precision)
    _assert_same(ref, got)
    assert f_ref == f_got and f_got > 0
    # second call, smaller and of another dimension: the array still holds
    # the first call's queue and counters
    print(f"noalloc uniform d=6 n=300 R=64 {precision}", flush=True)
    X2 = W.uniform_cloud(300, 6, seed=5)
    D2 = W.mc_directions(range(300), 64, 6, seed=12)
    ref2, got2, f_ref2, f_got2 = _both(vg, X2, D2, precision)
    _assert_same(ref2, got2)
    assert f_ref2 == f_got2 < f_got


def test_noalloc_without_status_output(vg):
    dev = torch.device("cuda", 0)
    X = W.uniform_cloud(200, 4, seed=3)
    D = W.mc_directions(range(200), 96, 4, seed=13)
    nodes, dirs = torch.from_numpy(X).to(dev), torch.from_numpy(D).to(dev)
    t0, i0, _ = vg.raycast_cells(nodes, dirs)
    t = torch.empty((200, 96), device=dev)
    i = torch.empty((200, 96), dtype=torch.int32, device=dev)
    vg.raycast_cells_noalloc(nodes, dirs, out=(t, i, None))
    torch.cuda.synchronize()
    assert torch.equal(t0.view(torch.int32), t.view(torch.int32))
    assert torch.equal(i0, i)


def test_noalloc_rejects_oversized_and_incircle_calls(vg):
    import ctypes

    dev = torch.device("cuda", 0)
    nodes = torch.rand((4097, 2), device=dev) * 0.5 + 0.25
    c = vg._ctx(dev)
    # 4097 cells x 1024 rays > 2^22: rejected before any launch (no pointer is read)
    rc = vg._lib.vg_raycast_cells_noalloc(c, 2, 4097, ctypes.c_void_p(nodes.data_ptr()), 1024,
                                          ctypes.c_void_p(nodes.data_ptr()), 0,
                                          ctypes.c_void_p(nodes.data_ptr()), ctypes.c_void_p(nodes.data_ptr()),
                                          None)
    assert rc == -1 and b"VG_NOALLOC_MAX_RAYS" in vg._lib.vg_last_error(c)
    rc = vg._lib.vg_raycast_cells_noalloc(c, 2, 16, ctypes.c_void_p(nodes.data_ptr()), 4,
                                          ctypes.c_void_p(nodes.data_ptr()), vg.VG_INCIRCLE,
                                          ctypes.c_void_p(nodes.data_ptr()), ctypes.c_void_p(nodes.data_ptr()),
                                          None)
    assert rc == -4
