"""GPU parity of vg_raycast_batched: an uneven batch of RayCast problems
(different d, node sets, ray counts and eta sizes, one problem without rays)
in one persistent launch.  Every problem is compared with the FP64 oracle and
bit for bit with the single-problem vg_raycast; a replay of the captured
graph (same buffers, eager work in between) must reproduce the first call."""
import numpy as np
import pytest
import torch

import oracle
import workloads as W
from tests.parity import compare_rays, runner_up_rays

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vg():
    import paper_2405_10050_amd as vg
    return vg


def _edge_problem(d, n, count, seed):
    """Edge rays of the oracle's Voronoi vertices: origin = vertex (rounded to
    FP32), eta = the edge's d generators, direction = SearchDirection."""
    X = W.uniform_cloud(n, d, seed=seed)
    mesh = oracle.explore(X, W.descent_draws(d))
    rng = np.random.default_rng(seed)
    pick = rng.choice(mesh["sigma"].shape[0], min(count, mesh["sigma"].shape[0]), replace=False)
    O, U, E = [], [], []
    for v in pick:
        sig = mesh["sigma"][v]
        o = rng.integers(d + 1)
        eta = np.delete(sig, o)
        O.append(mesh["coord"][v])
        U.append(oracle.search_direction(X, eta, sig[o]))
        E.append(eta)
    E = np.array(E, dtype=np.int32)
    return X, np.array(O).astype(np.float32), np.array(U).astype(np.float32), E[:, 0].copy(), E


def _generator_problem(d, n, m, seed):
    """Rays from generators in random directions, eta = {g}."""
    X = W.uniform_cloud(n, d, seed=seed)
    rng = np.random.default_rng(seed + 1)
    g = rng.integers(n, size=m).astype(np.int32)
    U = rng.standard_normal((m, d))
    U = (U / np.linalg.norm(U, axis=1, keepdims=True)).astype(np.float32) if m else \
        np.zeros((0, d), np.float32)
    return X, X[g].copy(), U, g, g[:, None].copy()


def _batch():
    return [
        _edge_problem(2, 500, 700, 1),
        _generator_problem(4, 3000, 20000, 2),
        _edge_problem(6, 200, 900, 3),
        _generator_problem(9, 120, 0, 4),       # no rays
        _generator_problem(16, 257, 1000, 5),
        _edge_problem(3, 400, 513, 6),           # ragged tile
        _generator_problem(5, 2000, 777, 7),
    ]


def _to_dev(problems, dev):
    out = []
    for X, O, U, g, E in problems:
        out.append(tuple(torch.from_numpy(np.ascontiguousarray(a)).to(dev) for a in (X, O, U, g, E)))
    return out


@pytest.mark.parametrize("clip", [True, False])
def test_batch_matches_oracle_and_single_calls(vg, clip):
    print(f"raycast_batched clip={clip}", flush=True)
    dev = torch.device("cuda", 0)
    host = _batch()
    problems = _to_dev(host, dev)
    res = vg.raycast_batched(problems, clip=clip)
    torch.cuda.synchronize()
    for q, ((X, O, U, g, E), (t, idx, st)) in enumerate(zip(host, res)):
        assert t.shape == (O.shape[0],)
        if O.shape[0] == 0:
            continue
        t_ref, idx_ref, t2_ref = oracle.raycast(X, O, U, g, excl=E, clip=clip)
        compare_rays(t.cpu().numpy(), idx.cpu().numpy(), t_ref, idx_ref, t2_ref, rtol=1e-5,
                     runner_up=runner_up_rays(X, O, U, g, E, clip, idx_ref))
        t1, i1, s1 = vg.raycast(*problems[q][:4], problems[q][4], clip=clip)
        assert torch.equal(t, t1) and torch.equal(idx, i1) and torch.equal(st, s1), f"problem {q}"


def test_graph_replays_reproduce_the_first_call(vg):
    dev = torch.device("cuda", 0)
    problems = _to_dev(_batch(), dev)
    res = vg.raycast_batched(problems, clip=True)
    torch.cuda.synchronize()
    first = [(t.clone(), i.clone(), s.clone()) for t, i, s in res]
    for rep in range(3):
        for t, i, s in res:  # scribble over the outputs between replays
            t.fill_(-1.0)
            i.fill_(-7)
            s.zero_()
        torch.cuda.synchronize()
        res = vg.raycast_batched(problems, clip=True, out=res)
        torch.cuda.synchronize()
        for q, ((t, i, s), (t0, i0, s0)) in enumerate(zip(res, first)):
            assert torch.equal(t, t0) and torch.equal(i, i0) and torch.equal(s, s0), (rep, q)


def test_batched_argument_errors(vg):
    dev = torch.device("cuda", 0)
    X = torch.rand(10, 17, device=dev)
    O = torch.rand(4, 17, device=dev)
    g = torch.zeros(4, dtype=torch.int32, device=dev)
    with pytest.raises(vg.VGError):
        vg.raycast_batched([(X, O, O, g, None)])  # d = 17 > VG_MAX_DIM
    X = torch.rand(10, 3, device=dev)
    O = torch.rand(4, 3, device=dev)
    E = torch.zeros((4, 4), dtype=torch.int32, device=dev)
    with pytest.raises(vg.VGError):
        vg.raycast_batched([(X, O, O, g, E)])  # n_excl = 4 > d
    assert vg.raycast_batched([]) == []
