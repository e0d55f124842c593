"""Comparison helpers for GPU-vs-oracle parity (used by the gpu tests).

Rays whose oracle gap (t2 - t1)/t1 is below 1e-9 are near-ties: several
answers are correct there (Sec. 2.2 assumes general position).  On every ray,
near-tie or not, t* must be within the tolerance of the oracle's (the tied
candidates' t agree to 1e-9).  The index must equal the oracle's, except on
a near-tie ray, where it may also be the oracle's runner-up: the winner of
the same RayCast run again by the oracle with the winner excluded (node
winners) or without the cube (face winners)."""
import numpy as np

import oracle


def runner_up_cells(X, cells, D, idx_ref):
    """Callable mask -> oracle runner-up index of the masked Monte-Carlo rays
    (ray k of listed cell c starts at x_{cells[c]}, direction D[c][k])."""
    X = np.asarray(X)
    cells = np.asarray(cells, dtype=np.int64).ravel()
    d = X.shape[1]
    U = np.asarray(D).reshape(-1, d)
    R = U.shape[0] // cells.size
    idx_ref = np.asarray(idx_ref).ravel()

    def f(mask):
        k = np.nonzero(mask)[0]
        cell = cells[k // R].astype(np.int32)
        return _runner_up(X, X[cell], U[k], cell, cell[:, None], True, idx_ref[k])

    return f


def runner_up_rays(X, origin, direction, gen, excl, clip, idx_ref):
    """Callable mask -> oracle runner-up index of the masked general rays
    (the arguments of oracle.raycast)."""
    X = np.asarray(X)
    d = X.shape[1]
    O = np.asarray(origin).reshape(-1, d)
    U = np.asarray(direction).reshape(-1, d)
    g = np.asarray(gen, dtype=np.int32).ravel()
    E = None if excl is None else np.asarray(excl, dtype=np.int32).reshape(O.shape[0], -1)
    idx_ref = np.asarray(idx_ref).ravel()

    def f(mask):
        k = np.nonzero(mask)[0]
        e = E[k] if E is not None else np.zeros((k.size, 0), dtype=np.int32)
        return _runner_up(X, O[k], U[k], g[k], e, clip, idx_ref[k])

    return f


def _runner_up(X, O, U, g, E, clip, win):
    out = np.full(win.size, -1, dtype=np.int32)
    node = win >= 0
    if node.any():
        ex = np.sort(np.concatenate([E[node], win[node][:, None]], axis=1), axis=1)
        _, j, _ = oracle.raycast(X, O[node], U[node], g[node], ex, clip=clip)
        out[node] = j
    if (~node).any():
        # a face (or no hit) won: the best node without the cube
        e = E[~node] if E.shape[1] else None
        _, j, _ = oracle.raycast(X, O[~node], U[~node], g[~node], e, clip=False)
        out[~node] = j
    return out


def compare_rays(t_gpu, idx_gpu, t_ref, idx_ref, t2_ref, rtol=1e-5, runner_up=None):
    """Index equal to the oracle's on every ray except near-ties, where it may
    be the oracle's winner or runner-up (``runner_up``: a callable as returned
    by runner_up_cells / runner_up_rays, required when a near-tie ray's index
    differs); t* within ``rtol`` relative on every ray with a hit; no-hit rays
    give t = inf.  Returns the number of near-tie rays and the largest
    relative t error."""
    t_gpu = np.asarray(t_gpu, dtype=np.float64).ravel()
    idx_gpu = np.asarray(idx_gpu).ravel()
    idx_ref = np.asarray(idx_ref).ravel()
    t_ref = np.asarray(t_ref).ravel()
    tie = oracle.near_tie(t_ref, np.asarray(t2_ref).ravel())
    diff = idx_gpu != idx_ref
    bad = diff & ~tie
    assert not bad.any(), (
        f"{int(bad.sum())} argmin mismatches, first at ray {int(np.nonzero(bad)[0][0])}: "
        f"gpu {idx_gpu[bad][:5]} oracle {idx_ref[bad][:5]}")
    other = diff & tie
    if other.any():
        assert runner_up is not None, (
            f"{int(other.sum())} near-tie rays differ from the oracle's winner and no runner-up was given")
        j2 = runner_up(other)
        wrong = idx_gpu[other] != j2
        assert not wrong.any(), (
            f"{int(wrong.sum())} near-tie rays are neither the oracle's winner nor its runner-up: "
            f"gpu {idx_gpu[other][wrong][:5]} winner {idx_ref[other][wrong][:5]} runner-up {j2[wrong][:5]}")
    ok = np.isfinite(t_ref)
    rel = np.abs(t_gpu[ok] - t_ref[ok]) / np.abs(t_ref[ok])
    worst = float(rel.max()) if rel.size else 0.0
    assert worst <= rtol, f"t* relative error {worst:.3e} > {rtol:.1e}"
    assert np.all(~np.isfinite(t_gpu[~ok])), "no-hit rays must report t = inf"
    return int(tie.sum()), worst


def tie_adjusted(t_ref, idx_ref, t2_ref, idx_gpu):
    """The oracle's per-ray results with each near-tie ray's index replaced by
    the GPU's (after compare_rays has checked it is a correct answer), for
    recomputing the oracle's Monte-Carlo sums on the GPU's assignment."""
    idx = np.asarray(idx_ref, dtype=np.int32).ravel().copy()
    tie = oracle.near_tie(np.asarray(t_ref).ravel(), np.asarray(t2_ref).ravel())
    g = np.asarray(idx_gpu).ravel()
    idx[tie] = g[tie]
    return np.asarray(t_ref, dtype=np.float64).ravel(), idx, np.asarray(t2_ref).ravel()
