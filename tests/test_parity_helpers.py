"""The parity helper itself (CPU, oracle only): on near-tie rays it accepts the
oracle's winner or runner-up and nothing else, and it checks t* there too."""
import numpy as np
import pytest

import oracle
from tests.parity import compare_rays, runner_up_cells, tie_adjusted


def _lattice_case():
    # an exact 2-D lattice with rays along lattice diagonals: many rays hit a
    # vertex shared by two or more bisectors (and corners of the cube)
    m = 5
    g = (np.stack(np.meshgrid(*[np.arange(m)] * 2, indexing="ij"), -1).reshape(-1, 2) + 0.5) / m
    X = g.astype(np.float32)
    n = X.shape[0]
    base = np.array([[1, 1], [1, -1], [-1, 1], [-1, -1], [2, 1], [1, 2]], dtype=np.float64)
    base /= np.linalg.norm(base, axis=1, keepdims=True)
    D = np.broadcast_to(base.astype(np.float32), (n, base.shape[0], 2)).copy()
    t, idx, t2 = oracle.raycast_cells(X, np.arange(n), D)
    return X, D, t, idx, t2


def test_runner_up_is_accepted_on_ties_only():
    X, D, t, idx, t2 = _lattice_case()
    n = X.shape[0]
    tie = oracle.near_tie(t, t2)
    assert tie.sum() > 0
    ru = runner_up_cells(X, np.arange(n), D, idx)
    j2 = ru(tie)
    assert np.all(j2 != idx[tie])
    # the runner-up's own t is the oracle's second-best value
    got = idx.copy()
    got[tie] = j2
    compare_rays(t, got, t, idx, t2, rtol=1e-12, runner_up=ru)
    # without a runner-up the differing tie rays are refused
    with pytest.raises(AssertionError):
        compare_rays(t, got, t, idx, t2, rtol=1e-12)
    # a third candidate on a tie ray is refused
    k = np.nonzero(tie)[0][0]
    bad = idx.copy()
    bad[k] = (max(idx[k], j2[np.nonzero(np.nonzero(tie)[0] == k)[0][0]]) + 7) % n
    with pytest.raises(AssertionError):
        compare_rays(t, bad, t, idx, t2, rtol=1e-12, runner_up=ru)
    # t* is checked on tie rays as well
    tt = t.copy()
    tt[k] *= 1.001
    with pytest.raises(AssertionError):
        compare_rays(tt, idx, t, idx, t2, rtol=1e-5, runner_up=ru)


def test_non_tie_mismatch_is_refused():
    X, D, t, idx, t2 = _lattice_case()
    tie = oracle.near_tie(t, t2)
    k = np.nonzero(~tie & (idx >= 0))[0][0]
    bad = idx.copy()
    bad[k] = (idx[k] + 1) % X.shape[0]
    with pytest.raises(AssertionError):
        compare_rays(t, bad, t, idx, t2, rtol=1e-5, runner_up=runner_up_cells(X, np.arange(X.shape[0]), D, idx))


def test_tie_adjusted_sums_follow_the_chosen_candidate():
    X, D, t, idx, t2 = _lattice_case()
    n = X.shape[0]
    tie = oracle.near_tie(t, t2)
    j2 = runner_up_cells(X, np.arange(n), D, idx)(tie)
    got = idx.copy()
    got[tie] = j2
    adj = oracle.mc_volume_area(X, np.arange(n), D, rays=tie_adjusted(t, idx, t2, got))
    assert np.array_equal(adj["idx"], got)
    ref = oracle.mc_volume_area(X, np.arange(n), D)
    # volumes do not depend on which tied candidate is named
    np.testing.assert_allclose(adj["volume"], ref["volume"], rtol=1e-9)
