"""Comparison helpers for GPU-vs-oracle parity (used by the gpu tests)."""
import numpy as np

import oracle


def compare_rays(t_gpu, idx_gpu, t_ref, idx_ref, t2_ref, rtol=1e-5):
    """Argmin bit-exact except on oracle near-ties (several answers are
    correct there); t* within ``rtol`` relative on the others.  Returns the
    number of excused rays and the largest relative t error."""
    t_gpu = np.asarray(t_gpu, dtype=np.float64).ravel()
    idx_gpu = np.asarray(idx_gpu).ravel()
    tie = oracle.near_tie(t_ref, t2_ref)
    bad = (idx_gpu != idx_ref) & ~tie
    assert not bad.any(), (
        f"{int(bad.sum())} argmin mismatches, first at ray {int(np.nonzero(bad)[0][0])}: "
        f"gpu {idx_gpu[bad][:5]} oracle {idx_ref[bad][:5]}")
    ok = ~tie & np.isfinite(t_ref)
    rel = np.abs(t_gpu[ok] - t_ref[ok]) / np.abs(t_ref[ok])
    worst = float(rel.max()) if rel.size else 0.0
    assert worst <= rtol, f"t* relative error {worst:.3e} > {rtol:.1e}"
    inf_ref = ~np.isfinite(t_ref)
    assert np.all(~np.isfinite(t_gpu[inf_ref])), "no-hit rays must report t = inf"
    return int(tie.sum()), worst
