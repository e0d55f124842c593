"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the bench.

This module only draws random numbers.  It holds none of the method's
arithmetic: no ray casting, no estimator, no geometry.  Everything it returns
is a NumPy array on the host (callers move it to the device themselves),
except ``mc_directions_device``, which draws very large direction sets on the
GPU with torch's seeded generator.

Conventions
-----------
* Point clouds are drawn in float64 and rounded to float32 once.  The float32
  array is *the* input of both the GPU path and the oracle (the oracle
  promotes it exactly to float64).
* A row in which some coordinate rounds to exactly 0.0 or 1.0 is drawn again,
  so every generator lies strictly inside the open unit cube (a generator on
  a face of the cube would give a zero-length Monte-Carlo ray).
* The Monte-Carlo directions of cell ``i`` are a pure function of
  ``(seed, i)``: cell ``i`` uses its own PCG64 stream seeded with
  ``SeedSequence([seed, i])``.  So any subset of cells can be regenerated on
  the host without drawing the others.  A direction is a standard normal
  vector divided by its norm (the uniform-on-the-sphere draw of Sec. 3.1),
  computed in float64 and rounded to float32.  Both sides use the rounded
  vector as given; it is not renormalised.
* ``philox_directions`` is the host side of the library's on-device draw
  (counter-based Philox4x32-10 and Box-Muller, keyed by (seed, cell, ray)):
  each side implements the same published generator, so the oracle can be
  given the directions of any seeded device run without reading them back.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "uniform_cloud",
    "gaussian_mixture_cloud",
    "jittered_lattice",
    "mc_directions",
    "mc_directions_device",
    "philox4x32_10",
    "philox_directions",
    "descent_draws",
    "uneven_batch_spec",
    "fd_generators",
    "WORKLOADS",
]


def _round_inside(pts64: np.ndarray) -> np.ndarray:
    """Round to float32; report rows that land on 0.0 or 1.0."""
    p32 = pts64.astype(np.float32)
    bad = np.any((p32 <= 0.0) | (p32 >= 1.0), axis=1)
    return p32, bad


def uniform_cloud(n: int, d: int, seed: int = 0) -> np.ndarray:
    """``n`` generators i.i.d. uniform in the open unit cube ``(0,1)^d``.

    Draw order: ``default_rng(seed).random((n, d))`` in float64, rounded to
    float32.  Rows that round onto a face are redrawn, in row order, from the
    same generator (this happens with probability about 6e-8 per coordinate).
    """
    rng = np.random.default_rng(seed)
    p64 = rng.random((n, d))
    p32, bad = _round_inside(p64)
    while bad.any():
        idx = np.nonzero(bad)[0]
        p32[idx], bad_new = _round_inside(rng.random((idx.size, d)))
        bad[:] = False
        bad[idx] = bad_new
    return np.ascontiguousarray(p32)


def gaussian_mixture_cloud(n: int = 100_000, d: int = 10, k: int = 8,
                           sigma: float = 0.05, seed: int = 0) -> np.ndarray:
    """Mixture of ``k`` isotropic Gaussians restricted to the unit cube.

    Draw order with ``rng = default_rng(seed)``: centres
    ``0.2 + 0.6 * rng.random((k, d))``; labels ``rng.integers(k, size=n)``;
    points ``centre[label] + sigma * rng.standard_normal((n, d))``.  Rows
    outside the open cube (after rounding to float32) are redrawn from their
    own component, in row order, until every row is inside (rejection, not
    clamping: clamping would put generators exactly on faces).
    """
    rng = np.random.default_rng(seed)
    centres = 0.2 + 0.6 * rng.random((k, d))
    labels = rng.integers(k, size=n)
    p64 = centres[labels] + sigma * rng.standard_normal((n, d))
    p32, bad = _round_inside(p64)
    while bad.any():
        idx = np.nonzero(bad)[0]
        q = centres[labels[idx]] + sigma * rng.standard_normal((idx.size, d))
        p32[idx], bad_new = _round_inside(q)
        bad[:] = False
        bad[idx] = bad_new
    return np.ascontiguousarray(p32)


def jittered_lattice(m: int, d: int, jitter: float = 1e-3, seed: int = 0) -> np.ndarray:
    """Cubic lattice ``h*(k + 1/2) + delta`` with ``h = 1/m`` and
    ``delta ~ U(-jitter*h, jitter*h)^d``; ``m**d`` generators in row-major
    lattice order (last axis fastest)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / m
    axes = [np.arange(m, dtype=np.float64)] * d
    grid = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1).reshape(-1, d)
    delta = rng.uniform(-jitter * h, jitter * h, size=grid.shape)
    p32, bad = _round_inside(h * (grid + 0.5) + delta)
    assert not bad.any()
    return np.ascontiguousarray(p32)


def _cell_directions(seed: int, cell: int, n_rays: int, d: int) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, int(cell)])))
    z = rng.standard_normal((n_rays, d))
    z /= np.sqrt(np.sum(z * z, axis=1, keepdims=True))
    return z.astype(np.float32)


def mc_directions(cells, n_rays: int, d: int, seed: int = 1) -> np.ndarray:
    """Unit directions for the Monte-Carlo rays of the listed cells.

    Returns float32 ``[len(cells)][n_rays][d]``; the block of cell ``i`` does
    not depend on which other cells are requested.
    """
    cells = np.asarray(cells, dtype=np.int64).ravel()
    out = np.empty((cells.size, n_rays, d), dtype=np.float32)
    for a, c in enumerate(cells):
        out[a] = _cell_directions(seed, c, n_rays, d)
    return out


def mc_directions_device(n_cells: int, n_rays: int, d: int, seed: int, device):
    """Unit directions ``[n_cells][n_rays][d]`` float32 drawn on a GPU with
    torch's seeded Philox generator (standard normal in float64, normalised,
    rounded to float32).  Used where the host draw would be too slow (the
    uneven batch holds about 6e9 numbers); the oracle reads host copies of
    the cells it checks."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    out = torch.empty((n_cells, n_rays, d), dtype=torch.float32, device=device)
    step = max(1, (1 << 26) // max(1, n_rays * d))
    for c0 in range(0, n_cells, step):
        c1 = min(n_cells, c0 + step)
        z = torch.randn((c1 - c0, n_rays, d), generator=g, dtype=torch.float64, device=device)
        z /= torch.sqrt((z * z).sum(dim=-1, keepdim=True))
        out[c0:c1] = z.float()
    return out


_PHILOX_M0, _PHILOX_M1 = 0xD2511F53, 0xCD9E8D57
_PHILOX_W0, _PHILOX_W1 = 0x9E3779B9, 0xBB67AE85


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11), vectorised:
    ``ctr`` uint32 ``[..., 4]``, ``key`` uint32 ``[..., 2]`` (broadcast);
    returns the four output words ``[..., 4]``.  Ten rounds; each round takes
    the high and low halves of M0 c0 and M1 c2 and bumps the key by the two
    Weyl constants."""
    c = np.array(ctr, dtype=np.uint64) & 0xFFFFFFFF
    k = np.array(key, dtype=np.uint64) & 0xFFFFFFFF
    c0, c1, c2, c3 = (c[..., i] for i in range(4))
    k0, k1 = k[..., 0], k[..., 1]
    mask = np.uint64(0xFFFFFFFF)
    for _ in range(10):
        p0 = np.uint64(_PHILOX_M0) * c0
        p1 = np.uint64(_PHILOX_M1) * c2
        c0, c1, c2, c3 = ((p1 >> np.uint64(32)) ^ c1 ^ k0, p1 & mask, (p0 >> np.uint64(32)) ^ c3 ^ k1, p0 & mask)
        k0 = (k0 + np.uint64(_PHILOX_W0)) & mask
        k1 = (k1 + np.uint64(_PHILOX_W1)) & mask
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def philox_directions(cells, n_rays: int, d: int, seed: int) -> np.ndarray:
    """Unit directions of the listed cells' Monte-Carlo rays as the library
    draws them on the device from ``seed`` (float32 ``[len(cells)][n_rays][d]``).

    Component k of ray r of cell c: Philox4x32-10 with counter
    ``(k // 4, r, c mod 2^32, c >> 32)`` and key ``(seed mod 2^32, seed >> 32)``
    gives words w0..w3; pair ``p = (k mod 4) // 2`` takes ``a = w[2p]``,
    ``b = w[2p+1]``; ``u1 = (a + 1/2) 2^-32``, ``u2 = b 2^-32``,
    ``rho = sqrt(-2 ln u1)``, ``theta = 2 pi u2`` (Box-Muller in float64);
    ``z_k = rho cos theta`` (k even) or ``rho sin theta`` (k odd).  Then
    ``s = z_0^2 + z_1^2 + ...`` summed in that order and ``u_k =
    float32(z_k / sqrt(s))``."""
    cells = np.asarray(cells, dtype=np.int64).ravel()
    nc = cells.size
    nj = (d + 3) // 4
    cell = np.broadcast_to(cells[:, None, None].astype(np.uint64), (nc, n_rays, nj))
    ray = np.broadcast_to(np.arange(n_rays, dtype=np.uint64)[None, :, None], (nc, n_rays, nj))
    j = np.broadcast_to(np.arange(nj, dtype=np.uint64)[None, None, :], (nc, n_rays, nj))
    ctr = np.stack([j, ray, cell & np.uint64(0xFFFFFFFF), cell >> np.uint64(32)], axis=-1)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    w = philox4x32_10(ctr, [seed & 0xFFFFFFFF, seed >> 32]).astype(np.float64)  # [nc, R, nj, 4]
    u1 = (w[..., 0::2] + 0.5) * 2.0 ** -32
    u2 = w[..., 1::2] * 2.0 ** -32
    rho = np.sqrt(-2.0 * np.log(u1))
    th = 6.283185307179586 * u2
    z = np.stack([rho * np.cos(th), rho * np.sin(th)], axis=-1).reshape(nc, n_rays, 4 * nj)[..., :d]
    s = np.zeros((nc, n_rays))
    for k in range(d):
        s = s + z[..., k] * z[..., k]
    return (z / np.sqrt(s)[..., None]).astype(np.float32)


def mc_radial_draws(cells, n_rays: int, m: int, seed: int = 3) -> np.ndarray:
    """The draws t ~ U(0, 1) of Algorithm 3's inner loop, ``m`` per ray, as
    float32 ``[len(cells)][n_rays][m]``; the block of cell ``i`` depends on
    ``(seed, i)`` only.  Values that round to 0 or 1 are redrawn."""
    cells = np.asarray(cells, dtype=np.int64).ravel()
    out = np.empty((cells.size, n_rays, m), dtype=np.float32)
    for a, c in enumerate(cells):
        rng = np.random.default_rng(np.random.SeedSequence([seed, int(c), 7]))
        v = rng.random((n_rays, m)).astype(np.float32)
        bad = (v <= 0) | (v >= 1)
        while bad.any():
            v[bad] = rng.random(int(bad.sum())).astype(np.float32)
            bad = (v <= 0) | (v >= 1)
        out[a] = v
    return out


def descent_draws(d: int, count: int = 64, seed: int = 2) -> np.ndarray:
    """Standard-normal float64 vectors ``[count][d]`` consumed, in order, by the
    ``Descent`` start of the exhaustive search (Algorithm 2): each step takes
    the next vector as its random search direction before projection."""
    return np.random.default_rng(seed).standard_normal((count, d))


def uneven_batch_spec(n_clouds: int = 64, seed: int = 0,
                      dims=(3, 4, 6, 8, 12, 16), n_lo: float = 1e3, n_hi: float = 2e5):
    """Specification of the uneven batch: a list of ``(d_c, N_c, cloud_seed)``.

    Draw order with ``rng = default_rng(seed)``: ``d_c = rng.choice(dims)``
    then ``N_c = int(exp(rng.uniform(ln n_lo, ln n_hi)))`` for each cloud in
    turn; cloud ``c`` then uses ``uniform_cloud(N_c, d_c, seed=1000 + c)``.
    """
    rng = np.random.default_rng(seed)
    spec = []
    for c in range(n_clouds):
        dc = int(rng.choice(np.asarray(dims)))
        nc = int(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi))))
        spec.append((dc, nc, 1000 + c))
    return spec


def fd_generators(n: int, count: int = 32, seed: int = 1) -> np.ndarray:
    """Indices of the generators whose coordinates are checked by finite
    differences: ``default_rng(seed).choice(n, count, replace=False)``."""
    return np.sort(np.random.default_rng(seed).choice(n, count, replace=False))


# Named workloads (sizes of the paper-shaped experiments used by tests and bench).
WORKLOADS = {
    "uniform_d2_n1000": dict(kind="uniform", n=1000, d=2, seed=0, rays_per_cell=128),
    "uniform_d6_n10000": dict(kind="uniform", n=10_000, d=6, seed=0),
    "gmm8_d10_n100000": dict(kind="gmm", n=100_000, d=10, seed=0, rays_per_cell=1024),
    "uneven64": dict(kind="uneven", n_clouds=64, seed=0, rays_per_cell=256),
    "uniform_d4_n50000": dict(kind="uniform", n=50_000, d=4, seed=0, rays_per_cell=512),
}
