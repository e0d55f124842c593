"""Pins of the oracle's Monte-Carlo estimators (Sec. 3.1, Algorithm 3) and of
their closed-form adjoint.

  * per ray, l^d = h * l^{d-1}/|n.u| with h the distance from x_i to the
    facet's plane, so volume = (1/d) sum_j h_ij area_ij (Sec. 3.3);
  * the cells tile the unit cube: volumes sum to 1 within Monte-Carlo error;
  * 2-D: exact polygon areas, edge lengths and second moments from
    half-plane clipping of the unit square;
  * jittered cubic lattice: volumes h^d, axis facets h^(d-1);
  * adjoint: central finite differences of the FP64 estimator with frozen
    directions, and the centroidal-energy identity grad = 2 V (x - c).
"""
import numpy as np
import pytest

import workloads as W


def _sample_se(per_ray_values):
    """Standard error of a mean over the last axis."""
    n = per_ray_values.shape[-1]
    return per_ray_values.std(axis=-1, ddof=1) / np.sqrt(n)


# ---------------------------------------------------------------------------
# exact 2-D cells by half-plane clipping (Sutherland-Hodgman)
# ---------------------------------------------------------------------------
def _clip(poly, a, b, lab):
    """Keep {y : a.y <= b}; poly is a list of (point, label-of-edge-to-next)."""
    out = []
    m = len(poly)
    for q in range(m):
        p0, l0 = poly[q]
        p1, _ = poly[(q + 1) % m]
        in0 = a @ p0 <= b
        in1 = a @ p1 <= b
        if in0:
            if in1:
                out.append((p0, l0))
            else:
                s = (b - a @ p0) / (a @ (p1 - p0))
                out.append((p0, l0))
                out.append((p0 + s * (p1 - p0), lab))
        elif in1:
            s = (b - a @ p0) / (a @ (p1 - p0))
            out.append((p0 + s * (p1 - p0), l0))
    return out


def _exact_cell_2d(X, i):
    sq = [(np.array([0.0, 0.0]), -2 - 2), (np.array([1.0, 0.0]), -2 - 1),
          (np.array([1.0, 1.0]), -2 - 3), (np.array([0.0, 1.0]), -2 - 0)]
    # edge labels follow the face codes: y=0 is 2*1+0, x=1 is 2*0+1, y=1 is 2*1+1, x=0 is 0
    poly = sq
    xi = X[i]
    for j in range(X.shape[0]):
        if j == i:
            continue
        a = X[j] - xi
        b = 0.5 * (X[j] @ X[j] - xi @ xi)
        poly = _clip(poly, a, b, j)
    P = np.array([p for p, _ in poly])
    area = 0.5 * abs(np.sum(P[:, 0] * np.roll(P[:, 1], -1) - np.roll(P[:, 0], -1) * P[:, 1]))
    lengths = {}
    second = 0.0
    for q, (p0, lab) in enumerate(poly):
        p1 = poly[(q + 1) % len(poly)][0]
        L = np.linalg.norm(p1 - p0)
        if L > 0:
            lengths[lab] = lengths.get(lab, 0.0) + L
        a0, a1 = p0 - xi, p1 - xi
        tri = 0.5 * abs(a0[0] * a1[1] - a0[1] * a1[0])
        second += tri / 6.0 * (a0 @ a0 + a1 @ a1 + a0 @ a1)
    return area, lengths, second


def test_per_ray_volume_area_identity(oracle_mod):
    for d, n in ((2, 80), (3, 150), (5, 200)):
        X = W.uniform_cloud(n, d, seed=d)
        X64 = X.astype(np.float64)
        cells = np.arange(0, n, 7)
        D = W.mc_directions(cells, 64, d, seed=11)
        r = oracle_mod.mc_volume_area(X, cells, D)
        cell_of_ray = np.repeat(cells, 64)
        h = np.empty(r["t"].size)
        for k, (i, j) in enumerate(zip(cell_of_ray, r["idx"])):
            if j >= 0:
                h[k] = 0.5 * np.linalg.norm(X64[j] - X64[i])
            else:
                kk, s = divmod(-2 - j, 2)
                h[k] = abs(s - X64[i, kk])
        assert np.allclose(r["w_vol"], h * r["w_area"], rtol=1e-11)
        # the cell-level form: V_i = (1/d) sum_j h_ij A_ij
        for c, i in enumerate(cells):
            acc = 0.0
            for (ii, j), A in r["facets"].items():
                if ii != i:
                    continue
                if j >= 0:
                    hij = 0.5 * np.linalg.norm(X64[j] - X64[i])
                else:
                    kk, s = divmod(-2 - j, 2)
                    hij = abs(s - X64[i, kk])
                acc += hij * A / d
            assert acc == pytest.approx(r["volume"][c], rel=1e-11)


@pytest.mark.parametrize("d,n,rays", [(2, 60, 256), (3, 80, 256), (4, 60, 256)])
def test_volumes_sum_to_one(oracle_mod, d, n, rays):
    X = W.uniform_cloud(n, d, seed=1)
    cells = np.arange(n)
    D = W.mc_directions(cells, rays, d, seed=2)
    r = oracle_mod.mc_volume_area(X, cells, D)
    S = oracle_mod.sphere_area(d)
    per_ray = (S / d) * r["w_vol"].reshape(n, rays)
    se = np.sqrt(np.sum(_sample_se(per_ray) ** 2))
    assert abs(r["volume"].sum() - 1.0) <= 5 * se
    assert se < 0.05


def test_2d_exact_polygons(oracle_mod):
    n, rays = 40, 512
    X = W.uniform_cloud(n, 2, seed=8)
    X64 = X.astype(np.float64)
    cells = np.arange(n)
    D = W.mc_directions(cells, rays, 2, seed=4)
    r = oracle_mod.mc_volume_area(X, cells, D)
    S = oracle_mod.sphere_area(2)
    vol_rays = (S / 2) * r["w_vol"].reshape(n, rays)
    en_rays = (S / 4) * r["w_energy"].reshape(n, rays)
    se_v = _sample_se(vol_rays)
    se_e = _sample_se(en_rays)
    idx = r["idx"].reshape(n, rays)
    wa = r["w_area"].reshape(n, rays)
    checked = 0
    for i in range(n):
        area, lengths, second = _exact_cell_2d(X64, i)
        assert abs(r["volume"][i] - area) <= 5 * se_v[i] + 1e-12
        assert abs(r["energy2"][i] - second) <= 5 * se_e[i] + 1e-12
        for lab, L in lengths.items():
            per_ray = S * wa[i] * (idx[i] == lab)
            est = per_ray.mean()
            assert est == pytest.approx(r["facets"].get((i, lab), 0.0), rel=1e-12, abs=1e-15)
            se = _sample_se(per_ray)
            if L > 0.02:  # facets hit by enough rays for a normal error
                assert abs(est - L) <= 5 * se + 1e-12, (i, lab, est, L, se)
                checked += 1
    assert checked > 3 * n


@pytest.mark.parametrize("d,m", [(2, 8), (3, 5)])
def test_jittered_lattice(oracle_mod, d, m):
    X = W.jittered_lattice(m, d, jitter=1e-3, seed=0)
    n = X.shape[0]
    rays = 512
    h = 1.0 / m
    cells = np.arange(n)
    D = W.mc_directions(cells, rays, d, seed=3)
    r = oracle_mod.mc_volume_area(X, cells, D)
    S = oracle_mod.sphere_area(d)
    se_v = _sample_se((S / d) * r["w_vol"].reshape(n, rays))
    assert np.all(np.abs(r["volume"] - h**d) <= 5 * se_v + 1e-2 * h**d)
    # second moment of a cube of side h about its centre: h^d * d h^2 / 12
    se_e = _sample_se((S / (d + 2)) * r["w_energy"].reshape(n, rays))
    assert np.all(np.abs(r["energy2"] - h**d * d * h * h / 12) <= 5 * se_e + 2e-2 * h**(d + 2))
    # facets toward the lattice neighbours along an axis (or a cube face)
    wa = r["w_area"].reshape(n, rays)
    idx = r["idx"].reshape(n, rays)
    checked = 0
    lat = np.stack(np.unravel_index(np.arange(n), (m,) * d), axis=1)
    strides = np.array([m ** (d - 1 - k) for k in range(d)])
    for i in range(0, n, 3):
        for k in range(d):
            for s, step in ((1, +1), (0, -1)):
                c = lat[i, k] + step
                j = i + step * strides[k] if 0 <= c < m else -2 - (2 * k + s)
                per_ray = S * wa[i] * (idx[i] == j)
                est, se = per_ray.mean(), _sample_se(per_ray)
                assert abs(est - h ** (d - 1)) <= 5 * se + 2e-2 * h ** (d - 1), (i, k, s)
                checked += 1
    assert checked > 0


# ---------------------------------------------------------------------------
# adjoint
# ---------------------------------------------------------------------------
def _loss(oracle_mod, X64, cells, D, gv, ge, ga_ray):
    r = oracle_mod.mc_volume_area(X64, cells, D)
    d = X64.shape[1]
    nr = D.shape[1]
    S = oracle_mod.sphere_area(d)
    L = gv @ r["volume"] + ge @ r["energy2"] + (S / nr) * (ga_ray @ r["w_area"])
    return L, r["idx"]


@pytest.mark.parametrize("d,n", [(2, 30), (3, 40), (4, 30)])
def test_adjoint_matches_central_differences(oracle_mod, d, n):
    X64 = W.uniform_cloud(n, d, seed=21).astype(np.float64)
    cells = np.arange(n)
    nr = 24
    D = W.mc_directions(cells, nr, d, seed=22)
    rng = np.random.default_rng(3)
    gv = rng.standard_normal(n)
    ge = rng.standard_normal(n)
    ga = rng.standard_normal(n * nr)
    r = oracle_mod.mc_volume_area(X64, cells, D)
    G = oracle_mod.mc_adjoint(X64, cells, D, r["t"], r["idx"], gv, ge, ga)
    h = 1e-6
    skipped = 0
    for i in range(n):
        for k in range(d):
            Xp = X64.copy()
            Xp[i, k] += h
            Xm = X64.copy()
            Xm[i, k] -= h
            Lp, ip = _loss(oracle_mod, Xp, cells, D, gv, ge, ga)
            Lm, im = _loss(oracle_mod, Xm, cells, D, gv, ge, ga)
            if not np.array_equal(ip, im):
                skipped += 1  # a ray changed facet: the area term jumps
                continue
            fd = (Lp - Lm) / (2 * h)
            assert fd == pytest.approx(G[i, k], rel=1e-5, abs=1e-7 * (1 + abs(fd)))
    assert skipped < n * d // 4


def test_centroidal_energy_gradient_identity(oracle_mod):
    """For the total second moment E = sum_i int_{C_i} |y - x_i|^2 dy,
    dE/dx_i = 2 V_i (x_i - c_i) (Du, Faber & Gunzburger, SIAM Rev. 1999): the
    moving-boundary terms of neighbouring cells cancel.  With Monte-Carlo
    estimates of V_i and c_i from the same rays the two sides agree up to the
    sampling error of the estimator."""
    d, m = 2, 6
    X = W.jittered_lattice(m, d, jitter=0.15, seed=1).astype(np.float64)
    n = X.shape[0]
    cells = np.arange(n)
    S = oracle_mod.sphere_area(d)
    errs = []
    for nr in (4096, 16384):
        D = W.mc_directions(cells, nr, d, seed=5)
        r = oracle_mod.mc_volume_area(X, cells, D)
        G = oracle_mod.mc_adjoint(X, cells, D, r["t"], r["idx"], None, np.ones(n), None)
        l = r["t"].reshape(n, nr)
        U = D.astype(np.float64)
        first = (S / nr) * np.einsum("ck,ckd->cd", l ** (d + 1) / (d + 1), U)  # int (y - x_i) dy
        pred = -2.0 * first  # 2 V (x - c) = -2 int (y - x_i) dy
        errs.append(np.linalg.norm(G - pred) / np.linalg.norm(pred))
    # unbiased: the discrepancy is sampling noise and halves when the rays quadruple
    assert errs[1] < 0.08
    assert 1.5 < errs[0] / errs[1] < 2.7


# ---------------------------------------------------------------------------
# integrals of a function f (Algorithm 3 with its inner loop)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d,n", [(2, 60), (3, 80), (5, 60)])
def test_function_integrals_reduce_to_volume_and_areas(oracle_mod, d, n):
    """f = 1 turns the facet integrals into the facet areas; with every draw
    t = 1 (t = 1/2) the volume integral is d (d 2^{1-d}) times the volume
    estimator, since t^{d-1} l^d then equals d times (2^{1-d} d times) the
    volume term l^d / d of the same ray."""
    X = W.uniform_cloud(n, d, seed=20 + d)
    cells = np.arange(0, n, 3)
    R, m = 128, 3
    D = W.mc_directions(cells, R, d, seed=21)
    one = lambda p: np.ones(p.shape[0])  # noqa: E731
    for tval, factor in ((1.0, d), (0.5, d * 0.5 ** (d - 1))):
        T = np.full((cells.size, R, m), tval)
        r = oracle_mod.mc_integrals(X, cells, D, T, one)
        assert np.allclose(r["F_V"], factor * r["volume"], rtol=1e-12)
        assert set(r["F"]) == set(r["facets"])
        for key, A in r["facets"].items():
            assert r["F"][key] == pytest.approx(A, rel=1e-12)


def _exact_linear_2d(X, i, c0, c):
    """Exact integrals of f(y) = c0 + c.y over cell i (area f(centroid)) and
    over its edges (per label: sum of segment length times f(midpoint))."""
    sq = [(np.array([0.0, 0.0]), -2 - 2), (np.array([1.0, 0.0]), -2 - 1),
          (np.array([1.0, 1.0]), -2 - 3), (np.array([0.0, 1.0]), -2 - 0)]
    poly = sq
    xi = X[i]
    for j in range(X.shape[0]):
        if j != i:
            poly = _clip(poly, X[j] - xi, 0.5 * (X[j] @ X[j] - xi @ xi), j)
    P = np.array([p for p, _ in poly])
    cross = P[:, 0] * np.roll(P[:, 1], -1) - np.roll(P[:, 0], -1) * P[:, 1]
    area = 0.5 * cross.sum()
    cen = np.array([((P[:, 0] + np.roll(P[:, 0], -1)) * cross).sum(),
                    ((P[:, 1] + np.roll(P[:, 1], -1)) * cross).sum()]) / (6.0 * area)
    cell = abs(area) * (c0 + c @ cen)
    edges = {}
    for q, (p0, lab) in enumerate(poly):
        p1 = poly[(q + 1) % len(poly)][0]
        L = np.linalg.norm(p1 - p0)
        if L > 0:
            edges[lab] = edges.get(lab, 0.0) + L * (c0 + c @ (0.5 * (p0 + p1)))
    return cell, edges


def test_function_integrals_2d_exact_polygons(oracle_mod):
    n, R, m = 30, 1024, 4
    X = W.uniform_cloud(n, 2, seed=9)
    X64 = X.astype(np.float64)
    cells = np.arange(n)
    D = W.mc_directions(cells, R, 2, seed=5)
    rng = np.random.default_rng(7)
    T = rng.random((n, R, m))
    c0, c = 0.3, np.array([1.7, -0.9])
    f = lambda p: c0 + p @ c  # noqa: E731
    r = oracle_mod.mc_integrals(X, cells, D, T, f)
    S = oracle_mod.sphere_area(2)
    # per-ray contributions, for the Monte-Carlo standard errors
    t = r["t"].reshape(n, R)
    pts = (1 - T[..., None]) * X64[:, None, None, :] + T[..., None] * (X64[:, None, :] + t[..., None] * D)[:, :, None, :]
    vol_ray = S * (f(pts.reshape(-1, 2)).reshape(n, R, m) * T * (t ** 2)[..., None]).mean(axis=2)
    se_v = _sample_se(vol_ray)
    idx = r["idx"].reshape(n, R)
    fa = (r["f_hit"] * r["w_area"].reshape(n, R)) * S
    checked = 0
    for i in range(n):
        cell, edges = _exact_linear_2d(X64, i, c0, c)
        assert vol_ray[i].mean() == pytest.approx(r["F_V"][i], rel=1e-12)
        assert abs(r["F_V"][i] - cell) <= 5 * se_v[i] + 1e-12, (i, r["F_V"][i], cell, se_v[i])
        for lab, val in edges.items():
            per_ray = fa[i] * (idx[i] == lab)
            assert per_ray.mean() == pytest.approx(r["F"].get((i, lab), 0.0), rel=1e-12, abs=1e-15)
            if (idx[i] == lab).sum() > 30:
                assert abs(per_ray.mean() - val) <= 5 * _sample_se(per_ray) + 1e-12, (i, lab)
                checked += 1
    assert checked > 2 * n
