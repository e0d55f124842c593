"""FP64 CPU oracle for the batched RayCast of the Voronoi Graph method
(Sikorski & Heida, arXiv 2405.10050).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library (``paper_2405_10050_amd``) and never imports it.

The arithmetic lives in ``vgoracle.c`` (plain C, FP64, OpenMP over independent
rays); this module compiles it with gcc, loads it with ctypes and adds the
Monte-Carlo sums of Sec. 3.1 / Algorithm 3 with NumPy in FP64.

Inputs are the float32 arrays the GPU receives, promoted exactly to float64.

Pins (what each function is checked against, in ``tests/test_oracle_*.py``):
  raycast / raycast_cells   bisection of nearest-generator membership along the
                            ray; incircle criterion of the hit (equidistant to
                            g and j, no node closer); Algorithm 1
                            (``raycast_incircle``); a lone generator exits
                            through a face of the cube.
  explore                   brute-force enumeration of empty circumspheres on
                            tiny inputs; 2-D Euler relation with an
                            independently computed hull; every edge seen by
                            exactly two vertices or once with an unbounded
                            ray; simplex volumes sum to the hull volume;
                            scipy's Delaunay on the 2-D workload.
  mc_volume_area            volume-from-areas identity of Sec. 3.3 per ray;
                            volumes sum to 1 within Monte-Carlo error; exact
                            2-D polygon areas and edge lengths from half-plane
                            clipping; the jittered cubic lattice.
  mc_adjoint                central finite differences of the FP64 estimator
                            with frozen directions; the centroidal-energy
                            gradient identity 2 V (x - c).
  star                      equals the vertices of ``explore`` that contain the
                            generator.
  explore_clipped           brute-force enumeration of the constraint sets
                            (generators and faces) on tiny inputs; 2-D closed
                            form V = 2N + 2; every cell's 2-D polygon from
                            half-plane clipping; 3-D cell volumes (convex
                            hulls of the cells' vertices) sum to 1; its
                            face-free vertices are the unbounded diagram's
                            vertices inside the cube; every edge seen by
                            exactly two vertices.
  hmc_integrals             f = 1 turns F into the areas and the cell integral
                            into the volume-from-areas identity; 2-D with
                            exact edge lengths: exact cell and edge integrals
                            of a linear f; 3-D with exact facet areas: f = 1
                            gives the convex-hull cell volumes.
  mc_integrals              f = 1 gives the facet areas, and t = 1 (t = 1/2)
                            gives d (d 2^{1-d}) times the volume, exactly;
                            2-D: exact cell and edge integrals of a linear f
                            (area times f at the centroid, length times f at
                            the midpoint) within Monte-Carlo error.
No oracle function is unpinned.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vgoracle.c")
_LIB = os.path.join(_HERE, "libvgoracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``vgoracle.c`` with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                               "-Wall", "-Wno-unused-function", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        lib.vgo_raycast.argtypes = [i32, i64, P, i64, P, P, P, P, i32, i32, P, P, P]
        lib.vgo_raycast_cells.argtypes = [i32, i64, P, i64, P, i32, P, P, P, P]
        lib.vgo_raycast_incircle.argtypes = [i32, i64, P, i64, P, P, P, i32, i32, P, P, P]
        lib.vgo_explore.argtypes = [i32, i64, P, P, i32, i32]
        lib.vgo_explore.restype = P
        for f in ("vgo_mesh_nv", "vgo_mesh_nb", "vgo_mesh_raycasts", "vgo_mesh_nn_calls",
                  "vgo_mesh_duplicates"):
            getattr(lib, f).argtypes = [P]
            getattr(lib, f).restype = i64
        lib.vgo_mesh_copy.argtypes = [P, P, P, P, P]
        lib.vgo_mesh_free.argtypes = [P]
        lib.vgo_circumcentre.argtypes = [i32, P, P, P]
        lib.vgo_search_direction.argtypes = [i32, P, P, i32, P]
        lib.vgo_mc_ray_weights.argtypes = [i32, i64, P, i64, P, i32, P, P, P, P, P, P]
        lib.vgo_mc_adjoint.argtypes = [i32, i64, P, i64, P, i32, P, P, P, dbl, P, P, P, P]
        lib.vgo_num_threads.restype = i32
        lib.vgo_set_threads.argtypes = [i32]
        lib.vgo_set_threads.restype = None
        lib.vgo_explore_clipped.argtypes = [i32, i64, P]
        lib.vgo_explore_clipped.restype = P
        lib.vgo_clipped_vertex.argtypes = [i32, i64, P, P, P]
        lib.vgo_explore_periodic.argtypes = [i32, i64, P, P, i32, P]
        lib.vgo_explore_periodic.restype = P
        lib.vgo_star.argtypes = [i32, i64, P, i32, P, i32, P, i64]
        lib.vgo_star.restype = i64
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def num_threads() -> int:
    return int(_load().vgo_num_threads())


def set_threads(k: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (the results do not
    depend on it)."""
    _load().vgo_set_threads(int(k))


def sphere_area(d: int) -> float:
    """S_{d-1} = 2 pi^{d/2} / Gamma(d/2), the area of the unit sphere in R^d
    (Sec. 3.1)."""
    return 2.0 * math.pi ** (d / 2.0) / math.gamma(d / 2.0)


# --------------------------------------------------------------------------
# O1: RayCast by definition
# --------------------------------------------------------------------------
def raycast(nodes, origin, direction, gen, excl=None, clip=True):
    """Brute-force RayCast of arbitrary rays (eq. (t) with the half-space
    restriction of Algorithm 1).  Returns float64 ``t`` (inf: no hit), int32
    ``idx`` and the second-smallest candidate ``t2``."""
    lib = _load()
    X = _f64(nodes)
    n, d = X.shape
    O = _f64(origin).reshape(-1, d)
    U = _f64(direction).reshape(-1, d)
    m = O.shape[0]
    g = _i32(gen).reshape(m)
    if excl is None:
        E, ne = None, 0
    else:
        E = _i32(excl).reshape(m, -1)
        ne = E.shape[1]
    t = np.empty(m)
    idx = np.empty(m, dtype=np.int32)
    t2 = np.empty(m)
    rc = lib.vgo_raycast(d, n, _p(X), m, _p(O), _p(U), _p(g), _p(E), ne, int(bool(clip)),
                         _p(t), _p(idx), _p(t2))
    assert rc == 0
    return t, idx, t2


def raycast_cells(nodes, cells, dirs):
    """Monte-Carlo rays of Algorithm 3: ray k of listed cell c starts at
    x_{cells[c]} with eta = {cells[c]} and is clipped to the unit cube.
    ``dirs`` is ``[len(cells)][n_rays][d]``.  Returns flat arrays of
    ``len(cells) * n_rays`` entries (cell-major)."""
    lib = _load()
    X = _f64(nodes)
    n, d = X.shape
    cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64).ravel())
    D = _f64(dirs).reshape(cells.size, -1, d)
    nr = D.shape[1]
    m = cells.size * nr
    t = np.empty(m)
    idx = np.empty(m, dtype=np.int32)
    t2 = np.empty(m)
    rc = lib.vgo_raycast_cells(d, n, _p(X), cells.size, _p(cells), nr, _p(D), _p(t), _p(idx),
                               _p(t2))
    assert rc == 0
    return t, idx, t2


def raycast_incircle(nodes, origin, direction, eta, heuristic=False):
    """Algorithm 1 (iterative incircle RayCast) with a brute-force ``nn``;
    clipping off.  ``eta`` is ``[m][n_eta]`` with ``eta[:,0]`` the generator
    x_0 of eq. (t).  Returns ``t``, ``idx`` and the number of ``nn`` calls."""
    lib = _load()
    X = _f64(nodes)
    n, d = X.shape
    O = _f64(origin).reshape(-1, d)
    U = _f64(direction).reshape(-1, d)
    m = O.shape[0]
    E = _i32(eta).reshape(m, -1)
    t = np.empty(m)
    idx = np.empty(m, dtype=np.int32)
    calls = np.empty(m, dtype=np.int64)
    rc = lib.vgo_raycast_incircle(d, n, _p(X), m, _p(O), _p(U), _p(E), E.shape[1],
                                  int(bool(heuristic)), _p(t), _p(idx), _p(calls))
    assert rc == 0
    return t, idx, calls


def near_tie(t, t2, rel: float = 1e-9):
    """Rays whose best and second-best candidates are within ``rel`` of each
    other: several answers are correct there, so argmin parity excuses them."""
    t = np.asarray(t)
    t2 = np.asarray(t2)
    with np.errstate(invalid="ignore"):
        return np.isfinite(t2) & ((t2 - t) <= rel * np.abs(t))


# --------------------------------------------------------------------------
# O2: Algorithm 2
# --------------------------------------------------------------------------
def explore(nodes, draws, mode: int = 0):
    """Exhaustive VoronoiGraph search (Algorithm 2) of the unbounded diagram.

    ``mode`` 0 casts rays by definition, 1 and 2 with Algorithm 1 without and
    with InitialHeuristic (then ``nn_calls`` counts its nearest-neighbour
    calls).  Returns a dict with ``sigma`` ``[V][d+1]`` (sorted tuples, in
    discovery order), ``coord`` ``[V][d]``, ``b_sigma``, ``b_omit`` and the
    counters ``raycasts``, ``nn_calls``, ``duplicates``."""
    lib = _load()
    X = _f64(nodes)
    n, d = X.shape
    W = _f64(draws).reshape(-1, d)
    h = lib.vgo_explore(d, n, _p(X), _p(W), W.shape[0], int(mode))
    if not h:
        raise RuntimeError("oracle explore failed (descent exhausted or singular vertex)")
    try:
        nv, nb = lib.vgo_mesh_nv(h), lib.vgo_mesh_nb(h)
        sig = np.empty((nv, d + 1), dtype=np.int32)
        coord = np.empty((nv, d))
        bsig = np.empty((nb, d + 1), dtype=np.int32)
        bomit = np.empty(nb, dtype=np.int32)
        lib.vgo_mesh_copy(h, _p(sig), _p(coord), _p(bsig), _p(bomit))
        return dict(sigma=sig, coord=coord, b_sigma=bsig, b_omit=bomit,
                    raycasts=int(lib.vgo_mesh_raycasts(h)), nn_calls=int(lib.vgo_mesh_nn_calls(h)),
                    duplicates=int(lib.vgo_mesh_duplicates(h)))
    finally:
        lib.vgo_mesh_free(h)


def explore_clipped(nodes):
    """Exhaustive search (Algorithm 2) of the diagram clipped to the unit
    cube, from the corner 0.  A vertex key holds d+1 sorted constraints:
    generator indices, and the code ``n + 2k + s`` for the face ``x_k = s``.
    Returns a dict with ``sigma`` ``[V][d+1]`` (discovery order), ``coord``
    ``[V][d]`` and the counters ``raycasts``, ``duplicates``."""
    lib = _load()
    X = _f64(nodes)
    n, d = X.shape
    h = lib.vgo_explore_clipped(d, n, _p(X))
    if not h:
        raise RuntimeError("oracle clipped explore failed (singular vertex)")
    try:
        nv = lib.vgo_mesh_nv(h)
        sig = np.empty((nv, d + 1), dtype=np.int32)
        coord = np.empty((nv, d))
        lib.vgo_mesh_copy(h, _p(sig), _p(coord), None, None)
        return dict(sigma=sig, coord=coord, raycasts=int(lib.vgo_mesh_raycasts(h)),
                    duplicates=int(lib.vgo_mesh_duplicates(h)))
    finally:
        lib.vgo_mesh_free(h)


_PERIODIC_FAIL = {-1: "nodes outside [0,1)^d, n * 3^d >= 2^31 or allocation",
                  -2: "a vertex ball reaches past the images in [-1,2]^d",
                  -3: "a vertex ball of radius >= 1/2 (key outside the shift range)",
                  -4: "singular vertex or Descent out of draws"}


def periodic_decode(keys, d):
    """Split periodic key entries ``i * 3^d + c(k)`` into node indices and
    lattice shifts ``k`` in ``{-1,0,1}^d`` (``c(k) = sum_a (k_a + 1) 3^a``)."""
    keys = np.asarray(keys, dtype=np.int64)
    S = 3 ** d
    ids = keys // S
    c = keys % S
    shift = np.stack([(c // 3 ** a) % 3 - 1 for a in range(d)], axis=-1).astype(np.int8)
    return ids.astype(np.int32), shift


def explore_periodic(nodes, draws):
    """Exhaustive search (Algorithm 2) of the periodic diagram of nodes in
    ``[0,1)^d`` (the torus R^d / Z^d).  A key entry is a node image
    ``x_i + k``, coded ``i * 3^d + c(k)``; a vertex key is translated so that
    its smallest node has ``k = 0`` and its coordinates are in that frame.
    Needs every vertex ball radius below 1/2.  Returns a dict with ``key``
    ``[V][d+1]`` (codes, sorted), ``sigma`` (node indices) and ``shift``
    (``[V][d+1][d]``) decoded from it, ``coord`` ``[V][d]``, and the counters
    ``raycasts``, ``duplicates``."""
    lib = _load()
    X = _f64(nodes)
    n, d = X.shape
    W = _f64(draws).reshape(-1, d)
    st = ctypes.c_int(0)
    h = lib.vgo_explore_periodic(d, n, _p(X), _p(W), W.shape[0], ctypes.byref(st))
    if not h:
        raise RuntimeError("oracle periodic explore failed: " + _PERIODIC_FAIL.get(st.value, str(st.value)))
    try:
        nv = lib.vgo_mesh_nv(h)
        key = np.empty((nv, d + 1), dtype=np.int32)
        coord = np.empty((nv, d))
        lib.vgo_mesh_copy(h, _p(key), _p(coord), None, None)
        sigma, shift = periodic_decode(key, d)
        return dict(key=key, sigma=sigma, shift=shift, coord=coord, raycasts=int(lib.vgo_mesh_raycasts(h)),
                    duplicates=int(lib.vgo_mesh_duplicates(h)))
    finally:
        lib.vgo_mesh_free(h)


def clipped_vertex(nodes, key):
    """The point fixed by the d+1 constraints ``key`` (clipped encoding)."""
    lib = _load()
    X = _f64(nodes)
    n, d = X.shape
    v = np.empty(d)
    if lib.vgo_clipped_vertex(d, n, _p(X), _p(_i32(np.sort(key))), _p(v)):
        raise ValueError("singular constraints")
    return v


def hmc_integrals(nodes, sigma, coord, areas, f):
    """Heuristic Monte-Carlo integrals (Sec. 3.3) over the clipped diagram.

    ``sigma``/``coord`` are the clipped vertex set (``explore_clipped``),
    ``areas`` a dict ``(i, j) -> A_ij`` of interface areas keyed like
    ``mc_volume_area``'s facets (``j`` a generator, or ``-2-(2k+s)`` for the
    face ``x_k = s``), ``f`` maps float64 points ``[P, d]`` to ``[P]``.  For
    every facet with an area:

      V_ij      = the vertices whose key holds both i and j (K_ij of them)
      y_ij      = K_ij^{-1} sum_k nu_k                       (its centroid)
      F_ij      = d/(d+1) K_ij^{-1} sum_k f(nu_k) A_ij + 1/(d+1) f(y_ij) A_ij
      h_ij      = distance of x_i to the facet's hyperplane: |x_j - x_i|/2,
                  or x_i,k (s = 0) / 1 - x_i,k (s = 1) for a face
      volume_i  = 1/d sum_j h_ij A_ij
      cell_i    = sum_j h_ij/d (d/(d+1) F_ij + 1/(d+1) A_ij f(x_i))

    the last being the pyramid rule of eq. (leibniz-int) applied to the
    pyramid over each facet with apex x_i.  Returns a dict with
    ``centroid`` and ``F`` (dicts keyed like ``areas``), ``cell`` and
    ``volume`` ``[n]``."""
    X = _f64(nodes)
    n, d = X.shape
    sig = np.asarray(sigma)
    P = _f64(coord)
    members = {}
    for v, row in enumerate(sig):
        for a in row:
            if a >= n:
                continue
            for b in row:
                if b == a:
                    continue
                j = int(b) if b < n else -2 - int(b - n)
                members.setdefault((int(a), j), []).append(v)
    fv = np.asarray(f(P), dtype=np.float64)
    fx = np.asarray(f(X), dtype=np.float64)
    keys = [k for k in areas if k in members]
    cent = {k: P[members[k]].mean(axis=0) for k in keys}
    fy = dict(zip(keys, np.asarray(f(np.array([cent[k] for k in keys]).reshape(-1, d)), dtype=np.float64)))
    F, cell, volume = {}, np.zeros(n), np.zeros(n)
    for (i, j) in keys:
        A = areas[(i, j)]
        F[(i, j)] = d / (d + 1) * fv[members[(i, j)]].mean() * A + fy[(i, j)] * A / (d + 1)
        if j >= 0:
            h = 0.5 * np.sqrt(((X[j] - X[i]) ** 2).sum())
        else:
            k, side = divmod(-2 - j, 2)
            h = X[i, k] if side == 0 else 1.0 - X[i, k]
        volume[i] += h * A / d
        cell[i] += h / d * (d / (d + 1) * F[(i, j)] + A * fx[i] / (d + 1))
    return dict(centroid=cent, F=F, cell=cell, volume=volume)


def star(nodes, i, draws, cap=200_000):
    """Vertices of the unbounded diagram whose generators include ``i``
    (sorted tuples ``[V_i][d+1]``): Algorithm 2 restricted to the edges that
    keep ``i``.  ``neighbours(star)`` are the Voronoi neighbours of ``i``."""
    lib = _load()
    X = _f64(nodes)
    n, d = X.shape
    W = _f64(draws).reshape(-1, d)
    out = np.empty((cap, d + 1), dtype=np.int32)
    nv = lib.vgo_star(d, n, _p(X), int(i), _p(W), W.shape[0], _p(out), cap)
    if nv < 0:
        raise RuntimeError("oracle star failed")
    return out[:nv].copy()


def circumcentre(nodes, sigma):
    lib = _load()
    X = _f64(nodes)
    d = X.shape[1]
    s = _i32(sigma)
    v = np.empty(d)
    assert lib.vgo_circumcentre(d, _p(X), _p(s), _p(v)) == 0
    return v


def search_direction(nodes, eta, omit):
    lib = _load()
    X = _f64(nodes)
    d = X.shape[1]
    e = _i32(eta)
    u = np.empty(d)
    assert lib.vgo_search_direction(d, _p(X), _p(e), int(omit), _p(u)) == 0
    return u


def sorted_rows(a):
    """Rows of an integer array in lexicographic order (for set comparison)."""
    a = np.asarray(a)
    if a.size == 0:
        return a.reshape(0, a.shape[1] if a.ndim == 2 else 0)
    order = np.lexsort(a.T[::-1])
    return a[order]


# --------------------------------------------------------------------------
# O3: Monte-Carlo estimators (Sec. 3.1, Algorithm 3 with f = 1, m = 0)
# --------------------------------------------------------------------------
def mc_volume_area(nodes, cells, dirs, rays=None):
    """Monte-Carlo volume, interface areas and second moment of the listed
    cells.

    With ``l`` = t* and ``S = S_{d-1}``:
      volume_i  = S/(d n) sum_k l_k^d
      area_ij   = S/n     sum_{k: j_k = j} l_k^{d-1} / |n_ij . u_k|
      energy2_i = S/((d+2) n) sum_k l_k^{d+2}     (= int_{C_i} |y - x_i|^2 dy)
    Facets toward the cube are keyed by the negative face code of the ray
    result.  Returns a dict with ``volume``, ``energy2`` (per listed cell),
    ``facets`` (dict ``(i, j) -> area``) and the per-ray ``t``, ``idx``,
    ``t2`` and ``w_vol``, ``w_area``, ``w_energy``.
    """
    lib = _load()
    X = _f64(nodes)
    n, d = X.shape
    cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64).ravel())
    D = _f64(dirs).reshape(cells.size, -1, d)
    nr = D.shape[1]
    if rays is None:
        t, idx, t2 = raycast_cells(X, cells, D)
    else:
        t, idx, t2 = rays
        t = _f64(t)
        idx = _i32(idx)
    m = t.size
    wv, wa, we = np.empty(m), np.empty(m), np.empty(m)
    rc = lib.vgo_mc_ray_weights(d, n, _p(X), cells.size, _p(cells), nr, _p(D), _p(t), _p(idx),
                                _p(wv), _p(wa), _p(we))
    assert rc == 0, "ray without a hit in a Monte-Carlo cell"
    S = sphere_area(d)
    volume = S / (d * nr) * wv.reshape(cells.size, nr).sum(axis=1)
    energy2 = S / ((d + 2) * nr) * we.reshape(cells.size, nr).sum(axis=1)
    facets = {}
    cell_of_ray = np.repeat(cells, nr)
    for k in range(m):
        key = (int(cell_of_ray[k]), int(idx[k]))
        facets[key] = facets.get(key, 0.0) + wa[k]
    for key in facets:
        facets[key] *= S / nr
    return dict(volume=volume, energy2=energy2, facets=facets, t=t, idx=idx, t2=t2,
                w_vol=wv, w_area=wa, w_energy=we)


def mc_integrals(nodes, cells, dirs, tsamp, f, rays=None):
    """Integrals of a function ``f`` over the listed cells and their facets,
    following Algorithm 3 (Sec. 3.1) with its inner loop of ``m`` draws:

      F_V[i]  = S/(n m) sum_k sum_s f((1 - t_ks) x_i + t_ks r_k) t_ks^{d-1} l_k^d
      F(i, j) = S/n     sum_{k: j_k = j} f(r_k) l_k^{d-1} / |n_ij . u_k|

    with ``l_k`` = t* of ray k, ``r_k = x_i + l_k u_k`` its hit point and
    ``t_ks = tsamp[c][k][s]`` in (0, 1) (``m = tsamp.shape[-1]``, possibly 0).
    The normalisation S/(n m) is Algorithm 3's: in polar coordinates about
    x_i the volume element is t^{d-1} l^d dt dS with t uniform on (0, 1), so
    no factor 1/d enters (the displayed equation for the integral of f
    carries one; with f = 1 and uniform t both agree only in expectation
    through E[t^{d-1}] = 1/d).
    ``f`` maps a float64 array [P, d] of points to [P] values.  Returns a
    dict with ``F_V`` (per listed cell, None when m = 0), ``F`` (dict
    ``(i, j) -> integral``) and the per-ray ``f_hit``."""
    base = mc_volume_area(nodes, cells, dirs, rays)
    X = _f64(nodes)
    n, d = X.shape
    cells = np.asarray(cells, dtype=np.int64).ravel()
    nc = cells.size
    D = _f64(dirs).reshape(nc, -1, d)
    nr = D.shape[1]
    t = base["t"].reshape(nc, nr)
    xi = X[cells][:, None, :]
    r = xi + t[..., None] * D  # hit points
    f_hit = np.asarray(f(r.reshape(-1, d)), dtype=np.float64).reshape(nc, nr)
    S = sphere_area(d)
    F = {}
    cell_of_ray = np.repeat(cells, nr)
    contrib = (f_hit.ravel() * base["w_area"])
    for k in range(contrib.size):
        key = (int(cell_of_ray[k]), int(base["idx"][k]))
        F[key] = F.get(key, 0.0) + contrib[k]
    for key in F:
        F[key] *= S / nr
    T = np.asarray(tsamp, dtype=np.float64).reshape(nc, nr, -1)
    m = T.shape[2]
    F_V = None
    if m > 0:
        pts = (1.0 - T[..., None]) * xi[:, :, None, :] + T[..., None] * r[:, :, None, :]
        fv = np.asarray(f(pts.reshape(-1, d)), dtype=np.float64).reshape(nc, nr, m)
        F_V = S / (nr * m) * (fv * T ** (d - 1) * (t ** d)[..., None]).sum(axis=(1, 2))
    return dict(F_V=F_V, F=F, f_hit=f_hit, volume=base["volume"], facets=base["facets"],
                t=base["t"], idx=base["idx"], t2=base["t2"], w_area=base["w_area"])


def mc_adjoint(nodes, cells, dirs, t, idx, g_volume=None, g_energy2=None, g_area_ray=None):
    """Closed-form gradient, with respect to all generator positions, of
    ``sum_c g_volume[c] volume_c + g_energy2[c] energy2_c + sum_k g_area_ray[k]
    area-term_k`` with frozen directions.  ``g_area_ray[k]`` is the upstream
    weight of the facet ray ``k`` contributes to.  Returns ``[n][d]`` float64."""
    lib = _load()
    X = _f64(nodes)
    n, d = X.shape
    cells = np.ascontiguousarray(np.asarray(cells, dtype=np.int64).ravel())
    D = _f64(dirs).reshape(cells.size, -1, d)
    nr = D.shape[1]
    grad = np.zeros((n, d))
    gv = None if g_volume is None else _f64(g_volume)
    ge = None if g_energy2 is None else _f64(g_energy2)
    ga = None if g_area_ray is None else _f64(g_area_ray)
    rc = lib.vgo_mc_adjoint(d, n, _p(X), cells.size, _p(cells), nr, _p(D), _p(_f64(t)),
                            _p(_i32(idx)), sphere_area(d), _p(gv), _p(ge), _p(ga), _p(grad))
    assert rc == 0
    return grad
