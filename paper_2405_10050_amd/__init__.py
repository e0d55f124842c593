"""MI355X (gfx950) batched RayCast for the Voronoi Graph method
(Sikorski & Heida, arXiv 2405.10050).

Thin Python binding of ``libvgraph.so`` (C ABI, ``include/vgraph.h``): it
checks tensors, passes device pointers and the current HIP stream, and
allocates outputs with torch.  All arithmetic runs in the library's HIP
kernels; there is no fallback.  Importing this package on a machine without
the built library raises ``ImportError``; calling it without a gfx950 GPU
raises ``VGError``.

Calls (names follow the paper's statement of the problem):
  raycast(nodes, origin, direction, gen, excl, clip)   RayCast of Sec. 2.2
  raycast_cells(nodes, dirs)                           Monte-Carlo rays of every cell
  raycast_cells(nodes, seed=s, rays_per_cell=R)        the same, directions drawn on the device
  dump_dirs(d, n_cells, R, seed)                       those directions, written out
  raycast_cells_noalloc(nodes, dirs, out=...)          raycast_cells with no device allocation
  mc_volume_area(nodes, dirs, neighbors=None)          Sec. 3.1 / Algorithm 3 estimators
  tuple_neighbors(sigma, n)                            cell adjacency from vertex tuples
  mc_integrals(nodes, dirs, res, f, tsamp)             integrals of f over cells and facets
  mc_backward(...), VoronoiMC                          adjoint / autograd Function
  raycast_batched(problems, clip)                      many RayCast problems, one launch
  raycast_cells_batched(problems)                      uneven batch of clouds
  explore(nodes, descent_draws)                        Algorithm 2 (VoronoiGraph)
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvgraph.so")

VG_CLIP = 1 << 0
VG_PREC_BF16X3 = 1 << 1
VG_NO_RECHECK = 1 << 2
VG_INCIRCLE = 1 << 3
VG_INIT_HEURISTIC = 1 << 4
VG_PERIODIC = 1 << 5
VG_SCAN_ORDER = 1 << 6
VG_INDEX_ORDER = 1 << 7

ST_NEAR_TIE = 1
ST_RECHECKED = 2
ST_NO_HIT = 4
ST_SUSPECT = 8
ST_FP64_TIE = 16
ST_BAD_INPUT = 32

MAX_DIM = 16
NOALLOC_MAX_RAYS = 1 << 22


class VGError(RuntimeError):
    pass


class _Stats(ctypes.Structure):
    _fields_ = [("rays", ctypes.c_int64), ("flagged", ctypes.c_int64),
                ("fp64_ties", ctypes.c_int64), ("tie_eps", ctypes.c_double),
                ("scan_launches", ctypes.c_int64), ("scan_ms", ctypes.c_double),
                ("nn_calls", ctypes.c_int64), ("nn_grid_calls", ctypes.c_int64),
                ("bad_input_rays", ctypes.c_int64), ("bad_node_values", ctypes.c_int64),
                ("scan_pairs", ctypes.c_int64)]


class _CellsProblem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("rays_per_cell", ctypes.c_int), ("n_nodes", ctypes.c_int64),
                ("nodes", ctypes.c_void_p), ("dirs", ctypes.c_void_p), ("t_out", ctypes.c_void_p),
                ("idx_out", ctypes.c_void_p), ("status_out", ctypes.c_void_p)]


class _RaysProblem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("n_excl", ctypes.c_int), ("n_nodes", ctypes.c_int64),
                ("nodes", ctypes.c_void_p), ("n_rays", ctypes.c_int64), ("origin", ctypes.c_void_p),
                ("dir", ctypes.c_void_p), ("gen", ctypes.c_void_p), ("excl", ctypes.c_void_p),
                ("t_out", ctypes.c_void_p), ("idx_out", ctypes.c_void_p),
                ("status_out", ctypes.c_void_p)]


EXPORTS = (
    "vg_create", "vg_destroy", "vg_set_stream", "vg_last_error", "vg_get_stats",
    "vg_set_profiling", "vg_raycast",
    "vg_raycast_cells", "vg_mc_volume_area", "vg_mc_backward", "vg_raycast_cells_batched",
    "vg_raycast_batched", "vg_mc_volume_area_nbr", "vg_tuple_neighbors", "vg_mc_sample_points",
    "vg_mc_integrals", "vg_hmc_centroids", "vg_hmc_integrals",
    "vg_explore", "vg_mesh_num_vertices", "vg_mesh_num_unbounded", "vg_mesh_num_raycasts",
    "vg_mesh_copy", "vg_mesh_free", "vg_mesh_num_nn_calls", "vg_raycast_cells_noalloc",
    "vg_raycast_cells_seeded", "vg_mc_volume_area_seeded", "vg_mc_backward_seeded", "vg_dump_dirs",
    "vg_peak_rate", "vg_raycast_f64",
)


def _load_lib():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                          "python paper_2405_10050_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, I64, U32, U64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    lib.vg_create.argtypes = [I, ctypes.POINTER(P)]
    lib.vg_destroy.argtypes = [P]
    lib.vg_destroy.restype = None
    lib.vg_set_stream.argtypes = [P, P]
    lib.vg_last_error.argtypes = [P]
    lib.vg_last_error.restype = ctypes.c_char_p
    lib.vg_get_stats.argtypes = [P, ctypes.POINTER(_Stats)]
    lib.vg_set_profiling.argtypes = [P, I]
    lib.vg_raycast.argtypes = [P, I, I64, P, I64, P, P, P, P, I, U32, P, P, P]
    lib.vg_raycast_f64.argtypes = [P, I, I64, P, I64, P, P, P, P, I, U32, P, P, P]
    lib.vg_raycast_cells.argtypes = [P, I, I64, P, I, P, U32, P, P, P]
    lib.vg_raycast_cells_noalloc.argtypes = [P, I, I64, P, I, P, U32, P, P, P]
    lib.vg_raycast_cells_seeded.argtypes = [P, I, I64, P, I, U64, U32, P, P, P]
    lib.vg_mc_volume_area_seeded.argtypes = [P, I, I64, P, I, U64, U32, P, P, P, P, P, P, P, P]
    lib.vg_mc_backward_seeded.argtypes = [P, I, I64, P, I, U64, P, P, P, P, P, P, P, P]
    lib.vg_dump_dirs.argtypes = [P, I, I64, I64, I, U64, P]
    lib.vg_peak_rate.argtypes = [P, I, ctypes.POINTER(ctypes.c_double)]
    lib.vg_mc_volume_area.argtypes = [P, I, I64, P, I, P, U32, P, P, P, P, P, P, P, P]
    lib.vg_mc_backward.argtypes = [P, I, I64, P, I, P, P, P, P, P, P, P, P, P]
    lib.vg_raycast_cells_batched.argtypes = [P, I, ctypes.POINTER(_CellsProblem), U32]
    lib.vg_raycast_batched.argtypes = [P, I, ctypes.POINTER(_RaysProblem), U32]
    lib.vg_mc_volume_area_nbr.argtypes = [P, I, I64, P, P, P, I, P, U32, P, P, P, P, P, P, P, P]
    lib.vg_tuple_neighbors.argtypes = [P, I, I64, I64, P, P, P, I64, ctypes.POINTER(I64)]
    lib.vg_mc_sample_points.argtypes = [P, I, I64, P, I, P, P, I, P, P]
    lib.vg_mc_integrals.argtypes = [P, I, I64, P, I, P, P, I, P, P, P, P, P, P]
    lib.vg_hmc_centroids.argtypes = [P, I, I64, P, I64, P, P, I, P, P, P, P]
    lib.vg_hmc_integrals.argtypes = [P, I, I64, P, I64, P, P, I, P, P, P, P, P, P, P, P]
    lib.vg_explore.argtypes = [P, I, I64, P, P, I, U32, ctypes.POINTER(P)]
    for f in ("vg_mesh_num_vertices", "vg_mesh_num_unbounded", "vg_mesh_num_raycasts", "vg_mesh_num_nn_calls"):
        getattr(lib, f).argtypes = [P]
        getattr(lib, f).restype = I64
    lib.vg_mesh_copy.argtypes = [P, P, P, P, P]
    lib.vg_mesh_free.argtypes = [P]
    lib.vg_mesh_free.restype = None
    return lib


_lib = _load_lib()
_ctxs: dict[int, ctypes.c_void_p] = {}


def _ctx(device: torch.device) -> ctypes.c_void_p:
    idx = device.index if device.index is not None else torch.cuda.current_device()
    c = _ctxs.get(idx)
    if c is None:
        c = ctypes.c_void_p()
        rc = _lib.vg_create(idx, ctypes.byref(c))
        if rc != 0:
            raise VGError(f"vg_create(device={idx}) failed with {rc}: no gfx950 device")
        _ctxs[idx] = c
    _lib.vg_set_stream(c, ctypes.c_void_p(torch.cuda.current_stream(idx).cuda_stream))
    return c


def _check(rc: int, ctx, what: str):
    if rc != 0:
        msg = _lib.vg_last_error(ctx).decode()
        raise VGError(f"{what} failed ({rc}): {msg}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev(t, dtype, name, device=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if not t.is_cuda:
        raise VGError(f"{name} must be a GPU tensor (no CPU path)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return t


def stats(device=None) -> dict:
    """Counters of the last raycast-type call on ``device`` (synchronises)."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    c = _ctx(dev)
    s = _Stats()
    _check(_lib.vg_get_stats(c, ctypes.byref(s)), c, "vg_get_stats")
    return dict(rays=s.rays, flagged=s.flagged, fp64_ties=s.fp64_ties, tie_eps=s.tie_eps,
                scan_launches=s.scan_launches, scan_ms=s.scan_ms, nn_calls=s.nn_calls,
                nn_grid_calls=s.nn_grid_calls, bad_input_rays=s.bad_input_rays,
                bad_node_values=s.bad_node_values, scan_pairs=s.scan_pairs)


def peak_rates(device=None) -> dict:
    """Measured FLOP/s of the FP32 MFMA, BF16 MFMA and FP64 vector-FMA pipes
    (short issue-bound kernels; synchronises)."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    c = _ctx(dev)
    out = {}
    for kind, name in enumerate(("fp32_mfma", "bf16_mfma", "fp64_fma")):
        v = ctypes.c_double(0.0)
        _check(_lib.vg_peak_rate(c, kind, ctypes.byref(v)), c, "vg_peak_rate")
        out[name] = v.value
    return out


def set_profiling(enable: bool, device=None) -> None:
    """Time every candidate-scan kernel with HIP events on the current stream
    (read back through ``stats()``); ``False`` stops and clears."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    c = _ctx(dev)
    _check(_lib.vg_set_profiling(c, int(bool(enable))), c, "vg_set_profiling")


def raycast(nodes, origin, direction, gen, excl=None, clip=True, recheck=True, incircle=False,
            heuristic=False):
    """RayCast of arbitrary rays; returns ``(t, idx, status)`` of length M.
    ``incircle=True`` casts them by Algorithm 1 with a grid index (d <= 6),
    ``heuristic=True`` starting from InitialHeuristic's point.  Float64
    ``origin`` and ``direction`` take the FP64-origin path (vg_raycast_f64,
    which synchronises)."""
    _dev(nodes, torch.float32, "nodes")
    dev = nodes.device
    n, d = nodes.shape
    f64 = isinstance(origin, torch.Tensor) and origin.dtype == torch.float64
    _dev(origin, torch.float64 if f64 else torch.float32, "origin", dev)
    _dev(direction, torch.float64 if f64 else torch.float32, "direction", dev)
    _dev(gen, torch.int32, "gen", dev)
    m = origin.shape[0]
    if origin.shape != (m, d) or direction.shape != (m, d) or gen.shape != (m,):
        raise ValueError("origin/direction must be [M, d] and gen [M]")
    ne = 0
    if excl is not None:
        _dev(excl, torch.int32, "excl", dev)
        if excl.dim() != 2 or excl.shape[0] != m:
            raise ValueError("excl must be [M, n_excl]")
        ne = excl.shape[1]
    t = torch.empty(m, dtype=torch.float32, device=dev)
    idx = torch.empty(m, dtype=torch.int32, device=dev)
    st = torch.empty(m, dtype=torch.uint8, device=dev)
    flags = ((VG_CLIP if clip else 0) | (0 if recheck else VG_NO_RECHECK) |
             (VG_INCIRCLE if incircle else 0) | (VG_INIT_HEURISTIC if heuristic else 0))
    c = _ctx(dev)
    if f64:
        if not recheck:
            raise ValueError("the FP64-origin path always rechecks")
        _check(_lib.vg_raycast_f64(c, d, n, _ptr(nodes), m, _ptr(origin), _ptr(direction), _ptr(gen),
                                   _ptr(excl), ne, flags, _ptr(t), _ptr(idx), _ptr(st)), c, "vg_raycast_f64")
        return t, idx, st
    _check(_lib.vg_raycast(c, d, n, _ptr(nodes), m, _ptr(origin), _ptr(direction), _ptr(gen),
                           _ptr(excl), ne, flags, _ptr(t), _ptr(idx), _ptr(st)), c, "vg_raycast")
    return t, idx, st


def _cells_flags(precision: str, recheck: bool, incircle: bool = False, order=None) -> int:
    if precision not in ("fp32", "bf16x3"):
        raise ValueError("precision must be 'fp32' or 'bf16x3'")
    if order not in (None, "scan", "index"):
        raise ValueError("order must be None, 'scan' or 'index'")
    return ((VG_PREC_BF16X3 if precision == "bf16x3" else 0) | (0 if recheck else VG_NO_RECHECK) |
            (VG_INCIRCLE if incircle else 0) | (VG_SCAN_ORDER if order == "scan" else 0) |
            (VG_INDEX_ORDER if order == "index" else 0))


def _rays_per_cell(dirs, n, d, dev, seed, rays_per_cell):
    """R of a call: from ``dirs`` [N, R, d], or ``rays_per_cell`` when the
    directions are drawn on the device from ``seed`` (``dirs`` None)."""
    if dirs is None:
        if seed is None or rays_per_cell is None:
            raise ValueError("without dirs, give seed and rays_per_cell (directions drawn on the device)")
        return int(rays_per_cell)
    _dev(dirs, torch.float32, "dirs", dev)
    if dirs.dim() != 3 or dirs.shape[0] != n or dirs.shape[2] != d:
        raise ValueError("dirs must be [N, R, d]")
    return dirs.shape[1]


def raycast_cells(nodes, dirs=None, precision="fp32", recheck=True, incircle=False, seed=None,
                  rays_per_cell=None, order=None):
    """Monte-Carlo rays of every cell: ``dirs`` is ``[N, R, d]``, or None with
    ``seed`` and ``rays_per_cell``: the directions are then drawn on the
    device (Philox4x32-10, see :func:`dump_dirs`) and never stored.
    ``order`` = "scan" / "index" forces the node order of the dense scan
    (default: scan order, with exact block skipping, for d <= 12 in FP32 and
    d <= 10 in BF16x3).  Returns
    ``(t, idx, status)`` shaped ``[N, R]``."""
    _dev(nodes, torch.float32, "nodes")
    dev = nodes.device
    n, d = nodes.shape
    R = _rays_per_cell(dirs, n, d, dev, seed, rays_per_cell)
    t = torch.empty((n, R), dtype=torch.float32, device=dev)
    idx = torch.empty((n, R), dtype=torch.int32, device=dev)
    st = torch.empty((n, R), dtype=torch.uint8, device=dev)
    c = _ctx(dev)
    flags = _cells_flags(precision, recheck, incircle, order)
    if dirs is None:
        _check(_lib.vg_raycast_cells_seeded(c, d, n, _ptr(nodes), R, int(seed) & (2 ** 64 - 1), flags,
                                            _ptr(t), _ptr(idx), _ptr(st)), c, "vg_raycast_cells_seeded")
    else:
        _check(_lib.vg_raycast_cells(c, d, n, _ptr(nodes), R, _ptr(dirs), flags, _ptr(t), _ptr(idx), _ptr(st)),
               c, "vg_raycast_cells")
    return t, idx, st


def dump_dirs(d, n_cells, rays_per_cell, seed, first_cell=0, device=None):
    """The directions the seeded calls draw for cells ``first_cell ..
    first_cell + n_cells - 1``, as a ``[n_cells, rays_per_cell, d]`` float32
    GPU tensor (bit for bit those of the kernels)."""
    dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
    out = torch.empty((n_cells, rays_per_cell, d), dtype=torch.float32, device=dev)
    c = _ctx(dev)
    _check(_lib.vg_dump_dirs(c, d, first_cell, n_cells, rays_per_cell, int(seed) & (2 ** 64 - 1), _ptr(out)),
           c, "vg_dump_dirs")
    return out


def raycast_cells_noalloc(nodes, dirs, precision="fp32", recheck=True, out=None):
    """:func:`raycast_cells` through the library's allocation-free entry
    point (its recheck queue and counters live in a fixed device array of
    the library; ``N * R <= NOALLOC_MAX_RAYS``).  ``out`` may pass
    preallocated ``(t, idx, status)`` ``[N, R]`` tensors (status may be
    None), so that the call itself allocates nothing."""
    _dev(nodes, torch.float32, "nodes")
    dev = nodes.device
    n, d = nodes.shape
    _dev(dirs, torch.float32, "dirs", dev)
    if dirs.dim() != 3 or dirs.shape[0] != n or dirs.shape[2] != d:
        raise ValueError("dirs must be [N, R, d]")
    R = dirs.shape[1]
    if out is None:
        out = (torch.empty((n, R), dtype=torch.float32, device=dev),
               torch.empty((n, R), dtype=torch.int32, device=dev),
               torch.empty((n, R), dtype=torch.uint8, device=dev))
    t, idx, st = out
    _dev(t, torch.float32, "t", dev)
    _dev(idx, torch.int32, "idx", dev)
    if st is not None:
        _dev(st, torch.uint8, "status", dev)
    if t.shape != (n, R) or idx.shape != (n, R) or (st is not None and st.shape != (n, R)):
        raise ValueError("out must hold [N, R] tensors")
    c = _ctx(dev)
    _check(_lib.vg_raycast_cells_noalloc(c, d, n, _ptr(nodes), R, _ptr(dirs), _cells_flags(precision, recheck),
                                         _ptr(t), _ptr(idx), _ptr(st)), c, "vg_raycast_cells_noalloc")
    return t, idx, st


@dataclass
class MCResult:
    volume: torch.Tensor       # [N]
    energy2: torch.Tensor      # [N]
    facet_j: torch.Tensor      # [N, R] (first facet_count[i] entries of row i)
    facet_area: torch.Tensor   # [N, R]
    facet_count: torch.Tensor  # [N]
    t: torch.Tensor            # [N, R]
    idx: torch.Tensor          # [N, R]
    status: torch.Tensor       # [N, R]
    seed: int | None = None    # directions drawn on the device from this seed (dirs None)

    def facets_coo(self):
        """Facets as host COO arrays ``(i, j, area)`` sorted by (i, j)."""
        cnt = self.facet_count.cpu().numpy()
        R = self.facet_j.shape[1]
        mask = np.arange(R)[None, :] < cnt[:, None]
        i = np.nonzero(mask)[0].astype(np.int32)
        return i, self.facet_j.cpu().numpy()[mask], self.facet_area.cpu().numpy()[mask]


def mc_volume_area(nodes, dirs=None, precision="fp32", facets=True, recheck=True, out=None,
                   neighbors=None, incircle=False, seed=None, rays_per_cell=None, order=None) -> MCResult:
    """Monte-Carlo cell volumes, second moments and interface areas
    (Sec. 3.1, Algorithm 3 with f = 1).  ``out`` may pass a previous
    ``MCResult`` of the same shape to reuse its buffers.  ``neighbors`` =
    ``(offsets [N+1] int64, nbr [nnz] int32)`` (e.g. from
    :func:`tuple_neighbors`) restricts each cell's scan to its neighbours;
    ``incircle=True`` casts the rays by Algorithm 1 with a grid index
    (d <= 6, FP32) instead of the dense scan.  ``dirs=None`` with ``seed``
    and ``rays_per_cell`` draws the directions on the device (no
    neighbours or incircle then)."""
    _dev(nodes, torch.float32, "nodes")
    dev = nodes.device
    n, d = nodes.shape
    R = _rays_per_cell(dirs, n, d, dev, seed, rays_per_cell)
    if out is None:
        out = MCResult(
            volume=torch.empty(n, dtype=torch.float32, device=dev),
            energy2=torch.empty(n, dtype=torch.float32, device=dev),
            facet_j=torch.empty((n, R), dtype=torch.int32, device=dev) if facets else None,
            facet_area=torch.empty((n, R), dtype=torch.float32, device=dev) if facets else None,
            facet_count=torch.empty(n, dtype=torch.int32, device=dev) if facets else None,
            t=torch.empty((n, R), dtype=torch.float32, device=dev),
            idx=torch.empty((n, R), dtype=torch.int32, device=dev),
            status=torch.empty((n, R), dtype=torch.uint8, device=dev))
    out.seed = int(seed) if dirs is None else None
    c = _ctx(dev)
    if dirs is None:
        if neighbors is not None:
            raise ValueError("neighbour lists need dirs")
        _check(_lib.vg_mc_volume_area_seeded(c, d, n, _ptr(nodes), R, int(seed) & (2 ** 64 - 1),
                                             _cells_flags(precision, recheck, incircle, order),
                                             _ptr(out.t), _ptr(out.idx), _ptr(out.status), _ptr(out.volume),
                                             _ptr(out.energy2), _ptr(out.facet_j), _ptr(out.facet_area),
                                             _ptr(out.facet_count)), c, "vg_mc_volume_area_seeded")
        return out
    if neighbors is None:
        _check(_lib.vg_mc_volume_area(c, d, n, _ptr(nodes), R, _ptr(dirs),
                                      _cells_flags(precision, recheck, incircle, order),
                                      _ptr(out.t), _ptr(out.idx), _ptr(out.status), _ptr(out.volume),
                                      _ptr(out.energy2), _ptr(out.facet_j), _ptr(out.facet_area),
                                      _ptr(out.facet_count)), c, "vg_mc_volume_area")
        return out
    off, nbr = neighbors
    _dev(off, torch.int64, "neighbor offsets", dev)
    _dev(nbr, torch.int32, "neighbor list", dev)
    if off.shape != (n + 1,) or nbr.dim() != 1:
        raise ValueError("neighbors must be (offsets [N+1], nbr [nnz])")
    _check(_lib.vg_mc_volume_area_nbr(c, d, n, _ptr(nodes), _ptr(off), _ptr(nbr), R, _ptr(dirs),
                                      _cells_flags(precision, recheck, incircle, order), _ptr(out.t), _ptr(out.idx),
                                      _ptr(out.status), _ptr(out.volume), _ptr(out.energy2),
                                      _ptr(out.facet_j), _ptr(out.facet_area), _ptr(out.facet_count)),
           c, "vg_mc_volume_area_nbr")
    return out


def tuple_neighbors(sigma, n_nodes):
    """Cell adjacency from Voronoi vertex tuples: ``sigma`` is a device int32
    tensor ``[V, d+1]`` (e.g. ``explore(...)["sigma"]`` moved to the GPU).
    Returns device tensors ``(offsets [n_nodes+1] int64, nbr [nnz] int32)``;
    row i lists, ascending, every generator that shares a vertex with i."""
    _dev(sigma, torch.int32, "sigma")
    if sigma.dim() != 2:
        raise ValueError("sigma must be [V, d+1]")
    dev = sigma.device
    V, L = sigma.shape
    off = torch.empty(n_nodes + 1, dtype=torch.int64, device=dev)
    cap = max(V * L * (L - 1), 1)
    nbr = torch.empty(cap, dtype=torch.int32, device=dev)
    nnz = ctypes.c_int64(0)
    c = _ctx(dev)
    _check(_lib.vg_tuple_neighbors(c, L - 1, n_nodes, V, _ptr(sigma), _ptr(off), _ptr(nbr), cap,
                                   ctypes.byref(nnz)), c, "vg_tuple_neighbors")
    return off, nbr[:nnz.value].clone()


@dataclass
class MCIntegrals:
    volume: torch.Tensor | None  # [N] integral of f over each cell (None without draws)
    facet_j: torch.Tensor        # [N, R] facet rows, as in MCResult
    facet: torch.Tensor          # [N, R] integral of f over each facet of the row
    facet_count: torch.Tensor    # [N]


def mc_integrals(nodes, dirs, res: MCResult, f, tsamp=None) -> MCIntegrals:
    """Integrals of ``f`` over every cell and facet (Algorithm 3, Sec. 3.1),
    from a forward result ``res`` of :func:`mc_volume_area` on the same
    ``dirs``.  ``f`` maps a float32 GPU tensor ``[P, d]`` of points to ``[P]``
    values; it is the integrand, called once between the library's two calls
    (sample points, then the weighted sums).  ``tsamp`` ``[N, R, m]`` float32
    in (0, 1) holds the draws of the inner loop (None: facet integrals
    only)."""
    _dev(nodes, torch.float32, "nodes")
    dev = nodes.device
    n, d = nodes.shape
    _dev(dirs, torch.float32, "dirs", dev)
    R = dirs.shape[1]
    if dirs.shape != (n, R, d) or res.t.shape != (n, R):
        raise ValueError("dirs must be [N, R, d] and res the forward result on them")
    m = 0
    if tsamp is not None:
        _dev(tsamp, torch.float32, "tsamp", dev)
        if tsamp.dim() != 3 or tsamp.shape[:2] != (n, R):
            raise ValueError("tsamp must be [N, R, m]")
        m = tsamp.shape[2]
    points = torch.empty((n, R, m + 1, d), dtype=torch.float32, device=dev)
    c = _ctx(dev)
    _check(_lib.vg_mc_sample_points(c, d, n, _ptr(nodes), R, _ptr(dirs), _ptr(res.t), m, _ptr(tsamp),
                                    _ptr(points)), c, "vg_mc_sample_points")
    fvals = f(points.view(-1, d))
    if not isinstance(fvals, torch.Tensor) or fvals.numel() != n * R * (m + 1):
        raise ValueError("f must return one value per point")
    fvals = fvals.to(device=dev, dtype=torch.float32).contiguous()
    out = MCIntegrals(
        volume=torch.empty(n, dtype=torch.float32, device=dev) if m > 0 else None,
        facet_j=torch.empty((n, R), dtype=torch.int32, device=dev),
        facet=torch.empty((n, R), dtype=torch.float32, device=dev),
        facet_count=torch.empty(n, dtype=torch.int32, device=dev))
    c = _ctx(dev)
    _check(_lib.vg_mc_integrals(c, d, n, _ptr(nodes), R, _ptr(res.t), _ptr(res.idx), m, _ptr(tsamp),
                                _ptr(fvals), _ptr(out.volume), _ptr(out.facet_j), _ptr(out.facet),
                                _ptr(out.facet_count)), c, "vg_mc_integrals")
    return out


@dataclass
class HMCResult:
    cell: torch.Tensor       # [N] heuristic integral of f over each cell
    volume: torch.Tensor     # [N] volume from the areas, sum_j h_ij A_ij / d
    facet: torch.Tensor      # [N, R] integral of f over each facet row of the forward result
    centroid: torch.Tensor   # [N, R, d] centroid of each facet's vertices
    kcount: torch.Tensor     # [N, R] number of those vertices


def hmc_integrals(nodes, mesh, res: MCResult, f) -> HMCResult:
    """Heuristic Monte-Carlo integrals of ``f`` (Sec. 3.3): the facet
    integrals from the vertices of each facet of the clipped diagram
    (``mesh`` = :func:`explore` with ``clip=True``) and its Monte-Carlo area
    in ``res`` (:func:`mc_volume_area`), and the cell integrals by the
    pyramid rule over the facets.  ``f`` maps float32 GPU points ``[P, d]``
    to ``[P]``; it is called on the vertices, the facet centroids and the
    generators."""
    _dev(nodes, torch.float32, "nodes")
    dev = nodes.device
    n, d = nodes.shape
    R = res.facet_j.shape[1]
    sig = torch.from_numpy(np.ascontiguousarray(mesh["sigma"], dtype=np.int32)).to(dev)
    coord = torch.from_numpy(np.ascontiguousarray(mesh["coord"], dtype=np.float64)).to(dev)
    V = sig.shape[0]
    if sig.shape != (V, d + 1) or coord.shape != (V, d):
        raise ValueError("mesh must hold sigma [V, d+1] and coord [V, d]")
    centroid = torch.empty((n, R, d), dtype=torch.float32, device=dev)
    kcount = torch.empty((n, R), dtype=torch.int32, device=dev)
    c = _ctx(dev)
    _check(_lib.vg_hmc_centroids(c, d, n, _ptr(nodes), V, _ptr(sig), _ptr(coord), R, _ptr(res.facet_j),
                                 _ptr(res.facet_count), _ptr(centroid), _ptr(kcount)), c, "vg_hmc_centroids")

    def values(p, count):
        v = f(p)
        if not isinstance(v, torch.Tensor) or v.numel() != count:
            raise ValueError("f must return one value per point")
        return v.to(device=dev, dtype=torch.float32).contiguous()

    fv = values(coord.to(torch.float32), V)
    fc = values(centroid.view(-1, d), n * R)
    fx = values(nodes, n)
    out = HMCResult(cell=torch.empty(n, dtype=torch.float32, device=dev),
                    volume=torch.empty(n, dtype=torch.float32, device=dev),
                    facet=torch.empty((n, R), dtype=torch.float32, device=dev),
                    centroid=centroid, kcount=kcount)
    _check(_lib.vg_hmc_integrals(c, d, n, _ptr(nodes), V, _ptr(sig), _ptr(fv), R, _ptr(res.facet_j),
                                 _ptr(res.facet_area), _ptr(res.facet_count), _ptr(fc), _ptr(fx),
                                 _ptr(out.facet), _ptr(out.cell), _ptr(out.volume)), c, "vg_hmc_integrals")
    return out


def mc_backward(nodes, dirs, res: MCResult, g_volume=None, g_energy2=None, g_facet_area=None, out=None):
    """Gradient with respect to the generator positions of
    ``<g_volume, volume> + <g_energy2, energy2> + <g_facet_area, facet_area>``
    with the directions frozen.  ``dirs=None``: the forward drew them on the
    device (``res.seed``).  Returns ``[N, d]`` float32 (written into ``out``
    when given)."""
    _dev(nodes, torch.float32, "nodes")
    dev = nodes.device
    n, d = nodes.shape
    R = res.t.shape[1]
    if dirs is None and res.seed is None:
        raise ValueError("dirs is None but the forward result has no seed")
    if dirs is not None and dirs.shape != (n, R, d):
        raise ValueError("dirs must be [N, R, d]")
    for name, g in (("g_volume", g_volume), ("g_energy2", g_energy2)):
        if g is not None:
            _dev(g, torch.float32, name, dev)
            if g.shape != (n,):
                raise ValueError(f"{name} must be [N]")
    if g_facet_area is not None:
        _dev(g_facet_area, torch.float32, "g_facet_area", dev)
        if g_facet_area.shape != (n, R) or res.facet_j is None:
            raise ValueError("g_facet_area must be [N, R] and the forward must have facets")
    if out is not None:
        _dev(out, torch.float32, "out", dev)
        if out.shape != (n, d):
            raise ValueError("out must be [N, d]")
    grad = out if out is not None else torch.empty((n, d), dtype=torch.float32, device=dev)
    c = _ctx(dev)
    if dirs is None:
        _check(_lib.vg_mc_backward_seeded(c, d, n, _ptr(nodes), R, res.seed & (2 ** 64 - 1), _ptr(res.t),
                                          _ptr(res.idx), _ptr(res.facet_j), _ptr(res.facet_count),
                                          _ptr(g_volume), _ptr(g_energy2), _ptr(g_facet_area), _ptr(grad)),
               c, "vg_mc_backward_seeded")
        return grad
    _check(_lib.vg_mc_backward(c, d, n, _ptr(nodes), R, _ptr(dirs), _ptr(res.t), _ptr(res.idx),
                               _ptr(res.facet_j), _ptr(res.facet_count), _ptr(g_volume),
                               _ptr(g_energy2), _ptr(g_facet_area), _ptr(grad)), c, "vg_mc_backward")
    return grad


class VoronoiMC(torch.autograd.Function):
    """``(volume, energy2, facet_area) = VoronoiMC.apply(nodes, dirs)``, or
    ``VoronoiMC.apply(nodes, None, precision, seed, rays_per_cell)`` with the
    directions drawn on the device.

    The forward is ``mc_volume_area``; the backward is the closed-form adjoint
    through the winning bisectors (``mc_backward``), directions frozen.
    ``facet_area[i, :facet_count[i]]`` are the areas of cell i's facets; the
    facet ids are available from ``VoronoiMC.last_result``."""

    last_result: MCResult | None = None

    @staticmethod
    def forward(ctx, nodes, dirs, precision="fp32", seed=None, rays_per_cell=None):
        res = mc_volume_area(nodes.detach().contiguous(), dirs, precision=precision, facets=True, seed=seed,
                             rays_per_cell=rays_per_cell)
        ctx.save_for_backward(nodes, dirs if dirs is not None else nodes.new_empty(0))
        ctx.seeded = dirs is None
        ctx.res = res
        VoronoiMC.last_result = res
        return res.volume, res.energy2, res.facet_area

    @staticmethod
    def backward(ctx, g_volume, g_energy2, g_facet_area):
        nodes, dirs = ctx.saved_tensors
        f = lambda g: None if g is None else g.contiguous().float()
        grad = mc_backward(nodes.detach().contiguous(), None if ctx.seeded else dirs, ctx.res, f(g_volume),
                           f(g_energy2), f(g_facet_area))
        return grad, None, None, None, None


def raycast_cells_batched(problems, precision="fp32", out=None, order=None):
    """Uneven batch in persistent launches (one per register class of d,
    captured into one graph): ``problems`` is
    a list of ``(nodes [N_c, d_c], dirs [N_c, R_c, d_c])``.  Returns a list of
    ``(t, idx, status)`` shaped ``[N_c, R_c]``; ``out`` may pass a previous
    result of the same batch to reuse its buffers (a repeated call on the same
    buffers replays the captured graph)."""
    probs = (_CellsProblem * len(problems))()
    outs = []
    dev = None
    for q, (nodes, dirs) in enumerate(problems):
        _dev(nodes, torch.float32, "nodes")
        dev = nodes.device if dev is None else dev
        _dev(dirs, torch.float32, "dirs", dev)
        n, d = nodes.shape
        R = dirs.shape[1]
        if dirs.shape != (n, R, d):
            raise ValueError("dirs must be [N, R, d]")
        if out is not None:
            t, idx, st = out[q]
            if t.shape != (n, R) or idx.shape != (n, R) or st.shape != (n, R):
                raise ValueError("out does not match the batch")
        else:
            t = torch.empty((n, R), dtype=torch.float32, device=dev)
            idx = torch.empty((n, R), dtype=torch.int32, device=dev)
            st = torch.empty((n, R), dtype=torch.uint8, device=dev)
        outs.append((t, idx, st))
        probs[q] = _CellsProblem(d, R, n, nodes.data_ptr(), dirs.data_ptr(), t.data_ptr(),
                                 idx.data_ptr(), st.data_ptr())
    if not problems:
        return outs
    c = _ctx(dev)
    _check(_lib.vg_raycast_cells_batched(c, len(problems), probs, _cells_flags(precision, True, order=order)),
           c, "vg_raycast_cells_batched")
    return outs


def raycast_batched(problems, clip=True, out=None):
    """Many independent RayCast problems in one persistent (graph-captured)
    launch plus one FP64 recheck.  ``problems`` is a list of tuples
    ``(nodes [N, d], origin [M, d], direction [M, d], gen [M], excl [M, n_excl]
    or None)``, each as in :func:`raycast` (problems may differ in d, N, M and
    n_excl).  Returns a list of ``(t, idx, status)`` of length M; ``out`` may
    pass a previous result of the same batch to reuse its buffers (a repeated
    call on the same buffers replays the captured graph)."""
    probs = (_RaysProblem * len(problems))()
    outs = []
    dev = None
    for q, pr in enumerate(problems):
        nodes, origin, direction, gen = pr[:4]
        excl = pr[4] if len(pr) > 4 else None
        _dev(nodes, torch.float32, "nodes")
        dev = nodes.device if dev is None else dev
        if nodes.device != dev:
            raise ValueError("all problems must be on one device")
        n, d = nodes.shape
        _dev(origin, torch.float32, "origin", dev)
        _dev(direction, torch.float32, "direction", dev)
        _dev(gen, torch.int32, "gen", dev)
        m = origin.shape[0]
        if origin.shape != (m, d) or direction.shape != (m, d) or gen.shape != (m,):
            raise ValueError("origin/direction must be [M, d] and gen [M]")
        ne = 0
        if excl is not None:
            _dev(excl, torch.int32, "excl", dev)
            if excl.dim() != 2 or excl.shape[0] != m:
                raise ValueError("excl must be [M, n_excl]")
            ne = excl.shape[1]
        if out is not None:
            t, idx, st = out[q]
            if t.shape != (m,) or idx.shape != (m,) or st.shape != (m,):
                raise ValueError("out does not match the batch")
        else:
            t = torch.empty(m, dtype=torch.float32, device=dev)
            idx = torch.empty(m, dtype=torch.int32, device=dev)
            st = torch.empty(m, dtype=torch.uint8, device=dev)
        outs.append((t, idx, st))
        probs[q] = _RaysProblem(d, ne, n, nodes.data_ptr(), m, origin.data_ptr(),
                                direction.data_ptr(), gen.data_ptr(),
                                excl.data_ptr() if excl is not None else None,
                                t.data_ptr(), idx.data_ptr(), st.data_ptr())
    if not problems:
        return outs
    c = _ctx(dev)
    _check(_lib.vg_raycast_batched(c, len(problems), probs, VG_CLIP if clip else 0), c,
           "vg_raycast_batched")
    return outs


def explore(nodes, descent_draws=None, clip=False, incircle=False, heuristic=False, periodic=False) -> dict:
    """Exhaustive search (Algorithm 2) of the unbounded diagram, or with
    ``clip=True`` of the diagram clipped to the unit cube (keys then hold
    ``n + 2k + s`` for the face ``x_k = s``; no draws needed).  With
    ``incircle=True`` (d <= 6) the edge rays are cast by Algorithm 1 with a
    grid index (``heuristic``: from InitialHeuristic's point) and
    ``nn_calls`` counts its queries.  Returns host arrays ``sigma [V, d+1]``,
    ``coord [V, d]`` (float64), ``b_sigma``, ``b_omit``, ``raycasts`` and
    ``nn_calls``.

    ``periodic=True`` (d <= 8, nodes in [0,1)^d) searches the periodic
    diagram (the torus R^d / Z^d): key entries are node images
    ``x_i + k`` coded ``i * 3^d + c(k)`` with ``c(k) = sum_a (k_a+1) 3^a``,
    each key translated so that its first (smallest) node has ``k = 0`` and
    ``coord`` in that frame.  The result then also holds ``key`` (the codes)
    with ``sigma`` the node indices and ``shift [V, d+1, d]`` int8 the
    ``k`` decoded from it."""
    _dev(nodes, torch.float32, "nodes")
    n, d = nodes.shape
    if descent_draws is None:
        draws = np.zeros((0, d))
    else:
        draws = np.ascontiguousarray(np.asarray(descent_draws, dtype=np.float64).reshape(-1, d))
    c = _ctx(nodes.device)
    mesh = ctypes.c_void_p()
    _check(_lib.vg_explore(c, d, n, _ptr(nodes), draws.ctypes.data_as(ctypes.c_void_p) if draws.size else None,
                           draws.shape[0],
                           (VG_CLIP if clip else 0) | (VG_INCIRCLE if incircle else 0) |
                           (VG_INIT_HEURISTIC if heuristic else 0) | (VG_PERIODIC if periodic else 0),
                           ctypes.byref(mesh)), c, "vg_explore")
    try:
        nv = _lib.vg_mesh_num_vertices(mesh)
        nb = _lib.vg_mesh_num_unbounded(mesh)
        sig = np.empty((nv, d + 1), dtype=np.int32)
        coord = np.empty((nv, d), dtype=np.float64)
        bsig = np.empty((nb, d + 1), dtype=np.int32)
        bomit = np.empty(nb, dtype=np.int32)
        P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        _check(_lib.vg_mesh_copy(mesh, P(sig), P(coord), P(bsig), P(bomit)), c, "vg_mesh_copy")
        out = dict(sigma=sig, coord=coord, b_sigma=bsig, b_omit=bomit,
                   raycasts=int(_lib.vg_mesh_num_raycasts(mesh)),
                   nn_calls=int(_lib.vg_mesh_num_nn_calls(mesh)))
        if periodic:
            S = 3 ** d
            key = sig.astype(np.int64)
            out["key"] = sig
            out["sigma"] = (key // S).astype(np.int32)
            out["shift"] = np.stack([(key % S) // 3 ** a % 3 - 1 for a in range(d)], axis=-1).astype(np.int8)
        return out
    finally:
        _lib.vg_mesh_free(mesh)
