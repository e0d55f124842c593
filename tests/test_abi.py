"""The C-ABI library loads on the host and exports every function that
include/vgraph.h declares (no compute call: this runs without a GPU)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vgraph.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("vg_create", "vg_raycast", "vg_raycast_cells", "vg_mc_volume_area",
                 "vg_mc_backward", "vg_raycast_cells_batched", "vg_raycast_batched",
                 "vg_mc_volume_area_nbr", "vg_tuple_neighbors", "vg_mc_sample_points",
                 "vg_mc_integrals", "vg_hmc_centroids", "vg_hmc_integrals",
                 "vg_explore"):
        assert want in names


def test_library_exports_every_declared_symbol():
    from paper_2405_10050_amd import LIB_PATH

    lib = ctypes.CDLL(LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\b(vg_[a-z0-9_]+)\b", out))
    assert set(_declared()) <= exported


def test_binding_names_match_exports():
    import paper_2405_10050_amd as vg

    assert set(vg.EXPORTS) == set(_declared())


def test_cpu_tensors_are_rejected():
    import pytest
    import torch

    import paper_2405_10050_amd as vg

    with pytest.raises(vg.VGError):
        vg.raycast_cells(torch.rand(4, 3), torch.rand(4, 2, 3))
