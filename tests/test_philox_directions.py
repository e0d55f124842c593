"""The host side of the on-device Monte-Carlo directions (workloads.philox_directions):
Philox4x32-10 against its published known-answer vectors, and the directions
against what a uniform draw on the unit sphere must satisfy (Sec. 3.1)."""
import json
import os

import numpy as np

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answer_vectors():
    kat = json.load(open(os.path.join(HERE, "golden", "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        out = W.philox4x32_10(ctr, key)
        assert [int(x) for x in out] == [int(x, 16) for x in v["out"]]


def test_directions_are_a_pure_function_of_seed_cell_and_ray():
    a = W.philox_directions([3, 7, 11], 40, 6, seed=9)
    b = W.philox_directions([11], 40, 6, seed=9)
    assert np.array_equal(a[2], b[0])
    c = W.philox_directions([3], 40, 6, seed=10)
    assert not np.array_equal(a[0], c[0])
    # the first components of a longer vector are not those of a shorter one
    # after normalisation, but the underlying draws are shared: d = 4 and 8
    # agree up to the norm on the first four components
    u4 = W.philox_directions([5], 16, 4, seed=1)[0].astype(np.float64)
    u8 = W.philox_directions([5], 16, 8, seed=1)[0].astype(np.float64)
    r = u8[:, :4] / u4
    assert np.allclose(r, r[:, :1], rtol=1e-6)


def test_directions_are_unit_vectors():
    for d in (2, 3, 5, 10, 16):
        u = W.philox_directions(np.arange(20), 64, d, seed=d).astype(np.float64)
        assert np.allclose(np.linalg.norm(u, axis=-1), 1.0, atol=4e-7)


def test_directions_are_isotropic():
    """Uniform on S^{d-1}: mean 0 and second moment I/d (each within a few
    standard errors of the sample), and the radial part is chi distributed
    with d degrees of freedom (E|z|^2 = d) -- checked through the first
    component's fourth moment 3/(d(d+2))."""
    for d in (2, 4, 10):
        u = W.philox_directions(np.arange(400), 500, d, seed=3).reshape(-1, d).astype(np.float64)
        m = u.shape[0]
        assert np.all(np.abs(u.mean(axis=0)) < 5 * np.sqrt(1.0 / d / m))
        S = u.T @ u / m
        se = np.sqrt(2.0 / (d * (d + 2)) / m)
        assert np.all(np.abs(np.diag(S) - 1.0 / d) < 5 * se + 1e-12)
        off = S[~np.eye(d, dtype=bool)]
        assert np.all(np.abs(off) < 5 * np.sqrt(1.0 / (d * (d + 2)) / m))
        m4 = np.mean(u[:, 0] ** 4)
        assert abs(m4 - 3.0 / (d * (d + 2))) < 0.05 * 3.0 / (d * (d + 2))
