"""Seeded generators: determinism and the sizes the workloads are defined by."""
import numpy as np

import oracle
from paper_1503_07192_amd import workloads as W


def test_grid32_shape_and_determinism():
    a, b = W.grid32(), W.grid32()
    assert a["n"] == 1024 and a["m"] == 1984 and a["k"] == 16
    for key in ("eu", "ev", "w", "part", "v1", "v2"):
        assert np.array_equal(a[key], b[key])
    assert a["w"].min() >= 1 and a["w"].max() <= 100
    assert np.bincount(a["part"]).tolist() == [64] * 16
    assert oracle.boundary(a["n"], a["eu"], a["ev"], a["part"]).sum() == 348


def test_grid256d_boundary_count():
    g = W.grid256d(queries=10)
    assert g["n"] == 65536 and g["k"] == 1024
    nd = g["m"] - 2 * 256 * 255
    assert 31_000 < nd < 34_000            # about half of the 65,025 cells
    assert g["w"].min() >= 1 and g["w"].max() <= 1000
    # diagonals add no boundary vertices: 27,900 as for the plain grid
    assert oracle.boundary(g["n"], g["eu"], g["ev"], g["part"]).sum() == 27_900


def test_rcb_partition_balanced():
    rng = np.random.default_rng(0)
    pts = rng.random((5000, 2))
    part, k = W.rcb_partition(pts, 5, rng)
    sizes = np.bincount(part, minlength=k)
    assert k == 32 and sizes.sum() == 5000 and sizes.min() > 100
