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


def test_superblock_numbering():
    part, k = W.block_partition(32, 32, 4, 4, sb=2)
    assert k == 64 and np.array_equal(np.bincount(part), [16] * 64)
    # ids 0..3 are the 2x2 blocks of the top-left 8x8 vertex square
    grid = part.reshape(32, 32)
    assert set(np.unique(grid[:8, :8])) == {0, 1, 2, 3}
    assert grid[0, 4] == 1 and grid[4, 0] == 2 and grid[0, 8] == 4


def test_morton_numbering():
    part, k = W.block_partition(64, 64, 4, 4, sb=0)
    assert k == 256 and np.array_equal(np.bincount(part), [16] * 256)
    blocks = part.reshape(64, 64)[::4, ::4]
    # aligned runs of 4^j ids are squares of 2^j x 2^j blocks, runs of 2 * 4^j
    # are 2^j x 2^(j+1)
    for run, (h, wd) in ((4, (2, 2)), (8, (2, 4)), (16, (4, 4)), (32, (4, 8)), (64, (8, 8))):
        for j in range(0, k, run):
            r, c = np.nonzero((blocks >= j) & (blocks < j + run))
            assert (r.max() - r.min() + 1, c.max() - c.min() + 1) == (h, wd), (run, j)
    assert np.array_equal(blocks[:2, :4], [[0, 1, 4, 5], [2, 3, 6, 7]])


def test_grid2048_small_share():
    g = W.grid2048(queries=1000, side=256, blk=16)
    assert g["k"] == 256 and g["share_k"] == 8
    # the share: the first 8 components in Z-order, a 2 x 4 block region
    sv = np.flatnonzero(g["part"] < 8)
    assert len(sv) == 8 * 256
    assert (sv // 256).max() < 32 and (sv % 256).max() < 64
    assert (g["part"][g["v1"]] < g["share_k"]).all()
    # connected: a spanning tree is kept
    import oracle
    d = oracle.dijkstra(g["n"], g["eu"], g["ev"], g["w"], [0])
    assert (d < oracle.O_INF).all()
    assert g["m"] == 2 * 256 * 255 - round(0.1 * 2 * 256 * 255)
