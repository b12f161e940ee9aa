"""Seeded synthetic inputs: graphs, partitions and query pairs.

This module only *draws* inputs.  It holds none of the method's arithmetic
(no boundary detection, no distances, no reordering), so both the HIP path
and the CPU oracle can be fed the very same arrays from it.

Every graph is undirected and given as an edge list ``(eu, ev, w)`` of int32
arrays; ``part[v]`` in ``[0, k)`` assigns vertex ``v`` to a component.  The
partitions are inputs here: the paper builds them with a separator-based
k-partition (Section 3) or METIS (Section 4); the workloads below prescribe
block or coordinate-bisection partitions instead.

Workloads (random streams come from ``SeedSequence(150307192 + cfg)``):

* ``grid32``    32x32 4-neighbour grid, weights U[1,100], 16 blocks of 8x8,
                1,000 uniform query pairs.
* ``grid256d``  256x256 grid plus one diagonal in each cell with probability
                1/2 (random orientation), weights U[1,1000], 1,024 blocks of
                8x8, 100,000 uniform query pairs.
* ``delaunay1m`` Delaunay triangulation of 1,000,000 uniform points,
                weight = rint(length * 1e6), recursive coordinate bisection
                to 4,096 components.
* ``grid2048``  2048x2048 grid, 10% of the non-spanning-tree edges deleted,
                lognormal(4,1) weights clipped to [1,1e5], 16,384 blocks of
                16x16 numbered along a Z-order curve; the single-GPU share
                is components [0, 512) (a 256 x 512-vertex region).
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 150307192


def streams(cfg: int, count: int = 4):
    """Independent generators for (weights, structure, partition, queries)."""
    ss = np.random.SeedSequence(SEED_BASE + cfg)
    return [np.random.default_rng(s) for s in ss.spawn(count)]


def grid_edges(rows: int, cols: int):
    """4-neighbour grid, vertex id = r*cols + c; horizontal edges then vertical."""
    ids = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    hu, hv = ids[:, :-1].ravel(), ids[:, 1:].ravel()
    vu, vv = ids[:-1, :].ravel(), ids[1:, :].ravel()
    eu = np.concatenate([hu, vu]).astype(np.int32)
    ev = np.concatenate([hv, vv]).astype(np.int32)
    return eu, ev


def morton_code(r, c, bits: int = 16):
    """Z-order (Morton) code of block (r, c): the bits of c and r interleaved,
    c in the even bit positions."""
    r = np.asarray(r, np.int64)
    c = np.asarray(c, np.int64)
    z = np.zeros(np.broadcast(r, c).shape, np.int64)
    for b in range(bits):
        z |= ((c >> b) & 1) << (2 * b)
        z |= ((r >> b) & 1) << (2 * b + 1)
    return z


def block_partition(rows: int, cols: int, br: int, bc: int, sb: int = 1):
    """Blocks of br x bc vertices.  With sb == 1 the component of (r, c) is
    (r // br) * ceil(cols / bc) + c // bc (blocks row by row).  With sb > 1 the
    blocks are numbered super-block by super-block, each super-block being
    sb x sb blocks numbered row by row inside it, so that runs of sb*sb
    consecutive ids are square regions.  With sb == 0 the blocks are numbered
    along a Z-order curve (ids = ranks of their Morton codes): every aligned
    run of 4^j consecutive ids is a 2^j x 2^j square of blocks and every run
    of 2 * 4^j a 2^j x 2^(j+1) rectangle, when the block grid is a power of
    two on each side."""
    r = np.arange(rows)[:, None] // br
    c = np.arange(cols)[None, :] // bc
    nbr, nbc = -(-rows // br), -(-cols // bc)
    if sb == 0:
        br_, bc_ = np.meshgrid(np.arange(nbr), np.arange(nbc), indexing="ij")
        rank = np.empty(nbr * nbc, np.int64)
        rank[np.argsort(morton_code(br_.ravel(), bc_.ravel()), kind="stable")] = np.arange(nbr * nbc)
        part = rank.reshape(nbr, nbc)[r, c].ravel().astype(np.int32)
    elif sb == 1:
        part = (r * nbc + c).ravel().astype(np.int32)
    else:
        assert nbr % sb == 0 and nbc % sb == 0
        sr, sc = r // sb, c // sb
        part = (((sr * (nbc // sb) + sc) * sb + r % sb) * sb + c % sb).ravel().astype(np.int32)
    return part, int(nbr * nbc)


def uniform_pairs(rng, n: int, q: int, lo: int = 0, hi: int | None = None):
    """q pairs: v1 uniform in [lo, hi), v2 uniform in [0, n).  v1 == v2 allowed."""
    hi = n if hi is None else hi
    v1 = rng.integers(lo, hi, size=q, dtype=np.int64).astype(np.int32)
    v2 = rng.integers(0, n, size=q, dtype=np.int64).astype(np.int32)
    return v1, v2


def _pack(name, n, eu, ev, w, part, k, v1=None, v2=None, **extra):
    d = dict(name=name, n=int(n), m=int(len(eu)),
             eu=np.ascontiguousarray(eu, np.int32),
             ev=np.ascontiguousarray(ev, np.int32),
             w=np.ascontiguousarray(w, np.int32),
             part=np.ascontiguousarray(part, np.int32), k=int(k))
    if v1 is not None:
        d["v1"] = np.ascontiguousarray(v1, np.int32)
        d["v2"] = np.ascontiguousarray(v2, np.int32)
    d.update(extra)
    return d


def grid32():
    rw, rs, rp, rq = streams(1)
    eu, ev = grid_edges(32, 32)
    w = rw.integers(1, 101, size=len(eu))
    part, k = block_partition(32, 32, 8, 8)
    v1, v2 = uniform_pairs(rq, 1024, 1000)
    return _pack("grid32", 1024, eu, ev, w, part, k, v1, v2)


def grid256d(queries: int = 100_000):
    rw, rs, rp, rq = streams(2)
    R = C = 256
    eu, ev = grid_edges(R, C)
    cell_r, cell_c = np.meshgrid(np.arange(R - 1), np.arange(C - 1), indexing="ij")
    cell_r, cell_c = cell_r.ravel(), cell_c.ravel()
    take = rs.random(cell_r.size) < 0.5
    orient = rs.integers(0, 2, size=cell_r.size)
    cr, cc, co = cell_r[take], cell_c[take], orient[take]
    # orientation 0: (r,c)-(r+1,c+1); orientation 1: (r,c+1)-(r+1,c)
    du = np.where(co == 0, cr * C + cc, cr * C + cc + 1)
    dv = np.where(co == 0, (cr + 1) * C + cc + 1, (cr + 1) * C + cc)
    eu = np.concatenate([eu, du.astype(np.int32)])
    ev = np.concatenate([ev, dv.astype(np.int32)])
    w = rw.integers(1, 1001, size=len(eu))
    part, k = block_partition(R, C, 8, 8)
    v1, v2 = uniform_pairs(rq, R * C, queries)
    return _pack("grid256d", R * C, eu, ev, w, part, k, v1, v2)


def rcb_partition(pts: np.ndarray, depth: int, rng, flo=0.47, fhi=0.53):
    """Recursive coordinate bisection: split each set on the longer side of
    its bounding box at rank round(len * f), f ~ U[flo, fhi]; 2**depth parts."""
    n = pts.shape[0]
    part = np.zeros(n, np.int32)
    sets = [np.arange(n)]
    for _ in range(depth):
        nxt = []
        fs = rng.uniform(flo, fhi, size=len(sets))
        for s, f in zip(sets, fs):
            p = pts[s]
            ext = p.max(axis=0) - p.min(axis=0)
            ax = int(np.argmax(ext))
            cut = int(round(len(s) * f))
            order = np.argpartition(p[:, ax], cut)
            nxt.append(s[order[:cut]])
            nxt.append(s[order[cut:]])
        sets = nxt
    for i, s in enumerate(sets):
        part[s] = i
    return part, len(sets)


def delaunay_graph(npts: int, cfg: int = 3, depth: int = 12, queries: int = 0):
    from scipy.spatial import Delaunay
    rw, rs, rp, rq = streams(cfg)
    pts = rs.random((npts, 2))
    tri = Delaunay(pts).simplices.astype(np.int64)
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [0, 2]]])
    e.sort(axis=1)
    e = np.unique(e[:, 0] * npts + e[:, 1])
    eu, ev = (e // npts).astype(np.int32), (e % npts).astype(np.int32)
    ln = np.hypot(*(pts[eu] - pts[ev]).T)
    w = np.rint(ln * 1e6).astype(np.int64)
    part, k = rcb_partition(pts, depth, rp)
    d = _pack("delaunay%d" % npts, npts, eu, ev, w, part, k)
    if queries:
        d["v1"], d["v2"] = uniform_pairs(rq, npts, queries)
    return d


def delaunay1m(queries: int = 0):
    return delaunay_graph(1_000_000, 3, 12, queries)


def grid2048(queries: int = 10_000_000, side: int = 2048, blk: int = 16,
             share_den: int = 32, sb: int = 0):
    """Grid with 10% of the edges deleted off a random spanning tree."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree
    rw, rs, rp, rq = streams(4)
    n = side * side
    eu, ev = grid_edges(side, side)
    m0 = len(eu)
    # Kruskal with a uniformly shuffled edge order == MST under distinct random keys
    perm = rs.permutation(m0)
    key = perm.astype(np.float64) + 1.0          # edge i gets key perm[i] + 1
    mst = minimum_spanning_tree(coo_matrix((key, (eu, ev)), shape=(n, n)).tocsr())
    tk = mst.tocoo()
    edge_of_key = np.argsort(perm)               # key - 1 -> edge index
    in_tree = np.zeros(m0, bool)
    in_tree[edge_of_key[(tk.data - 1.0).astype(np.int64)]] = True
    assert in_tree.sum() == n - 1
    non_tree = np.flatnonzero(~in_tree)
    ndel = int(round(0.1 * m0))
    drop = rs.choice(non_tree, size=ndel, replace=False)
    keep = np.ones(m0, bool)
    keep[drop] = False
    eu, ev = eu[keep], ev[keep]
    w = np.clip(np.rint(np.exp(4.0 + rw.standard_normal(len(eu)))), 1, 1e5).astype(np.int64)
    # blocks numbered along a Z-order curve (sb = 0; sb > 0: by super-blocks
    # of sb x sb blocks): runs of consecutive ids are compact regions, and the
    # share (the first k / share_den components) is one of them
    part, k = block_partition(side, side, blk, blk, sb)
    share_k = k // share_den
    share_v = np.flatnonzero(part < share_k).astype(np.int32)
    d = _pack("grid%d" % side, n, eu, ev, w, part, k, share_k=share_k,
              share_vertices=len(share_v))
    if queries:
        v1 = share_v[rq.integers(0, len(share_v), size=queries)]
        v2 = rq.integers(0, n, size=queries, dtype=np.int64).astype(np.int32)
        d["v1"], d["v2"] = np.ascontiguousarray(v1, np.int32), v2
    return d


# ---------------------------------------------------------------- small cases
def random_graph(rng, n: int, m: int, wlo: int = 0, whi: int = 20):
    """Arbitrary multigraph (self-loops and parallel edges allowed)."""
    if n == 0 or m == 0:
        e = np.zeros(0, np.int32)
        return e, e.copy(), e.copy()
    eu = rng.integers(0, n, size=m).astype(np.int32)
    ev = rng.integers(0, n, size=m).astype(np.int32)
    w = rng.integers(wlo, whi + 1, size=m).astype(np.int32)
    return eu, ev, w


def random_grid(rng, rows: int, cols: int, keep: float = 1.0, diag: float = 0.0,
                wlo: int = 1, whi: int = 100):
    eu, ev = grid_edges(rows, cols)
    if diag > 0 and rows > 1 and cols > 1:
        cr, cc = np.meshgrid(np.arange(rows - 1), np.arange(cols - 1), indexing="ij")
        cr, cc = cr.ravel(), cc.ravel()
        t = rng.random(cr.size) < diag
        eu = np.concatenate([eu, (cr[t] * cols + cc[t]).astype(np.int32)])
        ev = np.concatenate([ev, ((cr[t] + 1) * cols + cc[t] + 1).astype(np.int32)])
    sel = rng.random(len(eu)) < keep
    eu, ev = eu[sel], ev[sel]
    w = rng.integers(wlo, whi + 1, size=len(eu)).astype(np.int32)
    return eu, ev, w


def random_partition(rng, n: int, k: int):
    """Every one of the k parts is non-empty (needs n >= k)."""
    part = np.concatenate([np.arange(k), rng.integers(0, k, size=n - k)])
    return rng.permutation(part).astype(np.int32)
