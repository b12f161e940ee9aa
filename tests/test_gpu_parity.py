"""Parity of the HIP path with the CPU oracle, element by element (tolerance 0).

Every kernel output is compared with what the oracle computes from the same
seeded inputs: APSP(C) with Floyd-Warshall on the induced component, BG rows
with Dijkstra on G (Lemma 1 makes them equal), query answers with Dijkstra on
G (Lemma 3).  The Floyd-Warshall kernels are also driven directly on
adversarial matrices.  A value the kernels report is min(exact distance,
2^31-1): stored sums never wrap, so an exact distance at or above the
sentinel shows as the sentinel.
"""
import os

import numpy as np
import pytest

import oracle
from oracle import O_INF
from paper_1503_07192_amd import workloads as W

torch = pytest.importorskip("torch")
spq = pytest.importorskip("paper_1503_07192_amd.spq")

pytestmark = pytest.mark.gpu
INF32 = 2**31 - 1
# the options bench.py builds delaunay1m and grid2048 with (the autotuner's)
TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(spq.__file__)), "tune_cache.json")


def clamp32(d):
    d = np.asarray(d, np.int64)
    return np.where(d >= INF32, INF32, d).astype(np.int32)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()


def build(g, **kw):
    print("build %s n=%d m=%d k=%d" % (g.get("name", "?"), g["n"], len(g["eu"]), g["k"]), flush=True)
    idx = spq.build_index(g["n"], dev(g["eu"]), dev(g["ev"]), dev(g["w"]), dev(g["part"]), g["k"], **kw)
    torch.cuda.synchronize()
    return idx


def local_order(lay, c):
    """Vertices of component c in the index's local order."""
    vs = np.flatnonzero(lay["comp"] == c)
    return vs[np.argsort(lay["local"][vs], kind="stable")]


def check_layout(g, lay):
    n, k = g["n"], g["k"]
    assert np.array_equal(lay["comp"], g["part"])
    flag = oracle.boundary(n, g["eu"], g["ev"], g["part"])
    for c in range(k):
        vs = local_order(lay, c)
        assert np.array_equal(np.sort(lay["local"][vs]), np.arange(len(vs)))
        b = vs[: lay["nb"][c]]
        i = vs[lay["nb"][c]:]
        assert flag[b].all() and not flag[i].any()
        assert (np.diff(b) > 0).all() and (np.diff(i) > 0).all()
        assert lay["off"][c + 1] - lay["off"][c] == len(vs)
        assert lay["bgoff"][c + 1] - lay["bgoff"][c] == lay["nb"][c]


def check_components(g, idx, lay, comps=None):
    comps = list(range(g["k"])) if comps is None else list(comps)
    members, apsp = oracle.component_apsp(g["n"], g["eu"], g["ev"], g["w"], g["part"], g["k"],
                                          comps=comps)
    for c, mem, A in zip(comps, members, apsp):
        vs = local_order(lay, c)
        p = np.searchsorted(mem, vs)
        got = spq.index_component(idx, c, len(vs))
        want = clamp32(A[np.ix_(p, p)])
        assert np.array_equal(got, want), "component %d" % c


def check_components_all(g, idx, lay, chunk=2048):
    """Every APSP(C) against the oracle's Floyd-Warshall on the induced
    component, in chunks of components (large graphs)."""
    order = np.lexsort((lay["local"], lay["comp"]))   # vertices by (component, local index)
    off = lay["off"]
    for c0 in range(0, g["k"], chunk):
        comps = np.arange(c0, min(g["k"], c0 + chunk))
        members, apsp = oracle.component_apsp(g["n"], g["eu"], g["ev"], g["w"], g["part"], g["k"],
                                              comps=comps)
        for c, mem, A in zip(comps, members, apsp):
            vs = order[off[c]:off[c + 1]]
            p = np.searchsorted(mem, vs)
            got = spq.index_component(idx, int(c), len(vs))
            assert np.array_equal(got, clamp32(A[np.ix_(p, p)])), "component %d" % c
        print("components %d..%d match" % (comps[0], comps[-1]), flush=True)


def bg_vertices(lay):
    out = []
    for c in range(len(lay["nb"])):
        out.append(local_order(lay, c)[: lay["nb"][c]])
    return np.concatenate(out) if out else np.zeros(0, np.int64)


def check_bg_rows(g, idx, lay, rows):
    verts = bg_vertices(lay)
    V = len(verts)
    if V == 0:
        return
    rows = np.unique(np.asarray(rows))
    D = oracle.dijkstra(g["n"], g["eu"], g["ev"], g["w"], verts[rows])
    want = clamp32(D[:, verts])
    for r, wrow in zip(rows, want):
        got = spq.index_bg_rows(idx, int(r), 1, V)[0]
        assert np.array_equal(got, wrow), "BG row %d" % r


def run_queries(idx, v1, v2):
    out = spq.query_batch(idx, dev(v1), dev(v2))
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check_queries(g, idx, v1, v2):
    got = run_queries(idx, v1, v2)
    D = oracle.dijkstra(g["n"], g["eu"], g["ev"], g["w"], v1)
    want = clamp32(D[np.arange(len(v1)), v2])
    bad = np.flatnonzero(got != want)
    assert len(bad) == 0, "first mismatch pair %s: got %d want %d" % (
        (v1[bad[0]], v2[bad[0]]), got[bad[0]], want[bad[0]])


def check_pairs_by_source(g, idx, v1, v2, chunk=100):
    """check_queries on a large sample: one Dijkstra per distinct source,
    `chunk` sources at a time (the distance rows of a 4M-vertex graph are
    32 MB each)."""
    v1 = np.asarray(v1, np.int32)
    v2 = np.asarray(v2, np.int32)
    got = run_queries(idx, v1, v2)
    src, inv = np.unique(v1, return_inverse=True)
    for c0 in range(0, len(src), chunk):
        D = oracle.dijkstra(g["n"], g["eu"], g["ev"], g["w"], src[c0:c0 + chunk])
        sel = np.flatnonzero((inv >= c0) & (inv < c0 + chunk))
        want = clamp32(D[inv[sel] - c0, v2[sel]])
        bad = np.flatnonzero(got[sel] != want)
        assert len(bad) == 0, "first mismatch pair %s: got %d want %d" % (
            (v1[sel[bad[0]]], v2[sel[bad[0]]]), got[sel[bad[0]]], want[bad[0]])
    return len(src)


def all_pairs(n):
    a, b = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return a.ravel().astype(np.int32), b.ravel().astype(np.int32)


# ------------------------------------------------ Floyd-Warshall kernels
def random_symmetric(rng, N, ld, density, wlo, whi):
    A = np.full((ld, ld), INF32, np.int64)
    mask = np.triu(rng.random((N, N)) < density, 1)
    wts = rng.integers(wlo, whi + 1, size=(N, N))
    sub = np.where(mask, wts, INF32)
    sub = np.minimum(sub, sub.T)
    A[:N, :N] = sub
    np.fill_diagonal(A, 0)
    return A


def oracle_closure(A, N):
    d = np.where(A[:N, :N] == INF32, O_INF, A[:N, :N]).astype(np.int64)
    return clamp32(oracle.fw(d))


WEIGHTS = [("tiny", 0, 3), ("mid", 1, 10**6), ("nearinf", 2**30, INF32 - 1)]


@pytest.mark.parametrize("wname,wlo,whi", WEIGHTS, ids=[w[0] for w in WEIGHTS])
def test_fw_components_kernel(wname, wlo, whi):
    rng = np.random.default_rng(21)
    sizes = [1, 2, 3, 63, 64, 65, 100, 128, 129, 191, 200, 257, 300]
    mats, offs, lds, off = [], [], [], 0
    for N in sizes:
        ld = -(-N // 64) * 64
        dens = min(1.0, 4.0 / N) if N > 4 else 0.6
        mats.append(random_symmetric(rng, N, ld, dens, wlo, whi))
        offs.append(off)
        lds.append(ld)
        off += ld * ld
    data = np.concatenate([m.ravel() for m in mats]).astype(np.int32)
    d = dev(data)
    spq.fw_components(sizes, offs, lds, d)
    got = d.cpu().numpy()
    for N, m, o, ld in zip(sizes, mats, offs, lds):
        g = got[o:o + ld * ld].reshape(ld, ld)
        assert np.array_equal(g[:N, :N], oracle_closure(m, N)), "N=%d" % N


@pytest.mark.parametrize("pivot", [1, 2, 4])
@pytest.mark.parametrize("kc", [16, 32])
@pytest.mark.parametrize("tile", [64, 128])
@pytest.mark.parametrize("v", [1, 5, 64, 100, 129, 300, 520, 700])
def test_fw_dense_kernel(tile, v, kc, pivot):
    # pivot blocks of one, two or four tiles; the tiles left at the end form
    # smaller blocks (128-tiles: 1-6 tiles, e.g. 4 + 2; 64-tiles: up to 11,
    # 4 + 4 + 2 + 1)
    rng = np.random.default_rng(1000 + v + tile)
    ld = -(-v // tile) * tile
    for wlo, whi in [(0, 3), (1, 10**6), (2**30, INF32 - 1)]:
        A = random_symmetric(rng, v, ld, min(1.0, 3.0 / max(v, 1)), wlo, whi)
        d = dev(A.ravel())
        spq.fw_dense(v, ld, tile, d, kc=kc, pivot=pivot * tile)
        torch.cuda.synchronize()
        got = d.cpu().numpy().reshape(ld, ld)
        assert np.array_equal(got[:v, :v], oracle_closure(A, v)), (wlo, whi)
        # padding stays isolated
        if ld > v:
            assert (got[:v, v:] == INF32).all() and (got[v:, :v] == INF32).all()


def test_fw_dense_empty_and_dense_graph():
    rng = np.random.default_rng(3)
    v, ld = 200, 256
    A = np.full((ld, ld), INF32, np.int64)
    np.fill_diagonal(A, 0)
    d = dev(A.ravel())
    spq.fw_dense(v, ld, 128, d)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy().reshape(ld, ld)[:v, :v], clamp32(A[:v, :v]))
    B = random_symmetric(rng, v, ld, 1.0, 0, 1000)
    d = dev(B.ravel())
    spq.fw_dense(v, ld, 128, d)
    torch.cuda.synchronize()
    assert np.array_equal(d.cpu().numpy().reshape(ld, ld)[:v, :v], oracle_closure(B, v))


# ------------------------------------------------------------ the index
def small_cases():
    rng = np.random.default_rng(5)
    cases = []
    for t in range(12):
        R, C = int(rng.integers(2, 10)), int(rng.integers(2, 10))
        eu, ev, w = W.random_grid(rng, R, C, keep=0.85, diag=0.3, wlo=0, whi=30)
        n = R * C
        if t % 2:
            k = int(rng.integers(1, min(n, 7) + 1))
            part = W.random_partition(rng, n, k)
        else:
            part, k = W.block_partition(R, C, 3, 3)
        cases.append(dict(name="grid%d" % t, n=n, eu=eu, ev=ev, w=w, part=part, k=k))
    for t in range(8):
        n = int(rng.integers(1, 14))
        eu, ev, w = W.random_graph(rng, n, int(rng.integers(0, 30)), 0, 9)
        k = int(rng.integers(1, n + 1))
        cases.append(dict(name="multi%d" % t, n=n, eu=eu, ev=ev, w=w,
                          part=W.random_partition(rng, n, k), k=k))
    # components above one 64-tile: 2 and 3 tile rounds, k = 1 on 400 vertices
    eu, ev, w = W.random_grid(rng, 24, 24, keep=0.9, diag=0.2)
    part, k = W.block_partition(24, 24, 12, 12)
    cases.append(dict(name="blocks144", n=576, eu=eu, ev=ev, w=w, part=part, k=k))
    eu, ev, w = W.random_grid(rng, 20, 20, keep=0.95)
    cases.append(dict(name="k1_400", n=400, eu=eu, ev=ev, w=w, part=np.zeros(400, np.int32), k=1))
    eu, ev, w = W.random_grid(rng, 20, 30, keep=0.9, diag=0.3)
    cases.append(dict(name="rand2_600", n=600, eu=eu, ev=ev, w=w,
                      part=W.random_partition(rng, 600, 2), k=2))
    cases.append(dict(name="single", n=1, eu=np.zeros(0, np.int32), ev=np.zeros(0, np.int32),
                      w=np.zeros(0, np.int32), part=np.zeros(1, np.int32), k=1))
    cases.append(dict(name="noedges", n=10, eu=np.zeros(0, np.int32), ev=np.zeros(0, np.int32),
                      w=np.zeros(0, np.int32), part=np.arange(10, dtype=np.int32) % 3, k=3))
    return cases


CASES = small_cases()


@pytest.mark.parametrize("g", CASES, ids=[c["name"] for c in CASES])
def test_index_small_graphs_all_pairs(g):
    idx = build(g)
    lay = spq.index_layout(idx)
    check_layout(g, lay)
    check_components(g, idx, lay)
    st = spq.index_stats(idx)
    check_bg_rows(g, idx, lay, np.arange(st["v_bg"]))
    v1, v2 = all_pairs(g["n"])
    check_queries(g, idx, v1, v2)


def test_large_components_use_the_multi_workgroup_closure():
    rng = np.random.default_rng(66)
    eu, ev, w = W.random_grid(rng, 35, 40, keep=0.9, diag=0.2)
    n = 1400
    part = np.where(np.arange(n) < 1200, 0, 1 + (np.arange(n) % 3)).astype(np.int32)
    g = dict(name="bigcomp", n=n, eu=eu, ev=ev, w=w, part=part, k=4)
    for kw in ({}, {"plain": True}, {"bg_method": 2, "group_comps": 2}):
        idx = build(g, **kw)
        lay = spq.index_layout(idx)
        check_layout(g, lay)
        check_components(g, idx, lay)
        rng2 = np.random.default_rng(1)
        v1 = rng2.integers(0, n, 3000).astype(np.int32)
        v2 = rng2.integers(0, n, 3000).astype(np.int32)
        check_queries(g, idx, v1, v2)


def test_grid32_everything():
    g = W.grid32()
    idx = build(g)
    lay = spq.index_layout(idx)
    check_layout(g, lay)
    st = spq.index_stats(idx)
    assert st["v_bg"] == 348 and st["k"] == 16 and st["max_comp"] == 64
    check_components(g, idx, lay)
    check_bg_rows(g, idx, lay, np.arange(348))
    check_queries(g, idx, g["v1"], g["v2"])
    v1, v2 = all_pairs(g["n"])
    check_queries(g, idx, v1, v2)


def test_grid32_bg_tile_plain_and_repeat_are_bitwise_identical():
    g = W.grid32()
    a = build(g, bg_tile=64)
    b = build(g, bg_tile=128)
    c = build(g, bg_tile=128)
    d = build(g, plain=True)
    e = build(g, bg_tile=64, lookahead=False)
    f = build(g, bg_tile=64, inner_kc=32)
    ra, rb, rc, rd, re, rf = (spq.index_bg_rows(x, 0, 348, 348) for x in (a, b, c, d, e, f))
    assert np.array_equal(ra, rb) and np.array_equal(rb, rc) and np.array_equal(rb, rd)
    assert np.array_equal(ra, re) and np.array_equal(ra, rf)
    # pivot blocks of one tile, and of two without the lookahead (3 tiles of
    # 128: a two-tile block, then a one-tile block; 6 tiles of 64: three blocks)
    for kw in ({"bg_pivot": 128}, {"bg_pivot": 256, "lookahead": False}, {"bg_pivot": 256},
               {"bg_tile": 64, "bg_pivot": 64}, {"bg_tile": 64, "bg_pivot": 128, "lookahead": False},
               {"bg_tile": 64, "bg_pivot": 256}, {"bg_tile": 64, "bg_pivot": 256, "lookahead": False},
               {"bg_pivot": 512, "inner_kc": 32}):
        x = build(g, **kw)
        assert np.array_equal(spq.index_bg_rows(x, 0, 348, 348), ra), kw
    for comp in range(16):
        assert np.array_equal(spq.index_component(b, comp, 64), spq.index_component(d, comp, 64))
    v1, v2 = all_pairs(g["n"])
    qa, qb = run_queries(a, v1, v2), run_queries(b, v1, v2)
    assert np.array_equal(qa, qb)


def test_grid256d_full_size():
    """The benchmark workload: every component, sampled BG rows and queries."""
    g = W.grid256d()
    idx = build(g)
    lay = spq.index_layout(idx)
    check_layout(g, lay)
    st = spq.index_stats(idx)
    assert st["v_bg"] == 27_900 and st["k"] == 1024
    check_components(g, idx, lay)
    rng = np.random.default_rng(77)
    rows = np.concatenate([[0, 1, 27_899], rng.integers(0, 27_900, 200)])
    check_bg_rows(g, idx, lay, rows)
    q = len(g["v1"])
    out = run_queries(idx, g["v1"], g["v2"])
    assert out.shape == (q,)
    check_queries(g, idx, g["v1"][:3000], g["v2"][:3000])
    # the same pairs inside the full batch
    sub = run_queries(idx, g["v1"][:3000], g["v2"][:3000])
    assert np.array_equal(sub, out[:3000])
    # symmetry of the answers and d(v, v) = 0 over the whole batch
    rev = run_queries(idx, g["v2"], g["v1"])
    assert np.array_equal(rev, out)
    same = run_queries(idx, g["v1"], g["v1"])
    assert (same == 0).all()


def test_grid256d_every_bg_row_equals_dijkstra():
    """All 27,900 BG rows of the benchmark workload's flat closure against
    Dijkstra on G from each BG vertex (Lemma 1), in chunks of sources."""
    g = W.grid256d(queries=0)
    idx = build(g)
    lay = spq.index_layout(idx)
    verts = bg_vertices(lay)
    V = len(verts)
    assert V == 27_900
    for r0 in range(0, V, 2048):
        r1 = min(V, r0 + 2048)
        D = oracle.dijkstra(g["n"], g["eu"], g["ev"], g["w"], verts[r0:r1])
        got = spq.index_bg_rows(idx, r0, r1 - r0, V)
        bad = np.flatnonzero((got != clamp32(D[:, verts])).any(axis=1))
        assert len(bad) == 0, "BG row %d" % (r0 + bad[0])
        print("BG rows %d..%d match" % (r0, r1 - 1), flush=True)


def test_query_invalid_ids_and_empty_batch():
    g = W.grid32()
    idx = build(g)
    v1 = np.array([0, -1, 5, 1024, 3], np.int32)
    v2 = np.array([1, 2, 2000, 4, 3], np.int32)
    out = run_queries(idx, v1, v2)
    assert out[1] == spq.SPQ_BAD_PAIR and out[2] == spq.SPQ_BAD_PAIR and out[3] == spq.SPQ_BAD_PAIR
    assert out[4] == 0
    D = oracle.dijkstra(g["n"], g["eu"], g["ev"], g["w"], [0])
    assert out[0] == D[0, 1]
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    assert spq.query_batch(idx, e, e).numel() == 0
    # the host-array entry point gives the same answers, bad pairs included
    assert np.array_equal(spq.query_batch_host(idx, v1, v2), out)
    assert spq.query_batch_host(idx, v1[:0], v2[:0]).size == 0
    a, b = all_pairs(g["n"])
    assert np.array_equal(spq.query_batch_host(idx, a, b), run_queries(idx, a, b))


def test_build_errors():
    g = W.grid32()
    def expect(status, **over):
        h = dict(g)
        h.update(over)
        with pytest.raises(spq.SpqError) as ei:
            build(h)
        assert ei.value.name == status, ei.value
    bad = g["part"].copy()
    bad[7] = 16
    expect("SPQ_EINVAL", part=bad)
    w = g["w"].copy()
    w[3] = -1
    expect("SPQ_EINVAL", w=w)
    w = g["w"].copy()
    w[3] = INF32
    expect("SPQ_EINVAL", w=w)
    eu = g["eu"].copy()
    eu[0] = 1024
    expect("SPQ_EINVAL", eu=eu)
    expect("SPQ_EINVAL", part=np.where(g["part"] == 3, 4, g["part"]).astype(np.int32))
    w = g["w"].copy()
    w[:3] = 2**30
    expect("SPQ_ERANGE", w=w)
    # the index still builds after errors
    idx = build(g)
    assert spq.index_stats(idx)["v_bg"] == 348


# ------------------------------------------------------ two-level BG method
TWO_LEVEL = [c for c in CASES if c["k"] >= 1]


@pytest.mark.parametrize("g", TWO_LEVEL, ids=[c["name"] for c in TWO_LEVEL])
def test_two_level_small_graphs_all_pairs(g):
    for gc in sorted({1, 2, max(1, g["k"] // 2)}):
        idx = build(g, bg_method=2, group_comps=gc)
        st = spq.index_stats(idx)
        assert st["bg_method"] == 2 and st["ngroups"] == -(-g["k"] // gc)
        lay = spq.index_layout(idx)
        check_layout(g, lay)
        check_components(g, idx, lay)
        check_bg_rows(g, idx, lay, np.arange(st["v_bg"]))
        v1, v2 = all_pairs(g["n"])
        check_queries(g, idx, v1, v2)


@pytest.mark.parametrize("gc", [1, 2, 3, 4, 8, 16])
def test_grid32_two_level_equals_flat(gc):
    g = W.grid32()
    flat = build(g, bg_method=1)
    two = build(g, bg_method=2, group_comps=gc)
    assert np.array_equal(spq.index_bg_rows(flat, 0, 348, 348), spq.index_bg_rows(two, 0, 348, 348))
    v1, v2 = all_pairs(g["n"])
    assert np.array_equal(run_queries(flat, v1, v2), run_queries(two, v1, v2))


@pytest.mark.parametrize("l3", [1, 2, 3, 5, 16])
def test_grid32_level3_equals_flat(l3):
    # 16 groups of one component; BG2 closed by super-groups of l3 groups
    # (16: a single super-group, so no level-3 boundary at all)
    g = W.grid32()
    flat = build(g, bg_method=1)
    three = build(g, bg_method=2, group_comps=1, level3_groups=l3)
    st = spq.index_stats(three)
    assert st["groups3"] == -(-16 // l3)
    if l3 == 16:
        assert st["v_bg3"] == 0
    elif l3 == 1:   # super-groups of one group: every level-2 vertex is one of level 3
        assert st["v_bg3"] == st["v_bg2"]
    else:
        assert 0 < st["v_bg3"] < st["v_bg2"]
    assert np.array_equal(spq.index_bg_rows(flat, 0, 348, 348), spq.index_bg_rows(three, 0, 348, 348))
    v1, v2 = all_pairs(g["n"])
    assert np.array_equal(run_queries(flat, v1, v2), run_queries(three, v1, v2))


LEVEL3 = [c for c in CASES if c["k"] >= 3]


@pytest.mark.parametrize("g", LEVEL3, ids=[c["name"] for c in LEVEL3])
def test_level3_small_graphs_all_pairs(g):
    for gc, l3 in ((1, 1), (1, 2), (2, 1)):
        idx = build(g, bg_method=2, group_comps=gc, level3_groups=l3)
        st = spq.index_stats(idx)
        assert st["groups3"] == (-(-st["ngroups"] // l3) if st["v_bg2"] else 0)
        lay = spq.index_layout(idx)
        check_bg_rows(g, idx, lay, np.arange(st["v_bg"]))
        v1, v2 = all_pairs(g["n"])
        check_queries(g, idx, v1, v2)


def test_two_level_pair_list_in_several_launches():
    # 400 groups of one component: 80,200 group pairs, so the composition
    # runs over its pair list in several launches
    rng = np.random.default_rng(12)
    eu, ev, w = W.random_grid(rng, 40, 40, keep=0.9, diag=0.2)
    part, k = W.block_partition(40, 40, 2, 2)
    g = dict(name="pairs80k", n=1600, eu=eu, ev=ev, w=w, part=part, k=k)
    flat = build(g, bg_method=1)
    two = build(g, bg_method=2, group_comps=1, level3_groups=-1)
    st = spq.index_stats(two)
    assert st["ngroups"] == 400 and st["dominant_launches"] >= 2
    V = st["v_bg"]
    rows = np.random.default_rng(3).integers(0, V, 25)
    for r in rows:
        assert np.array_equal(spq.index_bg_rows(flat, int(r), 1, V), spq.index_bg_rows(two, int(r), 1, V))
    v1, v2 = all_pairs(g["n"])
    sel = np.random.default_rng(4).integers(0, len(v1), 200_000)
    assert np.array_equal(run_queries(flat, v1[sel], v2[sel]), run_queries(two, v1[sel], v2[sel]))
    check_queries(g, two, v1[sel[:3000]], v2[sel[:3000]])


def test_grid256d_two_level_equals_flat():
    g = W.grid256d()
    flat = build(g, bg_method=1)
    qf = run_queries(flat, g["v1"], g["v2"])
    rows = np.random.default_rng(8).integers(0, 27_900, 40)
    rf = [spq.index_bg_rows(flat, int(r), 1, 27_900) for r in rows]
    flat.free()
    # flat rounds without the lookahead overlap: the same matrix
    plain = build(g, bg_method=1, lookahead=False)
    assert np.array_equal(run_queries(plain, g["v1"], g["v2"]), qf)
    for r, want in zip(rows, rf):
        assert np.array_equal(spq.index_bg_rows(plain, int(r), 1, 27_900), want)
    plain.free()
    # pivot blocks of one tile (218 rounds) and two (109) instead of four (55)
    for pivot in (128, 256):
        one = build(g, bg_method=1, bg_pivot=pivot)
        assert np.array_equal(run_queries(one, g["v1"], g["v2"]), qf)
        for r, want in zip(rows, rf):
            assert np.array_equal(spq.index_bg_rows(one, int(r), 1, 27_900), want)
        one.free()
    # 256 groups of 4 components, BG2 closed by 16 super-groups (level 3)
    three = build(g, bg_method=2, group_comps=4, level3_groups=16)
    st = spq.index_stats(three)
    print({k: st[k] for k in ("ngroups", "v_bg2", "groups3", "v_bg3")}, flush=True)
    assert st["ngroups"] == 256 and st["groups3"] == 16 and 0 < st["v_bg3"] < st["v_bg2"]
    assert np.array_equal(run_queries(three, g["v1"], g["v2"]), qf)
    for r, want in zip(rows, rf):
        assert np.array_equal(spq.index_bg_rows(three, int(r), 1, 27_900), want)
    three.free()
    # the same with one-tile pivot blocks in the group, super-group and BG3
    # closures (two-tile blocks are the default)
    three = build(g, bg_method=2, group_comps=4, level3_groups=16, bg_pivot=128)
    assert np.array_equal(run_queries(three, g["v1"], g["v2"]), qf)
    for r, want in zip(rows[:10], rf[:10]):
        assert np.array_equal(spq.index_bg_rows(three, int(r), 1, 27_900), want)
    three.free()
    two = build(g, bg_method=2, group_comps=32)
    st = spq.index_stats(two)
    assert st["ngroups"] == 32 and st["v_bg2"] > 0
    assert np.array_equal(run_queries(two, g["v1"], g["v2"]), qf)
    for r, want in zip(rows, rf):
        assert np.array_equal(spq.index_bg_rows(two, int(r), 1, 27_900), want)
    two.free()
    # BG2 (and, at level 3, BG3) closed without the lookahead: the same matrix
    for kw in ({"group_comps": 32}, {"group_comps": 4, "level3_groups": 16}):
        nl = build(g, bg_method=2, lookahead=False, **kw)
        assert np.array_equal(run_queries(nl, g["v1"], g["v2"]), qf), kw
        for r, want in zip(rows[:10], rf[:10]):
            assert np.array_equal(spq.index_bg_rows(nl, int(r), 1, 27_900), want)
        nl.free()


# ------------------------------------------------ exactness certificate
def _path(n, wt, breaks, offset=0):
    eu = np.arange(offset, offset + n - 1, dtype=np.int32)
    return eu, eu + 1, np.full(n - 1, wt, np.int32)


@pytest.mark.parametrize("method", [1, 2])
def test_certificate_accepts_large_total_weight(method):
    # two disjoint 4-vertex paths, weights 5e8: total 3e9 >= INF, every
    # distance <= 1.5e9 < INF
    a = _path(4, 500_000_000, None, 0)
    b = _path(4, 500_000_000, None, 4)
    g = dict(name="bigpaths", n=8, eu=np.concatenate([a[0], b[0]]), ev=np.concatenate([a[1], b[1]]),
             w=np.concatenate([a[2], b[2]]), part=np.array([0, 0, 1, 1, 2, 2, 3, 3], np.int32), k=4)
    idx = build(g, bg_method=method, group_comps=2)
    lay = spq.index_layout(idx)
    check_components(g, idx, lay)
    check_bg_rows(g, idx, lay, np.arange(spq.index_stats(idx)["v_bg"]))
    v1, v2 = all_pairs(8)
    check_queries(g, idx, v1, v2)


@pytest.mark.parametrize("n", [5, 7, 9])
@pytest.mark.parametrize("method", [1, 2])
def test_certificate_rejects_unrepresentable_distance(n, method):
    # a path whose end-to-end distance (>= 2.4e9) does not fit below INF
    eu, ev, w = _path(n, 600_000_000, None)
    part = (np.minimum(np.arange(n) // 2, 2) if n < 9 else np.minimum(np.arange(n) // 2, 4)).astype(np.int32)
    g = dict(name="longpath", n=n, eu=eu, ev=ev, w=w, part=part, k=int(part.max()) + 1)
    with pytest.raises(spq.SpqError) as ei:
        build(g, bg_method=method, group_comps=1)
    assert ei.value.name == "SPQ_ERANGE"


# ------------------------------------------- Delaunay, 1M points, 4,096 parts
def check_layout_fast(g, lay, flag):
    """check_layout, vectorized for large graphs."""
    comp, local = lay["comp"], lay["local"]
    assert np.array_equal(comp, g["part"])
    order = np.lexsort((local, comp))
    c_sorted, l_sorted = comp[order], local[order]
    starts = lay["off"][:-1]
    assert np.array_equal(np.bincount(comp, minlength=g["k"]), np.diff(lay["off"]))
    assert np.array_equal(l_sorted, np.arange(g["n"]) - starts[c_sorted])
    assert np.array_equal(np.bincount(comp[flag], minlength=g["k"]), lay["nb"])
    isb = l_sorted < lay["nb"][c_sorted]
    assert np.array_equal(flag[order], isb)
    # ascending ids inside each (component, boundary flag) run
    key = c_sorted.astype(np.int64) * 2 + (~isb)
    same = key[1:] == key[:-1]
    assert (order[1:][same] > order[:-1][same]).all()


def test_delaunay1m_two_level():
    g = W.delaunay1m(queries=2000)
    print("delaunay1m: n=%d m=%d k=%d" % (g["n"], g["m"], g["k"]), flush=True)
    idx = build(g, tune_cache=TUNE_CACHE)   # the benchmark's configuration
    st = spq.index_stats(idx)
    print({k: st[k] for k in ("v_bg", "bg_method", "ngroups", "v_bg2", "groups3", "v_bg3",
                              "max_comp", "max_boundary", "bg_bytes", "ms_components",
                              "ms_bg_apsp")}, flush=True)
    assert st["bg_method"] == 2
    if st["v_bg2"] > 16384:   # BG2 closed by level 3
        assert st["groups3"] > 1 and 0 < st["v_bg3"] < st["v_bg2"]
    lay = spq.index_layout(idx)
    flag = oracle.boundary(g["n"], g["eu"], g["ev"], g["part"])
    assert st["v_bg"] == int(flag.sum())
    check_layout_fast(g, lay, flag)
    rng = np.random.default_rng(31)
    check_components_all(g, idx, lay)
    check_bg_rows(g, idx, lay, np.concatenate([[0, st["v_bg"] - 1], rng.integers(0, st["v_bg"], 30)]))
    # source-grouped query sample: 1,000 sources x 16 targets (the first of
    # each the source itself), then the workload's own first 2,000 pairs
    src = rng.integers(0, g["n"], 1000).astype(np.int32)
    v1 = np.repeat(src, 16)
    v2 = rng.integers(0, g["n"], v1.size).astype(np.int32)
    v2[::16] = v1[::16]
    check_pairs_by_source(g, idx, v1, v2)
    check_pairs_by_source(g, idx, g["v1"], g["v2"])
    got = run_queries(idx, v1[:2000], v2[:2000])
    D = oracle.dijkstra(g["n"], g["eu"], g["ev"], g["w"], src[:125])
    want = clamp32(D[np.repeat(np.arange(125), 16), v2[:2000]])
    assert np.array_equal(got, want)
    # the default group size (64 groups, level 3 on 30,021 level-2 vertices)
    idx.free()
    dflt = build(g)
    sd = spq.index_stats(dflt)
    assert sd["ngroups"] == 64 and sd["groups3"] > 1
    assert np.array_equal(run_queries(dflt, v1[:2000], v2[:2000]), want)


# --------------------------------------------------- share (one GPU's rows)
def share_vertices(g, share_comps):
    return np.flatnonzero(g["part"] < share_comps).astype(np.int32)


def check_share(g, idx, share_comps, nsrc=None, rng=None, uniform=True):
    lay = spq.index_layout(idx)
    st = spq.index_stats(idx)
    verts = bg_vertices(lay)
    if uniform:   # rows of the whole share groups
        bgend = int(lay["bgoff"][min(g["k"], st["share_groups"] * (-(-g["k"] // st["ngroups"])))])
    else:         # rows of the share's components
        bgend = int(lay["bgoff"][share_comps])
    rows = np.arange(bgend) if nsrc is None else rng.choice(bgend, min(nsrc, bgend), replace=False)
    if len(rows):
        check_bg_rows(g, idx, lay, rows)
    sv = share_vertices(g, share_comps)
    if nsrc is None:
        v1 = np.repeat(sv, g["n"]).astype(np.int32)
        v2 = np.tile(np.arange(g["n"]), len(sv)).astype(np.int32)
    else:
        src = rng.choice(sv, nsrc)
        v1 = np.repeat(src, 20).astype(np.int32)
        v2 = rng.integers(0, g["n"], v1.size).astype(np.int32)
    check_queries(g, idx, v1, v2)
    outside = np.flatnonzero(g["part"] >= share_comps)
    if len(outside):
        got = run_queries(idx, outside[:5].astype(np.int32), np.zeros(min(5, len(outside)), np.int32))
        assert (got == spq.SPQ_BAD_PAIR).all()


@pytest.mark.parametrize("blk", [-1, 0, 2, 3])
@pytest.mark.parametrize("share_comps,gc", [(1, 1), (2, 2), (3, 2), (8, 4)])
def test_share_small_grid(share_comps, gc, blk):
    """Share builds with the Bellman-Ford over single groups (-1), blocks of
    2 and 3 groups, and the automatic blocks (all 16 groups in one block at
    gc = 1)."""
    rng = np.random.default_rng(40 + share_comps)
    eu, ev, w = W.random_grid(rng, 16, 16, keep=0.9, diag=0.2, wlo=0, whi=50)
    part, k = W.block_partition(16, 16, 4, 4, sb=2)
    g = dict(name="sharegrid", n=256, eu=eu, ev=ev, w=w, part=part, k=k)
    idx = build(g, share_comps=share_comps, group_comps=gc, level3_groups=blk)
    st = spq.index_stats(idx)
    assert st["share_comps"] == share_comps and st["bf_rounds"] >= 1
    if blk != 0:
        assert st["bf_block_groups"] == min(max(blk, 1), st["ngroups"])
    lay = spq.index_layout(idx)
    check_layout(g, lay)
    check_components(g, idx, lay)
    check_share(g, idx, share_comps)


def size_groups(nb, budget):
    """Group count of the size rule: consecutive components join a group
    while it holds at most `budget` BG vertices."""
    groups, held = 0, 0
    for x in nb:
        if groups == 0 or (held > 0 and held + x > budget):
            groups, held = groups + 1, 0
        held += int(x)
    return groups


@pytest.mark.parametrize("gb", [1, 40, 64, 100, 200, 1000])
def test_grid32_size_groups_equal_flat(gb):
    g = W.grid32()
    flat = build(g, bg_method=1)
    two = build(g, bg_method=2, group_bg=gb)
    st = spq.index_stats(two)
    assert st["ngroups"] == size_groups(spq.index_layout(two)["nb"], gb)
    assert np.array_equal(spq.index_bg_rows(flat, 0, 348, 348), spq.index_bg_rows(two, 0, 348, 348))
    v1, v2 = all_pairs(g["n"])
    assert np.array_equal(run_queries(flat, v1, v2), run_queries(two, v1, v2))


@pytest.mark.parametrize("share_comps,gb", [(1, 10), (3, 25), (5, 60)])
def test_share_size_groups(share_comps, gb):
    rng = np.random.default_rng(60 + share_comps)
    eu, ev, w = W.random_grid(rng, 16, 16, keep=0.9, diag=0.2, wlo=0, whi=50)
    part, k = W.block_partition(16, 16, 4, 4, sb=2)
    g = dict(name="sharegrid", n=256, eu=eu, ev=ev, w=w, part=part, k=k)
    idx = build(g, share_comps=share_comps, group_bg=gb)
    st = spq.index_stats(idx)
    assert st["ngroups"] == size_groups(spq.index_layout(idx)["nb"], gb)
    check_share(g, idx, share_comps, uniform=False)


@pytest.mark.parametrize("blk", [-1, 2, 4])
def test_share_random_partition(blk):
    rng = np.random.default_rng(77)
    eu, ev, w = W.random_grid(rng, 12, 14, keep=0.8, diag=0.3, wlo=0, whi=20)
    n, k = 168, 9
    g = dict(name="sharerand", n=n, eu=eu, ev=ev, w=w, part=W.random_partition(rng, n, k), k=k)
    idx = build(g, share_comps=4, group_comps=2, level3_groups=blk)
    check_share(g, idx, 4)


@pytest.mark.parametrize("gc,blk", [(16, -1), (16, 0), (4, -1), (4, 2), (4, 4), (4, 5), (2, 8)])
def test_share_grid2048_small_equals_full_two_level(gc, blk):
    """The grid2048 recipe at 256x256 (256 components in Z-order, share =
    components [0, 8)): the share's BG rows and answers equal the full
    two-level index's, for groups of 16, 4 and 2 components and Bellman-Ford
    blocks of 1 to 8 groups."""
    g = W.grid2048(queries=2000, side=256, blk=16)
    full = build(g, bg_method=2, group_comps=16)
    share = build(g, share_comps=g["share_k"], group_comps=gc, level3_groups=blk)
    st = spq.index_stats(share)
    assert st["share_groups"] == -(-8 // gc)
    lay = spq.index_layout(share)
    nrows = int(lay["bgoff"][st["share_groups"] * gc])
    V = st["v_bg"]
    assert np.array_equal(spq.index_bg_rows(share, 0, nrows, V), spq.index_bg_rows(full, 0, nrows, V))
    assert np.array_equal(run_queries(share, g["v1"], g["v2"]), run_queries(full, g["v1"], g["v2"]))
    check_queries(g, share, g["v1"][:500], g["v2"][:500])


def test_grid2048_share_full_size():
    g = W.grid2048(queries=10_000_000)
    print("grid2048: n=%d m=%d k=%d share=%d" % (g["n"], g["m"], g["k"], g["share_k"]), flush=True)
    idx = build(g, share_comps=g["share_k"], tune_cache=TUNE_CACHE)   # the benchmark's configuration
    st = spq.index_stats(idx)
    print({k: st[k] for k in ("v_bg", "ngroups", "v_bg2", "share_groups", "bf_rounds", "bg_bytes",
                              "ms_components", "ms_bg_apsp")}, flush=True)
    # groups of the tuned size, a few of them cut in halves (one 128-tile
    # wider than the 99th percentile): at least k / 16 groups, 32 for the share
    assert st["v_bg"] == 883_500 and st["ngroups"] >= g["k"] // 16 and st["share_groups"] >= 32
    rng = np.random.default_rng(44)
    lay = spq.index_layout(idx)
    flag = oracle.boundary(g["n"], g["eu"], g["ev"], g["part"])
    check_layout_fast(g, lay, flag)
    check_components_all(g, idx, lay)
    bgend = int(lay["bgoff"][512])
    check_bg_rows(g, idx, lay, np.concatenate([[0, bgend - 1], rng.integers(0, bgend, 20)]))
    out = run_queries(idx, g["v1"], g["v2"])
    assert (out >= 0).all()
    # 500 share sources x 16 targets, then the batch's own first 2,000 pairs
    sv = np.flatnonzero(g["part"] < g["share_k"]).astype(np.int32)
    src = sv[rng.integers(0, len(sv), 500)]
    v1 = np.repeat(src, 16)
    v2 = rng.integers(0, g["n"], v1.size).astype(np.int32)
    check_pairs_by_source(g, idx, v1, v2)
    check_pairs_by_source(g, idx, g["v1"][:2000], g["v2"][:2000])
    assert np.array_equal(out[:2000], run_queries(idx, g["v1"][:2000], g["v2"][:2000]))


def test_cached_memory_release_and_rebuild():
    g = W.grid32()
    a = build(g)
    ra = spq.index_bg_rows(a, 0, 348, 348)
    a.free()
    b = build(g)                      # reuses the cached blocks
    assert np.array_equal(spq.index_bg_rows(b, 0, 348, 348), ra)
    b.free()
    spq.release_cached_memory()
    c = build(g)                      # fresh allocations
    assert np.array_equal(spq.index_bg_rows(c, 0, 348, 348), ra)


def test_two_level_degenerate_groups():
    """One group (no level-2 graph at all), groups cut off from every other
    group (empty B2), and disconnected pieces, against Dijkstra."""
    rng = np.random.default_rng(90)
    # four disjoint 6x6 grids; components are 3x3 blocks, 4 per grid
    parts_u, parts_v, parts_w, part = [], [], [], []
    for piece in range(4):
        eu, ev, w = W.random_grid(rng, 6, 6, keep=0.9, diag=0.3, wlo=0, whi=40)
        parts_u.append(eu + 36 * piece)
        parts_v.append(ev + 36 * piece)
        parts_w.append(w)
        pp, _ = W.block_partition(6, 6, 3, 3)
        part.append(pp + 4 * piece)
    g = dict(name="pieces", n=144, eu=np.concatenate(parts_u), ev=np.concatenate(parts_v),
             w=np.concatenate(parts_w), part=np.concatenate(part).astype(np.int32), k=16)
    v1, v2 = all_pairs(144)
    for gc in (4, 8, 16, 3):
        idx = build(g, bg_method=2, group_comps=gc)
        st = spq.index_stats(idx)
        if gc == 4:
            assert st["v_bg2"] == 0          # each group is one piece
        if gc == 16:
            assert st["ngroups"] == 1 and st["v_bg2"] == 0
        lay = spq.index_layout(idx)
        check_bg_rows(g, idx, lay, np.arange(st["v_bg"]))
        check_queries(g, idx, v1, v2)
    share = build(g, share_comps=5, group_comps=4)
    check_share(g, share, 5)


def test_big_components_closed_in_one_batch():
    # three consecutive components of 1,200 vertices (padded to 1,280: above
    # the one-workgroup limit) are closed by one batched launch sequence, a
    # fourth of another size alone; every component against the oracle and
    # the per-component (plain) build
    rng = np.random.default_rng(77)
    eu, ev, w = W.random_grid(rng, 40, 110, keep=0.9, diag=0.2, wlo=1, whi=500)
    col = np.arange(40 * 110) % 110
    part = np.where(col < 30, 0, np.where(col < 60, 1, np.where(col < 90, 2, 3))).astype(np.int32)
    g = dict(name="bigbatch", n=40 * 110, eu=eu, ev=ev, w=w, part=part, k=4)
    idx = build(g)
    lay = spq.index_layout(idx)
    assert spq.index_stats(idx)["max_comp"] == 1200
    check_components(g, idx, lay)
    plain = build(g, plain=True)
    for c in range(4):
        size = int(np.count_nonzero(lay["comp"] == c))
        assert np.array_equal(spq.index_component(idx, c, size), spq.index_component(plain, c, size))
    rng2 = np.random.default_rng(3)
    v1 = rng2.integers(0, g["n"], 3000).astype(np.int32)
    v2 = rng2.integers(0, g["n"], 3000).astype(np.int32)
    check_queries(g, idx, v1, v2)


def wide_group_graph():
    """48x48 grid: components 0 and 1 interleave on a 12x12 corner as a
    checkerboard (every vertex on the boundary, 72 each), the rest are 2x4
    blocks: in groups of two components every group fits one 128-tile but
    the first (144 BG vertices)."""
    rng = np.random.default_rng(91)
    R = C = 48
    eu, ev, w = W.random_grid(rng, R, C, keep=0.95, diag=0.1, wlo=1, whi=60)
    r, c = np.divmod(np.arange(R * C), C)
    part = np.empty(R * C, np.int32)
    corner = (r < 12) & (c < 12)
    part[corner] = ((r + c) % 2)[corner]
    top = ~corner & (r < 12)
    part[top] = 2 + (r[top] // 2) * 9 + (c[top] - 12) // 4
    low = r >= 12
    part[low] = 2 + 54 + ((r[low] - 12) // 2) * 12 + c[low] // 4
    k = int(part.max()) + 1
    assert k == 272 and np.bincount(part).min() >= 8
    return dict(name="widegroup", n=R * C, eu=eu, ev=ev, w=w, part=part, k=k)


@pytest.mark.parametrize("blk", [1, 4])
def test_share_cuts_the_wide_group(blk):
    """A share build in groups of two components (136 groups): the one group
    a tile wider than all others is cut into its two components, the
    Bellman-Ford blocks still cover the same runs of components, and the
    share's BG rows and answers equal the full two-level index's (which keeps
    the wide group) and Dijkstra's."""
    g = wide_group_graph()
    full = build(g, bg_method=2, group_comps=2, level3_groups=-1)
    fst = spq.index_stats(full)
    assert fst["ngroups"] == 136 and fst["v_bg_padded"] == 256
    share = build(g, share_comps=40, group_comps=2, level3_groups=blk)
    st = spq.index_stats(share)
    assert st["ngroups"] == 137 and st["v_bg_padded"] == 128 and st["share_groups"] == 21, st
    lay = spq.index_layout(share)
    nrows = int(lay["bgoff"][40])
    V = st["v_bg"]
    assert np.array_equal(spq.index_bg_rows(share, 0, nrows, V), spq.index_bg_rows(full, 0, nrows, V))
    sv = share_vertices(g, 40)
    rng = np.random.default_rng(6)
    v1 = sv[rng.integers(0, len(sv), 20000)]
    v2 = rng.integers(0, g["n"], 20000).astype(np.int32)
    assert np.array_equal(run_queries(share, v1, v2), run_queries(full, v1, v2))
    check_queries(g, share, v1[:2000], v2[:2000])
