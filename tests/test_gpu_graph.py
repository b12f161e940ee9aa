"""Builds captured as HIP graphs (SPQ_GRAPH) and their replays with new
weights (spq_reweight_index), against eager builds and the oracle.

A captured build must give bit-identical components, BG rows and answers; a
replay with new weights must give exactly what a fresh build on those
weights gives (and Dijkstra on G).  Replays run several times in a row with
eager work (queries, torch kernels, synchronizations) between them.
"""
import numpy as np
import pytest

import oracle
from paper_1503_07192_amd import workloads as W

torch = pytest.importorskip("torch")
spq = pytest.importorskip("paper_1503_07192_amd.spq")

from test_gpu_parity import (INF32, all_pairs, build, check_bg_rows, check_components,  # noqa: E402
                             check_queries, clamp32, dev, run_queries)

pytestmark = pytest.mark.gpu


def same_index(g, a, b, rows=None, pairs=None):
    """a and b hold the same components, BG rows and answers."""
    la, lb = spq.index_layout(a), spq.index_layout(b)
    for key in la:
        assert np.array_equal(la[key], lb[key]), key
    sa, sb = spq.index_stats(a), spq.index_stats(b)
    for c in range(g["k"]):
        size = int(np.count_nonzero(la["comp"] == c))
        assert np.array_equal(spq.index_component(a, c, size), spq.index_component(b, c, size)), c
    V = sa["v_bg"]
    assert V == sb["v_bg"]
    rows = np.arange(V) if rows is None else rows
    for r in rows:
        assert np.array_equal(spq.index_bg_rows(a, int(r), 1, V), spq.index_bg_rows(b, int(r), 1, V)), r
    v1, v2 = all_pairs(g["n"]) if pairs is None else pairs
    assert np.array_equal(run_queries(a, v1, v2), run_queries(b, v1, v2))


def grid_case(seed, R, C, blk, whi=100):
    rng = np.random.default_rng(seed)
    eu, ev, w = W.random_grid(rng, R, C, keep=0.9, diag=0.3, wlo=1, whi=whi)
    part, k = W.block_partition(R, C, blk, blk)
    return dict(name="grid%dx%d" % (R, C), n=R * C, eu=eu, ev=ev, w=w, part=part, k=k)


def bigcomp_case():
    rng = np.random.default_rng(66)
    eu, ev, w = W.random_grid(rng, 35, 40, keep=0.9, diag=0.2)
    n = 1400
    part = np.where(np.arange(n) < 1200, 0, 1 + (np.arange(n) % 3)).astype(np.int32)
    return dict(name="bigcomp", n=n, eu=eu, ev=ev, w=w, part=part, k=4)


GRAPH_CASES = [
    ("grid32_flat", lambda: W.grid32(), {}),
    ("grid32_flat_nolookahead", lambda: W.grid32(), {"lookahead": False}),
    ("grid32_flat_tile64_plain", lambda: W.grid32(), {"bg_tile": 64, "plain": True}),
    ("grid32_two_level", lambda: W.grid32(), {"bg_method": 2, "group_comps": 4}),
    ("grid30_two_level_ragged", lambda: grid_case(3, 30, 27, 5), {"bg_method": 2, "group_comps": 3}),
    ("grid30_level3", lambda: grid_case(3, 30, 27, 5),
     {"bg_method": 2, "group_comps": 2, "level3_groups": 3}),
    ("bigcomp_flat", bigcomp_case, {}),
    ("bigcomp_two_level", bigcomp_case, {"bg_method": 2, "group_comps": 2}),
    # four-tile pivot blocks: the 1,280-wide component closure runs 4 + 4 + 2
    ("bigcomp_pivot512", bigcomp_case, {"bg_pivot": 512}),
    ("grid30_level3_pivot512", lambda: grid_case(3, 30, 27, 5),
     {"bg_method": 2, "group_comps": 2, "level3_groups": 3, "bg_pivot": 512}),
    # group and super-group matrices of several tiles: their batched closures
    # take the lookahead inside the capture (4 groups of 4 tiles; 4
    # super-groups of 3 tiles)
    ("grid64_two_level_batch_lookahead", lambda: grid_case(5, 64, 64, 8),
     {"bg_method": 2, "group_comps": 16}),
    ("grid64_level3_batch_lookahead", lambda: grid_case(5, 64, 64, 8),
     {"bg_method": 2, "group_comps": 2, "level3_groups": 8}),
]


@pytest.mark.parametrize("name,make,kw", GRAPH_CASES, ids=[c[0] for c in GRAPH_CASES])
def test_graph_build_equals_eager(name, make, kw):
    g = make()
    eager = build(g, **kw)
    cap = build(g, graph=True, **kw)
    st = spq.index_stats(cap)
    assert st["graphs"] == (1 if st["bg_method"] == 1 else 3 if st["groups3"] else 2)
    assert st["graph_nodes"] > 0 and st["reweights"] == 0
    assert spq.index_stats(eager)["graphs"] == 0
    pairs = None
    if g["n"] > 1100:
        rng = np.random.default_rng(4)
        pairs = (rng.integers(0, g["n"], 20000).astype(np.int32),
                 rng.integers(0, g["n"], 20000).astype(np.int32))
    same_index(g, eager, cap, pairs=pairs)
    v1, v2 = pairs if pairs else all_pairs(g["n"])
    check_queries(g, cap, v1[:5000], v2[:5000])


def reweighted(g, seed, lo, hi):
    rng = np.random.default_rng(seed)
    h = dict(g)
    h["w"] = rng.integers(lo, hi + 1, size=len(g["eu"])).astype(np.int32)
    return h


@pytest.mark.parametrize("kw", [{}, {"bg_method": 2, "group_comps": 3},
                                {"bg_method": 2, "group_comps": 1, "level3_groups": 4}],
                         ids=["flat", "two_level", "level3"])
def test_reweight_replays_match_fresh_builds(kw):
    g = grid_case(11, 24, 26, 6)
    idx = build(g, graph=True, **kw)
    v1, v2 = all_pairs(g["n"])
    scratch = torch.zeros(1 << 20, dtype=torch.int32, device="cuda")
    seq = [reweighted(g, 100, 1, 1000), reweighted(g, 101, 0, 5), g, reweighted(g, 102, 1, 10**6)]
    for i, h in enumerate(seq):
        print("reweight %d" % i, flush=True)
        spq.reweight(idx, dev(h["w"]))
        got = run_queries(idx, v1, v2)
        # eager work between the replays
        scratch.add_(i)
        torch.cuda.synchronize()
        fresh = build(h, **kw)
        assert np.array_equal(got, run_queries(fresh, v1, v2)), "replay %d" % i
        same_index(h, idx, fresh, rows=np.arange(0, spq.index_stats(idx)["v_bg"], 7),
                   pairs=(v1[::13], v2[::13]))
        check_queries(h, idx, v1[::7], v2[::7])
        fresh.free()
    assert spq.index_stats(idx)["reweights"] == len(seq)
    assert int(scratch[0]) == sum(range(len(seq)))


def test_reweight_errors_leave_the_index_unchanged():
    g = grid_case(12, 12, 12, 4)
    idx = build(g, graph=True)
    v1, v2 = all_pairs(g["n"])
    before = run_queries(idx, v1, v2)
    bad = g["w"].copy()
    bad[5] = -1
    with pytest.raises(spq.SpqError) as ei:
        spq.reweight(idx, dev(bad))
    assert ei.value.name == "SPQ_EINVAL"
    bad[5] = INF32
    with pytest.raises(spq.SpqError) as ei:
        spq.reweight(idx, dev(bad))
    assert ei.value.name == "SPQ_EINVAL"
    assert np.array_equal(run_queries(idx, v1, v2), before)
    eager = build(g)
    with pytest.raises(spq.SpqError) as ei:
        spq.reweight(eager, dev(g["w"]))
    assert ei.value.name == "SPQ_EINVAL" and "SPQ_GRAPH" in str(ei.value)
    with pytest.raises(spq.SpqError):
        build(g, graph=True, profile=True)


def _two_paths(wt):
    eu = np.array([0, 1, 2, 4, 5, 6], np.int32)
    return dict(name="paths", n=8, eu=eu, ev=eu + 1, w=np.full(6, wt, np.int32),
                part=np.array([0, 0, 1, 1, 2, 2, 3, 3], np.int32), k=4)


def _long_path(n, wt):
    eu = np.arange(n - 1, dtype=np.int32)
    part = np.minimum(np.arange(n) // 2, 4).astype(np.int32)
    return dict(name="longpath", n=n, eu=eu, ev=eu + 1, w=np.full(n - 1, wt, np.int32), part=part,
                k=int(part.max()) + 1)


@pytest.mark.parametrize("method", [1, 2])
def test_reweight_certificate(method):
    kw = dict(bg_method=method, group_comps=2)
    v1, v2 = all_pairs(8)
    # captured without the certificate, replayed with weights that need it
    small, large = _two_paths(3), _two_paths(500_000_000)
    idx = build(small, graph=True, **kw)
    check_queries(small, idx, v1, v2)
    spq.reweight(idx, dev(large["w"]))
    check_queries(large, idx, v1, v2)
    spq.reweight(idx, dev(small["w"]))
    check_queries(small, idx, v1, v2)
    # captured with the certificate, replayed with and without it
    idx2 = build(large, graph=True, **kw)
    check_queries(large, idx2, v1, v2)
    spq.reweight(idx2, dev(small["w"]))
    check_queries(small, idx2, v1, v2)
    spq.reweight(idx2, dev(large["w"]))
    check_queries(large, idx2, v1, v2)
    # a replay whose distances cannot be represented invalidates the index
    p = _long_path(9, 1)
    idx3 = build(p, graph=True, **kw)
    a, b = all_pairs(9)
    check_queries(p, idx3, a, b)
    with pytest.raises(spq.SpqError) as ei:
        spq.reweight(idx3, dev(np.full(8, 600_000_000, np.int32)))
    assert ei.value.name == "SPQ_ERANGE"
    with pytest.raises(spq.SpqError) as ei:
        run_queries(idx3, a, b)
    assert ei.value.name == "SPQ_ERANGE"
    with pytest.raises(spq.SpqError) as ei:
        spq.reweight(idx3, dev(p["w"]))
    assert ei.value.name == "SPQ_ERANGE"


def test_grid256d_graph_build_and_reweight():
    g = W.grid256d(queries=20_000)
    v1, v2 = g["v1"], g["v2"]
    eager = build(g)
    want = run_queries(eager, v1, v2)
    eager.free()
    idx = build(g, graph=True)
    assert np.array_equal(run_queries(idx, v1, v2), want)
    h = reweighted(g, 7, 1, 1000)
    spq.reweight(idx, dev(h["w"]))
    got = run_queries(idx, v1, v2)
    fresh = build(h)
    assert np.array_equal(got, run_queries(fresh, v1, v2))
    fresh.free()
    check_queries(h, idx, v1[:2000], v2[:2000])
    spq.reweight(idx, dev(g["w"]))
    assert np.array_equal(run_queries(idx, v1, v2), want)


def test_streams_of_freed_indexes_are_reused():
    """A freed index hands its side and capture streams back to the library
    and later builds take them again.  Builds alive at the same time, builds
    made after frees (on reused streams), a capture and replays on a reused
    capture stream, and host-array queries (whose stream comes from the same
    cache) all agree with a build that uses no side stream."""
    g = W.grid32()
    v1, v2 = all_pairs(g["n"])
    base = build(g, bg_tile=64, lookahead=False)
    ref_rows = spq.index_bg_rows(base, 0, 348, 348)
    ref_q = run_queries(base, v1, v2)
    for rep in range(3):
        print("round %d" % rep, flush=True)
        a = build(g, bg_tile=64)
        b = build(g, bg_tile=64, graph=True)
        c = build(g, bg_method=2, group_comps=1, level3_groups=2)
        for x in (a, b, c):
            assert np.array_equal(spq.index_bg_rows(x, 0, 348, 348), ref_rows)
            assert np.array_equal(run_queries(x, v1, v2), ref_q)
        assert np.array_equal(spq.query_batch_host(a, v1[::5], v2[::5]), ref_q[::5])
        h = reweighted(g, 40 + rep, 1, 1000)
        spq.reweight(b, dev(h["w"]))
        fresh = build(h, bg_tile=64, lookahead=False)
        assert np.array_equal(run_queries(b, v1, v2), run_queries(fresh, v1, v2))
        for x in (a, b, c, fresh):
            x.free()
    check_queries(g, base, v1[::11], v2[::11])
    base.free()
    spq.release_cached_memory()
    again = build(g, bg_tile=64, graph=True)
    assert np.array_equal(run_queries(again, v1, v2), ref_q)


def test_batched_closures_with_lookahead_equal_flat():
    """The group closures (4 matrices of 512, 4 tiles each) and the
    super-group closures (4 of 384) run their rounds with the lookahead, a
    batch side by side: with two-tile and one-tile pivot blocks, and without
    the lookahead, every BG row and query equals the flat build's."""
    g = grid_case(5, 64, 64, 8)
    flat = build(g, bg_method=1, lookahead=False)
    V = spq.index_stats(flat)["v_bg"]
    assert V == 1504
    want_rows = spq.index_bg_rows(flat, 0, V, V)
    rng = np.random.default_rng(9)
    v1 = rng.integers(0, g["n"], 20000).astype(np.int32)
    v2 = rng.integers(0, g["n"], 20000).astype(np.int32)
    want_q = run_queries(flat, v1, v2)
    check_queries(g, flat, v1[:3000], v2[:3000])
    cases = [({"group_comps": 16}, 4, 0), ({"group_comps": 16, "bg_pivot": 128}, 4, 0),
             ({"group_comps": 16, "lookahead": False}, 4, 0),
             ({"group_comps": 2, "level3_groups": 8}, 32, 4),
             ({"group_comps": 2, "level3_groups": 8, "bg_pivot": 128}, 32, 4),
             ({"group_comps": 2, "level3_groups": 8, "lookahead": False}, 32, 4)]
    for kw, ngroups, groups3 in cases:
        x = build(g, bg_method=2, **kw)
        st = spq.index_stats(x)
        assert st["ngroups"] == ngroups and st["groups3"] == groups3, kw
        assert np.array_equal(spq.index_bg_rows(x, 0, V, V), want_rows), kw
        assert np.array_equal(run_queries(x, v1, v2), want_q), kw
        x.free()

