"""Shortest paths from the index (SPQ_PATHS): every returned path is a walk in
G from v1 to v2 whose edge weights sum to the Dijkstra distance.  Where several
shortest paths exist any one is valid, so the paths are checked, not matched.
"""
import numpy as np
import pytest

import oracle
from paper_1503_07192_amd import workloads as W

torch = pytest.importorskip("torch")
spq = pytest.importorskip("paper_1503_07192_amd.spq")

from test_gpu_parity import INF32, all_pairs, build, dev, small_cases  # noqa: E402

pytestmark = pytest.mark.gpu


def edge_weights(g):
    """Sorted keys u * n + v (both directions) and the lightest weight of each."""
    n = g["n"]
    eu, ev, w = (np.asarray(g[x], np.int64) for x in ("eu", "ev", "w"))
    keep = eu != ev
    u = np.concatenate([eu[keep], ev[keep]])
    v = np.concatenate([ev[keep], eu[keep]])
    ww = np.concatenate([w[keep], w[keep]])
    key = u * n + v
    order = np.lexsort((ww, key))
    key, ww = key[order], ww[order]
    first = np.ones(len(key), bool)
    first[1:] = key[1:] != key[:-1]
    return key[first], ww[first]


def check_paths(g, idx, v1, v2, max_len, allow_stall=False):
    paths, lens = spq.query_paths(idx, dev(v1), dev(v2), max_len)
    torch.cuda.synchronize()
    paths, lens = paths.cpu().numpy(), lens.cpu().numpy()
    src, inv = np.unique(v1, return_inverse=True)
    D = oracle.dijkstra(g["n"], g["eu"], g["ev"], g["w"], src)
    want = np.minimum(D[inv, v2], INF32)
    keys, wts = edge_weights(g)
    n = g["n"]
    stalled = 0
    for i in range(len(v1)):
        L = lens[i]
        if want[i] >= INF32:
            assert L == 0, (i, L)
            continue
        if L == -3 and allow_stall:
            stalled += 1
            continue
        assert L >= 1, (i, L, v1[i], v2[i], want[i])
        p = paths[i, :L].astype(np.int64)
        assert p[0] == v1[i] and p[-1] == v2[i]
        if L == 1:
            assert want[i] == 0
            continue
        k = p[:-1] * n + p[1:]
        pos = np.searchsorted(keys, k)
        assert (pos < len(keys)).all() and (keys[np.minimum(pos, len(keys) - 1)] == k).all(), "not a walk"
        assert wts[pos].sum() == want[i], (i, wts[pos].sum(), want[i])
    return lens, stalled


def test_grid32_paths():
    g = W.grid32()
    idx = build(g, paths=True)
    rng = np.random.default_rng(1)
    v1 = rng.integers(0, g["n"], 3000).astype(np.int32)
    v2 = rng.integers(0, g["n"], 3000).astype(np.int32)
    v1[:20] = v2[:20]
    lens, _ = check_paths(g, idx, v1, v2, 256)
    assert (lens[:20] == 1).all() and ((lens[20:] >= 2) | (v1[20:] == v2[20:])).all()
    # too little room: -2
    _, short = spq.query_paths(idx, dev(v1[20:40]), dev(v2[20:40]), 2)
    assert (short.cpu().numpy() == -2).all()
    # paths from the two-level store with level 3
    idx3 = build(g, paths=True, bg_method=2, group_comps=1, level3_groups=3)
    check_paths(g, idx3, v1[:1000], v2[:1000], 256)


CASES = small_cases()


@pytest.mark.parametrize("g", CASES, ids=[c["name"] for c in CASES])
def test_small_graph_paths_all_pairs(g):
    # weights from 0: the walk backs out of zero-weight dead ends
    idx = build(g, paths=True)
    v1, v2 = all_pairs(g["n"])
    lens, stalled = check_paths(g, idx, v1, v2, 4 * g["n"] + 4, allow_stall=True)
    assert stalled == 0


def test_paths_errors_and_share():
    rng = np.random.default_rng(41)
    eu, ev, w = W.random_grid(rng, 16, 16, keep=0.9, diag=0.2, wlo=1, whi=50)
    part, k = W.block_partition(16, 16, 4, 4, sb=2)
    g = dict(name="sharegrid", n=256, eu=eu, ev=ev, w=w, part=part, k=k)
    share = build(g, share_comps=4, group_comps=2, paths=True)
    sv = np.flatnonzero(part < 4).astype(np.int32)
    v1 = np.repeat(sv, 8).astype(np.int32)
    v2 = rng.integers(0, 256, len(v1)).astype(np.int32)
    check_paths(g, share, v1, v2, 257)
    outside = np.flatnonzero(part >= 4)[:5].astype(np.int32)
    _, lens = spq.query_paths(share, dev(outside), dev(outside), 16)
    assert (lens.cpu().numpy() == -1).all()
    bad = np.array([-1, 0, 300], np.int32)
    _, lens = spq.query_paths(share, dev(bad), dev(np.array([0, 256, 1], np.int32)), 16)
    assert (lens.cpu().numpy() == -1).all()
    plain = build(g)
    with pytest.raises(spq.SpqError) as ei:
        spq.query_paths(plain, dev(sv[:2]), dev(sv[:2]), 8)
    assert ei.value.name == "SPQ_EINVAL"


def test_paths_follow_reweighting():
    rng = np.random.default_rng(5)
    eu, ev, w = W.random_grid(rng, 20, 20, keep=0.9, diag=0.3, wlo=1, whi=100)
    part, k = W.block_partition(20, 20, 5, 5)
    g = dict(name="rw", n=400, eu=eu, ev=ev, w=w, part=part, k=k)
    idx = build(g, graph=True, paths=True, bg_method=2, group_comps=4)
    v1 = rng.integers(0, 400, 2000).astype(np.int32)
    v2 = rng.integers(0, 400, 2000).astype(np.int32)
    check_paths(g, idx, v1, v2, 401)
    h = dict(g)
    h["w"] = rng.integers(1, 10_000, len(eu)).astype(np.int32)
    spq.reweight(idx, dev(h["w"]))
    check_paths(h, idx, v1, v2, 401)


def test_delaunay1m_paths():
    g = W.delaunay1m()
    idx = build(g, paths=True, tune_cache=None)
    rng = np.random.default_rng(8)
    src = rng.integers(0, g["n"], 10).astype(np.int32)
    v1 = np.repeat(src, 10).astype(np.int32)
    v2 = rng.integers(0, g["n"], len(v1)).astype(np.int32)
    lens, stalled = check_paths(g, idx, v1, v2, 8192, allow_stall=True)
    assert stalled == 0 and (lens > 1).all()
