"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each pin would fail under a plausible mistake in the oracle: a dropped term
(no clique edges, no C1 = C2 correction), a wrong loop order in
Floyd-Warshall, distances in G where the induced component is meant, a
boundary taken from one edge end only.  The last group plants such mistakes
in copies of the oracle's steps and checks that the pins catch them.
"""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import O_INF
from paper_1503_07192_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


def all_pairs_dijkstra(n, eu, ev, w):
    return oracle.dijkstra(n, eu, ev, w, np.arange(n))


def tiny_graphs(count, seed=7, nmax=8, mmax=14):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        n = int(rng.integers(1, nmax + 1))
        m = int(rng.integers(0, mmax + 1))
        eu, ev, w = W.random_graph(rng, n, m, 0, 20)
        yield n, eu, ev, w


# ----------------------------------------------------------- brute force
def test_brute_force_matches_dijkstra_and_fw():
    """Definition of dist (Section 2) by path enumeration vs both algorithms."""
    for n, eu, ev, w in tiny_graphs(150):
        bf = oracle.brute_force_apsp(n, eu, ev, w)
        dj = all_pairs_dijkstra(n, eu, ev, w)
        fw = oracle.fw(oracle.dense_init(n, eu, ev, w))
        assert np.array_equal(bf, dj)
        assert np.array_equal(bf, fw)


def test_hand_example_distances():
    g = json.load(open(os.path.join(HERE, "golden", "hand6.json")))
    e = np.array(g["edges"])
    eu, ev, w = e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2].astype(np.int32)
    assert np.array_equal(all_pairs_dijkstra(g["n"], eu, ev, w), np.array(g["dist_G"]))
    assert np.array_equal(oracle.brute_force_apsp(g["n"], eu, ev, w), np.array(g["dist_G"]))


# ----------------------------------------------------------- closed forms
@pytest.mark.parametrize("c", [1, 7])
def test_grid_constant_weight_is_manhattan(c):
    R, C = 7, 9
    eu, ev = W.grid_edges(R, C)
    w = np.full(len(eu), c, np.int32)
    d = all_pairs_dijkstra(R * C, eu, ev, w)
    r, q = np.divmod(np.arange(R * C), C)
    man = np.abs(r[:, None] - r[None, :]) + np.abs(q[:, None] - q[None, :])
    assert np.array_equal(d, c * man)
    assert np.array_equal(oracle.fw(oracle.dense_init(R * C, eu, ev, w)), c * man)


def test_path_graph_prefix_sums():
    rng = np.random.default_rng(3)
    n = 40
    w = rng.integers(0, 1000, n - 1).astype(np.int32)
    eu = np.arange(n - 1, dtype=np.int32)
    ev = eu + 1
    ps = np.concatenate([[0], np.cumsum(w.astype(np.int64))])
    want = np.abs(ps[:, None] - ps[None, :])
    assert np.array_equal(all_pairs_dijkstra(n, eu, ev, w), want)
    # shuffled edge order and vertex relabelling do not matter
    perm = rng.permutation(n).astype(np.int32)
    eo = rng.permutation(n - 1)
    d2 = all_pairs_dijkstra(n, perm[eu[eo]], perm[ev[eo]], w[eo])
    assert np.array_equal(d2[np.ix_(perm, perm)], want)


def test_disconnected_and_zero_weights():
    n = 5
    eu = np.array([0, 1, 3], np.int32)
    ev = np.array([1, 2, 4], np.int32)
    w = np.array([0, 0, 5], np.int32)
    d = all_pairs_dijkstra(n, eu, ev, w)
    assert d[0, 2] == 0 and d[3, 4] == 5
    assert d[0, 3] == O_INF and d[2, 4] == O_INF


# ---------------------------------------------------- component APSP
def test_component_apsp_is_on_induced_subgraph():
    """APSP(C) is distances in C, not in G (remark before Lemma 1)."""
    g = json.load(open(os.path.join(HERE, "golden", "hand6.json")))
    e = np.array(g["edges"])
    eu, ev, w = e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2].astype(np.int32)
    part = np.array(g["part"], np.int32)
    members, apsp = oracle.component_apsp(g["n"], eu, ev, w, part, g["k"])
    assert members[0].tolist() == g["apsp_A_members"]
    assert np.array_equal(apsp[0], np.array(g["apsp_A"]))
    assert np.array_equal(apsp[1], np.array(g["apsp_B"]))
    assert oracle.boundary(g["n"], eu, ev, part).nonzero()[0].tolist() == g["boundary"]


def test_component_apsp_vs_brute_force_on_induced_graph():
    rng = np.random.default_rng(11)
    for _ in range(40):
        n = int(rng.integers(2, 16))
        eu, ev, w = W.random_graph(rng, n, int(rng.integers(0, 30)), 0, 50)
        k = int(rng.integers(1, min(n, 4) + 1))
        part = W.random_partition(rng, n, k)
        members, apsp = oracle.component_apsp(n, eu, ev, w, part, k)
        dG = all_pairs_dijkstra(n, eu, ev, w)
        for mem, A in zip(members, apsp):
            if len(mem) > 9:
                continue
            inside = np.isin(eu, mem) & np.isin(ev, mem)
            relabel = {int(v): i for i, v in enumerate(mem)}
            su = np.array([relabel[int(x)] for x in eu[inside]], np.int32)
            sv = np.array([relabel[int(x)] for x in ev[inside]], np.int32)
            bf = oracle.brute_force_apsp(len(mem), su, sv, w[inside])
            assert np.array_equal(A, bf)
            sub = dG[np.ix_(mem, mem)]
            assert (A >= sub).all()       # dist_C >= dist_G elementwise


# ------------------------------------------------------- Lemma 1 and 3
def partitioned_cases():
    rng = np.random.default_rng(5)
    cases = [("grid32", W.grid32())]
    for t in range(25):
        R, C = int(rng.integers(2, 9)), int(rng.integers(2, 9))
        eu, ev, w = W.random_grid(rng, R, C, keep=0.85, diag=0.3, wlo=0, whi=30)
        n = R * C
        k = int(rng.integers(1, min(n, 7) + 1))
        part = W.random_partition(rng, n, k) if t % 2 else W.block_partition(R, C, 3, 3)[0]
        if t % 2 == 0:
            k = int(part.max()) + 1
        cases.append(("g%d" % t, dict(n=n, eu=eu, ev=ev, w=w, part=part, k=k)))
    for t in range(10):
        n = int(rng.integers(1, 12))
        eu, ev, w = W.random_graph(rng, n, int(rng.integers(0, 25)), 0, 9)
        k = int(rng.integers(1, n + 1))
        cases.append(("r%d" % t, dict(n=n, eu=eu, ev=ev, w=w, part=W.random_partition(rng, n, k), k=k)))
    return cases


CASES = partitioned_cases()


def lemma1_holds(g, T):
    if len(T.bg_ids) == 0:
        return True
    dG = oracle.dijkstra(g["n"], g["eu"], g["ev"], g["w"], T.bg_ids)
    return np.array_equal(T.dbg, dG[:, T.bg_ids])


def lemma3_holds(g, T, v1, v2, query=oracle.query_alg2):
    dG = oracle.dijkstra(g["n"], g["eu"], g["ev"], g["w"], v1)
    return np.array_equal(query(T, v1, v2), dG[np.arange(len(v1)), v2])


def all_pairs(n):
    a, b = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    return a.ravel().astype(np.int32), b.ravel().astype(np.int32)


@pytest.mark.parametrize("name,g", CASES, ids=[c[0] for c in CASES])
def test_lemma1_bg_distances_equal_g_distances(name, g):
    T = oracle.preprocess(g["n"], g["eu"], g["ev"], g["w"], g["part"], g["k"])
    assert lemma1_holds(g, T)


@pytest.mark.parametrize("name,g", CASES, ids=[c[0] for c in CASES])
def test_lemma3_query_equals_g_distance(name, g):
    T = oracle.preprocess(g["n"], g["eu"], g["ev"], g["w"], g["part"], g["k"])
    if "v1" in g:
        v1, v2 = g["v1"], g["v2"]
    else:
        v1, v2 = all_pairs(g["n"])
    assert lemma3_holds(g, T, v1, v2)


def test_hand_example_tables_and_queries():
    g = json.load(open(os.path.join(HERE, "golden", "hand6.json")))
    e = np.array(g["edges"])
    G = dict(n=g["n"], eu=e[:, 0].astype(np.int32), ev=e[:, 1].astype(np.int32),
             w=e[:, 2].astype(np.int32), part=np.array(g["part"], np.int32), k=g["k"])
    T = oracle.preprocess(G["n"], G["eu"], G["ev"], G["w"], G["part"], G["k"])
    assert T.bg_ids.tolist() == g["bg_vertices"]
    assert np.array_equal(T.dbg, np.array(g["dist_BG"]))
    qs = np.array(g["queries"])
    out = oracle.query_alg2(T, qs[:, 0].astype(np.int32), qs[:, 1].astype(np.int32))
    assert out.tolist() == qs[:, 2].tolist()


# ----------------------------------------------------- special cases
def test_k1_reduces_to_floyd_warshall():
    """k = 1: no boundary, the query is its same-component term alone = FW on G."""
    rng = np.random.default_rng(2)
    eu, ev, w = W.random_grid(rng, 6, 7, keep=0.8, diag=0.2)
    n = 42
    part = np.zeros(n, np.int32)
    T = oracle.preprocess(n, eu, ev, w, part, 1)
    assert len(T.bg_ids) == 0
    fw = oracle.fw(oracle.dense_init(n, eu, ev, w))
    assert np.array_equal(T.apsp[0], fw)
    v1, v2 = all_pairs(n)
    assert np.array_equal(oracle.query_alg2(T, v1, v2), fw.ravel())


def test_kn_singletons_bg_is_g():
    """k = n: every non-isolated vertex is boundary and BG = G on them."""
    rng = np.random.default_rng(4)
    eu, ev, w = W.random_grid(rng, 5, 6, keep=0.7)
    n = 30
    part = np.arange(n, dtype=np.int32)
    T = oracle.preprocess(n, eu, ev, w, part, n)
    deg = np.bincount(np.concatenate([eu, ev]), minlength=n)
    assert T.bg_ids.tolist() == np.flatnonzero(deg > 0).tolist()
    fw = oracle.fw(oracle.dense_init(n, eu, ev, w))
    assert np.array_equal(T.dbg, fw[np.ix_(T.bg_ids, T.bg_ids)])


def test_metric_invariants_grid32():
    g = W.grid32()
    d = all_pairs_dijkstra(g["n"], g["eu"], g["ev"], g["w"])
    assert np.array_equal(d, d.T)
    assert (np.diag(d) == 0).all()
    assert (d[g["eu"], g["ev"]] <= g["w"]).all()
    for s in range(0, g["n"], 97):   # triangle inequality through s
        assert (d <= d[:, [s]] + d[[s], :]).all()


def test_partition_and_boundary_superset_invariance():
    rng = np.random.default_rng(9)
    eu, ev, w = W.random_grid(rng, 8, 8, keep=0.9, diag=0.4, wlo=1, whi=50)
    n = 64
    v1, v2 = all_pairs(n)
    answers = []
    for part, k in [W.block_partition(8, 8, 4, 4), W.block_partition(8, 8, 2, 8),
                    (W.random_partition(rng, n, 5), 5)]:
        T = oracle.preprocess(n, eu, ev, w, part, k)
        answers.append(oracle.query_alg2(T, v1, v2))
        extra = oracle.boundary(n, eu, ev, part) | (rng.random(n) < 0.3)
        T2 = oracle.preprocess(n, eu, ev, w, part, k, bflag=extra)
        answers.append(oracle.query_alg2(T2, v1, v2))
    for a in answers[1:]:
        assert np.array_equal(a, answers[0])


# --------------------------------------------------- planted mistakes
def test_planted_fw_wrong_loop_order_is_caught():
    def fw_k_inner(d):
        n = d.shape[0]
        for i in range(n):
            for j in range(n):
                for k in range(n):
                    if d[i, k] != O_INF and d[k, j] != O_INF and d[i, k] + d[k, j] < d[i, j]:
                        d[i, j] = d[i, k] + d[k, j]
        return d
    caught = False
    for n, eu, ev, w in tiny_graphs(150):
        bad = fw_k_inner(oracle.dense_init(n, eu, ev, w))
        if not np.array_equal(bad, oracle.brute_force_apsp(n, eu, ev, w)):
            caught = True
            break
    assert caught


def test_planted_missing_line13_is_caught():
    def query_no_line13(T, v1, v2):
        # same tables, but a component's own distance is never consulted:
        # emulate by handing Algorithm 2 a partition whose C1 = C2 check never fires
        out = []
        full = oracle.query_alg2(T, v1, v2)
        for a, b, f in zip(v1, v2, full):
            same = any(a in m and b in m for m in T.members)
            if same:
                # recompute the two min stages only
                c = [i for i, m in enumerate(T.members) if a in m][0]
                m, A = T.members[c], T.apsp[c]
                bl = np.searchsorted(m, T.bverts[c])
                base = sum(len(x) for x in T.bverts[:c])
                ia, ib = np.searchsorted(m, a), np.searchsorted(m, b)
                best = O_INF
                for j, b2 in enumerate(bl):
                    for i, b1 in enumerate(bl):
                        x = A[ia, b1], T.dbg[base + i, base + j], A[b2, ib]
                        if O_INF not in x:
                            best = min(best, sum(x))
                out.append(best)
            else:
                out.append(f)
        return np.array(out, np.int64)
    g = dict(n=42, part=np.zeros(42, np.int32), k=1)
    rng = np.random.default_rng(2)
    g["eu"], g["ev"], g["w"] = W.random_grid(rng, 6, 7, keep=0.8)
    T = oracle.preprocess(g["n"], g["eu"], g["ev"], g["w"], g["part"], g["k"])
    v1, v2 = all_pairs(42)
    assert lemma3_holds(g, T, v1, v2)
    assert not lemma3_holds(g, T, v1, v2, query=query_no_line13)


def test_planted_bg_without_clique_edges_is_caught():
    g = W.grid32()
    T = oracle.preprocess(g["n"], g["eu"], g["ev"], g["w"], g["part"], g["k"])
    bgidx = {int(v): i for i, v in enumerate(T.bg_ids)}
    keep = np.array([int(u) in bgidx and int(v) in bgidx and u != v
                     for u, v in zip(g["eu"], g["ev"])])
    bu = np.array([bgidx[int(x)] for x in g["eu"][keep]], np.int32)
    bv = np.array([bgidx[int(x)] for x in g["ev"][keep]], np.int32)
    T.dbg = oracle.bg_apsp(T.bg_ids, bu, bv, g["w"][keep])
    assert not lemma1_holds(g, T)


def test_planted_one_sided_boundary_is_caught():
    g = W.grid32()
    part = g["part"]
    cross = part[g["eu"]] != part[g["ev"]]
    one_sided = np.zeros(g["n"], bool)
    one_sided[g["eu"][cross]] = True          # forgets the ev end
    T = oracle.preprocess(g["n"], g["eu"], g["ev"], g["w"], part, g["k"], bflag=one_sided)
    assert not lemma3_holds(g, T, g["v1"], g["v2"])


def test_planted_g_distances_in_component_table_is_caught():
    """A table holding dist_G instead of dist_C fails the induced-subgraph pin."""
    gd = json.load(open(os.path.join(HERE, "golden", "hand6.json")))
    dG = np.array(gd["dist_G"])
    wrong_A = dG[np.ix_([0, 1, 2], [0, 1, 2])]
    assert not np.array_equal(wrong_A, np.array(gd["apsp_A"]))


def test_int32_sentinel_mapping():
    d = np.array([0, 5, O_INF], np.int64)
    assert oracle.to_int32_distance(d).tolist() == [0, 5, 2**31 - 1]
    with pytest.raises(OverflowError):
        oracle.to_int32_distance(np.array([2**31 - 1], np.int64))
