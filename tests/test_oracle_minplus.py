"""Pins of the oracle's (min, +) product against facts that do not come from it.

The product C[i][j] = min over k of A[i][k] + B[k][j] is how distance tables
compose through a separating vertex set (the two stages of Algorithm 2, and
the group-level composition of the two-level BG).  Each pin would fail under a
plausible mistake: max for min, an operand read transposed, the last k
dropped, INF treated as a number.  The last tests plant such mistakes in
copies of the product and check that the pins catch them.
"""
import numpy as np

import oracle
from oracle import O_INF
from paper_1503_07192_amd import workloads as W


def rand_table(rng, n, p, lo=0, hi=50, inf_frac=0.3):
    A = rng.integers(lo, hi, size=(n, p)).astype(np.int64)
    A[rng.random((n, p)) < inf_frac] = O_INF
    return A


def identity(n):
    I = np.full((n, n), O_INF, np.int64)
    np.fill_diagonal(I, 0)
    return I


def check_identity(mp, rng):
    for n, K, p in ((1, 1, 1), (3, 5, 2), (7, 4, 9), (16, 17, 3)):
        A = rand_table(rng, n, K)
        B = rand_table(rng, K, p)
        assert np.array_equal(mp(A, identity(K)), A)
        assert np.array_equal(mp(identity(K), B), B)


def walks_upto_two_edges(n, eu, ev, w):
    """Shortest walk of at most two edges, enumerated edge by edge."""
    adj = [[] for _ in range(n)]
    for u, v, x in zip(eu.tolist(), ev.tolist(), w.tolist()):
        adj[u].append((v, x))
        adj[v].append((u, x))
    best = np.full((n, n), O_INF, np.int64)
    for s in range(n):
        best[s, s] = 0
        for u, x1 in adj[s]:
            best[s, u] = min(best[s, u], x1)
            for t, x2 in adj[u]:
                best[s, t] = min(best[s, t], x1 + x2)
    return best


def check_two_edge_walks(mp, count=60, seed=11):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        n = int(rng.integers(1, 9))
        eu, ev, w = W.random_graph(rng, n, int(rng.integers(0, 15)), 0, 20)
        W0 = oracle.dense_init(n, eu, ev, w)
        assert np.array_equal(mp(W0, W0), walks_upto_two_edges(n, eu, ev, w))


def check_closed_form(mp, rng, n=6, K=11, p=5):
    # A[i][k] = a_i + c_k, B[k][j] = d_k + b_j: C[i][j] = a_i + b_j + min_k (c_k + d_k)
    a, c = rng.integers(0, 100, n), rng.integers(0, 100, K)
    d, b = rng.integers(0, 100, K), rng.integers(0, 100, p)
    A = (a[:, None] + c[None, :]).astype(np.int64)
    B = (d[:, None] + b[None, :]).astype(np.int64)
    want = a[:, None] + b[None, :] + (c + d).min()
    assert np.array_equal(mp(A, B), want)


def test_identity_element():
    check_identity(oracle.minplus, np.random.default_rng(1))


def test_square_is_walks_of_at_most_two_edges():
    check_two_edge_walks(oracle.minplus)


def test_repeated_squaring_reaches_brute_force_distances():
    rng = np.random.default_rng(5)
    for _ in range(40):
        n = int(rng.integers(1, 9))
        eu, ev, w = W.random_graph(rng, n, int(rng.integers(0, 15)), 0, 20)
        D = oracle.dense_init(n, eu, ev, w)
        for _ in range(3):  # walks of up to 8 edges cover every simple path of n <= 8
            D = oracle.minplus(D, D)
        assert np.array_equal(D, oracle.brute_force_apsp(n, eu, ev, w))


def test_closed_form_sum_of_row_and_column_terms():
    check_closed_form(oracle.minplus, np.random.default_rng(2))


def test_transpose_and_associativity():
    rng = np.random.default_rng(3)
    A, B, C = rand_table(rng, 5, 7), rand_table(rng, 7, 4), rand_table(rng, 4, 6)
    assert np.array_equal(oracle.minplus(A, B).T, oracle.minplus(B.T.copy(), A.T.copy()))
    assert np.array_equal(oracle.minplus(oracle.minplus(A, B), C),
                          oracle.minplus(A, oracle.minplus(B, C)))


def test_empty_inner_dimension_and_all_inf_rows():
    C = oracle.minplus(np.zeros((3, 0), np.int64), np.zeros((0, 4), np.int64))
    assert C.shape == (3, 4) and (C == O_INF).all()
    rng = np.random.default_rng(4)
    A = rand_table(rng, 4, 6)
    A[2, :] = O_INF
    A[[0, 1, 3], 0] = 7
    C = oracle.minplus(A, rand_table(rng, 6, 5, inf_frac=0.0))
    assert (C[2] == O_INF).all()
    assert (C[[0, 1, 3]] < O_INF).all()


# ----------------------------------------------------- planted mistakes
def planted(kind):
    def mp(A, B):
        n, K = A.shape
        p = B.shape[1]
        C = np.full((n, p), O_INF if kind != "max" else -1, np.int64)
        for i in range(n):
            for j in range(p):
                ks = range(K - 1) if kind == "drop_last" else range(K)
                for k in ks:
                    x = A[k, i] if kind == "transposed" else A[i, k]
                    y = B[k, j]
                    s = O_INF if (x == O_INF or y == O_INF) else x + y
                    if kind == "inf_as_number":  # int64 addition that wraps past O_INF
                        s = (int(x) + int(y) + 2**63) % 2**64 - 2**63
                    C[i, j] = max(C[i, j], s) if kind == "max" else min(C[i, j], s)
        return C
    return mp


def caught(check, mp, *args):
    try:
        check(mp, *args)
    except AssertionError:
        return True
    return False


def test_planted_mistakes_are_caught():
    rng = lambda: np.random.default_rng(1)
    assert caught(check_identity, planted("max"), rng())
    assert caught(check_identity, planted("drop_last"), rng())
    assert caught(check_closed_form, planted("transposed"), rng(), 8, 8, 8)
    assert caught(check_identity, planted("inf_as_number"), rng())
    # and the correct copy passes the same checks
    assert not caught(check_identity, planted("none"), rng())
    assert not caught(check_closed_form, planted("none"), rng())
