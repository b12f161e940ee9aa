"""CPU oracle for the planar shortest-path query structure.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use it; the product library never does.  It shares no code with the
HIP path (its heavy loops live in ``oracle.c``, compiled with gcc).

All distances are int64; ``O_INF`` (int64 max) means "no path".

What it computes, each from its definition in the paper:

* ``dijkstra``        single-source distances in G (Section 2 definitions,
                      Dijkstra's algorithm from Section 1).
* ``brute_force_apsp`` exhaustive enumeration of simple paths (tiny graphs);
                      the length of a path is the sum of its edge weights,
                      dist is the minimum over paths (Section 2).
* ``boundary``        vertices with a neighbour in another component
                      (Section 2, definition of the boundary).
* ``component_apsp``  APSP(C) on the subgraph *induced* by each component
                      (Algorithm 1, Phase 2) by Floyd-Warshall on a matrix
                      initialised to wt / infinity (Section 4).
* ``boundary_graph``  BG: vertices = all boundary vertices; edges = the edges of
                      G between boundary vertices plus, for every pair of
                      boundary vertices of one component, an edge weighted by
                      their distance inside that component (Algorithm 1,
                      Phase 2 second step and Phase 3 first step).
* ``bg_apsp``         SSSP in BG from each requested BG vertex by Dijkstra
                      (Algorithm 1, Phase 3).
* ``query_alg2``      Algorithm 2 evaluated literally on those tables.
* ``minplus``         the (min, +) product of two distance tables: how
                      distances compose through a separating vertex set (the
                      two stages of Algorithm 2; the composition of the
                      two-level BG applies it one level up).

Pins (in tests/test_oracle_pins.py): brute force on tiny graphs; closed forms
on grids and paths; for ``minplus``, its identity element, walks of at most
two edges enumerated edge by edge, repeated squaring reaching the
brute-force distances, a closed form and the transpose identity; Lemma 1 (BG distances equal G distances); Lemma 3 (the
query equals the G distance); the k = 1 and k = n reductions; invariance under
partition and boundary superset; metric invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

O_INF = np.iinfo(np.int64).max
HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

LIB_NATIVE = os.path.join(HERE, "liboracle_native.so")

_lib = None
_native = False


def build(force: bool = False, native: bool = False) -> str:
    """Compile oracle.c with gcc: oracle/liboracle.so (-O2, portable), or with
    native=True oracle/liboracle_native.so (-O3 -march=native, for timing the
    oracle on the host that runs it; built there, never shipped)."""
    out = LIB_NATIVE if native else LIB
    flags = ["-O3", "-march=native"] if native else ["-O2"]
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(SRC):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *flags, "-std=c11", "-shared", "-fPIC", "-pthread",
                               SRC, "-o", tmp])
        os.replace(tmp, out)
    return out


def configure(native: bool):
    """Select the build the functions below call (before their first use):
    the portable one (tests) or the -O3 -march=native one (CPU timing)."""
    global _lib, _native
    if _lib is not None and native != _native:
        raise RuntimeError("oracle library already loaded")
    _native = native


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build(force=_native, native=_native))
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C")
        L.oracle_dijkstra.restype = ctypes.c_int
        L.oracle_dijkstra.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, i32p,
                                      ctypes.c_int64, i32p, i64p, ctypes.c_int32]
        L.oracle_fw.restype = None
        L.oracle_fw.argtypes = [ctypes.c_int32, i64p]
        L.oracle_fw_many.restype = None
        L.oracle_fw_many.argtypes = [ctypes.c_int32, i32p, i64p, i64p, ctypes.c_int32]
        L.oracle_minplus.restype = None
        L.oracle_minplus.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, i64p, i64p,
                                     i64p]
        L.oracle_query_alg2.restype = None
        L.oracle_query_alg2.argtypes = [ctypes.c_int64, i32p, i32p, i32p, i32p, i32p, i64p,
                                        i64p, i32p, i32p, ctypes.c_int32, i64p, i64p]
        _lib = L
    return _lib


def _threads(nthreads):
    return int(nthreads) if nthreads else max(1, min(16, os.cpu_count() or 1))


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


# ------------------------------------------------------------------ G-level
def dijkstra(n, eu, ev, w, sources, nthreads=None):
    """dist_G(s, v) for every s in sources, as an int64 [len(sources), n] array."""
    src = _i32(np.atleast_1d(sources))
    out = np.empty((len(src), n), np.int64)
    rc = lib().oracle_dijkstra(int(n), len(eu), _i32(eu), _i32(ev), _i32(w),
                               len(src), src, out, _threads(nthreads))
    if rc != 0:
        raise ValueError("oracle_dijkstra: invalid graph or sources")
    return out


def dense_init(n, eu, ev, w):
    """Distance matrix before any relaxation: 0 on the diagonal, the lightest
    parallel edge where an edge exists, O_INF elsewhere (Section 4)."""
    d = np.full((n, n), O_INF, np.int64)
    for u, v, x in zip(np.asarray(eu).tolist(), np.asarray(ev).tolist(), np.asarray(w).tolist()):
        if u != v:
            if x < d[u, v]:
                d[u, v] = x
            if x < d[v, u]:
                d[v, u] = x
    np.fill_diagonal(d, 0)
    return d


def fw(d):
    """Floyd-Warshall in place on an int64 matrix (O_INF = no edge)."""
    d = np.ascontiguousarray(d, np.int64)
    lib().oracle_fw(d.shape[0], d)
    return d


def brute_force_apsp(n, eu, ev, w):
    """Minimum over all simple paths of the sum of edge weights (n <= 9)."""
    assert n <= 9, "brute force is for tiny graphs"
    adj = [[] for _ in range(n)]
    for u, v, x in zip(np.asarray(eu).tolist(), np.asarray(ev).tolist(), np.asarray(w).tolist()):
        adj[u].append((v, x))
        adj[v].append((u, x))
    best = np.full((n, n), O_INF, np.int64)
    for s in range(n):
        best[s, s] = 0
        seen = [False] * n
        seen[s] = True

        def walk(u, length):
            for v, x in adj[u]:
                if not seen[v]:
                    L = length + x
                    if L < best[s, v]:
                        best[s, v] = L
                    seen[v] = True
                    walk(v, L)
                    seen[v] = False
        walk(s, 0)
    return best


# ------------------------------------------------------- partition tables
def boundary(n, eu, ev, part):
    """True for vertices with at least one neighbour in another component."""
    eu, ev, part = np.asarray(eu), np.asarray(ev), np.asarray(part)
    cross = part[eu] != part[ev]
    flag = np.zeros(n, bool)
    flag[eu[cross]] = True
    flag[ev[cross]] = True
    return flag


class Tables:
    """Preprocessing output in the oracle's own layout.

    members[c]   vertices of component c in ascending id order
    apsp[c]      int64 distances in the subgraph induced by members[c]
    bverts[c]    boundary vertices of c, ascending id (a subset of members[c])
    bg_ids       all boundary vertices, component by component (BG vertex order)
    """


def component_apsp(n, eu, ev, w, part, k, comps=None, nthreads=None):
    """APSP(C) of the induced subgraph of every (or each listed) component."""
    eu, ev, w, part = (np.asarray(a) for a in (eu, ev, w, part))
    comps = list(range(k)) if comps is None else list(comps)
    order = np.argsort(part, kind="stable")
    starts = np.searchsorted(part[order], np.arange(k + 1))
    inside = (part[eu] == part[ev]) & (eu != ev)
    ieu, iev, iw = eu[inside], ev[inside], w[inside]
    ipart = part[ieu]
    members, sizes = [], []
    for c in comps:
        members.append(np.sort(order[starts[c]:starts[c + 1]]))
        sizes.append(len(members[-1]))
    sizes = np.asarray(sizes, np.int32)
    offs = np.zeros(len(comps) + 1, np.int64)
    offs[1:] = np.cumsum(sizes.astype(np.int64) ** 2)
    data = np.full(int(offs[-1]), O_INF, np.int64)
    pos = np.full(n, -1, np.int64)
    eorder = np.argsort(ipart, kind="stable")
    estarts = np.searchsorted(ipart[eorder], np.arange(k + 1))
    for idx, c in enumerate(comps):
        mem = members[idx]
        N = len(mem)
        pos[mem] = np.arange(N)
        mat = data[offs[idx]:offs[idx + 1]].reshape(N, N)
        sel = eorder[estarts[c]:estarts[c + 1]]
        a, b, x = pos[ieu[sel]], pos[iev[sel]], iw[sel].astype(np.int64)
        np.minimum.at(mat, (a, b), x)
        np.minimum.at(mat, (b, a), x)
        mat[np.arange(N), np.arange(N)] = 0
    lib().oracle_fw_many(len(comps), sizes, offs[:-1].copy(), data, _threads(nthreads))
    return members, [data[offs[i]:offs[i + 1]].reshape(sizes[i], sizes[i])
                     for i in range(len(comps))]


def boundary_graph(n, eu, ev, w, part, k, members, apsp, bflag=None):
    """BG as an edge list on BG ids 0..V-1, plus the BG vertex order.

    bflag may be any superset of the boundary (used by the invariance pin)."""
    eu, ev, w, part = (np.asarray(a) for a in (eu, ev, w, part))
    if bflag is None:
        bflag = boundary(n, eu, ev, part)
    bverts = [m[bflag[m]] for m in members]
    bg_ids = np.concatenate(bverts) if bverts else np.zeros(0, np.int64)
    bgidx = np.full(n, -1, np.int64)
    bgidx[bg_ids] = np.arange(len(bg_ids))
    # edges of G between boundary vertices (the induced part of BG)
    keep = (bgidx[eu] >= 0) & (bgidx[ev] >= 0) & (eu != ev)
    parts_u = [bgidx[eu[keep]]]
    parts_v = [bgidx[ev[keep]]]
    parts_w = [w[keep].astype(np.int64)]
    # clique edges: weight dist_C(b, b') for boundary pairs of one component
    for m, b, A in zip(members, bverts, apsp):
        if len(b) < 2:
            continue
        loc = np.searchsorted(m, b)
        sub = A[np.ix_(loc, loc)]
        iu, ju = np.triu_indices(len(b), 1)
        x = sub[iu, ju]
        fin = x != O_INF
        parts_u.append(bgidx[b[iu[fin]]])
        parts_v.append(bgidx[b[ju[fin]]])
        parts_w.append(x[fin])
    bu = np.concatenate(parts_u).astype(np.int32)
    bv = np.concatenate(parts_v).astype(np.int32)
    bw = np.concatenate(parts_w)
    if len(bw) and bw.max() >= np.iinfo(np.int32).max:
        raise OverflowError("BG edge weight beyond int32")
    return bg_ids, bverts, bu, bv, bw.astype(np.int32)


def bg_apsp(bg_ids, bu, bv, bw, sources=None, nthreads=None):
    """Phase 3: Dijkstra in BG from each listed BG id (default: all)."""
    V = len(bg_ids)
    src = np.arange(V) if sources is None else np.asarray(sources)
    if V == 0:
        return np.zeros((0, 0), np.int64)
    return dijkstra(V, bu, bv, bw, src, nthreads)


def preprocess(n, eu, ev, w, part, k, bflag=None, nthreads=None):
    """Algorithm 1 in full (small graphs): APSP(C) for all C, BG, APSP_BG."""
    T = Tables()
    T.members, T.apsp = component_apsp(n, eu, ev, w, part, k, nthreads=nthreads)
    T.bg_ids, T.bverts, T.bu, T.bv, T.bw = boundary_graph(n, eu, ev, w, part, k,
                                                          T.members, T.apsp, bflag)
    T.dbg = bg_apsp(T.bg_ids, T.bu, T.bv, T.bw, nthreads=nthreads)
    T.n, T.k = n, k
    return T


def query_alg2(T, v1, v2):
    """Algorithm 2 for each pair, on the tables of ``preprocess``."""
    n, k = T.n, T.k
    comp = np.zeros(n, np.int32)
    pos = np.zeros(n, np.int32)
    for c, m in enumerate(T.members):
        comp[m] = c
        pos[m] = np.arange(len(m))
    csize = np.array([len(m) for m in T.members], np.int32)
    moff = np.zeros(k, np.int64)
    if k > 1:
        moff[1:] = np.cumsum(csize.astype(np.int64) ** 2)[:-1]
    apsp = np.concatenate([a.ravel() for a in T.apsp]) if k else np.zeros(0, np.int64)
    bstart = np.zeros(k + 1, np.int32)
    bstart[1:] = np.cumsum([len(b) for b in T.bverts])
    blocal = np.concatenate([np.searchsorted(m, b) for m, b in zip(T.members, T.bverts)]
                            ).astype(np.int32) if k else np.zeros(0, np.int32)
    V = len(T.bg_ids)
    dbg = np.ascontiguousarray(T.dbg, np.int64) if V else np.zeros(1, np.int64)
    v1, v2 = _i32(v1), _i32(v2)
    out = np.empty(len(v1), np.int64)
    lib().oracle_query_alg2(len(v1), v1, v2, comp, pos, csize, moff, np.ascontiguousarray(apsp),
                            bstart, _i32(blocal), V, dbg.ravel(), out)
    return out


def minplus(A, B):
    """(min, +) product of int64 tables (O_INF = no path): C[i][j] = min over
    k of A[i][k] + B[k][j]."""
    A = np.ascontiguousarray(A, np.int64)
    B = np.ascontiguousarray(B, np.int64)
    if A.ndim != 2 or B.ndim != 2 or A.shape[1] != B.shape[0]:
        raise ValueError("minplus: shapes %s and %s do not chain" % (A.shape, B.shape))
    C = np.empty((A.shape[0], B.shape[1]), np.int64)
    if C.size:
        lib().oracle_minplus(A.shape[0], A.shape[1], B.shape[1], A, B, C)
    return C


def to_int32_distance(d):
    """Map oracle distances onto the int32 convention: no path -> 2**31-1.

    Raises if a finite distance does not fit below that sentinel."""
    d = np.asarray(d, np.int64)
    fin = d != O_INF
    if fin.any() and d[fin].max() >= np.iinfo(np.int32).max:
        raise OverflowError("finite distance >= int32 sentinel")
    out = d.copy()
    out[~fin] = np.iinfo(np.int32).max
    return out.astype(np.int32)
