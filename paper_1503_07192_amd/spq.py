"""Python binding of the C-ABI in include/spq.h (argument marshalling only).

Every computation runs in the HIP kernels of ``libspq.so``; this module only
checks and converts arguments.  There is no fallback: if the library is not
built, ``load()`` raises.

Device arrays are torch tensors on the current HIP device (int32,
contiguous); streams default to torch's current stream.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libspq.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "spq.h")

SPQ_INF = 2147483647
SPQ_BAD_PAIR = -1
SPQ_NO_LOOKAHEAD = 1
SPQ_GRAPH = 2
SPQ_PATHS = 4
SPQ_MP_BLOCKED = 0
SPQ_MP_DENSE = 1
SPQ_STATIC_PAIRS = 1 << 20
STATUS = {0: "SPQ_OK", 1: "SPQ_EINVAL", 2: "SPQ_ENOMEM", 3: "SPQ_EDEVICE", 4: "SPQ_ERANGE",
          5: "SPQ_EBUSY"}


class SpqError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status
        self.name = STATUS.get(status, str(status))


class BuildOpts(ctypes.Structure):
    _fields_ = [("bg_tile", ctypes.c_int32), ("profile", ctypes.c_int32),
                ("plain", ctypes.c_int32), ("bg_method", ctypes.c_int32),
                ("group_comps", ctypes.c_int32), ("share_comps", ctypes.c_int32),
                ("inner_kc", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("level3_groups", ctypes.c_int32), ("group_bg", ctypes.c_int32),
                ("bg_pivot", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("k", ctypes.c_int32), ("m", ctypes.c_int64),
                ("v_bg", ctypes.c_int32), ("v_bg_padded", ctypes.c_int32),
                ("max_comp", ctypes.c_int32), ("max_boundary", ctypes.c_int32),
                ("comp_bytes", ctypes.c_int64), ("bg_bytes", ctypes.c_int64),
                ("relax_comp", ctypes.c_double), ("relax_bg", ctypes.c_double),
                ("relax_comp_exec", ctypes.c_double), ("relax_bg_exec", ctypes.c_double),
                ("relax_dominant", ctypes.c_double), ("dominant_launches", ctypes.c_int64),
                ("ms_dominant", ctypes.c_float),
                ("bg_method", ctypes.c_int32), ("ngroups", ctypes.c_int32),
                ("v_bg2", ctypes.c_int32), ("share_comps", ctypes.c_int32),
                ("share_groups", ctypes.c_int32), ("bf_rounds", ctypes.c_int32),
                ("ms_partition", ctypes.c_float), ("ms_components", ctypes.c_float),
                ("ms_bg_assembly", ctypes.c_float), ("ms_bg_apsp", ctypes.c_float),
                ("graphs", ctypes.c_int32), ("reweights", ctypes.c_int32),
                ("graph_nodes", ctypes.c_int64), ("groups3", ctypes.c_int32),
                ("v_bg3", ctypes.c_int32), ("bf_block_groups", ctypes.c_int32)]


_lib = None
P = ctypes.c_void_p
I32, I64 = ctypes.c_int32, ctypes.c_int64
_SIGS = {
    "spq_build_index": (I32, [I32, I64, P, P, P, P, I32, ctypes.POINTER(BuildOpts), P,
                              ctypes.POINTER(P)]),
    "spq_build_index_host": (I32, [I32, I64, P, P, P, P, I32, ctypes.POINTER(BuildOpts),
                                   ctypes.POINTER(P)]),
    "spq_query_batch": (I32, [P, I64, P, P, P, P]),
    "spq_query_batch_host": (I32, [P, I64, P, P, P]),
    "spq_query_batch_host_static": (I32, [P, I64, P, P, P, P]),
    "spq_reweight_index": (I32, [P, P, P]),
    "spq_query_paths": (I32, [P, I64, P, P, I32, P, P, P]),
    "spq_index_stats": (I32, [P, ctypes.POINTER(Stats)]),
    "spq_index_layout": (I32, [P, P, P, P, P, P]),
    "spq_index_component": (I32, [P, I32, P]),
    "spq_index_bg_rows": (I32, [P, I32, I32, P]),
    "spq_free_index": (None, [P]),
    "spq_release_cached_memory": (None, []),
    "spq_last_error": (ctypes.c_char_p, []),
    "spq_fw_components": (I32, [I32, P, P, P, P, P]),
    "spq_fw_dense": (I32, [I32, I32, I32, I32, I32, P, P]),
    "spq_valu_rates": (I32, [P, P]),
    "spq_minplus_batched": (I32, [I32, I32, P, P, I32, I32, P, P, P, I64, P, I32, P, I32, I32, P,
                                  I64, P]),
    "spq_minplus_rows": (I32, [I32, P, I32, P, P, I64, P, P, P, P]),
    "spq_minplus_gather": (I32, [I32, P, P, I32, I32, P, P, I64, P, P, P]),
    "spq_server_create": (I32, [P, I32, I64, I64, P]),
    "spq_server_submit": (I32, [P, I64, P, P, P, P]),
    "spq_server_poll": (I32, [P, I64, I32, P, P]),
    "spq_server_stats": (I32, [P, P, P]),
    "spq_server_destroy": (None, [P]),
}


def header_functions():
    """Names of the functions declared in include/spq.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spq_\w+)\s*\(", text)))


def load():
    """The built library; raises if it is missing (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libspq.so is not built: run `python -m paper_1503_07192_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def release_cached_memory():
    """Frees device memory cached from released indexes."""
    load().spq_release_cached_memory()


def last_error() -> str:
    return load().spq_last_error().decode()


def _check(st):
    if st != 0:
        raise SpqError(st, last_error())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_i32(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a torch tensor on the HIP device" % name)
    if t.dtype != torch.int32 or not t.is_contiguous():
        raise TypeError("%s must be contiguous int32" % name)
    return ctypes.c_void_p(t.data_ptr())


class Index:
    """Owns an spq_index (freed with the object)."""

    def __init__(self, handle, n, k):
        self._h = handle
        self.n, self.k = n, k

    @property
    def handle(self):
        if not self._h:
            raise ValueError("index already freed")
        return self._h

    def free(self):
        if self._h:
            load().spq_free_index(self._h)
            self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _opts(n, m, k, bg_tile=0, profile=False, plain=False, bg_method=0, group_comps=0,
          share_comps=0, inner_kc=0, lookahead=True, graph=False, level3_groups=0, group_bg=0,
          paths=False, bg_pivot=0, tune_cache=None):
    if tune_cache:
        from . import autotune
        tuned = autotune.lookup(tune_cache, n, m, k, share_comps)
        bg_tile = bg_tile or tuned.get("bg_tile", 0)
        inner_kc = inner_kc or tuned.get("inner_kc", 0)
        bg_method = bg_method or tuned.get("bg_method", 0)
        group_comps = group_comps or tuned.get("group_comps", 0)
        level3_groups = level3_groups or tuned.get("level3_groups", 0)
        group_bg = group_bg or tuned.get("group_bg", 0)
        bg_pivot = bg_pivot or tuned.get("bg_pivot", 0)
    opts = BuildOpts(bg_tile=bg_tile, profile=int(bool(profile)), plain=int(bool(plain)),
                     bg_method=int(bg_method), group_comps=int(group_comps),
                     share_comps=int(share_comps), inner_kc=int(inner_kc),
                     flags=(0 if lookahead else SPQ_NO_LOOKAHEAD) | (SPQ_GRAPH if graph else 0) |
                     (SPQ_PATHS if paths else 0),
                     level3_groups=int(level3_groups), group_bg=int(group_bg),
                     bg_pivot=int(bg_pivot))
    return opts


def build_index(n, eu, ev, w, part, k, stream=None, **kw) -> Index:
    """Algorithm 1 on device tensors; see spq_build_index.

    Options (keywords, see spq_build_opts): bg_tile, profile, plain,
    bg_method, group_comps, share_comps, inner_kc, lookahead, level3_groups,
    group_bg, bg_pivot;
    graph: capture Phases 2-3 as HIP graphs kept for reweight();
    paths: keep the graph's adjacency for query_paths();
    tune_cache: path of an autotuner cache (paper_1503_07192_amd.autotune);
    options it holds for this device and problem size fill in the ones left
    at 0 here."""
    L = load()
    m = int(eu.numel())
    opts = _opts(int(n), m, int(k), **kw)
    h = ctypes.c_void_p()
    st = L.spq_build_index(int(n), m, _dev_i32(eu, "eu"), _dev_i32(ev, "ev"), _dev_i32(w, "w"),
                           _dev_i32(part, "part"), int(k), ctypes.byref(opts), _stream(stream),
                           ctypes.byref(h))
    _check(st)
    return Index(h, int(n), int(k))


def build_index_host(n, eu, ev, w, part, k, **kw) -> Index:
    """Algorithm 1 on host (numpy) arrays, synchronous; see
    spq_build_index_host.  Options as build_index."""
    eu, ev, w, part = (np.ascontiguousarray(a, np.int32) for a in (eu, ev, w, part))
    m = len(eu)
    if len(ev) != m or len(w) != m or len(part) != int(n):
        raise ValueError("eu, ev, w need m entries and part n")
    opts = _opts(int(n), m, int(k), **kw)
    h = ctypes.c_void_p()
    _check(load().spq_build_index_host(int(n), m, eu.ctypes.data, ev.ctypes.data, w.ctypes.data,
                                       part.ctypes.data, int(k), ctypes.byref(opts),
                                       ctypes.byref(h)))
    return Index(h, int(n), int(k))


def reweight(index: Index, w, stream=None):
    """New edge weights (device int32, the build's edge order) for an index
    built with graph=True; see spq_reweight_index."""
    _check(load().spq_reweight_index(index.handle, _dev_i32(w, "w"), _stream(stream)))
    return index


def query_batch(index: Index, v1, v2, out=None, stream=None):
    """Algorithm 2 for every pair; returns the int32 device tensor `out`."""
    import torch
    q = int(v1.numel())
    if int(v2.numel()) != q:
        raise ValueError("v1 and v2 differ in length")
    if out is None:
        out = torch.empty(q, dtype=torch.int32, device=v1.device)
    elif int(out.numel()) != q:
        raise ValueError("out has the wrong length")
    _check(load().spq_query_batch(index.handle, q, _dev_i32(v1, "v1"), _dev_i32(v2, "v2"),
                                  _dev_i32(out, "out"), _stream(stream)))
    return out


def query_paths(index: Index, v1, v2, max_len, stream=None):
    """One shortest path per pair (index built with paths=True); returns the
    device tensors (paths [q, max_len], lens [q]), see spq_query_paths."""
    import torch
    q = int(v1.numel())
    if int(v2.numel()) != q:
        raise ValueError("v1 and v2 differ in length")
    paths = torch.full((q, int(max_len)), -1, dtype=torch.int32, device=v1.device)
    lens = torch.empty(q, dtype=torch.int32, device=v1.device)
    _check(load().spq_query_paths(index.handle, q, _dev_i32(v1, "v1"), _dev_i32(v2, "v2"),
                                  int(max_len), _dev_i32(paths, "paths"), _dev_i32(lens, "lens"),
                                  _stream(stream)))
    return paths, lens


def query_batch_host(index: Index, v1, v2):
    """Algorithm 2 on host (numpy) pairs; returns a numpy int32 array."""
    v1 = np.ascontiguousarray(v1, np.int32)
    v2 = np.ascontiguousarray(v2, np.int32)
    if v1.shape != v2.shape or v1.ndim != 1:
        raise ValueError("v1 and v2 must be 1-d and equally long")
    out = np.empty_like(v1)
    _check(load().spq_query_batch_host(index.handle, len(v1), v1.ctypes.data, v2.ctypes.data,
                                       out.ctypes.data))
    return out


def query_batch_host_static(index: Index, v1, v2, stream=None):
    """Algorithm 2 on host (numpy) pairs through the library's fixed device
    staging (no allocation; at most SPQ_STATIC_PAIRS pairs); returns a numpy
    int32 array.  See spq_query_batch_host_static."""
    v1 = np.ascontiguousarray(v1, np.int32)
    v2 = np.ascontiguousarray(v2, np.int32)
    if v1.shape != v2.shape or v1.ndim != 1:
        raise ValueError("v1 and v2 must be 1-d and equally long")
    out = np.empty_like(v1)
    _check(load().spq_query_batch_host_static(index.handle, len(v1), v1.ctypes.data,
                                              v2.ctypes.data, out.ctypes.data, _stream(stream)))
    return out


class Server:
    """The library's continuous-batching server (spq_server_*) on a built
    index: requests of host (numpy) pairs are queued, coalesced into launches
    on `slots` streams by a native worker thread, and answered into numpy
    arrays; `mem_bytes` is its device (and pinned) pool, 12 bytes per pair in
    flight."""

    def __init__(self, index: Index, slots: int = 4, slot_pairs: int = 65536,
                 mem_bytes: int = 64 << 20):
        h = ctypes.c_void_p()
        _check(load().spq_server_create(index.handle, int(slots), int(slot_pairs), int(mem_bytes),
                                        ctypes.byref(h)))
        self.handle = h.value
        self.index = index   # the index must outlive the server
        self._held = {}      # ticket -> (v1, v2, out): alive until answered

    def submit(self, v1, v2) -> int:
        """Queues the pairs (v1[i], v2[i]); returns the request's ticket."""
        v1 = np.ascontiguousarray(v1, np.int32)
        v2 = np.ascontiguousarray(v2, np.int32)
        if v1.shape != v2.shape or v1.ndim != 1:
            raise ValueError("v1 and v2 must be 1-d and equally long")
        out = np.empty_like(v1)
        t = ctypes.c_int64()
        _check(load().spq_server_submit(self.handle, len(v1), v1.ctypes.data, v2.ctypes.data,
                                        out.ctypes.data, ctypes.byref(t)))
        self._held[t.value] = (v1, v2, out)
        return t.value

    def poll(self, ticket: int, wait: bool = False):
        """(answers, latency in seconds) once the request is complete, else
        None; wait=True blocks until it is.  A ticket is answered once."""
        done = ctypes.c_int32()
        lat = ctypes.c_double()
        _check(load().spq_server_poll(self.handle, int(ticket), int(bool(wait)),
                                      ctypes.byref(done), ctypes.byref(lat)))
        if not done.value:
            return None
        return self._held.pop(ticket)[2], lat.value

    def stats(self) -> dict:
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(load().spq_server_stats(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return {"launches": a.value, "pairs": b.value}

    def close(self):
        """Answers everything submitted, then frees the server."""
        if self.handle:
            load().spq_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def index_stats(index: Index) -> dict:
    s = Stats()
    _check(load().spq_index_stats(index.handle, ctypes.byref(s)))
    return {name: getattr(s, name) for name, _ in Stats._fields_}


def index_layout(index: Index) -> dict:
    n, k = index.n, index.k
    comp = np.empty(n, np.int32)
    local = np.empty(n, np.int32)
    nb = np.empty(k, np.int32)
    off = np.empty(k + 1, np.int32)
    bgoff = np.empty(k + 1, np.int32)
    _check(load().spq_index_layout(index.handle, comp.ctypes.data, local.ctypes.data,
                                   nb.ctypes.data, off.ctypes.data, bgoff.ctypes.data))
    return dict(comp=comp, local=local, nb=nb, off=off, bgoff=bgoff)


def index_component(index: Index, c: int, size: int):
    out = np.empty((size, size), np.int32)
    _check(load().spq_index_component(index.handle, int(c), out.ctypes.data))
    return out


def index_bg_rows(index: Index, row0: int, nrows: int, v_bg: int):
    out = np.empty((nrows, v_bg), np.int32)
    _check(load().spq_index_bg_rows(index.handle, int(row0), int(nrows), out.ctypes.data))
    return out


def fw_components(size, off, ld, data, stream=None):
    size = np.ascontiguousarray(size, np.int32)
    off = np.ascontiguousarray(off, np.int64)
    ld = np.ascontiguousarray(ld, np.int32)
    _check(load().spq_fw_components(len(size), size.ctypes.data, off.ctypes.data, ld.ctypes.data,
                                    _dev_i32(data, "data"), _stream(stream)))
    return data


def fw_dense(v, ld, tile, data, stream=None, kc=0, pivot=0):
    _check(load().spq_fw_dense(int(v), int(ld), int(tile), int(pivot), int(kc),
                               _dev_i32(data, "data"), _stream(stream)))
    return data


def valu_rates(stream=None):
    """Measured issue rates on the current device, see spq_valu_rates:
    {"v_add_u32": lane-ops/s, "v_min3_u32": lane-ops/s, "relax_loop": relax/s (LDS
    operands), "relax_regs": relax/s (register operands)}."""
    out = (ctypes.c_double * 4)()
    _check(load().spq_valu_rates(out, _stream(stream)))
    return {"v_add_u32": out[0], "v_min3_u32": out[1], "relax_loop": out[2],
            "relax_regs": out[3]}


def minplus_batched(layout, nv, nk, vp, kp, R, D, ldd, M, pairs, out, cb=1, ldo=0, stream=None,
                    assoc=0, Dt=None):
    """Group-level composition products on device tensors (see
    spq_minplus_batched): nv, nk per group and pairs [(S1, S2), ...] on the
    host; R, D, Dt (D transposed, for assoc 1 and 2), M, out int32 device
    tensors.  Synchronous."""
    import torch
    nv = np.ascontiguousarray(nv, np.int32)
    nk = np.ascontiguousarray(nk, np.int32)
    pairs = np.ascontiguousarray(np.asarray(pairs, np.int32).reshape(-1, 2))
    if nv.shape != nk.shape or nv.ndim != 1:
        raise ValueError("nv and nk must be 1-d and equally long")
    dptr = _dev_i32(D, "D") if D is not None else ctypes.c_void_p(0)
    dtptr = _dev_i32(Dt, "Dt") if Dt is not None else ctypes.c_void_p(0)
    _check(load().spq_minplus_batched(int(layout), len(nv), nv.ctypes.data, nk.ctypes.data,
                                      int(vp), int(kp), _dev_i32(R, "R"), dptr, dtptr, int(ldd),
                                      _dev_i32(M, "M"), len(pairs), pairs.ctypes.data, int(assoc),
                                      int(cb), _dev_i32(out, "out"), int(ldo), _stream(stream)))
    return out


def minplus_rows(nk, kp, A, C, ldc, cnt, rows=None, own=None, stream=None):
    """The in-place intra-block product of the share's Bellman-Ford rounds on
    device tensors (see spq_minplus_rows): nk, cnt, rows and own on the
    host.  Synchronous."""
    nk = np.ascontiguousarray(nk, np.int32)
    cnt = np.ascontiguousarray(cnt, np.int32)
    rows = np.ascontiguousarray(rows if rows is not None else np.zeros(0), np.int32)
    if nk.shape != cnt.shape or nk.ndim != 1:
        raise ValueError("nk and cnt must be 1-d and equally long")
    own_p = None
    if own is not None:
        own = np.ascontiguousarray(own, np.int32)
        if own.shape != (int(nk.sum()),):
            raise ValueError("own must hold sum(nk) rows")
        own_p = own.ctypes.data
    _check(load().spq_minplus_rows(len(nk), nk.ctypes.data, int(kp), _dev_i32(A, "A"),
                                   _dev_i32(C, "C"), int(ldc), cnt.ctypes.data, rows.ctypes.data,
                                   own_p, _stream(stream)))
    return C


def minplus_gather(nk, nout, kp, np_, Aout, C, ldc, own, out, stream=None):
    """The last product of the share's Bellman-Ford stage on device tensors
    (see spq_minplus_gather): nk, nout, own and out on the host.
    Synchronous."""
    nk = np.ascontiguousarray(nk, np.int32)
    nout = np.ascontiguousarray(nout, np.int32)
    own = np.ascontiguousarray(own, np.int32)
    out = np.ascontiguousarray(out, np.int32)
    if nk.shape != nout.shape or nk.ndim != 1:
        raise ValueError("nk and nout must be 1-d and equally long")
    if own.shape != (int(nk.sum()),) or out.shape != (int(nout.sum()),):
        raise ValueError("own / out must hold sum(nk) / sum(nout) rows")
    _check(load().spq_minplus_gather(len(nk), nk.ctypes.data, nout.ctypes.data, int(kp), int(np_),
                                     _dev_i32(Aout, "Aout"), _dev_i32(C, "C"), int(ldc),
                                     own.ctypes.data, out.ctypes.data, _stream(stream)))
    return C
