"""The C-ABI library on the CPU: it loads, exports what include/spq.h declares,
and rejects bad arguments before touching a device."""
import ctypes

import pytest

from paper_1503_07192_amd import spq


def test_library_exports_every_header_symbol():
    L = spq.load()
    names = spq.header_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(spq._SIGS)


def test_argument_errors_without_device():
    L = spq.load()
    h = ctypes.c_void_p()
    assert L.spq_build_index(0, 0, None, None, None, None, 1, None, None, ctypes.byref(h)) == 1
    assert "n >= 1" in spq.last_error()
    assert L.spq_build_index(5, 0, None, None, None, None, 6, None, None, ctypes.byref(h)) == 1
    assert "empty" in spq.last_error()
    assert L.spq_build_index(5, 3, None, None, None, None, 2, None, None, ctypes.byref(h)) == 1
    opts = spq.BuildOpts(bg_tile=96)
    assert L.spq_build_index(5, 0, None, None, None, ctypes.c_void_p(8), 2, ctypes.byref(opts),
                             None, ctypes.byref(h)) == 1
    assert "bg_tile" in spq.last_error()
    opts = spq.BuildOpts(bg_pivot=192)
    assert L.spq_build_index(5, 0, None, None, None, ctypes.c_void_p(8), 2, ctypes.byref(opts),
                             None, ctypes.byref(h)) == 1
    assert "bg_pivot" in spq.last_error()
    assert L.spq_build_index(5, 0, None, None, None, None, 2, None, None, None) == 1
    assert L.spq_build_index_host(0, 0, None, None, None, None, 1, None, ctypes.byref(h)) == 1
    assert "n >= 1" in spq.last_error()
    assert L.spq_build_index_host(5, 3, None, None, None, ctypes.c_void_p(8), 2, None,
                                  ctypes.byref(h)) == 1
    assert "null input" in spq.last_error()
    assert L.spq_build_index_host(5, 0, None, None, None, None, 2, None, None) == 1
    assert L.spq_query_batch(None, 3, None, None, None, None) == 1
    assert L.spq_query_batch_host(None, 3, None, None, None) == 1
    assert L.spq_query_paths(None, 3, None, None, 8, None, None, None) == 1
    assert L.spq_fw_dense(10, 10, 3, 0, 0, None, None) == 1
    assert L.spq_fw_dense(10, 8, 64, 0, 0, None, None) == 1
    assert L.spq_fw_dense(10, 64, 64, 0, 8, None, None) == 1
    assert L.spq_fw_dense(10, 128, 64, 192, 0, None, None) == 1
    assert "pivot" in spq.last_error()
    assert L.spq_fw_dense(0, 0, 64, 128, 0, None, None) == 0
    assert L.spq_fw_components(-1, None, None, None, None, None) == 1
    assert L.spq_valu_rates(None, None) == 1
    assert L.spq_index_stats(None, None) == 1
    assert L.spq_reweight_index(None, None, None) == 1
    part = ctypes.c_void_p(8)
    for flags, share, profile, msg in ((8, 0, 0, "unknown flags"),
                                       (spq.SPQ_GRAPH, 1, 0, "SPQ_GRAPH"),
                                       (spq.SPQ_GRAPH, 0, 1, "SPQ_GRAPH")):
        opts = spq.BuildOpts(flags=flags, share_comps=share, profile=profile)
        assert L.spq_build_index(5, 0, None, None, None, part, 2, ctypes.byref(opts), None,
                                 ctypes.byref(h)) == 1
        assert msg in spq.last_error()
    L.spq_free_index(None)


def test_minplus_hooks_reject_bad_arguments_without_device():
    import numpy as np
    L = spq.load()
    dummy = ctypes.c_void_p(8)
    nv = np.array([100, 128], np.int32)
    nk = np.array([5, 0], np.int32)
    pairs = np.array([0, 1, 1, 1], np.int32)

    def call(layout=0, groups=2, nv=nv, nk=nk, vp=128, kp=128, ldd=5, npairs=2, pairs=pairs,
             cb=8, ldo=0, assoc=0, Dt=None):
        return L.spq_minplus_batched(layout, groups, nv.ctypes.data, nk.ctypes.data, vp, kp, dummy,
                                     dummy, Dt, ldd, dummy, npairs, pairs.ctypes.data, assoc, cb,
                                     dummy, ldo, None)
    assert call(layout=2) == 1 and "layout" in spq.last_error()
    assert call(vp=100) == 1 and "multiples of 128" in spq.last_error()
    assert call(nv=np.array([129, 1], np.int32)) == 1 and "group 0" in spq.last_error()
    assert call(ldd=4) == 1 and "ldd" in spq.last_error()
    assert call(cb=0) == 1 and "cb" in spq.last_error()
    assert call(layout=1, ldo=227) == 1 and "ldo" in spq.last_error()
    assert call(pairs=np.array([0, 1, 0, 1], np.int32)) == 1 and "repeats" in spq.last_error()
    assert call(pairs=np.array([0, 2, 0, 1], np.int32)) == 1 and "outside" in spq.last_error()
    assert call(npairs=0) == 0
    assert call(assoc=3) == 1 and "assoc" in spq.last_error()
    assert call(layout=1, ldo=228, assoc=1) == 1 and "assoc" in spq.last_error()
    assert call(assoc=1) == 1 and "Dt" in spq.last_error()
    cnt = np.array([-1, 0], np.int32)
    assert L.spq_minplus_rows(2, nk.ctypes.data, 100, dummy, dummy, 128, cnt.ctypes.data, None,
                              None, None) == 1
    assert L.spq_minplus_rows(2, nk.ctypes.data, 128, dummy, dummy, 128,
                              np.array([6, 0], np.int32).ctypes.data, None, None, None) == 1
    assert "listed rows" in spq.last_error()
    assert L.spq_minplus_rows(2, nk.ctypes.data, 128, dummy, dummy, 128,
                              np.array([2, 0], np.int32).ctypes.data, None, None, None) == 1
    assert "rows is NULL" in spq.last_error()
    rows = np.array([1, 5], np.int32)
    assert L.spq_minplus_rows(2, nk.ctypes.data, 128, dummy, dummy, 128,
                              np.array([2, 0], np.int32).ctypes.data, rows.ctypes.data, None,
                              None) == 1
    assert "outside its group" in spq.last_error()
    own = np.array([0, 1, 2, -3, 4], np.int32)
    assert L.spq_minplus_rows(2, nk.ctypes.data, 128, dummy, dummy, 128, cnt.ctypes.data, None,
                              own.ctypes.data, None) == 1
    assert "negative row" in spq.last_error()
    nout = np.array([3, 0], np.int32)
    out = np.array([7, 8, 9], np.int32)
    own = np.arange(5, dtype=np.int32)

    def gather(nk=nk, nout=nout, kp=128, np_=128, ldc=128, own=own, out=out):
        return L.spq_minplus_gather(2, nk.ctypes.data, nout.ctypes.data, kp, np_, dummy, dummy, ldc,
                                    own.ctypes.data if own is not None else None,
                                    out.ctypes.data if out is not None else None, None)
    assert gather(np_=100) == 1 and "multiples of 128" in spq.last_error()
    assert gather(ldc=64) == 1 and "ldc" in spq.last_error()
    assert gather(nout=np.array([129, 0], np.int32)) == 1 and "nout" in spq.last_error()
    assert gather(own=None) == 1 and "null row list" in spq.last_error()
    assert gather(out=np.array([7, -8, 9], np.int32)) == 1 and "negative row" in spq.last_error()


def test_python_binding_rejects_host_tensors():
    torch = pytest.importorskip("torch")
    x = torch.zeros(4, dtype=torch.int32)
    with pytest.raises(TypeError):
        spq.build_index(4, x, x, x, x, 1)


def test_struct_layouts_match_header(tmp_path):
    """The ctypes mirrors of spq_build_opts and spq_stats match the C header."""
    import subprocess
    fields = [f for f, _ in spq.Stats._fields_]
    src = ["#include <stdio.h>", "#include <stddef.h>", '#include "spq.h"', "int main(void) {",
           'printf("%zu %zu\\n", sizeof(spq_build_opts), sizeof(spq_stats));']
    src += ['printf("%%zu\\n", offsetof(spq_stats, %s));' % f for f in fields]
    src += ["return 0; }"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", str(spq.HEADER.rsplit("/", 1)[0]), str(c), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    assert int(out[0]) == ctypes.sizeof(spq.BuildOpts)
    assert int(out[1]) == ctypes.sizeof(spq.Stats)
    for f, off in zip(fields, out[2:]):
        assert int(off) == getattr(spq.Stats, f).offset, f


def test_server_rejects_bad_arguments_without_device():
    """spq_server_*: null server, index, ticket or output pointer, negative
    sizes; destroy(NULL) is a no-op."""
    L = spq.load()
    h = ctypes.c_void_p()
    assert L.spq_server_create(None, 4, 1024, 1 << 20, None) == 1
    assert "out is NULL" in spq.last_error()
    assert L.spq_server_create(None, 4, 1024, 1 << 20, ctypes.byref(h)) == 1
    assert "index is NULL" in spq.last_error() and h.value is None
    t = ctypes.c_int64()
    assert L.spq_server_submit(None, 3, None, None, None, ctypes.byref(t)) == 1
    assert L.spq_server_submit(ctypes.c_void_p(8), 3, None, None, None, None) == 1
    assert "null argument" in spq.last_error()
    d = ctypes.c_int32()
    assert L.spq_server_poll(None, 1, 0, ctypes.byref(d), None) == 1
    assert L.spq_server_stats(None, None, None) == 1
    L.spq_server_destroy(None)
