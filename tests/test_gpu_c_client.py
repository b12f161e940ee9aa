"""The C ABI from a plain C program (tests/c_client/spq_client.c, built with
gcc against include/spq.h and libspq.so): host-array build, host-array
queries with and without allocation and through the library's server,
answers equal to Dijkstra on G
(Algorithm 1 then Algorithm 2, Lemma 3)."""
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_1503_07192_amd import spq, workloads as W

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def test_c_client_grid32(tmp_path):
    exe = tmp_path / "spq_client"
    libdir = os.path.dirname(spq.LIB_PATH)
    subprocess.check_call(["gcc", "-O2", "-I", os.path.dirname(spq.HEADER),
                           os.path.join(HERE, "c_client", "spq_client.c"), "-o", str(exe),
                           "-L", libdir, "-lspq", "-Wl,-rpath," + libdir])
    g = W.grid32()
    rng = np.random.default_rng(17)
    v1 = np.concatenate([g["v1"], rng.integers(0, g["n"], 3000)]).astype(np.int32)
    v2 = np.concatenate([g["v2"], rng.integers(0, g["n"], 3000)]).astype(np.int32)
    v1[5] = -1  # a bad pair: SPQ_BAD_PAIR in its slot
    inp, outp = tmp_path / "in.bin", tmp_path / "out.bin"
    hdr = np.array([g["n"], len(g["eu"]), g["k"], len(v1)], np.int32)
    np.concatenate([hdr, g["eu"], g["ev"], g["w"], g["part"], v1, v2]).astype("<i4").tofile(inp)
    print("c client on grid32", flush=True)
    res = subprocess.run([str(exe), str(inp), str(outp)], capture_output=True, text=True,
                         timeout=120)
    assert res.returncode == 0, res.stderr
    assert "v_bg=348" in res.stdout
    out = np.fromfile(outp, "<i4").reshape(3, len(v1))
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
    assert "served: %d pairs" % len(v1) in res.stdout
    D = oracle.dijkstra(g["n"], g["eu"], g["ev"], g["w"], np.maximum(v1, 0))
    want = D[np.arange(len(v1)), v2].astype(np.int32)
    want[5] = spq.SPQ_BAD_PAIR
    assert np.array_equal(out[0], want)
