"""spq_query_batch_host_static, the query entry point that allocates nothing
(its staging is a fixed device array of the library), against
spq_query_batch_host on the same index: bit-identical answers on two calls
in a row, the second with a smaller batch; device memory unchanged across
calls; sizes above SPQ_STATIC_PAIRS rejected."""
import numpy as np
import pytest

from paper_1503_07192_amd import spq, workloads as W

pytestmark = pytest.mark.gpu


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()


def _index(g, **kw):
    return spq.build_index(g["n"], dev(g["eu"]), dev(g["ev"]), dev(g["w"]), dev(g["part"]), g["k"],
                           **kw)


@pytest.mark.parametrize("kw", [{}, {"bg_method": 2, "group_comps": 3}])
def test_static_query_equals_host_query(kw):
    import torch
    g = W.grid32()
    rng = np.random.default_rng(11)
    v1 = rng.integers(0, g["n"], 5000).astype(np.int32)
    v2 = rng.integers(0, g["n"], 5000).astype(np.int32)
    v1[7], v2[9] = -3, g["n"]  # bad pairs: SPQ_BAD_PAIR in their slots
    idx = _index(g, **kw)
    print("grid32 static query", kw, flush=True)
    for q in (5000, 1234):  # the second call smaller than the first
        got = spq.query_batch_host_static(idx, v1[:q], v2[:q])
        want = spq.query_batch_host(idx, v1[:q], v2[:q])
        assert np.array_equal(got, want), q
    assert got[7] == spq.SPQ_BAD_PAIR and got[9] == spq.SPQ_BAD_PAIR
    # once set up, a call leaves the device's free memory as it found it
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for q in (3000, 17):
        spq.query_batch_host_static(idx, v1[:q], v2[:q])
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    idx.free()


def test_static_query_limits():
    g = W.grid32()
    idx = _index(g)
    print("grid32 static query limits", flush=True)
    big = np.zeros(spq.SPQ_STATIC_PAIRS + 1, np.int32)
    with pytest.raises(spq.SpqError) as e:
        spq.query_batch_host_static(idx, big, big)
    assert e.value.name == "SPQ_EINVAL" and "SPQ_STATIC_PAIRS" in str(e.value)
    assert len(spq.query_batch_host_static(idx, big[:0], big[:0])) == 0
    # the largest batch the array holds, on a stream of the caller
    import torch
    rng = np.random.default_rng(5)
    v1 = rng.integers(0, g["n"], spq.SPQ_STATIC_PAIRS).astype(np.int32)
    v2 = rng.integers(0, g["n"], spq.SPQ_STATIC_PAIRS).astype(np.int32)
    s = torch.cuda.Stream()
    got = spq.query_batch_host_static(idx, v1, v2, stream=s)
    assert np.array_equal(got, spq.query_batch_host(idx, v1, v2))
    idx.free()
