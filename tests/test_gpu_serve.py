"""Serving on the GPU: every request's answers are the same alone and in the
mix of concurrently served requests (tolerance 0), and match Dijkstra."""
import numpy as np
import pytest

import oracle
from paper_1503_07192_amd import serve, workloads as W

torch = pytest.importorskip("torch")
spq = pytest.importorskip("paper_1503_07192_amd.spq")

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.int32)).cuda()


@pytest.mark.parametrize("method", [1, 2])
def test_served_mix_equals_alone(method):
    g = W.grid256d(queries=0)
    print("serve test: build grid256d method %d" % method, flush=True)
    idx = spq.build_index(g["n"], dev(g["eu"]), dev(g["ev"]), dev(g["w"]), dev(g["part"]), g["k"],
                          bg_method=method, group_comps=64)
    torch.cuda.synchronize()
    rng = np.random.default_rng(12)
    reqs = serve.poisson_stream(rng, 2e7, 150, g["n"], max_log2=12.0)
    ex = serve.GpuExecutor(idx, 4, 2048)
    sched = serve.Scheduler(ex, 4, 2048, 12 * 3000)   # small budget: requests get cut
    done = serve.run_stream(sched, reqs)
    assert len(done) == len(reqs)
    assert sched.launches < sum(r.size for r in reqs)
    assert any(len(r.launches) > 1 for r in reqs)
    for r in reqs:
        alone = spq.query_batch(idx, dev(r.v1), dev(r.v2)).cpu().numpy()
        assert np.array_equal(alone, r.result), r.rid
    # a sample against Dijkstra on G
    for r in reqs[:5]:
        D = oracle.dijkstra(g["n"], g["eu"], g["ev"], g["w"], r.v1[:20])
        assert np.array_equal(r.result[:20], D[np.arange(min(20, r.size)), r.v2[:20]])
    s = serve.summarize(done, sched)
    assert s["latency_ms_p99"] >= s["latency_ms_p50"] > 0
    one = serve.poisson_stream(rng, 1e5, 3, g["n"], max_log2=6.0)
    serve.OneAtATime(idx).run(one)
    for r in one:
        alone = spq.query_batch(idx, dev(r.v1), dev(r.v2)).cpu().numpy()
        assert np.array_equal(alone, r.result)
