"""The components-vs-k study: every partition's index answers the query batch
with the distances in G (Dijkstra, Lemma 3), and the sizes move the way the
block sides dictate."""
import numpy as np
import pytest

import oracle

pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_study_every_k_equals_dijkstra():
    from paper_1503_07192_amd import study, workloads as W
    rows = study.run(blocks=(64, 32, 16, 8), queries=1000, log=lambda s: print(s, flush=True),
                     answers=True)
    assert [r["k"] for r in rows] == [16, 64, 256, 1024]
    g = W.grid256d(queries=0)
    v1, v2 = rows[0]["v1"], rows[0]["v2"]
    D = oracle.dijkstra(g["n"], g["eu"], g["ev"], g["w"], v1)
    want = np.minimum(D[np.arange(len(v1)), v2], 2**31 - 1).astype(np.int32)
    for r in rows:
        assert np.array_equal(r["answers"], want), "k = %d" % r["k"]
        assert r["answers_identical"]
    # smaller components: less APSP(C), more boundary vertices, smaller |B(C)|
    for a, b in zip(rows, rows[1:]):
        assert a["comp_bytes"] > b["comp_bytes"]
        assert a["v_bg"] < b["v_bg"]
        assert a["mean_boundary"] > b["mean_boundary"]
    assert rows[3]["v_bg"] == 27900
