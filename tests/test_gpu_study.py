"""The components-vs-k study: every partition gives the same answers, and the
sizes move the way the block sides dictate."""
import pytest

pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_study_small():
    from paper_1503_07192_amd import study
    rows = study.run(blocks=(32, 16, 8), queries=2000, log=lambda s: None)
    assert all(r["answers_identical"] for r in rows)
    assert [r["k"] for r in rows] == [64, 256, 1024]
    # smaller components: less APSP(C), more boundary vertices, smaller |B(C)|
    assert rows[0]["comp_bytes"] > rows[1]["comp_bytes"] > rows[2]["comp_bytes"]
    assert rows[0]["v_bg"] < rows[1]["v_bg"] < rows[2]["v_bg"]
    assert rows[0]["mean_boundary"] > rows[1]["mean_boundary"] > rows[2]["mean_boundary"]
    assert rows[2]["v_bg"] == 27900
