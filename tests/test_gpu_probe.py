"""spq_valu_rates: the measured issue rates the relaxation peak rests on."""
import pytest

spq = pytest.importorskip("paper_1503_07192_amd.spq")

pytestmark = pytest.mark.gpu


def test_valu_rates_are_measured():
    r = spq.valu_rates()
    for kind in ("v_add_u32", "v_min3_u32", "relax_loop"):
        v = r[kind]
        print(kind, v, flush=True)
        assert v["per_s"] > 0
        assert 0.3e9 < v["clock_hz"] < 4.0e9
        # at most two lane-operations (relaxations) per lane per clock
        assert 0 < v["per_lane_clock"] < 2.5
