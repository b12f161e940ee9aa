"""spq_valu_rates: the measured issue rates the relaxation peak rests on."""
import pytest

spq = pytest.importorskip("paper_1503_07192_amd.spq")

pytestmark = pytest.mark.gpu


def test_valu_rates_are_measured():
    r = spq.valu_rates()
    print(r, flush=True)
    lane_cycles = 256 * 64 * 2.4e9   # MI355X: 256 CUs x 64 lanes x 2.4 GHz
    for kind in ("v_add_u32", "v_min3_u32", "relax_loop", "relax_regs"):
        # at most two operations (relaxations) per lane and clock
        assert 0 < r[kind] < 2.2 * lane_cycles
