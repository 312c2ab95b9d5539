"""The associative-detachment sweep of section 3 (C = 0, 0.1, 1/6) on the GPU:
a short run of the batch, checked against Eq. (1), whose sigma g does not depend
on the energy, so detachments per O- push scale as C."""
import math

import numpy as np
import pytest

from paper_0705_0497_amd import inputs as I


@pytest.mark.gpu
def test_detachment_rate_scales_with_the_metastable_fraction():
    from paper_0705_0497_amd import csweep, binding as B
    res = csweep.run(n_total=30000, max_cycles=20, avg_cycles=10)
    mem = res["members"]
    assert [m["C"] for m in mem] == list(csweep.C_VALUES)
    assert mem[0]["ad_events"] == 0
    for m in mem:
        assert all(v > 0 for v in m["centre_density_m3"].values())
        assert len(m["current_a_m2"]) == 400 and math.isfinite(m["power_w_m2"])
    # detachments per O- push over the averaging window: C n(O2) sigma g dt_i per push
    d = csweep.fig34_discharge(0.1, 0)
    n_o2 = d.p / (1.380649e-23 * 300.0)
    sg = I.eq1_sigma0_m2() * math.sqrt(2 * 1.602176634e-19 / (I.M_OMINUS * I.M_O2 / (I.M_OMINUS + I.M_O2)))
    per_push = [m["ad_events_window"] / max(m["o_minus_pushes_window"], 1) for m in mem[1:]]
    for m, r in zip(mem[1:], per_push):
        p = 1.0 - math.exp(-m["C"] * n_o2 * sg * d.ksub * d.dt)
        n = m["o_minus_pushes_window"]
        assert abs(r * n - p * n) <= 4 * math.sqrt(n * p) + 1, (m["C"], r, p)
