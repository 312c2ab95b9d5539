"""The numbers the paper prints (tests/golden/paper_values.txt, each with its
citation) are the ones the inputs and experiments use."""
import math
import os

import numpy as np

from paper_0705_0497_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))


def golden():
    out = {}
    for line in open(os.path.join(HERE, "golden", "paper_values.txt")):
        if line.strip() and not line.startswith("#"):
            key, value, unit = line.split()[:3]
            out[key] = (float(value), unit)
    return out


def test_eq1_coefficient_and_exponent():
    g = golden()
    assert g["ad_sigma_coefficient"][1] == "cm^2"
    assert I.eq1_sigma0_m2() == g["ad_sigma_coefficient"][0] * 1e-4
    e = np.array([0.01, 1.0, 4.0, 100.0])
    tab = I.power_law(e, I.eq1_sigma0_m2(), 0.0, -g["ad_sigma_exponent"][0], 0.0)
    np.testing.assert_allclose(tab, g["ad_sigma_coefficient"][0] * 1e-4 * e ** g["ad_sigma_exponent"][0], rtol=1e-14)


def test_background_and_thresholds():
    g = golden()
    assert I.config(1).t_gas == g["gas_temperature"][0]
    ext = {p.name: p for p in I.make_processes_extended()}
    assert ext["e-diss6.4"].e_th == g["dissociation_threshold_1"][0]
    assert ext["e-diss8.6"].e_th == g["dissociation_threshold_2"][0]


def test_cx_bridge_bounds():
    g = golden()
    e = I.energy_grid()
    sm = 1e-18 * np.ones_like(e)
    sm[e > 1.0] = 3e-18                           # a step inside the bridge shows where it is bridged
    cx = I.cx_from_momentum_transfer(sm)
    lo, hi = g["cx_bridge_low"][0], g["cx_bridge_high"][0]
    assert np.all(cx[e <= lo] == 0.5e-18) and np.all(cx[e >= hi] == 1.5e-18)
    mid = (e > lo) & (e < hi)
    assert np.all((cx[mid] > 0.5e-18) & (cx[mid] < 1.5e-18))


def test_section3_discharge_and_metastable_fraction():
    from paper_0705_0497_amd import csweep
    g = golden()
    d = csweep.fig34_discharge(1.0 / 6.0, 0)
    assert d.L == g["fig34_gap"][0] * 1e-2
    assert d.f == g["fig34_frequency"][0] * 1e6
    assert d.p == g["fig34_pressure"][0]
    assert d.U == g["fig34_voltage"][0]
    assert abs(csweep.C_VALUES[-1] - g["fig4_metastable_fraction"][0]) < 1e-9
    assert g["fig4_measured_density"][1] == "cm^-3" and math.isfinite(g["fig4_measured_density"][0])
