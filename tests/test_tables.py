"""The paper's cross-section models as table generators (section 2), checked
against their closed forms and limits (host only)."""
import math

import numpy as np
import pytest

from paper_0705_0497_amd import inputs as I

A0 = 5.29177210903e-11
EH = 27.211386245988


@pytest.mark.parametrize("r_x", [3.0, 5.3, 12.0])
def test_landau_zener_limits_and_crossing_energy(r_x):
    geo = 4 * math.pi * (r_x * A0) ** 2                     # the high-energy limit 4 pi R_x^2
    assert abs(I.landau_zener([1e9], r_x)[0] / geo - 1) < 1e-7
    # at E = 1 / R_x (Hartree), the Coulomb energy of the crossing, the cross section doubles
    assert abs(I.landau_zener([EH / r_x], r_x)[0] / (2 * geo) - 1) < 1e-12
    # low energies: sigma E -> 4 pi R_x E_h (Coulomb focusing)
    e = 1e-6
    assert abs(I.landau_zener([e], r_x)[0] * e / (4 * math.pi * r_x * A0 ** 2 * EH) - 1) < 1e-5
    tab = I.landau_zener_table(r_x)
    assert np.all(np.diff(tab) < 0) and tab.shape == (I.TABLE_N,)


def test_charge_exchange_bridge():
    e = I.energy_grid()
    sm = 3e-19 * (e / 1.0) ** -0.4 + 1e-20
    cx = I.cx_from_momentum_transfer(sm)
    out = (e <= 0.251) | (e >= 8.5)
    np.testing.assert_array_equal(cx[out], 0.5 * sm[out])
    mid = ~out
    # linear in E between the two ends, meeting sigma_m / 2 there
    lo, hi = 0.5 * np.interp(np.log([0.251, 8.5]), np.log(e), sm)
    np.testing.assert_allclose(cx[mid], lo + (hi - lo) * (e[mid] - 0.251) / (8.5 - 0.251), rtol=1e-12)
    f = lambda x: 3e-19 * np.asarray(x) ** -0.4 + 1e-20
    cx2 = I.cx_from_momentum_transfer(f)
    np.testing.assert_array_equal(cx2[out], 0.5 * f(e[out]))
    assert abs(cx2[mid][0] - (0.5 * f(0.251) + (0.5 * f(8.5) - 0.5 * f(0.251)) * (e[mid][0] - 0.251) / 8.249)) \
        < 1e-12 * cx2[mid][0]
    with pytest.raises(ValueError):
        I.cx_from_momentum_transfer(np.ones(3))


def test_eq1_associative_detachment_table():
    """Eq. (1): 5.96e-16 cm^2 / sqrt(E [eV]) on the table grid."""
    e = I.energy_grid()
    tab = I.power_law_table(I.eq1_sigma0_m2(), 0.0, 0.5, 0.0)
    np.testing.assert_allclose(tab, 5.96e-20 / np.sqrt(e), rtol=1e-13)
