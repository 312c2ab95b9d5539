"""Energy moments of the GPU against the FP64 oracle (the paper's stated output:
the potential and the distribution functions of e, O- and O2+; abstract and
section 1).

What the diagnostics record: per cell the number of particles and the sum of
their kinetic energies (2^-20 eV units), per species the energy distribution on
256 log bins from 1e-3 to 1e3 eV, per electrode the energies of the absorbed
particles, and per node the potential summed over the steps.

* From one canonical state, one step on both sides: the sample of the start
  state (counts exact, energy sums within FP32-vs-FP64 rounding, bins exact
  outside the 1e-6 band at the bin edges), the electrode distributions of the
  step's absorptions (exact), the potential sum (1e-12).
* After many GPU steps, at working and large size: the oracle samples the very
  state the GPU's diagnostics saw, so the comparison stays exact however far
  the run has gone.
"""
import numpy as np
import pytest

from oracle import pyoracle as po
from paper_0705_0497_amd import inputs as I
from tests import helpers as H

pytestmark = pytest.mark.gpu

EDGES = 10.0 ** (-3.0 + 6.0 * np.arange(po.NBIN + 1) / po.NBIN)


def _energies(st, s, species):
    m = species[s].mass
    v2 = st["vx"].astype(np.float64) ** 2 + st["vy"].astype(np.float64) ** 2 + st["vz"].astype(np.float64) ** 2
    return 0.5 * m * v2 / H.QE


def _edf_band(e):
    """Particles whose energy lies within 1e-6 (relative) of a bin edge."""
    e = e[e > 0]
    k = np.searchsorted(EDGES, e)
    near = np.zeros(len(e), bool)
    for kk in (k - 1, k):
        kk = np.clip(kk, 0, len(EDGES) - 1)
        near |= np.abs(e - EDGES[kk]) <= 1e-6 * e
    return int(near.sum())


def _check_sample(mg, mo, states, species):
    """One diagnostic sample of the same state on both sides."""
    assert mg["ndiag"] == mo["ndiag"] == 1
    np.testing.assert_array_equal(mg["ecnt"], mo["ecnt"])
    for s in range(3):
        # per particle the FP32 energy differs from the FP64 one by a few ulp, and
        # each side rounds e 2^20 to an integer: |diff| <= 1 unit + 3e-7 e per particle
        tol = mo["ecnt"][s] + 3e-7 * np.abs(mo["esum"][s].astype(np.float64))
        diff = np.abs(mg["esum"][s].astype(np.float64) - mo["esum"][s].astype(np.float64))
        assert np.all(diff <= tol), (s, float(np.max(diff - tol)))
        band = _edf_band(_energies(states[s], s, species))
        moved = int(np.abs(mg["edf"][s] - mo["edf"][s]).sum())
        assert moved <= 2 * band, (s, moved, band)
        assert mg["edf"][s].sum() == mo["edf"][s].sum() == len(states[s]["id"])


@pytest.mark.parametrize("step0", [0, 20])
def test_energy_moments_single_step(step0):
    d = I.config(1, diag_every=1)
    procs = I.make_processes()
    st, nid, _ = H.canonical_from_oracle(d, procs, seed_steps=30)
    o = H.oracle_from_canonical(d, procs, st, nid, step0)
    g = H.gpu_from_canonical(d, procs, st, nid, step0)
    o.reset_moments()
    g.moments(reset=True)
    o.step(1)
    g.step(1)
    mo, mg = o.moments(), g.moments()
    _check_sample(mg, mo, st, d.species())
    # the step's absorptions at each electrode, binned by their energy
    np.testing.assert_array_equal(mg["iedf"], mo["iedf"])
    assert mo["iedf"].sum() > 0
    # charge and potential summed over the step: the same state, the same field
    assert mg["nacc"] == mo["nacc"] == 1
    np.testing.assert_array_equal(mg["sum_q"], mo["sumQ"])
    assert np.max(np.abs(mg["sum_phi"] - mo["sumphi"])) <= 1e-12 * np.max(np.abs(mo["sumphi"]))


def test_energy_moments_of_ragged_stores():
    """Stores whose sizes leave 1, 2 and 3 slots after the last full group of the
    four slots a thread reads at once: every particle is sampled once."""
    d = I.config(1, diag_every=1)
    procs = I.make_processes()
    st, nid, step = H.canonical_from_oracle(d, procs, seed_steps=30)
    trimmed = []
    for s in range(3):
        n = len(st[s]["id"])
        keep = n - (n - (s + 1)) % 4
        trimmed.append({k: v[:keep] for k, v in st[s].items()})
    assert [len(t["id"]) % 4 for t in trimmed] == [1, 2, 3]
    o = H.oracle_from_canonical(d, procs, trimmed, nid, step)
    g = H.gpu_from_canonical(d, procs, trimmed, nid, step)
    o.reset_moments()
    g.moments(reset=True)
    o.step(1)
    g.step(1)
    _check_sample(g.moments(), o.moments(), trimmed, d.species())


def _state_moments_after(cfg, steps, **kw):
    """The GPU runs `steps` steps, then records one diagnostic sample of its state;
    the oracle samples the same state."""
    from paper_0705_0497_amd.binding import Discharge
    d = I.config(cfg, diag_every=steps)
    procs = I.make_processes()
    g = Discharge(d, procs, **kw)
    g.load_uniform()
    g.step(steps)
    states = [g.get_particles(s) for s in range(3)]
    g.moments(reset=True)
    g.step(1)                                        # diagnostics sample the step's start state
    mg = g.moments()
    o = po.Oracle(d, d.species(), procs)
    for s in range(3):
        o.set_particles(s, states[s][0], states[s][1])
    o.reset_moments()
    o.sample_moments()
    mo = o.moments()
    g.sync()
    return d, mg, mo, [st for st, _ in states]


def test_energy_moments_of_a_late_state_match_the_oracle():
    # the 128-cell discharge after five rf cycles
    d, mg, mo, states = _state_moments_after(1, 5 * 400)
    _check_sample(mg, mo, states, d.species())


@pytest.mark.parametrize("cfg,steps", [(2, 2000), (3, 39)])
def test_energy_moments_full_size(cfg, steps):
    """Working (512 cells, 6e5+ particles, one rf cycle in) and large (4096 cells,
    4.8e7+ particles) discharges in the benchmark's launch shape."""
    d, mg, mo, states = _state_moments_after(cfg, steps, block=1024)
    _check_sample(mg, mo, states, d.species())
