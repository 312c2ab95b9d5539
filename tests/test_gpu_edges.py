"""Edge cases of the hot path against the oracle, one step element by element:
the largest grid the library takes (8192 cells: the LDS of one block and the
field block's register tiles at their limits, electrons crossing ~60 cells per
step), the smallest (2 cells), an empty electron store that fills with
detachment products, and a few particles per species (a ragged last group)."""
import numpy as np
import pytest

from oracle import pyoracle as po
from paper_0705_0497_amd import inputs as I
from tests import helpers as H

pytestmark = pytest.mark.gpu
EVCAP = 1 << 20


def _max_displacement(before, after):
    # largest |x_after - x_before| in cells over the ids present in both states
    b = {int(i): float(c) + float(f) for i, c, f in zip(before["id"], before["cell"], before["off"])}
    d = [abs(x - b[int(i)]) for i, x in zip(after["id"], after["xi"]) if int(i) in b]
    return max(d, default=0.0)


def _one_step(d, procs, st, nid, step, **kw):
    o = H.oracle_from_canonical(d, procs, st, nid, step)
    g = H.gpu_from_canonical(d, procs, st, nid, step, event_capacity=EVCAP, **kw)
    o.log_events(True)
    o.step(1)
    g.step(1)
    bad, band = H.compare_events(g.events(), o.events())
    assert not bad, f"decisions differ outside the band: {bad[:10]}"
    for s in range(3):
        gs, nid_g = g.get_particles(s)
        os_ = o.get_particles(s)
        # the FP32 offset carries a few ulps (2^-24 relative) of the step's displacement: at 8192
        # cells electrons cross up to ~100 cells per step, beyond what the fixed 1e-5 cell allows
        pos_tol = H.POS_TOL + 2.0 ** -22 * _max_displacement(st[s], os_)
        dx, dv = H.compare_states(gs, os_, d.species()[s], skip=band, s=s)
        assert dx <= pos_tol and dv <= H.VEL_TOL, (s, dx, pos_tol, dv)
        np.testing.assert_array_equal(g.hist()[s], po.deposit_canonical(d.ng, gs["cell"], gs["off"]))
        assert g.count(s) == o.count(s) or band
    if not band:
        np.testing.assert_array_equal(g.counters()[:po.C_CLAMP], o.counters()[:po.C_CLAMP])
    return o, g


@pytest.mark.parametrize("ng,n_total", [(2, 3000), (8192, 20000)])
def test_extreme_grids(ng, n_total):
    d = I.config(1, ng=ng, n_total=n_total)
    procs = H.neutralising(I.make_processes())
    st, nid, sidx = H.canonical_from_oracle(d, procs, 10)
    assert sidx % d.ksub == 0                  # the compared step pushes the ions too
    _one_step(d, procs, st, nid, sidx)


def test_empty_electron_store_fills_with_products():
    # no electrons loaded: the first ion step detaches O- (Eq. (1), made frequent) into the empty store
    d = I.config(1, counts=(0, 4000, 4000), n_plus0=1e12)
    procs = I.make_processes()
    for p in procs:
        if p.target == "O2a":
            p.sigma = p.sigma * 50.0
    st, nid, sidx = H.canonical_from_oracle(d, procs, 0)
    assert len(st[0]["id"]) == 0
    o, g = _one_step(d, procs, st, nid, 0)
    assert g.count(0) > 0 and g.count(0) == o.count(0)


@pytest.mark.parametrize("n", [1, 9, 17])
def test_few_particles_per_species(n):
    # n = 8 k + 1: the last 8-slot group of each species holds one particle
    d = I.config(1, counts=(n, n, n), n_plus0=1e9)
    procs = I.make_processes()
    st, nid, sidx = H.canonical_from_oracle(d, procs, 0)
    for step in (0, 1):
        _one_step(d, procs, st, nid, step)


@pytest.mark.parametrize("block,grid,sort_every", [(1024, 0, 7), (256, 2048, 3), (512, 5, 0)])
def test_cost_balanced_push_ranges_deposit_every_electron_once(block, grid, sort_every):
    """The electron push cuts the store where the previous launch's measured cost
    reaches equal fractions: after every step the electron charge histogram is
    exactly the deposit of the electron state (a range gap leaves electrons out,
    an overlap deposits them twice), also when reordering shrinks the store between
    launches and when most of a large grid gets empty ranges."""
    from paper_0705_0497_amd.binding import Discharge
    d = I.config(2)
    g = Discharge(d, I.make_processes(), block=block, grid=grid, sort_every=sort_every)
    g.load_uniform()
    c0 = g.counters()
    for k in range(24):
        g.step(1)
        st, _ = g.get_particles(0)
        np.testing.assert_array_equal(g.hist()[0], po.deposit_canonical(d.ng, st["cell"], st["off"]),
                                      err_msg=f"step {k}")
    assert g.counters()[0] > c0[0]
    g.close()
