"""GPU (HIP, gfx950) against the FP64 oracle.

Single steps are compared element by element from identical canonical states:
positions to 1e-5 cell, velocities to 1e-5 of max(|v|, thermal speed), collision
decisions identical outside the 1e-6 band the oracle reports, charge histograms
bit-exact.  Longer runs are compared statistically and by exact properties
(determinism, resume, bookkeeping).
"""
import math

import numpy as np
import pytest

from oracle import pyoracle as po
from paper_0705_0497_amd import inputs as I
from tests import helpers as H

pytestmark = pytest.mark.gpu

EVCAP = 1 << 21


def _pair(d, procs, step0, seed_steps=0, event_capacity=EVCAP, **kw):
    st, nid, sidx = H.canonical_from_oracle(d, procs, seed_steps)
    step = step0 if step0 is not None else sidx
    o = H.oracle_from_canonical(d, procs, st, nid, step)
    g = H.gpu_from_canonical(d, procs, st, nid, step, event_capacity=event_capacity, **kw)
    return o, g, st


def test_initial_deposit_and_field_match_oracle():
    d = I.config(1)
    procs = I.make_processes()
    o, g, st = _pair(d, procs, 0)
    np.testing.assert_array_equal(g.hist(), o.hist())                     # bit-exact deposit
    for s in range(3):
        np.testing.assert_array_equal(g.hist()[s], po.deposit_canonical(d.ng, st[s]["cell"], st[s]["off"]))
    # field of the same histograms: GPU double scan vs oracle Thomas
    g.set_step(137)
    o.set_step(137)
    g.prepare(True)
    o.prepare(True)
    phi_g, e_g = g.field()
    phi_o, e_o = o.field()
    assert np.max(np.abs(phi_g - phi_o)) <= 1e-12 * np.max(np.abs(phi_o))
    assert np.max(np.abs(e_g - e_o)) <= 1e-6 * np.max(np.abs(e_o))
    for s in range(3):                                                   # leapfrog start
        gs, os_ = g.get_particles(s)[0], o.get_particles(s)
        dx, dv = H.compare_states(gs, os_, d.species()[s], s=s)
        assert dx == 0.0 and dv < 1e-6


@pytest.mark.parametrize("step0,neut", [(0, False), (1, False), (0, True), (20, True)])
def test_single_step_element_by_element(step0, neut):
    d = I.config(1)
    procs = I.make_processes()
    if neut:
        procs = H.neutralising(procs)
    o, g, st = _pair(d, procs, step0, seed_steps=30 if neut else 0)
    o.log_events(True)
    o.step(1)
    g.step(1)
    gev = g.events()
    bad, band = H.compare_events(gev, o.events())
    assert not bad, f"decisions differ outside the band: {bad[:10]}"
    assert len(band) <= max(3, len(gev) // 1000)
    for s in range(3):
        gs, nid_g = g.get_particles(s)
        dx, dv = H.compare_states(gs, o.get_particles(s), d.species()[s], skip=band, s=s)
        assert dx <= H.POS_TOL and dv <= H.VEL_TOL, (s, dx, dv)
        if not band:
            assert nid_g == o.next_id(s)
        # charge bit-exact against the oracle's deposit of the GPU state
        np.testing.assert_array_equal(g.hist()[s], po.deposit_canonical(d.ng, gs["cell"], gs["off"]))
    if not band:
        np.testing.assert_array_equal(g.counters()[:po.C_CLAMP], o.counters()[:po.C_CLAMP])


def test_products_and_pairing_over_an_ion_cycle():
    """Twenty steps with frequent neutralisation: bookkeeping exact each step,
    ids dense and unique, histograms the deposit of the state."""
    d = I.config(1)
    procs = H.neutralising(I.make_processes())
    o, g, st = _pair(d, procs, None, seed_steps=10)
    kinds = [p.kind for p in procs]
    ev = lambda c, k: sum(int(c[po.C_EVENT + i]) for i, kk in enumerate(kinds) if kk == k)
    N = [g.count(s) for s in range(3)]
    c0 = g.counters()
    paired = 0
    for _ in range(2 * d.ksub):
        g.step(1)
        c1 = g.counters()
        dc = c1 - c0
        A = [dc[po.C_ABS0 + s] + dc[po.C_ABSL + s] for s in range(3)]
        N1 = [g.count(s) for s in range(3)]
        assert N1[0] == N[0] - A[0] + ev(dc, "ionize") - ev(dc, "attach") + ev(dc, "detach")
        assert N1[1] == N[1] - A[1] + ev(dc, "ionize") - dc[po.C_PAIRED]
        assert N1[2] == N[2] - A[2] + ev(dc, "attach") - ev(dc, "neutralize") - ev(dc, "detach")
        assert dc[po.C_PAIRED] + dc[po.C_DEFICIT] == ev(dc, "neutralize")
        paired += dc[po.C_PAIRED]
        Q = g.hist()
        for s in range(3):
            gs, nid = g.get_particles(s)
            assert Q[s].sum() == (1 << 32) * N1[s]
            ids = np.sort(gs["id"])
            assert len(np.unique(ids)) == len(ids) and (len(ids) == 0 or ids[-1] < nid)
        N, c0 = N1, c1
    assert paired > 0


def test_pairing_takes_every_partner_a_cell_has():
    """Table 1 (17): each neutralisation removes one O2+ of the O-'s cell, the one
    with the smallest (pairing draw, id) among those there before the step; a cell
    with more events than O2+ gives them all and counts the rest as a deficit.  The
    same O2+ leave on both sides, cell by cell."""
    from paper_0705_0497_amd.binding import Discharge, F_EXT_FIELD
    neut = I.Process("n", 2, "neutralize", "grid+", 0.0, I.M_O2PLUS, I.power_law_table(4e-14, 0, 0.5, 0), {})
    ng = 8
    # cell 2: 3 O2+ among 300 O- (its nodes carry the density of 1500 O2+ each from cells
    # 1 and 3); cell 5: 3000 O2+, 300 O-; cell 6: 40 O2+ and 300 O-, densities from cell 7
    xpos = np.concatenate([np.full(3, 2.5), np.full(1500, 1.99), np.full(1500, 3.01), np.full(3000, 5.5),
                           np.full(40, 6.5), np.full(2000, 7.01)])
    xneg = np.concatenate([np.full(300, 2.5), np.full(300, 5.5), np.full(300, 6.5)])
    npos, nneg = len(xpos), len(xneg)
    weight = 6.25e12
    d = I.config(1, L=0.025, ng=ng, p=2000.0, c_meta=1.0, diag_every=0, sort_every=0,
                 n_plus0=weight * npos / 0.025, counts=(1, npos, 1))
    sp = [I.Species(-1.0, I.ELECTRON_MASS, 3.0, 0, 1), I.Species(1.0, I.M_O2PLUS, 0.026, npos, npos),
          I.Species(-1.0, I.M_OMINUS, 0.026, nneg, nneg)]

    def canon(x):
        cell = np.floor(x).astype(np.int32)
        z = np.zeros(len(x), np.float32)
        return dict(cell=cell, off=(x - cell).astype(np.float32), vx=z, vy=z, vz=z,
                    id=np.arange(len(x), dtype=np.uint32), cd=np.ones(len(x), np.int32))
    st = [canon(np.zeros(0)), canon(xpos), canon(xneg)]
    nid = [0, npos, nneg]
    o = H.oracle_from_canonical(d, [neut], st, nid, 0, species=sp, flags=po.F_EXT_FIELD, e_ext=(0.0, 0.0))
    g = Discharge(d, [neut], species=sp, flags=F_EXT_FIELD, e_ext=(0.0, 0.0), sort_every=0)
    for s in range(3):
        g.set_particles(s, st[s], nid[s])
    g.set_step(0)
    g.prepare(False)
    o.step(1)
    g.step(1)
    for s in (1, 2):
        np.testing.assert_array_equal(np.sort(g.get_particles(s)[0]["id"]), np.sort(o.get_particles(s)["id"]))
    gc, oc = g.counters(), o.counters()
    for c in (po.C_PAIRED, po.C_DEFICIT, po.C_EVENT):
        assert gc[c] == oc[c], (c, gc[c], oc[c])
    left = np.bincount(np.floor(H.xi_of(g.get_particles(1)[0])).astype(int), minlength=ng)
    k = np.bincount(np.floor(xneg[np.isin(np.arange(nneg), g.get_particles(2)[0]["id"], invert=True)]).astype(int),
                    minlength=ng)
    assert k[2] > 3 and k[6] > 40 and k[5] > 3
    assert left[2] == 0 and left[6] == 0 and left[5] == 3000 - k[5]
    assert gc[po.C_DEFICIT] == (k[2] - 3) + (k[6] - 40)
    np.testing.assert_array_equal(g.hist(), o.hist())


def test_multi_step_trajectories_stay_close():
    """Same draws on both sides: after 40 steps most particles still agree."""
    d = I.config(1)
    procs = I.make_processes()
    o, g, st = _pair(d, procs, 0)
    o.step(40)
    g.step(40)
    for s in range(3):
        gs, os_ = H.by_id(g.get_particles(s)[0]), H.by_id(o.get_particles(s))
        common, gi, oi = np.intersect1d(gs["id"], os_["id"], return_indices=True)
        assert len(common) >= 0.98 * max(len(gs["id"]), len(os_["id"]))
        dx = np.abs(H.xi_of(gs)[gi] - H.xi_of(os_)[oi])
        assert np.mean(dx < 1e-3) > 0.95


def _run_gpu(d, procs, steps, **kw):
    from paper_0705_0497_amd.binding import Discharge
    g = Discharge(d, procs, **kw)
    g.load_uniform()
    g.step(steps)
    return g, [H.by_id(g.get_particles(s)[0]) for s in range(3)], g.hist()


def _same(a, b):
    for s in range(3):
        for k in ("cell", "off", "vx", "vy", "vz", "id", "cd"):
            np.testing.assert_array_equal(a[s][k], b[s][k])


def test_determinism_across_repeats_blocks_and_sort_interval():
    d = I.config(1)
    procs = H.neutralising(I.make_processes())
    _, a, qa = _run_gpu(d, procs, 300)
    _, b, qb = _run_gpu(d, procs, 300)
    _same(a, b)
    np.testing.assert_array_equal(qa, qb)
    _, c, qc = _run_gpu(d, procs, 300, block=256, grid=7, sort_every=7)
    _same(a, c)
    np.testing.assert_array_equal(qa, qc)
    _, e, qe = _run_gpu(d, procs, 300, block=1024, sort_every=0)
    _same(a, e)
    _, f, qf = _run_gpu(d, procs, 300, sort_every=11, sort_kind=1)     # order-preserving compaction
    _same(a, f)
    np.testing.assert_array_equal(qa, qf)


def test_multi_step_calls_equal_single_steps():
    """pic_step(h, n) solves the field of each next electron-only step inside the
    electron reduction; n calls of one step never do.  Both reach the same state,
    field, moments and counters bit for bit, at two grid sizes (one and several
    node columns of the reduction)."""
    from paper_0705_0497_amd.binding import Discharge
    for d in (I.config(1), I.config(1, ng=2500, n_total=60000)):
        procs = H.neutralising(I.make_processes())
        a = Discharge(d, procs)
        b = Discharge(d, procs)
        a.load_uniform()
        b.load_uniform()
        a.step(157)
        for _ in range(157):
            b.step(1)
        _same([H.by_id(a.get_particles(s)[0]) for s in range(3)], [H.by_id(b.get_particles(s)[0]) for s in range(3)])
        np.testing.assert_array_equal(a.hist(), b.hist())
        for x, y in zip(a.field(), b.field()):
            np.testing.assert_array_equal(x, y)
        ma, mb = a.moments(), b.moments()
        for k in ma:
            np.testing.assert_array_equal(ma[k], mb[k], err_msg=k)
        np.testing.assert_array_equal(a.counters(), b.counters())


def test_resume_is_bitwise():
    from paper_0705_0497_amd.binding import Discharge
    d = I.config(1)
    procs = H.neutralising(I.make_processes())
    _, a, qa = _run_gpu(d, procs, 250)
    g, _, _ = _run_gpu(d, procs, 110)
    st = [g.get_particles(s) for s in range(3)]
    r = Discharge(d, procs)
    for s in range(3):
        r.set_particles(s, st[s][0], st[s][1])
    r.set_step(g.step_index)
    r.prepare(False)
    r.step(140)
    _same(a, [H.by_id(r.get_particles(s)[0]) for s in range(3)])
    np.testing.assert_array_equal(qa, r.hist())


def test_gpu_loader_statistics():
    from scipy import stats
    from paper_0705_0497_amd.binding import Discharge
    d = I.config(2)
    g = Discharge(d, I.make_processes())
    g.load_uniform()
    o = po.Oracle(d, d.species(), I.make_processes())
    for s, sp in enumerate(d.species()):
        st, nid = g.get_particles(s)
        assert len(st["id"]) == sp.count and nid == sp.count
        assert stats.kstest(H.xi_of(st) / d.ng, "uniform").pvalue > 1e-4
        assert sorted(st["id"].tolist()) == list(range(sp.count))
    # positions are exact lattice points: identical to the oracle's loader
    o.load_uniform()
    for s in range(3):
        gs, os_ = H.by_id(g.get_particles(s)[0]), H.by_id(o.canonical(s))
        np.testing.assert_array_equal(gs["cell"], os_["cell"])
        np.testing.assert_array_equal(gs["off"], os_["off"])
        assert np.max(np.abs(gs["vy"] - os_["vy"]) / H.thermal_speed(d.species()[s])) < 1e-5


def test_ballistic_flight_fp32():
    from paper_0705_0497_amd.binding import Discharge, F_EXT_FIELD, F_NO_COLL
    d = I.config(1)
    E0 = -50.0
    sp = [I.Species(-1.0, I.ELECTRON_MASS, 3.0, 0, 64), I.Species(1.0, I.M_O2PLUS, 0.026, 0, 64),
          I.Species(-1.0, I.M_OMINUS, 0.026, 0, 64)]
    g = Discharge(d, [], species=sp, flags=F_EXT_FIELD | F_NO_COLL, e_ext=(E0, 0.0))
    rng = np.random.default_rng(2)
    xi0 = rng.uniform(20, 40, 16)
    v0 = rng.uniform(-1e5, 1e5, 16)
    cell = np.floor(xi0).astype(np.int32)
    z = np.zeros(16, np.float32)
    g.set_particles(0, dict(cell=cell, off=(xi0 - cell).astype(np.float32), vx=v0.astype(np.float32), vy=z, vz=z,
                            id=np.arange(16, dtype=np.uint32), cd=np.ones(16, np.int32)), 16)
    for s in (1, 2):
        g.set_particles(s, dict(cell=np.zeros(0, np.int32), off=z[:0], vx=z[:0], vy=z[:0], vz=z[:0],
                                id=np.zeros(0, np.uint32), cd=np.zeros(0, np.int32)), 0)
    g.prepare(True)
    n = 200
    g.step(n)
    st = H.by_id(g.get_particles(0)[0])
    a = QE_ = 1.602176634e-19 * (-E0) / I.ELECTRON_MASS
    t = n * d.dt
    expect = (xi0 * (d.L / d.ng) + (v0.astype(np.float32).astype(float) * t + 0.5 * a * t * t)) / (d.L / d.ng)
    np.testing.assert_allclose(H.xi_of(st), expect, atol=2e-3)   # FP32 offsets over 200 steps
    np.testing.assert_allclose(st["vx"], v0 + a * (n - 0.5) * d.dt, rtol=1e-5)


def _decisions(ev, s, ids=None):
    """(id, code) of the species' decision records, sorted by id (vectorised)."""
    r = ev[ev[:, 1] == s]
    r = r[r[:, 3] != -4]
    if ids is not None:
        r = r[np.isin(r[:, 2], ids)]
    o = np.argsort(r[:, 2], kind="stable")
    return r[o, 2], r[o, 3]


def _band_of(oev, s):
    b = oev[(oev[:, 4] != 0) & ((oev[:, 1] == s) | ((s == 0) & (oev[:, 1] == 3)))]
    return set(b[:, 2].tolist())


@pytest.mark.parametrize("cfg", [2, 3])
def test_full_size_single_step(cfg):
    """Working and large discharges in the benchmark's launch shape, one ion step and
    one electron step.  The oracle holds every ion (so the O2+ density that the O-
    see, the O- collision bound, neutralisation, detachment and the pairing of the
    ion step are the GPU's) and a sample of the electrons, in the GPU's own field;
    decisions and states are compared for every species, the wall distributions of
    the ions exactly, and the deposit is exact on the whole state."""
    from paper_0705_0497_amd.binding import Discharge
    d = I.config(cfg)
    procs = I.make_processes()
    g = Discharge(d, procs, event_capacity=1 << 26, block=1024)     # bench.py's push block
    g.load_uniform()
    g.step(2 * d.ksub)               # the next step is an ion step, with a re-ordering just before it
    for step_kind in ("ion", "electron"):
        n = g.step_index
        assert (n % d.ksub == 0) == (step_kind == "ion")
        states = [g.get_particles(s) for s in range(3)]
        Q = g.hist()
        for s in range(3):
            np.testing.assert_array_equal(Q[s], po.deposit_canonical(d.ng, states[s][0]["cell"], states[s][0]["off"]))
        rng = np.random.default_rng(cfg * 10 + n)
        samples = []
        o = po.Oracle(d, d.species(), procs)
        for s in range(3):
            st, nid = states[s]
            if s == 0:
                k = rng.choice(len(st["id"]), size=min(50000, len(st["id"])), replace=False)
                st = {key: v[k] for key, v in st.items()}
            samples.append(st)
            o.set_particles(s, st, nid)
        o.set_hist(Q)
        o.set_step(n)
        o.log_events(True)
        o.reset_moments()
        g.clear_events()
        g.moments(reset=True)
        gc0 = g.counters()
        g.step(1)
        o.step(1)
        gev = g.events()
        oev = o.events()
        check = (0, 1, 2) if step_kind == "ion" else (0,)
        for s in check:
            ids = samples[s]["id"]
            band = _band_of(oev, s)
            gi, gc = _decisions(gev, s, ids)
            oi, oc = _decisions(oev, s)
            if s == 2 and step_kind == "ion":
                assert len(oi) > 10, "the ion step has O- collision candidates"
            keep_g = ~np.isin(gi, list(band)) if band else np.ones(len(gi), bool)
            keep_o = ~np.isin(oi, list(band)) if band else np.ones(len(oi), bool)
            np.testing.assert_array_equal(gi[keep_g], oi[keep_o], err_msg=f"cfg {cfg} species {s}: candidates")
            np.testing.assert_array_equal(gc[keep_g], oc[keep_o], err_msg=f"cfg {cfg} species {s}: channels")
            gs = H.by_id(g.get_particles(s)[0])
            os_ = H.by_id(o.get_particles(s))
            keep = np.isin(os_["id"], ids)                      # the pre-step particles, no products
            os_ = {k2: v[keep] for k2, v in os_.items()}
            gk = np.isin(gs["id"], ids)
            gs = {k2: v[gk] for k2, v in gs.items()}
            skip = {(s, i) for i in band}
            dx, dv = H.compare_states(gs, os_, d.species()[s], skip=skip, s=s)
            assert dx <= H.POS_TOL and dv <= H.VEL_TOL, (cfg, step_kind, s, dx, dv)
        if step_kind == "ion":
            # every ion of both sides: the same partners removed, the same wall energies
            gc_, oc_ = g.counters() - gc0, o.counters()
            assert gc_[po.C_PAIRED] == oc_[po.C_PAIRED] and gc_[po.C_DEFICIT] == oc_[po.C_DEFICIT] == 0
            mg, mo = g.moments(), o.moments()
            np.testing.assert_array_equal(mg["iedf"][1:], mo["iedf"][1:])
        g.sync()


def _profile():
    x = np.linspace(0.0, 1.0, 17)
    bump = np.sin(np.pi * x)
    dens = np.stack([2e14 + 4e14 * bump, 3e14 + 9e14 * bump, 1e14 + 5e14 * bump ** 2])
    mean = np.stack([1.0 + 3.0 * bump, 0.04 + 0.5 * x, np.full_like(x, 0.039)])
    return x, dens, mean


def test_profile_loader_matches_oracle():
    from paper_0705_0497_amd.binding import Discharge
    d = I.config(1, n_total=60000)
    procs = I.make_processes()
    x, dens, mean = _profile()
    o = po.Oracle(d, d.species(), procs)
    o.load_profile(x, dens, mean)
    o.prepare(True)
    g = Discharge(d, procs)
    assert g.load_profiles(x, dens, mean)
    for s in range(3):
        gs, os_ = g.get_particles(s)[0], o.get_particles(s)
        assert len(gs["id"]) == len(os_["id"]) > 1000
        dx, dv = H.compare_states(gs, os_, d.species()[s], s=s)
        assert dx == 0.0 and dv < 1e-5, (s, dx, dv)                 # same cells, same lattice offsets
    np.testing.assert_array_equal(g.hist(), o.hist())
    phi_g, _ = g.field()
    phi_o, _ = o.field()
    assert np.max(np.abs(phi_g - phi_o)) <= 1e-12 * np.max(np.abs(phi_o))


def test_profile_loader_falls_back_to_uniform_on_invalid_input():
    from paper_0705_0497_amd.binding import Discharge
    d = I.config(1)
    procs = I.make_processes()
    x, dens, mean = _profile()
    mean[0, 3] = -1.0                                                 # a negative mean energy
    g = Discharge(d, procs)
    assert g.load_profiles(x, dens, mean) is False
    u = Discharge(d, procs)
    u.load_uniform()
    for s in range(3):
        a, b = H.by_id(g.get_particles(s)[0]), H.by_id(u.get_particles(s)[0])
        for k in ("cell", "off", "vx", "vy", "vz", "id", "cd"):
            np.testing.assert_array_equal(a[k], b[k])


def test_current_density_and_power_match_oracle():
    # section 3: displacement plus conduction current at the driven electrode per rf phase
    d = I.config(1)
    procs = I.make_processes()
    o, g, st = _pair(d, procs, 0, event_capacity=0)
    o.reset_moments()
    g.moments(reset=True)
    n = 60
    o.step(n)
    g.step(n)
    co, mg = o.current(), g.moments()
    assert np.array_equal(mg["current_n"], co["jcnt"]) and co["jcnt"].sum() == n - 1
    jo, jg = co["jsum"], mg["current"]
    dt = 1.0 / (d.f * d.steps_per_cycle)
    one = H.QE * d.weight / dt                       # one superparticle charge per step
    scale = np.max(np.abs(jo))
    close = np.abs(jg - jo) <= 1e-6 * scale
    assert np.mean(close) >= 0.9
    assert np.all(np.abs(jg - jo) <= 1e-6 * scale + 2 * one)
    assert mg["power_n"] == co["pn"]
    assert abs(mg["power_sum"] - co["psum"]) <= 1e-5 * abs(d.U) * scale * n + 2 * abs(d.U) * one


@pytest.mark.parametrize("step0", [0, 20])
def test_extended_channels_single_step_element_by_element(step0):
    # eleven Table 1 channels, with O- elastic scattering (8) and direct detachment (19)
    # made frequent so that one ion step exercises them on both sides
    d = I.config(1)
    procs = H.neutralising(I.make_processes_extended())
    for k, p in enumerate(procs):
        if p.name == "O--el":
            p.sigma = p.sigma * 30.0
        if p.name == "O--dd":                     # threshold within the thermal O- energies
            procs[k] = I.Process("O--dd", 2, "detach", "O2", 0.02, I.M_O2,
                                 I.power_law_table(1e-18, 1.0, 0.5, 0.02), {})
    o, g, st = _pair(d, procs, step0, seed_steps=30)
    o.log_events(True)
    o.step(1)
    g.step(1)
    gev = g.events()
    oev = o.events()
    names = [p.name for p in procs]
    for nm in ("O--el", "O--dd", "e-diss6.4", "e-diss8.6"):
        assert np.sum(oev[:, 3] == names.index(nm)) >= 3, nm
    bad, band = H.compare_events(gev, oev)
    assert not bad, f"decisions differ outside the band: {bad[:10]}"
    for s in range(3):
        gs, nid_g = g.get_particles(s)
        dx, dv = H.compare_states(gs, o.get_particles(s), d.species()[s], skip=band, s=s)
        assert dx <= H.POS_TOL and dv <= H.VEL_TOL, (s, dx, dv)
        np.testing.assert_array_equal(g.hist()[s], po.deposit_canonical(d.ng, gs["cell"], gs["off"]))
    if not band:
        np.testing.assert_array_equal(g.counters()[:po.C_CLAMP], o.counters()[:po.C_CLAMP])


@pytest.mark.gpu
@pytest.mark.parametrize("step0", [0, 20])
def test_electron_ion_channels_single_step_element_by_element(step0):
    # all sixteen channels; Table 1 (16) and (22) with sigma ~ E^-1/2 large enough that one ion
    # step holds several of each, and the pairing removes their partners
    d = I.config(1)
    procs = H.neutralising(I.make_processes_full())
    for k, p in enumerate(procs):
        if p.name == "e-recomb":
            procs[k] = I.Process("e-recomb", 0, "recomb", "grid+", 0.0, I.M_O2PLUS,
                                 I.power_law_table(1e-13, 0.0, 0.5, 0.0), {})
        if p.name == "e-edet":
            procs[k] = I.Process("e-edet", 0, "edetach", "grid-", 1.461, I.M_OMINUS,
                                 I.power_law_table(1e-14, 0.0, 0.5, 1.461), {})
    o, g, st = _pair(d, procs, step0, seed_steps=30)
    o.log_events(True)
    o.step(1)
    g.step(1)
    gev = g.events()
    oev = o.events()
    names = [p.name for p in procs]
    ei = oev[oev[:, 1] == 3]
    for nm in ("e-recomb", "e-edet"):
        assert np.sum(ei[:, 3] == names.index(nm)) >= 3, nm
    assert np.sum(ei[:, 3] == -1) >= 3                      # null collisions of the test
    bad, band = H.compare_events(gev, oev)
    assert not bad, f"decisions differ outside the band: {bad[:10]}"
    for s in range(3):
        gs, nid_g = g.get_particles(s)
        dx, dv = H.compare_states(gs, o.get_particles(s), d.species()[s], skip=band, s=s)
        assert dx <= H.POS_TOL and dv <= H.VEL_TOL, (s, dx, dv)
        np.testing.assert_array_equal(g.hist()[s], po.deposit_canonical(d.ng, gs["cell"], gs["off"]))
    if not band:
        gc, oc = g.counters(), o.counters()
        np.testing.assert_array_equal(gc[:po.C_CLAMP], oc[:po.C_CLAMP])
        np.testing.assert_array_equal(gc[po.C_EICAND:po.C_DEFICIT_NEG + 1], oc[po.C_EICAND:po.C_DEFICIT_NEG + 1])
        assert all(g.count(s) == o.count(s) for s in range(3))


def _with_a1(factor=20.0):
    # the eight workload channels plus O2(a1Delta_g) excitation (Table 1 (14)), boosted so that
    # a few steps give a production profile; index of the new channel
    procs = H.neutralising(I.make_processes())
    a1 = next(p for p in I.make_processes_full() if p.name == "e-a1")
    a1.sigma = a1.sigma * factor
    k = max(i for i, p in enumerate(procs) if p.species == 0) + 1
    procs.insert(k, a1)
    return procs, k


META = dict(diffusion=0.1, quench_rate=20.0, surface_loss=0.05)


@pytest.mark.gpu
def test_metastable_tally_and_solve_match_the_event_positions():
    """O2(a) production from the GPU's own events: the tally is the exact deposit of the
    electrons that excited O2(a), and the device solve equals the oracle's solver on it."""
    d = I.config(1)
    procs, ka1 = _with_a1(factor=80.0)
    o, g, st = _pair(d, procs, None, seed_steps=30)      # continue after the seed run: fresh draws
    g.metastable_config(ka1, META["diffusion"], META["quench_rate"], META["surface_loss"])
    o.metastable_config(ka1, META["diffusion"], META["quench_rate"], META["surface_loss"])
    g.clear_events()
    o.log_events(True)
    steps = 1                                # the events' positions are those after this step
    g.step(steps)
    o.step(steps)
    gev = g.events()
    hits = gev[(gev[:, 1] == 0) & (gev[:, 3] == ka1)][:, 2]
    assert len(hits) >= 20
    n_g = g.metastable_update()
    n_o = o.metastable_update()
    gs, _ = g.get_particles(0)
    sel = np.isin(gs["id"], hits)
    assert sel.sum() == len(hits)           # excitation keeps the electron
    tally = po.deposit_canonical(d.ng, gs["cell"][sel], gs["off"][sel])
    dx = d.L / d.ng
    vol = np.full(d.ng + 1, dx)
    vol[0] = vol[-1] = dx / 2
    prod = d.weight * (tally / 2.0 ** 32) / (vol * steps * d.dt)
    vbar = math.sqrt(8 * 1.380649e-23 * d.t_gas / (math.pi * I.M_O2))
    h = META["surface_loss"] * vbar / (2 * (2 - META["surface_loss"]))
    n_exp = po.metastable_solve(d.ng, dx, META["diffusion"], META["quench_rate"], h, prod)
    np.testing.assert_allclose(n_g, n_exp, rtol=1e-12, atol=0)
    # the oracle's own update from its FP64 positions: the same events, positions within 1e-5 cell
    np.testing.assert_allclose(n_g, n_o, rtol=5e-4)


@pytest.mark.gpu
def test_detachment_on_the_resolved_density_single_step():
    """Eq. (1) detachment against the O2(a) profile the GPU solved: the oracle takes the
    GPU's state and profile after the production steps, then both run the ion step."""
    d = I.config(1)
    procs, ka1 = _with_a1()
    for p in procs:
        if p.target == "O2a":
            p.sigma = p.sigma * 300.0            # Eq. (1) made frequent at the small O2(a) densities
    st, nid, sidx = H.canonical_from_oracle(d, procs, 30)
    assert sidx % d.ksub == 0
    # continue after the seed run (its draws are not replayed): production steps, then an ion step
    g = H.gpu_from_canonical(d, procs, st, nid, sidx + 1, event_capacity=EVCAP)
    g.metastable_config(ka1, META["diffusion"], META["quench_rate"], META["surface_loss"])
    g.step(d.ksub - 1)
    n_g = g.metastable_update()
    assert n_g.max() > 1.3 * n_g.min()         # a profile, not the uniform start
    gst = [g.get_particles(s) for s in range(3)]
    o = H.oracle_from_canonical(d, procs, [x[0] for x in gst], [x[1] for x in gst], sidx + d.ksub)
    o.metastable_config(ka1, META["diffusion"], META["quench_rate"], META["surface_loss"])
    o.metastable_set(n_g)
    g.clear_events()
    o.log_events(True)
    o.step(1)                                    # the ion step, detachment on the resolved field
    g.step(1)
    gev, oev = g.events(), o.events()
    ad = [i for i, p in enumerate(procs) if p.target == "O2a"][0]
    assert np.sum(oev[:, 3] == ad) >= 3
    bad, band = H.compare_events(gev, oev)
    assert not bad, f"decisions differ outside the band: {bad[:10]}"
    for s in range(3):
        gs, _ = g.get_particles(s)
        dx_, dv = H.compare_states(gs, o.get_particles(s), d.species()[s], skip=band, s=s)
        assert dx_ <= H.POS_TOL and dv <= H.VEL_TOL, (s, dx_, dv)


def _full_set_for_runs():
    # all sixteen channels with the electron-ion rates and the O2(a) production raised so that two rf
    # cycles of the small discharge feel them; index of the O2(a) source channel
    procs = I.make_processes_full()
    for k, p in enumerate(procs):
        if p.name == "e-recomb":
            procs[k] = I.Process("e-recomb", 0, "recomb", "grid+", 0.0, I.M_O2PLUS,
                                 I.power_law_table(2e-15, 0.0, 0.5, 0.0), {})
        if p.name == "e-edet":
            procs[k] = I.Process("e-edet", 0, "edetach", "grid-", 1.461, I.M_OMINUS,
                                 I.power_law_table(2e-15, 0.0, 0.5, 1.461), {})
        if p.name == "e-a1":
            p.sigma = p.sigma * 100.0
    return procs, [p.name for p in procs].index("e-a1")


def test_full_channel_set_with_resolved_o2a_agrees_statistically():
    """Sixteen channels and the O2(a) profile solved after the first rf cycle (each side from
    its own production): node densities over the second cycle, 16 seeds per side, per node
    and species at the thresholds of the other ensemble tests (tests/test_gpu_statistics.py),
    and the electron-ion event counts within 3 sigma."""
    from paper_0705_0497_amd.binding import Discharge
    d = I.config(1)
    procs, ka1 = _full_set_for_runs()
    names = [p.name for p in procs]
    M = 16
    res = {"gpu": [], "orc": []}
    ev = {"gpu": [], "orc": []}
    cols = [po.C_EVENT + names.index("e-recomb"), po.C_EVENT + names.index("e-edet")]
    for m in range(M):
        dd = I.config(1, seed=9100 + m)
        o = po.Oracle(dd, dd.species(), procs)
        o.load_uniform()
        o.prepare(True)
        o.metastable_config(ka1, META["diffusion"], META["quench_rate"], META["surface_loss"])
        o.step(d.steps_per_cycle)
        o.metastable_update()
        o.reset_moments()
        c0 = o.counters()
        o.step(d.steps_per_cycle)
        res["orc"].append(o.moments()["sumQ"] / d.steps_per_cycle / 2.0 ** 32)
        ev["orc"].append((o.counters() - c0)[cols])
        g = Discharge(dd, procs)
        g.load_uniform()
        g.metastable_config(ka1, META["diffusion"], META["quench_rate"], META["surface_loss"])
        g.step(d.steps_per_cycle)
        g.metastable_update()
        g.moments(reset=True)
        c0 = g.counters()
        g.step(d.steps_per_cycle)
        res["gpu"].append(g.moments()["sum_q"] / d.steps_per_cycle / 2.0 ** 32)
        ev["gpu"].append((g.counters() - c0)[cols])
        g.close()
    G, O = np.array(res["gpu"]), np.array(res["orc"])
    mid = slice(int(0.45 * d.ng), int(0.55 * d.ng) + 1)
    alpha = lambda a: a[:, 2, mid].sum(1) / a[:, 0, mid].sum(1)
    H.judge_ensembles(G, O, alpha(G), alpha(O), "sixteen channels, resolved O2(a), second cycle")
    eg, eo = np.array(ev["gpu"], float), np.array(ev["orc"], float)
    assert np.all(eo.sum(0) > 50), eo
    z, _ = H.welch_z(eg, eo)
    assert np.all(np.abs(z) <= 3.0), (z, eg.mean(0), eo.mean(0))
