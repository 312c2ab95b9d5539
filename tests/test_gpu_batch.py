"""Batched discharges: one launch per kernel per step over many members, one
HIP graph per rf cycle, and the autotuner.  A member advanced in a batch must
reach exactly the state of the same discharge advanced alone (same random
streams; launch shapes and re-ordering change the storage order only), so
everything is compared bit for bit, matched by particle id."""
import numpy as np
import pytest

from paper_0705_0497_amd import inputs as I
from tests import helpers as H

pytestmark = pytest.mark.gpu

SPC = 40


def _members(spec, **over):
    """Small sweep members: (index, ksub, superparticles) with 40 steps per cycle."""
    return [I.sweep_member(j, steps_per_cycle=SPC, ksub=k, n_total=n, diag_every=10, sort_every=20, **over)
            for j, k, n in spec]


def _snapshot(g):
    parts = [H.by_id(g.get_particles(s)[0]) for s in range(3)]
    m = g.moments()
    return {"parts": parts, "hist": g.hist(), "counters": g.counters(), "moments": m, "step": g.step_index}


def _same(a, b, who):
    assert a["step"] == b["step"], who
    for s in range(3):
        assert len(a["parts"][s]["id"]) == len(b["parts"][s]["id"]), (who, s)
        for k in ("cell", "off", "vx", "vy", "vz", "id", "cd"):
            np.testing.assert_array_equal(a["parts"][s][k], b["parts"][s][k], err_msg=f"{who} species {s} {k}")
    np.testing.assert_array_equal(a["hist"], b["hist"], err_msg=who)
    np.testing.assert_array_equal(a["counters"], b["counters"], err_msg=who)
    for k in ("sum_q", "sum_phi", "esum", "ecnt", "edf", "iedf", "nacc", "ndiag", "current", "current_n",
              "power_sum", "power_n"):
        np.testing.assert_array_equal(a["moments"][k], b["moments"][k], err_msg=f"{who} {k}")


def _alone(ds, procs, stream, steps):
    from paper_0705_0497_amd.binding import Discharge
    out = []
    for d in ds:
        g = Discharge(d, procs, stream=stream)
        g.load_uniform()
        g.step(steps)
        out.append(_snapshot(g))
        g.close()
    return out


def _loaded(ds, procs, stream):
    from paper_0705_0497_amd.binding import Discharge
    mem = [Discharge(d, procs, stream=stream) for d in ds]
    for g in mem:
        g.load_uniform()
    return mem


SPEC = [(0, 2, 6000), (1, 4, 15000), (2, 5, 3000), (3, 8, 9000), (4, 10, 4000)]


def test_batch_member_equals_discharge_alone_graph_replays():
    import torch
    from paper_0705_0497_amd.binding import Batch
    stream = torch.cuda.Stream()
    ds = _members(SPEC)
    procs = H.neutralising(I.make_processes())
    ref1 = _alone(ds, procs, stream, SPC)
    ref3 = _alone(ds, procs, stream, 3 * SPC)
    mem = _loaded(ds, procs, stream)
    b = Batch(mem, block=256, sort_every=10, use_graph=True)
    print("batch: 5 members, graph, cycle 1", flush=True)
    b.step_cycles(1)
    b.sync()
    for m, g in enumerate(mem):
        _same(_snapshot(g), ref1[m], f"member {m} after 1 cycle")
    print("batch: cycles 2-3 (two more replays after eager work)", flush=True)
    b.step_cycles(2)
    b.sync()
    for m, g in enumerate(mem):
        _same(_snapshot(g), ref3[m], f"member {m} after 3 cycles")
    b.close()


def test_batch_direct_launches_and_launch_shapes():
    import torch
    from paper_0705_0497_amd.binding import Batch
    stream = torch.cuda.Stream()
    ds = _members(SPEC[:3])
    procs = H.neutralising(I.make_processes())
    ref = _alone(ds, procs, stream, 2 * SPC)
    for kw in ({"block": 1024, "sort_every": 0, "use_graph": False},
               {"block": 512, "sort_every": 20, "use_graph": False, "grid": 3},
               {"block": 256, "sort_every": 40, "use_graph": True, "grid": 1},
               # more blocks than tiles: the balanced electron cuts give every block one tile,
               # and compaction every 10 steps changes the tile count between launches
               {"block": 256, "sort_every": 10, "use_graph": True, "grid": 2048}):
        print("batch shapes", kw, flush=True)
        mem = _loaded(ds, procs, stream)
        b = Batch(mem, **kw)
        b.step_cycles(2)
        b.sync()
        for m, g in enumerate(mem):
            _same(_snapshot(g), ref[m], f"member {m} {kw}")
        b.close()
        for g in mem:
            g.close()


def test_autotuner_picks_a_candidate_and_keeps_results():
    import torch
    from paper_0705_0497_amd.binding import Batch
    stream = torch.cuda.Stream()
    ds = _members(SPEC[:2])
    procs = I.make_processes()
    mem = _loaded(ds, procs, stream)
    b = Batch(mem, block=512, sort_every=20, use_graph=True)
    print("autotune window 20", flush=True)
    t = b.autotune(window=20)
    b.step_cycles(1)
    b.sync()
    trials = t["trials"]
    assert len(trials) == 6                                  # 3 blocks x sort_every in {10, 20}
    assert {(x["block"], x["sort_every"]) for x in trials} == {(bs, s) for bs in (256, 512, 1024) for s in (10, 20)}
    assert all(x["ms_per_step"] > 0 for x in trials)
    best = min(trials, key=lambda x: x["ms_per_step"])
    cfg = b.config()
    assert (cfg["block"], cfg["sort_every"]) == (best["block"], best["sort_every"])
    steps = mem[0].step_index
    assert steps % SPC == 0 and steps == 6 * 20 + SPC
    ref = _alone(ds, procs, stream, steps)
    for m, g in enumerate(mem):
        _same(_snapshot(g), ref[m], f"member {m} after autotune")
    b.close()


def test_batch_validation_and_busy_members():
    import torch
    from paper_0705_0497_amd import binding as B
    stream = torch.cuda.Stream()
    procs = I.make_processes()
    ds = _members(SPEC[:2])
    mem = _loaded(ds, procs, stream)
    other = B.Discharge(ds[0], procs, stream=torch.cuda.Stream())
    with pytest.raises(B.PicError) as e:
        B.Batch([mem[0], other])
    assert e.value.code == B.PIC_EINVAL                      # members on different streams
    bad = B.Discharge(_members([(5, 3, 2000)])[0], procs, stream=stream)   # ksub 3 does not divide 40
    with pytest.raises(B.PicError):
        B.Batch([mem[0], bad])
    with pytest.raises(B.PicError):
        B.Batch([mem[0], mem[0]])
    with pytest.raises(B.PicError):
        B.Batch(mem, sort_every=7)                           # does not divide the cycle
    b = B.Batch(mem, sort_every=20)
    b.step_cycles(1)
    with pytest.raises(B.PicError) as e:
        mem[0].get_particles(0)
    assert e.value.code == B.PIC_EBUSY
    b.sync()
    assert mem[0].step_index == SPC
    mem[0].step(1)                                           # off the cycle boundary
    with pytest.raises(B.PicError):
        b.step_cycles(1)
    b.close()


def _full_channels():
    # all sixteen channels, the electron-ion ones with sigma ~ E^-1/2 large enough to act in a few
    # cycles; index of the O2(a) production channel
    procs = I.make_processes_full()
    for k, p in enumerate(procs):
        if p.kind in ("recomb", "edetach"):
            procs[k] = I.Process(p.name, 0, p.kind, p.target, p.e_th, p.target_mass,
                                 I.power_law_table(3e-15, 0.0, 0.5, p.e_th), {})
    return procs, [p.name for p in procs].index("e-a1")


def test_batch_with_all_channels_and_resolved_o2a_equals_alone():
    """Members with the electron-ion channels and the O2(a) profile (updated after the first
    cycle on both sides) reach bit for bit the states of the same discharges run alone."""
    import torch
    from paper_0705_0497_amd.binding import Batch, Discharge
    stream = torch.cuda.Stream()
    ds = _members(SPEC[:3])
    procs, ka1 = _full_channels()
    meta = (ka1, 0.1, 20.0, 0.05)
    ref = []
    for d in ds:
        g = Discharge(d, procs, stream=stream)
        g.load_uniform()
        g.metastable_config(*meta)
        g.step(SPC)
        n_a = g.metastable_update()
        g.step(SPC)
        ref.append((_snapshot(g), n_a))
        g.close()
    mem = _loaded(ds, procs, stream)
    for g in mem:
        g.metastable_config(*meta)
    b = Batch(mem, block=256, sort_every=10, use_graph=True)
    b.step_cycles(1)
    b.sync()
    for m, g in enumerate(mem):
        np.testing.assert_array_equal(g.metastable_update(), ref[m][1], err_msg=f"member {m} O2(a)")
    b.step_cycles(1)
    b.sync()
    for m, g in enumerate(mem):
        snap = _snapshot(g)
        _same(snap, ref[m][0], f"member {m}")
        names = [p.name for p in procs]
        c = snap["counters"]
        assert c[18 + names.index("e-recomb")] + c[18 + names.index("e-edet")] > 0, m
    b.close()


def test_batch_members_of_mixed_sizes_match_the_oracle():
    """One batched rf cycle against the FP64 oracle, element by element: three members
    of different cells, sizes, voltages and pressures on a four-step cycle (the time
    step of the 128-cell workload, ions every second step, neutralisation boosted so
    that pairing acts), each set from an oracle state.  Decisions identical outside
    the 1e-6 band, positions and velocities to 1e-5, charge the exact deposit."""
    import dataclasses
    import torch
    from oracle import pyoracle as po
    from paper_0705_0497_amd.binding import Batch
    stream = torch.cuda.Stream()
    procs = H.neutralising(I.make_processes())
    base = I.config(1)
    spc = 4
    f = base.f * base.steps_per_cycle / spc                   # the same dt as the 128-cell workload
    ds = [dataclasses.replace(base, ng=ng, U=U, p=p, n_total=n, seed=8800 + j, f=f, steps_per_cycle=spc,
                              ksub=2, diag_every=0, sort_every=0, capacity_factor=8.0)
          for j, (ng, U, p, n) in enumerate([(64, 150.0, 10.0, 6000), (128, 250.0, 20.0, 30000),
                                              (256, 350.0, 40.0, 60000)])]
    mem, orc, nid0, paired = [], [], [], 0
    for d in ds:
        st, nid, step = H.canonical_from_oracle(d, procs, seed_steps=8)
        assert step % spc == 0
        orc.append(H.oracle_from_canonical(d, procs, st, nid, step))
        mem.append(H.gpu_from_canonical(d, procs, st, nid, step, event_capacity=1 << 20, stream=stream))
        nid0.append(nid)
    b = Batch(mem, block=256, sort_every=2, use_graph=True)
    for o in orc:
        o.log_events(True)
        o.step(spc)
    b.step_cycles(1)
    b.sync()
    for m, (g, o, d) in enumerate(zip(mem, orc, ds)):
        gev, oev = g.events(), o.events()
        band = H.band_ids(oev)
        key_o = {(int(r[0]), int(r[1]), int(r[2])): int(r[3]) for r in oev if r[3] not in (-4, -5)}
        key_g = {(int(r[0]), int(r[1]), int(r[2])): int(r[3]) for r in gev}
        pre = lambda k: k[2] < nid0[m][k[1] if k[1] < 3 else 0]
        # without a decision in the band every particle, products included, must agree
        keep = (lambda k: (k[1], k[2]) not in band) if not band else (lambda k: (k[1], k[2]) not in band and pre(k))
        bad = [(k, key_o.get(k), key_g.get(k)) for k in set(key_o) | set(key_g) if keep(k) and key_o.get(k) != key_g.get(k)]
        assert not bad, (m, bad[:10])
        assert len(key_g) > 100 and len(band) <= 3, (m, len(key_g), len(band))
        for s in range(3):
            gs, nid_g = g.get_particles(s)
            os_ = o.get_particles(s)
            if band:
                gs = {k: v[gs["id"] < nid0[m][s]] for k, v in gs.items()}
                os_ = {k: v[os_["id"] < nid0[m][s]] for k, v in os_.items()}
            else:
                assert nid_g == o.next_id(s)
            dx, dv = H.compare_states(gs, os_, d.species()[s], skip=band, s=s)
            assert dx <= H.POS_TOL and dv <= H.VEL_TOL, (m, s, dx, dv)
            full, _ = g.get_particles(s)
            np.testing.assert_array_equal(g.hist()[s], po.deposit_canonical(d.ng, full["cell"], full["off"]))
        gc, oc = g.counters(), o.counters()
        if not band:
            np.testing.assert_array_equal(gc[po.C_PUSH:po.C_CLAMP], oc[po.C_PUSH:po.C_CLAMP])
        paired += int(oc[po.C_PAIRED])
    assert paired > 0
    b.close()
