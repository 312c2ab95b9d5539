"""Shared pieces of the GPU-vs-oracle tests."""
import math

import numpy as np
from scipy import stats

from oracle import pyoracle as po
from paper_0705_0497_amd import inputs as I

QE = 1.602176634e-19
POS_TOL = 1e-5          # cells
VEL_TOL = 1e-5          # relative to max(|v|, thermal speed of the species)


def thermal_speed(sp):
    return math.sqrt(max(sp.t0_ev, 0.026) * QE / sp.mass)


def canonical_from_oracle(d, procs, seed_steps=0, species=None):
    """Oracle-loaded state (after the leapfrog start), rounded to the FP32 record."""
    o = po.Oracle(d, species or d.species(), procs)
    o.load_uniform()
    o.prepare(True)
    if seed_steps:
        o.step(seed_steps)
    st = [o.canonical(s) for s in range(3)]
    nid = [o.next_id(s) for s in range(3)]
    return st, nid, o.step_index


def oracle_from_canonical(d, procs, st, nid, step, species=None, **kw):
    o = po.Oracle(d, species or d.species(), procs, **kw)
    for s in range(3):
        o.set_particles(s, st[s], nid[s])
    o.set_step(step)
    o.prepare(False)
    return o


def gpu_from_canonical(d, procs, st, nid, step, species=None, **kw):
    from paper_0705_0497_amd.binding import Discharge
    g = Discharge(d, procs, species=species, **kw)
    for s in range(3):
        g.set_particles(s, st[s], nid[s])
    g.set_step(step)
    g.prepare(False)
    return g


def by_id(st):
    o = np.argsort(st["id"], kind="stable")
    return {k: v[o] for k, v in st.items()}


def xi_of(st):
    if "xi" in st:
        return st["xi"]
    return st["cell"].astype(np.float64) + st["off"].astype(np.float64)


def band_ids(oracle_events):
    """(species, id) pairs whose decision fell within the 1e-6 band; an electron-ion
    test in the band (species 3) marks the electron (species 0) as well."""
    ev = oracle_events
    out = set(map(tuple, ev[ev[:, 4] != 0][:, [1, 2]].tolist()))
    return out | {(0, i) for s, i in out if s == 3}


def compare_events(gpu_ev, orc_ev):
    """Decisions of one step: identical outside the oracle's 1e-6 band."""
    band = band_ids(orc_ev)
    o = {(int(r[1]), int(r[2])): int(r[3]) for r in orc_ev if r[3] != -4}
    g = {(int(r[1]), int(r[2])): int(r[3]) for r in gpu_ev}
    bad = [(k, o.get(k), g.get(k)) for k in set(o) | set(g) if o.get(k) != g.get(k) and k not in band]
    return bad, band


def compare_states(gst, ost, sp, skip=frozenset(), s=0):
    """Positions (cells) and velocities of matching ids; returns worst errors."""
    g, o = by_id(gst), by_id(ost)
    gi, oi = g["id"].astype(np.int64), o["id"].astype(np.int64)
    keep_g = np.array([(s, int(i)) not in skip for i in gi], bool)
    keep_o = np.array([(s, int(i)) not in skip for i in oi], bool)
    g = {k: v[keep_g] for k, v in g.items()}
    o = {k: v[keep_o] for k, v in o.items()}
    assert np.array_equal(g["id"], o["id"]), "live id sets differ outside the band"
    dx = np.abs(xi_of(g) - xi_of(o))
    vth = thermal_speed(sp)
    worst_v = 0.0
    for k in ("vx", "vy", "vz"):
        ref = np.maximum(np.abs(o[k].astype(np.float64)), vth)
        worst_v = max(worst_v, float(np.max(np.abs(g[k].astype(np.float64) - o[k]) / ref, initial=0.0)))
    if s == 0:
        assert np.array_equal(g["cd"] & 0xFFFF, o["cd"] & 0xFFFF), "free-flight countdowns differ"
    return float(np.max(dx, initial=0.0)), worst_v


def neutralising(procs, factor=3e4):
    for p in procs:
        if p.kind == "neutralize":
            p.sigma = p.sigma * factor
    return procs


def welch_z(g, o):
    """Normal-equivalent z of the Welch t statistic of two samples (axis 0), and the
    mask of the entries with a variance."""
    M1, M2 = g.shape[0], o.shape[0]
    v1, v2 = g.var(0, ddof=1) / M1, o.var(0, ddof=1) / M2
    se2 = v1 + v2
    live = se2 > 0
    t = np.zeros_like(se2)
    t[live] = (g.mean(0)[live] - o.mean(0)[live]) / np.sqrt(se2[live])
    dof = np.full_like(se2, 1.0)
    dof[live] = se2[live] ** 2 / (v1[live] ** 2 / (M1 - 1) + v2[live] ** 2 / (M2 - 1))
    p = 2.0 * stats.t.sf(np.abs(t), dof)
    z = np.sign(t) * stats.norm.isf(p / 2.0)
    return z, live


def perm_quantile(G, O, q=0.999, nperm=2000, seed=0):
    """Quantile q of the mean z^2 over the nodes when the gpu / oracle labels are
    exchanged at random among all runs: the null distribution of the statistic for
    two samples of one distribution, with the correlation of the nodes included."""
    X = np.concatenate([G, O])
    M1 = G.shape[0]
    rng = np.random.Generator(np.random.PCG64(seed))
    vals = np.empty(nperm)
    for k in range(nperm):
        idx = rng.permutation(X.shape[0])
        z, live = welch_z(X[idx[:M1]], X[idx[M1:]])
        vals[k] = np.mean(z[live] ** 2)
    return float(np.quantile(vals, q))


def judge_ensembles(G, O, ag, ao, what):
    """Cycle averages of M runs per side, G and O [M][...], and their central
    electronegativities ag, ao [M]: at most 1 % of the entries beyond |z| = 3, the
    mean z^2 below the 99.9 % quantile of its relabelling distribution, alpha
    within 3."""
    G2, O2 = G.reshape(G.shape[0], -1), O.reshape(O.shape[0], -1)
    z, live = welch_z(G2, O2)
    # a node that is empty on every run of both sides (no variance) must agree exactly
    dead = ~live
    np.testing.assert_array_equal(G2.mean(0)[dead], O2.mean(0)[dead])
    zl = z[live]
    K = zl.size
    beyond = float(np.mean(np.abs(zl) > 3.0))
    mz2 = float(np.mean(zl ** 2))
    # the chi^2 99.9 % bound holds for independent nodes; the profiles fluctuate
    # coherently (neighbouring nodes and species move together), so the bound is the
    # 99.9 % quantile of the same statistic under random relabelling of the runs
    chi2 = stats.chi2.ppf(0.999, K) / K
    bound = perm_quantile(G2, O2)
    za, _ = welch_z(ag[:, None], ao[:, None])
    msg = (f"{what}: {K} nodes, {beyond:.4f} beyond 3, mean z^2 {mz2:.3f} (99.9 % under relabelling "
           f"{bound:.3f}; chi^2 of independent nodes {chi2:.3f}), alpha z {za[0]:.2f}")
    print(msg)
    assert beyond <= 0.01, msg
    assert mz2 <= bound, msg
    assert abs(za[0]) <= 3.0, msg
