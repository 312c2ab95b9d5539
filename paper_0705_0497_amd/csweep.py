"""Associative detachment sweep: the discharge of section 3 (Figs. 3-5: L = 2.5 cm,
f = 13.6 MHz, p = 13.8 Pa, U = 250 V) at C = n(O2(a)) / n(O2) = 0, 0.1 and 1/6,
run as one batch to the periodic steady state.

The paper's cross sections are not available, so this is a qualitative analogue
of Figs. 3-5, not a reproduction: the seeded synthetic tables of inputs.py, with
ion-ion neutralisation from the two-channel Landau-Zener model (section 2) at a
crossing radius R_x chosen here (the paper fits R_x to measured high-energy
cross sections that are not given), and Eq. (1) for associative detachment.
Reported per C: cycle-averaged density profiles of e, O- and O2+, their values
at the centre of the gap, the electronegativity n(O-) / n(e) there, the rf-phase
resolved current density at the driven electrode and the mean power <U j>.

Everything here is orchestration: the discharges advance in the HIP kernels.
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import sys
import time

import numpy as np

from . import binding as B
from . import inputs as I
from . import warmstart as W

C_VALUES = (0.0, 0.1, 1.0 / 6.0)
R_X_BOHR = 5.3      # 4 pi R_x^2 = 1.0e-18 m^2 (1e-14 cm^2) at high energies


def fig34_discharge(c_meta, seed, n_total=120000, ng=128):
    """The section 3 discharge in the 128-cell form of the warm-start family
    (400 steps per rf cycle, ions every 10 steps)."""
    d = I.config(1, L=0.025, ng=ng, U=250.0, f=13.6e6, p=13.8, c_meta=float(c_meta), seed=int(seed),
                 n_total=int(n_total), diag_every=20, sort_every=20)
    c = d.species_counts()
    return dataclasses.replace(d, name=f"fig34-C{c_meta:.3f}",
                               capacities=(60 * c[0] + 4096, 60 * c[1] + 4096, 8 * c[2] + 4096))


def processes(r_x=R_X_BOHR):
    """The eight workload channels with Landau-Zener neutralisation."""
    procs = I.make_processes()
    out = []
    for p in procs:
        if p.kind == "neutralize":
            p = dataclasses.replace(p, sigma=I.landau_zener_table(r_x), params=dict(model="landau-zener", r_x=r_x))
        out.append(p)
    return out


def C_EVENT_AD(procs):
    """Counter index of the associative-detachment events (Eq. (1), target O2(a))."""
    return B.C_EVENT + [p.target for p in procs].index("O2a")


def run(c_values=C_VALUES, n_total=120000, max_cycles=3000, avg_cycles=100, seed0=7000, log=None):
    import torch
    stream = torch.cuda.Stream()
    procs = processes()
    members = []
    for j, c in enumerate(c_values):
        g = B.Discharge(fig34_discharge(c, seed0 + j, n_total), procs, stream=stream, max_products=1 << 16)
        g.load_uniform()
        members.append(g)
    t0 = time.perf_counter()
    conv, _, cycles = W.run_batch(members, max_cycles, log=log)
    # profiles and currents averaged over avg_cycles more cycles at the steady state
    batch = B.Batch(members, block=512, sort_every=20, use_graph=True)
    c_start = []
    for g in members:
        g.moments(reset=True)
        c_start.append(g.counters())
    batch.step_cycles(avg_cycles)
    batch.sync()
    batch.close()
    out = {"c_values": list(c_values), "converged_at": conv, "cycles_to_steady": cycles,
           "avg_cycles": avg_cycles, "r_x_bohr": R_X_BOHR, "n_total": n_total, "members": []}
    i_ad = C_EVENT_AD(procs)
    for c, g, c0 in zip(c_values, members, c_start):
        m = g.moments(reset=True)
        dwin = g.counters() - c0
        dens, mean = W.cycle_profiles(g, m)
        k = len(W.XS) // 2
        cur = m["current"] / np.maximum(m["current_n"], 1)
        cnt = g.counters()
        out["members"].append({
            "C": c,
            "centre_density_m3": {"e": float(dens[0, k]), "O-": float(dens[2, k]), "O2+": float(dens[1, k])},
            "electronegativity_centre": float(dens[2, k] / max(dens[0, k], 1.0)),
            "profiles_x": W.XS[::16].tolist(),
            "profiles_m3": {"e": dens[0, ::16].tolist(), "O-": dens[2, ::16].tolist(), "O2+": dens[1, ::16].tolist()},
            "mean_energy_centre_ev": {"e": float(mean[0, k]), "O-": float(mean[2, k]), "O2+": float(mean[1, k])},
            "current_a_m2": cur.tolist(),
            "power_w_m2": float(m["power_sum"] / max(m["power_n"], 1)),
            "ad_events": int(cnt[i_ad]),
            "ad_events_window": int(dwin[i_ad]),
            "o_minus_pushes_window": int(dwin[B.C_PUSH + 2]),
            "counts": [g.count(s) for s in range(3)],
        })
    out["gpu_seconds"] = time.perf_counter() - t0
    ref = np.asarray(out["members"][0]["current_a_m2"])
    for mem in out["members"]:
        j = np.asarray(mem["current_a_m2"])
        mem["current_rms_diff_vs_C0"] = float(np.sqrt(np.mean((j - ref) ** 2)) / max(np.sqrt(np.mean(ref ** 2)), 1e-30))
    return out


# O2(a1Delta_g) transport (order-of-magnitude values, not from the paper): diffusion
# from O2 self-diffusion, 0.2 cm^2/s at 1 atm (D p = 2.0 m^2 Pa / s); quenching by
# O2 at 1.5e-24 m^3/s; loss probability 5e-3 per collision with an electrode
DP_O2A = 2.0
K_QUENCH = 1.5e-24
GAMMA_O2A = 5e-3


def processes_with_a1(r_x=R_X_BOHR):
    """processes() plus O2(a1Delta_g) excitation (Table 1 (14)) as the last electron
    channel; returns the list and that channel's index."""
    procs = processes(r_x)
    a1 = next(p for p in I.make_processes_full() if p.name == "e-a1")
    k = max(i for i, p in enumerate(procs) if p.species == 0) + 1
    procs.insert(k, a1)
    return procs, k


def resolved(n_total=120000, c0=1.0 / 6.0, window=100, min_updates=20, max_updates=60, tol=0.01, seed0=7100,
             log=None):
    """The section 3 discharge with the O2(a) density solved from its own production
    (updated every window cycles), beside the same discharge with the uniform
    n = c0 n(O2); both start from c0 and run as one batch until, after at least
    min_updates, the profile changes by less than tol between updates and the
    electron density of both members passes the convergence test."""
    import torch
    stream = torch.cuda.Stream()
    procs, ka1 = processes_with_a1()
    members = []
    for j in range(2):
        g = B.Discharge(fig34_discharge(c0, seed0 + j, n_total), procs, stream=stream, max_products=1 << 16)
        g.load_uniform()
        members.append(g)
    d = members[0].d
    n_o2 = d.p / (1.380649e-23 * d.t_gas)
    res_g = members[1]
    res_g.metastable_config(ka1, DP_O2A / d.p, K_QUENCH * n_o2, GAMMA_O2A)
    t0 = time.perf_counter()
    batch = B.Batch(members, block=512, sort_every=20, use_graph=True)
    history, n_a, prev = [], None, None
    mons = [W.Monitor() for _ in members]
    for g in members:
        g.moments(reset=True)
    for u in range(max_updates):
        for w in range(window // W.WINDOW):
            batch.step_cycles(W.WINDOW)
            batch.sync()
            for mon, g in zip(mons, members):
                mon.add(g.moments(reset=True)["sum_q"][0], u * window + (w + 1) * W.WINDOW)
        n_a = res_g.metastable_update()
        change = float(np.abs(n_a - prev).sum() / np.abs(n_a).sum()) if prev is not None else 1.0
        history.append({"cycle": (u + 1) * window, "n_a_centre": float(n_a[d.ng // 2]),
                        "n_a_edge": float(n_a[0]), "change": change})
        if log:
            log(f"update {u + 1}: n(O2a) centre {n_a[d.ng // 2]:.3e}, edge {n_a[0]:.3e}, change {change:.4f}")
        # the plasma follows the new profile: stop once both hold still
        steady = all(len(m.passed) >= 2 and m.passed[-1] and m.passed[-2] for m in mons)
        if u + 1 >= min_updates and change < tol and steady:
            break
        prev = n_a
    for g in members:
        g.moments(reset=True)
    batch.step_cycles(window)
    batch.sync()
    batch.close()
    out = {"c0": c0, "window": window, "updates": len(history), "history": history,
           "transport": {"D_m2_s": DP_O2A / d.p, "quench_rate_s": K_QUENCH * n_o2, "gamma": GAMMA_O2A},
           "n_o2": n_o2, "n_a": n_a.tolist(), "members": []}
    for name, g in (("uniform", members[0]), ("resolved", members[1])):
        m = g.moments(reset=True)
        dens, mean = W.cycle_profiles(g, m)
        k = len(W.XS) // 2
        ne = dens[0]
        above = W.XS[ne >= 0.5 * ne.max()]
        out["members"].append({
            "name": name,
            "centre_density_m3": {"e": float(dens[0, k]), "O-": float(dens[2, k]), "O2+": float(dens[1, k])},
            "electronegativity_centre": float(dens[2, k] / max(dens[0, k], 1.0)),
            "fwhm_ne_over_L": float(above.max() - above.min()) if len(above) else 0.0,
            "profiles_x": W.XS[::16].tolist(),
            "profiles_m3": {"e": dens[0, ::16].tolist(), "O-": dens[2, ::16].tolist(), "O2+": dens[1, ::16].tolist()},
        })
    out["gpu_seconds"] = time.perf_counter() - t0
    return out


def markdown(res):
    lines = ["| C | converged at cycle | n_e centre [m^-3] | n_O- centre | n_O2+ centre | n_O- / n_e | "
             "power <U j> [W/m^2] | current rms diff vs C = 0 |",
             "|---|---|---|---|---|---|---|---|"]
    for mem, cv in zip(res["members"], res["converged_at"]):
        d = mem["centre_density_m3"]
        lines.append(f"| {mem['C']:.3f} | {cv} | {d['e']:.3e} | {d['O-']:.3e} | {d['O2+']:.3e} | "
                     f"{mem['electronegativity_centre']:.2f} | {mem['power_w_m2']:.3g} | "
                     f"{mem['current_rms_diff_vs_C0']:.3f} |")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", default=None, help="write the results as JSON here")
    ap.add_argument("--n-total", type=int, default=120000)
    ap.add_argument("--max-cycles", type=int, default=3000)
    ap.add_argument("--avg-cycles", type=int, default=100)
    ap.add_argument("--resolved", action="store_true",
                    help="O2(a) solved from its own production instead of the C sweep")
    args = ap.parse_args(argv)
    log = lambda s: print(s, file=sys.stderr, flush=True)
    if args.resolved:
        res = resolved(n_total=args.n_total, log=log)
        text = "\n".join(f"| {m['name']} | {m['centre_density_m3']['e']:.3e} | {m['centre_density_m3']['O-']:.3e} | "
                         f"{m['centre_density_m3']['O2+']:.3e} | {m['electronegativity_centre']:.3f} | "
                         f"{m['fwhm_ne_over_L']:.3f} |" for m in res["members"])
        text = ("| O2(a) | n_e centre | n_O- centre | n_O2+ centre | n_O- / n_e | FWHM of n_e / L |\n"
                "|---|---|---|---|---|---|\n" + text)
    else:
        res = run(n_total=args.n_total, max_cycles=args.max_cycles, avg_cycles=args.avg_cycles, log=log)
        text = markdown(res)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(res, f)
    print(text, flush=True)


if __name__ == "__main__":
    main()
