"""Throughput of the 1D3V oxygen PIC-MCC step on one MI355X.

Workload: the large single discharge (4096 cells, L = 4 cm, U = 500 V,
p = 100 Pa, 8e6 e + 2.4e7 O2+ + 1.6e7 O- loaded, 2000 steps per rf cycle, ions
every 20 steps).  One bench "step" is one rf cycle: 2000 electron steps with 100
ion steps, field solves, MCC, deposits, products, store re-ordering and moments.  Inputs (seeded synthetic tables, uniform loading) are resident on the
GPU before the timed region starts.

Prints one JSON line.  Roofline of the dominant kernel (electron
push+MCC+deposit): algorithmic bytes per launch / mean launch duration from
HIP events on the handle's stream.  cpu_baseline: the FP64 oracle on a bounded
sample of the same workload on the host cores (one process per core, each on
1/16 of the particles for 120 steps), timed before the GPU is initialised.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

BYTES_PUSH = 24          # read + write the position (cell word, offset) and vx
BYTES_CAND = 20          # at a collision candidate (a free-flight end): read id, read + write vy, vz
HBM_PEAK_GBS = 8000.0    # MI355X HBM3E


def push_alg_bytes(dc, procs=None):
    """Algorithmic HBM bytes of the electron push over a counter difference dc:
    24 B per push and 20 B per collision candidate, the per-unit figures of the
    streaming sweep this MCC has to make (the amortised re-ordering bytes belong
    to the sort kernels, not to this one)."""
    from paper_0705_0497_amd import binding as B
    return BYTES_PUSH * int(dc[B.C_PUSH]) + BYTES_CAND * int(dc[B.C_CAND])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "push_electron_cfg3_pmc.md")
KERNEL_SOURCE = os.path.join(ROOT, "paper_0705_0497_amd", "csrc", "kernels.hip")


def measured_traffic(particles_per_launch):
    """HBM bytes per electron-push launch from the committed rocprofv3 --pmc
    summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain 1 GiB copy), scaled
    to this run's particles per launch; None when the kernel source changed since."""
    try:
        text = open(TRAFFIC_SUMMARY).read()
    except OSError:
        return None
    src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()[:16]
    m_hash = re.search(r"kernels\.hip sha256\[:16\]:\s*([0-9a-f]{16})", text)
    m_bpp = re.search(r"HBM bytes per electron push:\s*([0-9.]+)", text)
    if not m_hash or not m_bpp or m_hash.group(1) != src:
        return None
    return float(m_bpp.group(1)) * particles_per_launch


def _native_oracle():
    """The oracle's C source built for this host (-O3 -march=native, no FMA
    contraction, no fast-math: IEEE arithmetic in the source's order) into a
    temporary directory; returns the library path."""
    import subprocess
    import tempfile
    from oracle import pyoracle as po
    out = os.path.join(tempfile.mkdtemp(prefix="oracle_native_"), "liboracle_native.so")
    subprocess.check_call(["gcc", "-O3", "-march=native", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                           *po.SOURCES, "-o", out, "-lm"])
    return out


def _oracle_worker(lib_path, frac, seed, steps, barrier, results):
    """One oracle on 1/frac of the superparticles of the large discharge: load,
    then time `steps` steps after every worker is ready."""
    import dataclasses
    from oracle import pyoracle as po
    from paper_0705_0497_amd import inputs as I
    po.LIB_PATH = lib_path
    d = I.config(3, seed=seed)
    d = dataclasses.replace(d, counts=tuple(c // frac for c in d.species_counts()))
    o = po.Oracle(d, d.species(), I.make_processes())
    o.load_uniform()
    o.prepare(True)
    c0 = o.counters()
    if barrier is not None:
        barrier.wait()
    t0 = time.time()
    o.step(steps)
    t1 = time.time()
    results.put((int((o.counters() - c0)[0:3].sum()), t0, t1))


def cpu_baseline(steps=120):
    """The FP64 oracle as it stands on the host: one thread on 1/16 of the
    superparticles of the large discharge, then one independent oracle per
    core, each on its own 1/16 (another seed), started together.  value = the
    all-core aggregate (pushes / wall time of the common window)."""
    import multiprocessing as mp
    lib_path = _native_oracle()
    ctx = mp.get_context("spawn")
    cores = min(len(os.sched_getaffinity(0)), 16)      # the host share of one GPU
    frac = 16

    def run(n):
        q = ctx.Queue()
        bar = ctx.Barrier(n) if n > 1 else None
        ps = [ctx.Process(target=_oracle_worker, args=(lib_path, frac, 3001 + k, steps, bar, q)) for k in range(n)]
        for p in ps:
            p.start()
        res = [q.get() for _ in ps]
        for p in ps:
            p.join()
        pushes = sum(r[0] for r in res)
        wall = max(r[2] for r in res) - min(r[1] for r in res)
        return pushes, wall

    p1, w1 = run(1)
    pn, wn = run(cores)
    return {"value": pn / wn, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{cores} independent FP64 oracles at once, each the large discharge with 1/{frac} of its "
                      f"superparticles (3e6, own seed), {steps} steps incl. {steps // 20} ion steps: {pn} pushes "
                      f"in {wn:.1f} s; built -O3 -march=native -ffp-contract=off",
            "single_thread": {"value": p1 / w1, "pushes": p1, "seconds": w1}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50, help="timed rf cycles")
    ap.add_argument("--warmup", type=int, default=5, help="untimed rf cycles")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--block", type=int, default=1024,
                    help="push block size (1024: one block per CU, half the partial histograms of 512)")
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--sort", choices=("compact", "cell"), default="compact",
                    help="periodic re-ordering: order-preserving compaction or counting sort by cell")
    ap.add_argument("--sort-every", type=int, default=2000)
    ap.add_argument("--workload", choices=("single", "sweep", "warmstart", "working", "mlp"), default="single",
                    help="single: the 4096-cell discharge; sweep: 64 discharges advanced as one batch; "
                         "warmstart: learned warm start against cold starts; working: the 512-cell "
                         "discharge, host-enqueued steps against the cycle graph; mlp: the network kernels alone")
    ap.add_argument("--train-runs", type=int, default=256, help="warmstart: training discharges")
    ap.add_argument("--test-runs", type=int, default=16, help="warmstart: held-out discharges")
    ap.add_argument("--members", type=int, default=64, help="sweep: discharges in the batch")
    ap.add_argument("--tune-window", type=int, default=200, help="sweep: autotuner trial length [steps]")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: one discharge runs on one GPU; --gpus {args.gpus} is not supported "
              "(the decomposition over several GPUs is designed, not implemented)", file=sys.stderr)
        sys.exit(2)

    base = None
    if args.workload == "single" and not args.no_cpu_baseline:
        # on the host cores before the GPU is touched (the workers are fresh interpreters)
        log("bench: timing the FP64 oracle on the host cores (bounded sample)")
        base = cpu_baseline()
        log(f"bench: oracle {base['value']:.3e} particle-steps/s on {base['cores']} cores")

    import torch
    from paper_0705_0497_amd import inputs as I
    from paper_0705_0497_amd.binding import Discharge, C_PUSH, C_CAND, C_REDRAW, C_EVENT, C_PAIRED, C_DEFICIT

    torch.cuda.set_device(0)
    if args.workload == "sweep":
        return sweep(args)
    if args.workload == "working":
        return working(args)
    if args.workload == "mlp":
        return mlp(args)
    if args.workload == "warmstart":
        return warmstart(args)
    d = I.config(3)
    procs = I.make_processes()
    log(f"bench: loading {d.name} ({sum(d.species_counts())} superparticles, {d.ng} cells)")
    g = Discharge(d, procs, block=args.block, grid=args.grid, sort_every=args.sort_every,
                  sort_kind=1 if args.sort == "compact" else 0)
    g.load_uniform()
    g.sync()
    spc = d.steps_per_cycle
    for c in range(args.warmup):
        g.step(spc)
        g.sync()
        log(f"bench: warmup cycle {c + 1}/{args.warmup} done")
    c0 = g.counters()
    n_start = sum(g.count(s) for s in range(3))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_push = 0.0
    for c in range(args.steps):
        mp, mt, _ = g.step_timed(spc)
        ms_push += mp
        if (c + 1) % 10 == 0 or c + 1 == args.steps:
            log(f"bench: timed cycle {c + 1}/{args.steps}")
    g.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    c1 = g.counters()
    dc, dc_all = c1 - c0, c1
    pushes = int(dc[C_PUSH:C_PUSH + 3].sum())
    value = pushes / elapsed
    launches = args.steps * spc
    alg_bytes = push_alg_bytes(dc, procs)
    per_launch = alg_bytes / launches
    mean_ms = ms_push / launches
    achieved = per_launch / (mean_ms * 1e-3) / 1e9
    counts = [g.count(s) for s in range(3)]
    traffic = measured_traffic(int(dc[C_PUSH]) / launches)
    # every superparticle counted at every electron step (ions included although they move every k_sub)
    physical = 0.5 * (n_start + sum(counts)) * launches / elapsed
    out = {
        "metric": "particle-steps/s (push+deposit+MCC); rf cycles to steady state, warm vs cold",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "4096-cell O2 CCP, L=4 cm, U=500 V, p=100 Pa, 8e6 e + 2.4e7 O2+ + 1.6e7 O-",
                   "step": "one rf cycle = 2000 electron steps, ions every 20",
                   "reorder": f"{args.sort} every {args.sort_every} steps",
                   "cells": d.ng, "superparticles_loaded": int(sum(d.species_counts())),
                   "superparticles_end": counts, "electron_pushes": int(dc[C_PUSH]),
                   "ion_pushes": int(dc[C_PUSH + 1] + dc[C_PUSH + 2]),
                   "electron_candidates": int(dc[C_CAND]),
                   # Table 1 (17): every neutralisation removes one O2+ of its cell; a deficit
                   # would be an event that found none (counted over the whole run)
                   "neutralisations": int(sum(dc_all[C_EVENT + i] for i, p in enumerate(procs)
                                              if p.kind == "neutralize")),
                   "o2plus_partners_removed": int(dc_all[C_PAIRED]), "partner_deficit": int(dc_all[C_DEFICIT]),
                   "parallelism": "single GPU"},
        "pushes_per_step": pushes / launches,
        "physical_particle_steps_per_s": physical,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_source": ("not counted in this run: HBM bytes per push from the committed "
                                        "rocprofv3 --pmc FETCH_SIZE/WRITE_SIZE summary "
                                        "(profiles/push_electron_cfg3_pmc.md, copy-calibrated) times this "
                                        "run's pushes per launch; null when the kernel source differs"),
                     "kernel": f"k_push<{args.block or 512},0> electron push+MCC+deposit",
                     "bytes_per_launch": per_launch, "mean_launch_ms": mean_ms},
    }
    if base is not None:
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)


def sweep(args):
    """64 discharges (U ~ U[100, 600] V, p ~ logU[5, 100] Pa, 256..1024 cells,
    5e4..2e6 superparticles per species) advanced as one batch: one launch per
    kernel per step, one HIP graph per rf cycle; ion subcycling per member from
    the physics-valid rule, block size and re-ordering interval from the
    autotuner.  One bench step = one rf cycle of the whole batch."""
    import torch
    from paper_0705_0497_amd import inputs as I
    from paper_0705_0497_amd import binding as B

    procs = I.make_processes()
    stream = torch.cuda.Stream()
    members, ksubs = [], []
    for j in range(args.members):
        d = I.sweep_member(j, diag_every=100)
        k = B.pic_ksub_select(B.make_config(d), B.make_species(d.species()), 3.0 * d.n_plus0, d.U)
        d = I.sweep_member(j, diag_every=100, ksub=k)
        g = B.Discharge(d, procs, stream=stream)
        g.load_uniform()
        members.append(g)
        ksubs.append(k)
    loaded = sum(sum(g.d.species_counts()) for g in members)
    log(f"bench: sweep of {len(members)} discharges, {loaded} superparticles, ksub {sorted(set(ksubs))}")
    b = B.Batch(members, block=512, sort_every=100, use_graph=True)
    t0 = time.perf_counter()
    tune = b.autotune(window=args.tune_window)
    b.sync()
    log(f"bench: autotune {time.perf_counter() - t0:.1f} s -> {tune['best']}")
    spc = members[0].d.steps_per_cycle
    for c in range(args.warmup):
        b.step_cycles(1)
        b.sync()
        log(f"bench: warmup cycle {c + 1}/{args.warmup} done")
    c0 = [g.counters() for g in members]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c in range(args.steps):
        b.step_cycles(1)
        if (c + 1) % 5 == 0 or c + 1 == args.steps:
            b.sync()
            log(f"bench: timed cycle {c + 1}/{args.steps}")
    b.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    dc = [g.counters() - a for g, a in zip(members, c0)]
    end_counts = [sum(g.count(s) for s in range(3)) for g in members]
    pushes = sum(int(x[B.C_PUSH:B.C_PUSH + 3].sum()) for x in dc)
    push_e = sum(int(x[B.C_PUSH]) for x in dc)
    alg = sum(push_alg_bytes(x, procs) for x in dc)
    achieved = alg / elapsed / 1e9
    cfg = b.config()
    out = {
        "metric": "particle-steps/s (push+deposit+MCC); rf cycles to steady state, warm vs cold",
        "value": pushes / elapsed,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched sweep of {len(members)} O2 CCP discharges (L=2.5 cm, U 100-600 V, "
                               "p 5-100 Pa, 256-1024 cells, 5e4-2e6 superparticles per species)",
                   "step": "one rf cycle of every member = 2000 electron steps", "cells": [g.ng for g in members],
                   "ksub": ksubs, "superparticles_loaded": loaded, "superparticles_end": sum(end_counts),
                   "electron_pushes": push_e,
                   "ion_pushes": pushes - push_e, "autotuned": cfg, "autotune_trials": tune["trials"],
                   "graph": "one HIP graph per rf cycle", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole batched step (algorithmic push bytes over wall time)"},
    }
    print(json.dumps(out), flush=True)
    b.close()


def working(args):
    """The 512-cell working-size discharge (L=2.5 cm, U=400 V, p=40 Pa, 6e5
    superparticles, 2000 steps per rf cycle, ions every 20): with ~1.7e5 pushes per
    step the launches, not HBM, set the pace, so the same discharge is advanced
    both ways a caller can: steps enqueued from the host (pic_step) and a
    one-member batch that replays one HIP graph per rf cycle.  value = pushes per
    second of the graph path; one bench step = one rf cycle."""
    import torch
    from paper_0705_0497_amd import binding as B
    from paper_0705_0497_amd import inputs as I
    procs = I.make_processes()
    d = I.config(2)
    d = I.config(2, capacities=tuple(40 * c for c in d.species_counts()))   # the discharge grows ~10x
    stream = torch.cuda.Stream()

    def make():
        g = B.Discharge(d, procs, stream=stream, sort_kind=B.SORT_COMPACT, sort_every=2000, max_products=1 << 18)
        g.load_uniform()                     # loads and starts the leapfrog
        return g

    def timed(advance, sync, g):
        for c in range(args.warmup):
            advance()
        sync()
        c0 = g.counters()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for c in range(args.steps):
            advance()
            if (c + 1) % 10 == 0:
                sync()
                log(f"bench: timed cycle {c + 1}/{args.steps}")
        sync()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        dc = g.counters() - c0
        return int(dc[B.C_PUSH:B.C_PUSH + 3].sum()), el

    spc = d.steps_per_cycle
    g1 = make()
    p_host, t_host = timed(lambda: g1.step(spc), g1.sync, g1)
    log(f"bench: host-enqueued steps {p_host / t_host:.3e} pushes/s")
    g1.close()
    g2 = make()
    b = B.Batch([g2], block=512, sort_every=2000, use_graph=True)
    tune = b.autotune(window=200)                 # block size and re-ordering interval, ~1 rf cycle of trials
    b.sync()
    log(f"bench: autotune -> {tune['best']}")
    p_graph, t_graph = timed(lambda: b.step_cycles(1), b.sync, g2)
    log(f"bench: cycle graph {p_graph / t_graph:.3e} pushes/s")
    counts = [g2.count(s) for s in range(3)]
    b.close()
    g2.close()
    out = {
        "metric": "particle-steps/s (push+deposit+MCC); rf cycles to steady state, warm vs cold",
        "value": p_graph / t_graph,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * t_graph / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "512-cell O2 CCP, L=2.5 cm, U=400 V, p=40 Pa, 6e5 superparticles",
                   "step": "one rf cycle = 2000 electron steps, ions every 20",
                   "path": "one-member batch, one HIP graph per rf cycle", "autotuned": tune["best"],
                   "host_enqueued": {"value": p_host / t_host, "ms_per_step": 1e3 * t_host / args.steps},
                   "superparticles_end": counts, "parallelism": "single GPU"},
    }
    print(json.dumps(out), flush=True)


def mlp(args):
    """The warm-start network's kernels alone: one training step (forward,
    backward, Adam) on batches of 8192 of a synthetic training set of the
    learned part's size (256 discharges x 512 points, inputs (U, log p, x/L),
    smooth targets), then forward passes over the whole set.  value = training
    samples per second; the roofline is MFMA bf16 on the counted multiply-adds
    (2 flops each: 3.98e5 per sample forward, twice that backward)."""
    import numpy as np
    import torch
    from paper_0705_0497_amd import binding as B
    from paper_0705_0497_amd import warmstart as W
    rng = np.random.Generator(np.random.PCG64(17))
    pts = W.sample_points(256, 13)
    X = np.concatenate([W.features(U, p) for U, p in pts])
    a = rng.standard_normal((1, 6)).astype(np.float32)
    T = np.tanh(X[:, :1] * a + np.sin(3.0 * X[:, 2:3] + X[:, 1:2] * a)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    Td = torch.from_numpy(T).cuda()
    batch = 8192
    net = B.Network(batch, params=W.init_params(0))
    n = len(X)
    flop_fwd = 2.0 * (3 * 256 + 3 * 256 * 256 + 256 * 6)

    def epoch():
        for b0 in range(0, n, batch):
            net.backward(Xd[b0:b0 + batch], Td[b0:b0 + batch], want_loss=False)
            net.adam(1e-3)

    for _ in range(args.warmup):
        epoch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        epoch()
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    steps = args.steps * ((n + batch - 1) // batch)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        net.forward(Xd)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    rate = args.steps * n / t_train
    tflops = 3.0 * flop_fwd * rate / 1e12
    out = {
        "metric": "training samples/s of the warm-start network (forward + backward + Adam)",
        "value": rate, "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * t_train / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "MLP 3 -> 4 x 256 GELU -> 6, batches of 8192 over 256 x 512 samples",
                   "step": "one epoch (16 training steps)", "training_step_us": 1e6 * t_train / steps,
                   "forward_samples_per_s": args.steps * n / t_fwd, "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "achieved": tflops, "peak": 2500.0, "unit": "TFLOP/s",
                     "frac": tflops / 2500.0, "traffic": None,
                     "kernel": "training step (all network kernels over wall time)"},
    }
    print(json.dumps(out), flush=True)
    net.close()


def warmstart(args):
    """Learned warm start: training profiles from batched cold runs carried to a
    long horizon (their late average), the network trained on the GPU, then every
    held-out (U, p) run cold, warm and cold again (other random streams) in one
    batch to a common horizon.  value = particle-steps/s of that evaluation batch;
    the rf cycles to the steady state (the cold run's late average: every 100-cycle
    average of e and O2+ within 5 % from then on), cold and warm, and the profile
    errors are in config; the earlier 1 %-per-20-cycles test is reported beside."""
    import numpy as np
    from paper_0705_0497_amd import warmstart as W
    t0 = time.perf_counter()
    r = W.experiment(W.sample_points(args.train_runs, 11), W.sample_points(args.test_runs, 12),
                     n_total=40000, horizon=3000, late=500, epochs=1500, reference=True,
                     log=lambda m: log(f"bench: [{time.perf_counter() - t0:5.0f} s] {m}"))
    rows = r["rows"]
    cold = [x["cold_cycles"] for x in rows]
    warm = [x["warm_cycles"] for x in rows]
    both = [(c, w) for c, w in zip(cold, warm) if c is not None and w is not None]
    r25 = [(x["cold_cycles_r25"], x["warm_cycles_r25"]) for x in rows]
    r25b = [(c, w) for c, w in r25 if c is not None and w is not None]
    err = np.array([x["density_error"] for x in rows])
    ok = [max(x["density_error"][:2]) < 0.05 for x in rows]
    out = {
        "metric": "particle-steps/s (push+deposit+MCC); rf cycles to steady state, warm vs cold",
        "value": r["pushes"]["eval"] / r["seconds"]["eval"],
        "unit": "particle-steps/s",
        "n_gpus": 1, "steps": r["eval_cycles"], "warmup": 0,
        "ms_per_step": 1e3 * r["seconds"]["eval"] / r["eval_cycles"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+bf16", "data": "synthetic",
        "config": {"workload": f"learned warm start: {args.train_runs} training + {args.test_runs} held-out "
                               "128-cell O2 CCP discharges (L=2.5 cm, U 200-350 V, p 12-17 Pa log-uniform, "
                               "4e4 superparticles loaded, every run to 3000 rf cycles)",
                   "step": "one rf cycle of the evaluation batch (cold, warm and reference members together)",
                   "horizon_cycles": r["horizon"], "late_average_cycles": r["late"],
                   "train_horizon_cycles": r["train_horizon"],
                   "cycles_cold": cold, "cycles_warm": warm,
                   "cycles_ratio_total": sum(c for c, _ in both) / max(1, sum(w for _, w in both)),
                   "cycles_ratio_median": float(np.median([c / w for c, w in both])) if both else None,
                   "points_settled_both": len(both),
                   "r25_cycles_cold_warm": r25,
                   "r25_cycles_ratio_total": sum(c for c, _ in r25b) / max(1, sum(w for _, w in r25b)),
                   "density_error_median": {"e": float(np.median(err[:, 0])), "O2+": float(np.median(err[:, 1])),
                                            "O-": float(np.median(err[:, 2]))},
                   "density_error_max": {"e": float(err[:, 0].max()), "O2+": float(err[:, 1].max()),
                                         "O-": float(err[:, 2].max())},
                   "within_5pct_e_and_O2+": int(sum(ok)),
                   "cold_vs_cold_error_median": {k: float(np.median([x["reference_density_error"][s] for x in rows]))
                                                 for s, k in enumerate(("e", "O2+", "O-"))},
                   "points": [{k: v for k, v in x.items()} for x in rows],
                   "loss_first_last": [r["loss"][0], r["loss"][-1]],
                   "seconds": r["seconds"], "parallelism": "single GPU"},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
