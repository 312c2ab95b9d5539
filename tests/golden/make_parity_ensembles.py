"""Writes the FP64 oracle ensembles that the GPU's cycle-averaged densities are
compared with (per node and species, z-scores over independent seeds).  Calls
only the oracle.

Three protocols, each from the uniform quasi-neutral load of its workload:

  cfg1_20cycles  128-cell discharge (2.5 cm, 200 V, 20 Pa, 3e4 superparticles),
                 node charges averaged over its 20 rf cycles; 32 seeds.
  cfg1_steady    the same discharge at its periodic steady state: 1000 rf
                 cycles run, then averaged over the next 100; 32 seeds.
  cfg2_window    512-cell discharge (2.5 cm, 400 V, 40 Pa, 6e5 superparticles),
                 averaged over rf cycles 2-6 (it is still growing); 16 seeds.

Each output row: seed, central electronegativity alpha (O- over e summed over
the central 10 % of the nodes), then 3 x (ng + 1) cycle-averaged node charges
(e, O2+, O-) in superparticles.

    python tests/golden/make_parity_ensembles.py [protocol ...] [--workers N]

About 50 minutes on 8 cores for all three (the steady state dominates).
"""
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

PROTOCOLS = {
    # name: (workload, seeds, cycles run before the window, cycles averaged)
    "cfg1_20cycles": (1, list(range(9300, 9332)), 0, 20),
    "cfg1_steady": (1, list(range(9400, 9432)), 1000, 100),
    "cfg2_window": (2, list(range(9500, 9516)), 1, 5),
}


def path_of(name):
    return os.path.join(HERE, f"ens_{name}.txt")


def alpha_centre(q, ng):
    mid = slice(int(0.45 * ng), int(0.55 * ng) + 1)
    return q[2, mid].sum() / q[0, mid].sum()


def one(job):
    name, seed = job
    from oracle import pyoracle as po
    from paper_0705_0497_amd import inputs as I
    cfg, _, skip, avg = PROTOCOLS[name]
    d = I.config(cfg, seed=seed)
    o = po.Oracle(d, d.species(), I.make_processes())
    o.load_uniform()
    o.prepare(True)
    if skip:
        o.step(skip * d.steps_per_cycle)
    o.reset_moments()
    o.step(avg * d.steps_per_cycle)
    q = o.moments()["sumQ"] / (avg * d.steps_per_cycle) / 4294967296.0
    return name, seed, alpha_centre(q, d.ng), q


def main():
    args = [a for a in sys.argv[1:] if not a.startswith("--")]
    workers = os.cpu_count() or 1
    if "--workers" in sys.argv:
        workers = int(sys.argv[sys.argv.index("--workers") + 1])
        args = [a for a in args if a != str(workers)]
    names = args or list(PROTOCOLS)
    # longest jobs first
    jobs = [(n, s) for n in sorted(names, key=lambda n: -PROTOCOLS[n][2] - PROTOCOLS[n][3]) for s in PROTOCOLS[n][1]]
    rows = {n: {} for n in names}
    with mp.Pool(min(workers, len(jobs))) as pool:
        for name, seed, alpha, q in pool.imap_unordered(one, jobs):
            rows[name][seed] = (alpha, q)
            print(f"{name} seed {seed} done", flush=True)
    for name in names:
        cfg, seeds, skip, avg = PROTOCOLS[name]
        with open(path_of(name), "w") as f:
            f.write(f"# oracle ensemble {name}: workload {cfg}, cycles {skip + 1}..{skip + avg} averaged; "
                    "written by make_parity_ensembles.py\n")
            f.write("# seed alpha_centre then 3 x (ng + 1) node charges (e, O2+, O-) in superparticles\n")
            for seed in seeds:
                alpha, q = rows[name][seed]
                f.write(f"{seed} {alpha:.10e} " + " ".join(f"{v:.9e}" for v in q.ravel()) + "\n")
        print("wrote", path_of(name))


if __name__ == "__main__":
    main()
