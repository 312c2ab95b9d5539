"""Writes cfg2_oracle_ensemble.txt: the FP64 oracle's cycle-averaged node densities
of the 512-cell discharge (2.5 cm, 400 V, 40 Pa, 6e5 superparticles, the eight
workload channels) over its second rf cycle, for 8 seeds, summed onto 32 coarse
bins per species, plus the electronegativity of the central 10 % of nodes.
Calls only the oracle; the GPU test compares its own ensemble with this one.

    python tests/golden/make_cfg2_ensemble.py      (about a minute on 8 cores)
"""
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SEEDS = list(range(9200, 9208))
BINS = 32


def one(seed):
    from oracle import pyoracle as po
    from paper_0705_0497_amd import inputs as I
    d = I.config(2, seed=seed)
    o = po.Oracle(d, d.species(), I.make_processes())
    o.load_uniform()
    o.prepare(True)
    o.step(d.steps_per_cycle)
    o.reset_moments()
    o.step(d.steps_per_cycle)
    q = o.moments()["sumQ"] / d.steps_per_cycle          # [3][ng+1] fixed-point charge per node
    coarse = q[:, :d.ng].reshape(3, BINS, -1).sum(-1)
    mid = slice(int(0.45 * d.ng), int(0.55 * d.ng) + 1)
    alpha = q[2, mid].sum() / q[0, mid].sum()
    return seed, coarse, alpha


def main():
    with mp.Pool(min(len(SEEDS), os.cpu_count() or 1)) as pool:
        res = pool.map(one, SEEDS)
    path = os.path.join(HERE, "cfg2_oracle_ensemble.txt")
    with open(path, "w") as f:
        f.write("# oracle ensemble, 512-cell discharge, second rf cycle; written by make_cfg2_ensemble.py\n")
        f.write("# seed alpha_centre then 3 x 32 coarse-bin charge sums (e, O2+, O-) in 2^-32 units\n")
        for seed, coarse, alpha in res:
            f.write(f"{seed} {alpha:.10e} " + " ".join(f"{v:.10e}" for v in coarse.ravel()) + "\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
