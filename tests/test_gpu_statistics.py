"""Cycle-averaged densities of the GPU against stored FP64 oracle ensembles
(section 3: the discharge is characterised by its cycle-averaged profiles).

Trajectories of a stochastic method decorrelate within ~10^2 steps, so many-
cycle parity is statistical: independent seeds per side, the same seeds on
both sides, the cycle-averaged charge of every node and species compared by
its z-score

    z = (mean_gpu - mean_oracle) / sqrt(var_gpu / M + var_oracle / M),

turned into the normal quantile of the same Welch t probability (the variances
are estimated from M seeds).  Pass: at most 1 % of the nodes beyond 3, the mean
z^2 below the 99.9 % quantile of its distribution when the gpu / oracle labels
are exchanged at random among the 2M runs (for independent nodes that is the
chi^2 bound; the nodes of a profile fluctuate together, which widens it), and
the central electronegativity (O- over e in the middle 10 % of the gap) within 3.
The same seeds run on both sides; while their trajectories are still correlated
(the first cycles) the z-scores come out smaller than for independent runs.

The oracle ensembles are written by tests/golden/make_parity_ensembles.py,
which calls only the oracle; the GPU runs the same protocols here.
"""
import os

import numpy as np
import pytest
from paper_0705_0497_amd import inputs as I
from tests.helpers import judge_ensembles as _judge

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TWO32 = 4294967296.0


def _load(name):
    rows = [line.split() for line in open(os.path.join(GOLDEN, f"ens_{name}.txt")) if not line.startswith("#")]
    seeds = [int(r[0]) for r in rows]
    alpha = np.array([float(r[1]) for r in rows])
    q = np.array([[float(x) for x in r[2:]] for r in rows]).reshape(len(rows), 3, -1)
    return seeds, alpha, q


def _alpha(q, ng):
    mid = slice(int(0.45 * ng), int(0.55 * ng) + 1)
    return q[:, 2, mid].sum(1) / q[:, 0, mid].sum(1)


def _gpu_batch(cfg, seeds, skip, avg, capacity_factor=8.0):
    """The protocol on the GPU: all seeds as members of one batch (each member
    reaches the state it reaches alone), cycle-averaged node charges.  The
    discharges grow from their load; the slots reserved do not change results."""
    import torch
    from paper_0705_0497_amd.binding import Batch, Discharge
    stream = torch.cuda.Stream()
    procs = I.make_processes()
    ds = [I.config(cfg, seed=s, capacity_factor=capacity_factor) for s in seeds]
    mem = [Discharge(d, procs, stream=stream) for d in ds]
    for g in mem:
        g.load_uniform()
    b = Batch(mem, sort_every=20)
    if skip:
        b.step_cycles(skip)
        b.sync()
    for g in mem:
        g.moments(reset=True)
    b.step_cycles(avg)
    b.sync()
    spc = ds[0].steps_per_cycle
    q = np.array([g.moments()["sum_q"] / (avg * spc) / TWO32 for g in mem])
    b.close()
    for g in mem:
        g.close()
    return q, ds[0].ng


@pytest.mark.parametrize("name,cfg", [("cfg1_20cycles", 1), ("cfg2_window", 2)])
def test_cycle_averaged_densities_per_node(name, cfg):
    """128-cell discharge over its 20 rf cycles (32 seeds); 512-cell discharge over
    rf cycles 2-6 (16 seeds)."""
    seeds, ao, O = _load(name)
    skip, avg = {"cfg1_20cycles": (0, 20), "cfg2_window": (1, 5)}[name]
    G, ng = _gpu_batch(cfg, seeds, skip, avg)
    _judge(G, O, _alpha(G, ng), ao, name)


def test_cycle_averaged_densities_at_periodic_steady_state():
    """128-cell discharge after 1000 rf cycles, averaged over the next 100 (32 seeds)."""
    seeds, ao, O = _load("cfg1_steady")
    G, ng = _gpu_batch(1, seeds, 1000, 100)
    _judge(G, O, _alpha(G, ng), ao, "cfg1_steady")
