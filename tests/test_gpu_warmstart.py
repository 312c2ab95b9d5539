"""What the learned warm start gains over the plain method: a network trained
on the GPU (BF16 MFMA kernels) from the converged profiles of batched cold runs
loads held-out discharges close to their steady state; the plain method, run
until its convergence test holds, evaluates both starts.  Small version of the
benchmark experiment (8 training runs, 2 held-out points)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_warm_start_converges_faster_to_the_same_state():
    from paper_0705_0497_amd import warmstart as W
    train = [(U, p) for U in (160.0, 230.0, 300.0) for p in (15.0, 28.0)] + [(195.0, 20.0), (265.0, 20.0)]
    test = [(210.0, 18.0), (250.0, 24.0)]
    max_cycles = 1600
    r = W.experiment(train, test, n_total=100000, max_cycles=max_cycles, epochs=1500,
                     log=lambda m: print("warm start:", m, flush=True))
    assert r["loss"][-1][1] < 0.05 * r["loss"][0][1]
    for row in r["rows"]:
        print(row, flush=True)
        assert row["warm_cycles"] is not None
        cold = row["cold_cycles"] if row["cold_cycles"] is not None else max_cycles
        assert 3 * row["warm_cycles"] <= cold, row
        # a warm run keeps what the prediction got wrong once it drifts by less than the
        # convergence test's 1 % per 20 cycles, so agreement follows the prediction: an
        # 8-run network reaches ~10 %; the benchmark's 64-run network is held to 5 %
        assert row["density_error"][0] < 0.15 and row["density_error"][1] < 0.15, row   # e and O2+
