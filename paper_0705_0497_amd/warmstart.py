"""Learned warm start: batched runs to the periodic steady state generate
cycle-averaged profiles; the network of include/mlp.h learns (U, p, x/L) ->
profiles on the GPU; new discharges are loaded from its prediction
(pic_load_profiles) instead of uniformly, and the plain method evaluates the
result.

The paper computes the quasi-stationary state reached after many rf cycles and
reports cycle-averaged densities and energies across the gap (section 3); it
has no network.  Everything here is orchestration: every step of the method,
the network's forward and backward passes and Adam run in the HIP kernels.

Profiles: 512 points x/L in [0, 1]; per species (e, O-, O2+ in the network's
order) the cycle-averaged density from the charge sums at the nodes and the
mean kinetic energy per cell from the sampled energy sums.

Steady state and cycles to reach it.  Runs advance in windows of 10 rf cycles
to a common horizon.  The steady state of a held-out point is the average of
its cold run over the last `late` cycles before the horizon.  A run has reached
it at cycle c when every 100-cycle moving average of its e and O2+ densities from
c to the horizon lies within 5 % (relative L1) of that average (100 cycles: at
the low-density points of the family 50-cycle averages of two cold runs with
different random streams already scatter by several %).  The earlier
convergence test (n_e changing by less than 1 % over 20 cycles, twice in a row,
reading R25) is reported beside it: the plasma density relaxes over 10^2-10^3
cycles and passes that test long before the profiles stop moving.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import binding as B
from . import inputs as I

QE = 1.602176634e-19
NPTS = 512
XS = np.linspace(0.0, 1.0, NPTS)
U_MAX = 600.0
P_MIN, P_MAX = 5.0, 100.0
NET_SPECIES = (0, 2, 1)          # network outputs e, O-, O2+ -> library species indices
WINDOW, LAG, TOL = 10, 20, 0.01
DENS_FLOOR = 1e10                # m^-3, floor of the log densities


def features(U, p, x=XS):
    """Network inputs (U / U_max, log p scaled to [-1, 1], x / L) for every x."""
    lp = 2.0 * (math.log(p) - math.log(P_MIN)) / (math.log(P_MAX) - math.log(P_MIN)) - 1.0
    return np.stack([np.full_like(x, U / U_MAX), np.full_like(x, lp), x], 1).astype(np.float32)


def family(U, p, seed, n_total=60000, **over):
    """One discharge of the warm-start family: the 128-cell, 2.5 cm gap form with
    400 steps per rf cycle and ions every 10 steps, at voltage U and pressure p."""
    d = I.config(1, U=float(U), p=float(p), seed=int(seed), n_total=int(n_total), diag_every=20, sort_every=20,
                 **over)
    c = d.species_counts()
    return dataclasses.replace(d, capacities=(60 * c[0] + 4096, 60 * c[1] + 4096, 8 * c[2] + 4096))


def cycle_profiles(g, m):
    """Profiles on XS from the moments m = g.moments() of a window of cycles:
    densities [3][NPTS] (m^-3, library species order) and mean energies [3][NPTS] (eV)."""
    d = g.d
    ng = d.ng
    dx = d.L / ng
    vol = np.full(ng + 1, dx)
    vol[0] = vol[-1] = 0.5 * dx
    nodes = np.arange(ng + 1) / ng
    centres = (np.arange(ng) + 0.5) / ng
    nacc = max(int(m["nacc"]), 1)
    dens = np.zeros((3, NPTS))
    mean = np.zeros((3, NPTS))
    for s in range(3):
        n = d.weight * 2.0 ** -32 * m["sum_q"][s] / nacc / vol
        dens[s] = np.interp(XS, nodes, n)
        cnt = m["ecnt"][s].astype(np.float64)
        e = np.where(cnt > 0, m["esum"][s] * 2.0 ** -20 / np.maximum(cnt, 1), np.nan)
        ok = np.isfinite(e)
        if ok.sum() >= 2:
            mean[s] = np.interp(XS, centres[ok], e[ok])
        else:
            mean[s] = 1.5 * d.species()[s].t0_ev if d.species()[s].t0_ev > 0 else 0.04
    return dens, mean


def to_targets(dens, mean):
    """[NPTS][6] raw network targets: log densities and mean energies (e, O-, O2+)."""
    out = np.zeros((NPTS, 6))
    for k, s in enumerate(NET_SPECIES):
        out[:, k] = np.log(np.maximum(dens[s], DENS_FLOOR))
        out[:, 3 + k] = mean[s]
    return out


def from_targets(y):
    """Inverse of to_targets: densities and mean energies [3][NPTS] in library order."""
    dens = np.zeros((3, len(y)))
    mean = np.zeros((3, len(y)))
    for k, s in enumerate(NET_SPECIES):
        dens[s] = np.exp(y[:, k])
        mean[s] = np.maximum(y[:, 3 + k], 1e-3)
    return dens, mean


class Monitor:
    """Convergence of one discharge from 10-cycle window sums of n_e."""

    def __init__(self):
        self.windows = []
        self.passed = []
        self.converged_at = None

    def add(self, ne_window, cycle):
        self.windows.append(np.asarray(ne_window, dtype=np.float64))
        ok = False
        if len(self.windows) >= 3:
            a, b = self.windows[-1], self.windows[-3]
            ok = float(np.abs(a - b).sum()) < TOL * float(np.abs(a).sum())
        self.passed.append(ok)
        if self.converged_at is None and len(self.passed) >= 2 and self.passed[-1] and self.passed[-2]:
            self.converged_at = cycle
        return self.converged_at


def run_batch(members, max_cycles, log=None):
    """Advances Discharge members as one batch (one launch per kernel per step,
    a HIP graph per rf cycle) in windows of 10 rf cycles until every member has
    converged or max_cycles have run.  Returns per member the convergence cycle
    (None if not reached) and the profiles of the window at convergence (of the
    last window if not reached), and the cycles run."""
    batch = B.Batch(members, block=512, sort_every=20, use_graph=True)
    for g in members:
        g.moments(reset=True)
    mons = [Monitor() for _ in members]
    prof = [None] * len(members)
    cycles = 0
    while cycles < max_cycles:
        batch.step_cycles(WINDOW)
        batch.sync()
        cycles += WINDOW
        for i, g in enumerate(members):
            m = g.moments(reset=True)
            if mons[i].converged_at is None:
                mons[i].add(m["sum_q"][0], cycles)
                prof[i] = cycle_profiles(g, m)
        done = sum(mon.converged_at is not None for mon in mons)
        if log and (cycles % 100 == 0 or done == len(members)):
            log(f"cycle {cycles}: {done}/{len(members)} converged")
        if done == len(members):
            break
    batch.close()
    return [mon.converged_at for mon in mons], prof, cycles


def make_members(points, procs, stream, n_total=60000, seed0=5000, warm=None):
    """Discharge objects for (U, p) points, loaded uniformly or from profiles."""
    out = []
    for j, (U, p) in enumerate(points):
        g = B.Discharge(family(U, p, seed0 + j, n_total), procs, stream=stream, max_products=1 << 16)
        if warm is None:
            g.load_uniform()
        else:
            dens, mean = warm[j]
            used = g.load_profiles(XS, dens, mean)
            if not used:
                raise RuntimeError("warm-start profile rejected")
        out.append(g)
    return out


@dataclasses.dataclass
class Standardizer:
    mu: np.ndarray
    sd: np.ndarray

    @classmethod
    def fit(cls, T):
        return cls(T.mean(0), np.maximum(T.std(0), 1e-6))

    def fwd(self, T):
        return (T - self.mu) / self.sd

    def inv(self, Z):
        return Z * self.sd + self.mu


def init_params(seed):
    """Uniform(+-1/sqrt(fan_in)) weights and biases (seeded)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for o, i in ((256, 3), (256, 256), (256, 256), (256, 256), (6, 256)):
        s = 1.0 / math.sqrt(i)
        parts.append(rng.uniform(-s, s, size=o * i))
        parts.append(rng.uniform(-s, s, size=o))
    return np.concatenate(parts).astype(np.float32)


def train_network(X, T, epochs=2000, lr=2e-3, batch=8192, seed=0, log=None):
    """Trains the network on the GPU (BF16 MFMA kernels, Adam) from inputs X
    [N][3] and raw targets T [N][6]; returns the network, the standardiser and
    the loss history."""
    import torch
    std = Standardizer.fit(T)
    Z = std.fwd(T).astype(np.float32)
    net = B.Network(min(batch, len(X)), params=init_params(seed))
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    Zd = torch.from_numpy(np.ascontiguousarray(Z)).cuda()
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    hist = []
    n = len(X)
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        for b0 in range(0, n, batch):
            idx = perm[b0:b0 + batch]
            want = (ep % 100 == 0 or ep == epochs - 1) and b0 == 0
            loss = net.backward(Xd[idx], Zd[idx], want_loss=want)
            net.adam(lr * (0.5 * (1.0 + math.cos(math.pi * ep / epochs))) + 1e-5)
            if want:
                hist.append((ep, loss))
                if log:
                    log(f"epoch {ep}: loss {loss:.4g}")
    return net, std, hist


def predict(net, std, U, p):
    """Predicted profiles (densities, mean energies [3][NPTS], library order)."""
    import torch
    y = net.forward(torch.from_numpy(features(U, p)).cuda()).cpu().numpy().astype(np.float64)
    return from_targets(std.inv(y))


def profile_error(a, b):
    """Relative L1 difference of two density profiles (b the reference)."""
    return float(np.abs(a - b).sum() / max(np.abs(b).sum(), 1e-300))


def sample_points(n, seed, U=(200.0, 350.0), p=(12.0, 17.0)):
    """(U, p) pairs: U uniform, p log-uniform (seeded).  The default range is
    where cold runs of the family settle within a few thousand rf cycles: below
    ~10 Pa the discharge of the synthetic tables goes out, above ~20 Pa its
    density still creeps by more than a percent per thousand cycles at 4000."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Us = rng.uniform(U[0], U[1], n)
    ps = np.exp(rng.uniform(math.log(p[0]), math.log(p[1]), n))
    return [(float(a), float(b)) for a, b in zip(Us, ps)]


SMOOTH = 10                      # windows in the moving average of the steady-state test (100 cycles)
SETTLE_TOL = 0.05                # relative L1 band of e and O2+ around the steady state


def run_to_horizon(members, horizon, late, log=None):
    """Advances Discharge members as one batch (a HIP graph per rf cycle) for
    `horizon` rf cycles in windows of WINDOW cycles.  Returns per member the
    window-averaged node charges [n_windows][3][ng + 1] (superparticles per node)
    and the profiles (densities, mean energies) averaged over the last `late`
    cycles."""
    batch = B.Batch(members, block=512, sort_every=20, use_graph=True)
    for g in members:
        g.moments(reset=True)
    nwin = horizon // WINDOW
    q = [np.zeros((nwin, 3, g.ng + 1)) for g in members]
    acc = [None] * len(members)
    for k in range(nwin):
        batch.step_cycles(WINDOW)
        batch.sync()
        for i, g in enumerate(members):
            m = g.moments(reset=True)
            q[i][k] = m["sum_q"] / max(int(m["nacc"]), 1) * 2.0 ** -32
            if (nwin - k) * WINDOW <= late:                 # a window of the late average
                if acc[i] is None:
                    acc[i] = {key: np.array(m[key], dtype=np.float64) for key in ("sum_q", "esum", "ecnt")}
                    acc[i]["nacc"] = int(m["nacc"])
                else:
                    for key in ("sum_q", "esum", "ecnt"):
                        acc[i][key] += m[key]
                    acc[i]["nacc"] += int(m["nacc"])
        if log and ((k + 1) * WINDOW) % 100 == 0:
            log(f"cycle {(k + 1) * WINDOW} of {horizon}")
    batch.close()
    prof = [cycle_profiles(g, a) for g, a in zip(members, acc)]
    return q, prof


def r25_cycles(qwin):
    """Cycle at which the 1 %-over-20-cycles test on n_e first held twice in a row."""
    mon = Monitor()
    for k in range(len(qwin)):
        if mon.add(qwin[k][0], (k + 1) * WINDOW) is not None:
            return mon.converged_at
    return None


def settle_cycles(qwin, ref_q, tol=SETTLE_TOL, smooth=SMOOTH):
    """First cycle from which every moving average over `smooth` windows of the
    e and O2+ node densities stays within `tol` (relative L1) of ref_q [3][ng+1];
    None if the last one does not."""
    n = len(qwin)
    ok = np.zeros(n, bool)
    for k in range(smooth - 1, n):
        avg = qwin[k - smooth + 1:k + 1].mean(0)
        ok[k] = all(profile_error(avg[s], ref_q[s]) <= tol for s in (0, 1))
    if not ok[-1]:
        return None
    k = n - 1
    while k - 1 >= smooth - 1 and ok[k - 1]:
        k -= 1
    return (k + 1) * WINDOW


def experiment(train_pts, test_pts, n_total=30000, horizon=3000, late=500, epochs=1500, reference=True, log=None,
               train_horizon=None):
    """Trains on the late-averaged profiles of cold runs at train_pts (carried to
    train_horizon cycles, by default the evaluation horizon, the last `late`
    averaged), then runs every test point cold, warm (loaded from the prediction)
    and, with reference=True, cold again with other random streams, all in one
    batch to `horizon` cycles.  Per point: cycles to the steady state (the cold
    run's late average) of each run, the R25 convergence cycles beside them, and
    the late-average profile errors of the warm and reference runs against the
    cold run."""
    if train_horizon is None:
        train_horizon = horizon
    import time
    import torch
    procs = I.make_processes()
    stream = torch.cuda.Stream()
    t0 = time.perf_counter()
    prof_tr, push_data = [], 0
    for b0 in range(0, len(train_pts), 64):
        pts = train_pts[b0:b0 + 64]
        train = make_members(pts, procs, stream, n_total=n_total, seed0=7000 + b0)
        _, prof = run_to_horizon(train, train_horizon, late,
                                 log=(lambda m, b0=b0: log(f"training runs {b0}-{b0 + len(pts) - 1}: {m}")) if log else None)
        prof_tr += prof
        push_data += sum(int(g.counters()[B.C_PUSH:B.C_PUSH + 3].sum()) for g in train)
        for g in train:
            g.close()
    t_data = time.perf_counter() - t0
    X = np.concatenate([features(U, p) for U, p in train_pts])
    T = np.concatenate([to_targets(*pr) for pr in prof_tr])
    t0 = time.perf_counter()
    net, std, hist = train_network(X, T, epochs=epochs, log=log)
    t_train = time.perf_counter() - t0
    warm = [predict(net, std, U, p) for U, p in test_pts]
    cold_m = make_members(test_pts, procs, stream, n_total=n_total, seed0=9000)
    warm_m = make_members(test_pts, procs, stream, n_total=n_total, seed0=9000, warm=warm)
    ref_m = make_members(test_pts, procs, stream, n_total=n_total, seed0=9500) if reference else []
    t0 = time.perf_counter()
    qw, prof = run_to_horizon(cold_m + warm_m + ref_m, horizon, late,
                              log=(lambda m: log(f"evaluation: {m}")) if log else None)
    t_eval = time.perf_counter() - t0
    n = len(test_pts)
    rows = []
    for j, (U, p) in enumerate(test_pts):
        ref_q = qw[j][-(late // WINDOW):].mean(0)          # the steady state: the cold run's late average
        (dc, ec), (dw, ew) = prof[j], prof[n + j]
        row = {"U": U, "p": p,
               "cold_cycles": settle_cycles(qw[j], ref_q), "warm_cycles": settle_cycles(qw[n + j], ref_q),
               "cold_cycles_r25": r25_cycles(qw[j]), "warm_cycles_r25": r25_cycles(qw[n + j]),
               "density_error": [profile_error(dw[s], dc[s]) for s in range(3)],
               "energy_error": [profile_error(ew[s], ec[s]) for s in range(3)],
               "predicted_density_error": [profile_error(warm[j][0][s], dc[s]) for s in range(3)]}
        if reference:
            row["reference_cycles"] = settle_cycles(qw[2 * n + j], ref_q)
            row["reference_density_error"] = [profile_error(prof[2 * n + j][0][s], dc[s]) for s in range(3)]
        rows.append(row)
    push_eval = sum(int(g.counters()[B.C_PUSH:B.C_PUSH + 3].sum()) for g in cold_m + warm_m + ref_m)
    for g in cold_m + warm_m + ref_m:
        g.close()
    return {"train_points": len(train_pts), "loss": hist, "rows": rows, "horizon": horizon, "late": late,
            "train_horizon": train_horizon, "seconds": {"data": t_data, "train": t_train, "eval": t_eval},
            "eval_cycles": horizon, "pushes": {"data": push_data, "eval": push_eval}, "net": net, "std": std}
