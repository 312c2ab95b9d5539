"""Seeded synthetic inputs for the 1D3V oxygen PIC-MCC discharge.

This module only *describes* inputs: discharge parameters, species data and
cross-section tables written on a fixed log-spaced energy grid.  It holds none
of the method's arithmetic (no push, no collision, no field solve); both the
HIP library and the FP64 oracle receive what it produces as plain data.

Paper basis (Bronold et al., ICPIG 2007):
  * geometry and drive: 1D gap 0 <= x <= L, one electrode at U sin(2 pi f t),
    the other grounded, O2 background at T = 300 K (section 2);
  * species e, O-, O2+ (section 2) and the reaction list of Table 1;
  * associative detachment cross section, Eq. (1):
    sigma_ad(E) = 5.96e-16 cm^2 / sqrt(E[eV])  ->  sigma0 = 5.96e-20 m^2, b = 1/2.
The paper's measured cross sections are not available (Fig. 2 is an image and
its sources are not at hand), so every other table is a seeded synthetic
stand-in of the form sigma0 * (1 - E_th/E)^a * (E/E0)^(-b), E0 = 1 eV.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# --- physical data handed to both sides (SI, CODATA 2018; e and k_B exact) ---
ELEMENTARY_CHARGE = 1.602176634e-19
BOLTZMANN = 1.380649e-23
ELECTRON_MASS = 9.1093837015e-31
ATOMIC_MASS_UNIT = 1.66053906660e-27
M_O2 = 31.9988 * ATOMIC_MASS_UNIT
M_O = 15.9994 * ATOMIC_MASS_UNIT
M_O2PLUS = M_O2 - ELECTRON_MASS
M_OMINUS = M_O + ELECTRON_MASS

# species indices (fixed roles of the three simulated species, section 2)
ELECTRON, O2PLUS, OMINUS = 0, 1, 2
SPECIES_NAMES = ("e", "O2+", "O-")

# cross-section energy grid: n log-spaced points from emin to emax [eV]
TABLE_EMIN = 1.0e-3
TABLE_EMAX = 1.0e3
TABLE_N = 512

# process kinds and collision targets (string names; each binding maps them
# to its own enumeration)
KINDS = ("elastic", "excite", "ionize", "attach", "cx", "neutralize", "detach", "ion_elastic", "recomb", "edetach")
TARGETS = ("O2", "O2a", "grid+", "grid-")   # background O2, metastable O2(a), O2+ / O- grid densities

TABLE_SEED = 0x5EED0001


@dataclasses.dataclass
class Process:
    """One collision channel of Table 1 with its cross-section table.

    species      index of the projectile species (ELECTRON, O2PLUS, OMINUS)
    kind         one of KINDS
    target       one of TARGETS
    e_th         threshold energy [eV] (0 for none)
    target_mass  mass of the collision partner [kg]
    sigma        cross sections [m^2] on the TABLE_N-point log grid
    params       generator parameters (sigma0, a, b, e_th), for documentation
    """
    name: str
    species: int
    kind: str
    target: str
    e_th: float
    target_mass: float
    sigma: np.ndarray
    params: dict


@dataclasses.dataclass
class Species:
    charge: float        # in units of e
    mass: float          # kg
    t0_ev: float         # loading temperature [eV]
    count: int           # superparticles loaded
    capacity: int        # superparticle slots reserved


@dataclasses.dataclass
class Discharge:
    """Parameters of one discharge (one simulation)."""
    name: str
    L: float                 # gap [m]
    ng: int                  # cells
    U: float                 # voltage amplitude [V]
    f: float                 # rf frequency [Hz]
    p: float                 # gas pressure [Pa]
    steps_per_cycle: int
    ksub: int                # ion subcycling factor
    cycles: int
    n_plus0: float           # loaded O2+ density [m^-3]
    frac_minus: float        # n(O-)/n(O2+) at loading
    te0: float = 3.0         # electron loading temperature [eV]
    ti0: float = 0.026       # ion loading temperature [eV]
    c_meta: float = 0.1      # metastable fraction C, n(O2(a)) = C n(O2)
    t_gas: float = 300.0     # K
    n_total: int = 30000     # superparticles over all species
    sort_every: int = 20
    diag_every: int = 20
    seed: int = 1
    capacity_factor: float = 4.0
    counts: Optional[tuple] = None   # explicit (e, O2+, O-) counts, if given
    capacities: Optional[tuple] = None   # explicit slots per species, if given

    @property
    def dt(self) -> float:
        return 1.0 / (self.f * self.steps_per_cycle)

    def species_counts(self):
        """Superparticle counts per species under one common weight.

        One weight per discharge keeps every reaction charge-exact per event:
        the counts are split in proportion to the loaded densities."""
        if self.counts is not None:
            return tuple(int(c) for c in self.counts)
        n_minus = self.frac_minus * self.n_plus0
        n_e = self.n_plus0 - n_minus
        tot = self.n_plus0 + n_minus + n_e
        c_plus = int(round(self.n_total * self.n_plus0 / tot))
        c_minus = int(round(self.n_total * n_minus / tot))
        c_e = self.n_total - c_plus - c_minus
        return (c_e, c_plus, c_minus)

    @property
    def weight(self) -> float:
        """Physical particles per superparticle per m^2 of electrode area."""
        c_plus = self.species_counts()[O2PLUS]
        return self.n_plus0 * self.L / c_plus

    def species(self) -> List[Species]:
        ce, cp, cm = self.species_counts()
        if self.capacities is not None:
            caps = [int(c) for c in self.capacities]
        else:
            caps = [max(1024, int(math.ceil(c * self.capacity_factor))) for c in (ce, cp, cm)]
        return [
            Species(-1.0, ELECTRON_MASS, self.te0, ce, caps[0]),
            Species(+1.0, M_O2PLUS, self.ti0, cp, caps[1]),
            Species(-1.0, M_OMINUS, self.ti0, cm, caps[2]),
        ]


def energy_grid() -> np.ndarray:
    k = np.arange(TABLE_N, dtype=np.float64)
    return TABLE_EMIN * (TABLE_EMAX / TABLE_EMIN) ** (k / (TABLE_N - 1))


def power_law(e, sigma0, a, b, e_th, e0=1.0) -> np.ndarray:
    """sigma0 (1 - e_th/E)^a (E/e0)^(-b) for E > e_th, else 0 (E in eV, sigma in m^2)."""
    e = np.asarray(e, dtype=np.float64)
    out = np.zeros_like(e)
    m = e > e_th
    out[m] = sigma0 * (1.0 - e_th / e[m]) ** a * (e[m] / e0) ** (-b)
    return out


def power_law_table(sigma0, a, b, e_th, e0=1.0) -> np.ndarray:
    """power_law on the TABLE_N-point grid."""
    return power_law(energy_grid(), sigma0, a, b, e_th, e0)


def eq1_sigma0_m2() -> float:
    """Eq. (1): 5.96e-16 cm^2 / sqrt(E[eV]) written in m^2 at E = 1 eV."""
    return 5.96e-16 * 1e-4


# ---- the paper's cross-section models as table generators (section 2) --------
BOHR_M = 5.29177210903e-11          # Bohr radius [m]
HARTREE_EV = 27.211386245988        # Hartree energy [eV]


def landau_zener(e, r_x):
    """Two-channel Landau-Zener cross section of ion-ion neutralisation,
    sigma_n = 4 pi R_x^2 (1 + 1 / (R_x E)), read in atomic units: R_x in Bohr
    radii, E the relative energy in Hartree, sigma in Bohr^2 (1 / R_x is the
    Coulomb energy at the crossing radius).  E in eV, result in m^2."""
    e = np.asarray(e, dtype=np.float64)
    return 4.0 * math.pi * (r_x * BOHR_M) ** 2 * (1.0 + HARTREE_EV / (r_x * e))


def landau_zener_table(r_x) -> np.ndarray:
    """landau_zener on the TABLE_N-point grid."""
    return landau_zener(energy_grid(), r_x)


def cx_from_momentum_transfer(sigma_m, e_lo=0.251, e_hi=8.5) -> np.ndarray:
    """(O2+, O2) charge exchange from a momentum-transfer cross section sigma_m
    (callable of E [eV] -> m^2, or an array on the table grid): sigma_cx = sigma_m / 2
    below e_lo and above e_hi, linear in E in between."""
    e = energy_grid()
    sm = np.asarray(sigma_m(e) if callable(sigma_m) else sigma_m, dtype=np.float64)
    if sm.shape != e.shape:
        raise ValueError("sigma_m must be given on the table grid")
    f = (lambda x: 0.5 * np.asarray(sigma_m(x), dtype=np.float64)) if callable(sigma_m) else \
        (lambda x: 0.5 * np.interp(np.log(x), np.log(e), sm))
    lo, hi = float(f(np.array([e_lo]))[0]), float(f(np.array([e_hi]))[0])
    out = 0.5 * sm
    mid = (e > e_lo) & (e < e_hi)
    out[mid] = lo + (hi - lo) * (e[mid] - e_lo) / (e_hi - e_lo)
    return out


# Windows of the synthetic parameters.  Generic orders of magnitude chosen so
# that the seeded discharge is sustained; not fitted to any measured data.
_WINDOWS = {
    # name: (kind, species, target, target_mass, sigma0 log-window, a, b, e_th)
    "e-elastic": ("elastic", ELECTRON, "O2", M_O2, (3e-20, 1e-19), (0.0, 0.0), (0.0, 0.3), (0.0, 0.0)),
    "e-vib": ("excite", ELECTRON, "O2", M_O2, (3e-21, 3e-20), (0.5, 2.0), (0.5, 1.5), (0.15, 0.5)),
    "e-exc": ("excite", ELECTRON, "O2", M_O2, (5e-21, 3e-20), (0.5, 2.0), (0.0, 0.4), (6.4, 8.6)),
    "e-ion": ("ionize", ELECTRON, "O2", M_O2, (1e-20, 4e-20), (1.0, 2.0), (0.0, 0.3), (10.0, 14.0)),
    "e-att": ("attach", ELECTRON, "O2", M_O2, (1e-22, 1e-21), (0.5, 2.0), (0.5, 1.5), (3.0, 6.0)),
    "O2+-cx": ("cx", O2PLUS, "O2", M_O2, (2e-19, 6e-19), (0.0, 0.0), (0.0, 0.5), (0.0, 0.0)),
    "O--neut": ("neutralize", OMINUS, "grid+", M_O2PLUS, (1e-18, 5e-18), (0.0, 0.0), (0.5, 1.0), (0.0, 0.0)),
}


def make_processes(seed: int = TABLE_SEED, ad_eq1: bool = True) -> List[Process]:
    """The eight seeded channels: 5 electron, 1 O2+, 2 O- (table order = selection order)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    procs = []
    for name, (kind, sp, tgt, tm, s0w, aw, bw, ew) in _WINDOWS.items():
        s0 = float(math.exp(rng.uniform(math.log(s0w[0]), math.log(s0w[1]))))
        a = float(rng.uniform(*aw))
        b = float(rng.uniform(*bw))
        eth = float(rng.uniform(*ew))
        procs.append(Process(name, sp, kind, tgt, eth, tm, power_law_table(s0, a, b, eth),
                             dict(sigma0=s0, a=a, b=b, e_th=eth)))
    if ad_eq1:
        s0, a, b, eth = eq1_sigma0_m2(), 0.0, 0.5, 0.0
    else:
        s0 = float(math.exp(rng.uniform(math.log(3e-20), math.log(9e-20))))
        a, b, eth = 0.0, 0.5, 0.0
    procs.append(Process("O--ad", OMINUS, "detach", "O2a", eth, M_O2, power_law_table(s0, a, b, eth),
                         dict(sigma0=s0, a=a, b=b, e_th=eth)))
    return procs


# Table 1 channels beyond the eight of the workloads (seeded with their own stream):
# the two dissociation thresholds of rows (12), (13) as separate channels, O- elastic
# scattering on O2 (8) and direct detachment O- + O2 -> O + O2 + e (19)
_EXTRA_WINDOWS = {
    "e-diss6.4": ("excite", ELECTRON, "O2", M_O2, (5e-21, 3e-20), (0.5, 2.0), (0.0, 0.4), (6.4, 6.4)),
    "e-diss8.6": ("excite", ELECTRON, "O2", M_O2, (5e-21, 3e-20), (0.5, 2.0), (0.0, 0.4), (8.6, 8.6)),
    "O--el": ("ion_elastic", OMINUS, "O2", M_O2, (1e-19, 5e-19), (0.0, 0.0), (0.0, 0.5), (0.0, 0.0)),
    "O--dd": ("detach", OMINUS, "O2", M_O2, (1e-21, 1e-20), (0.5, 2.0), (0.0, 0.5), (1.5, 3.0)),
}


def make_processes_extended(seed: int = TABLE_SEED) -> List[Process]:
    """Eleven channels: e elastic (7), vibrational (10), dissociation at 6.4 eV (12) and
    8.6 eV (13), ionisation (21), attachment (18); O2+ charge exchange (9); O-
    neutralisation (17), elastic (8), direct detachment (19), associative detachment (20)."""
    base = {p.name: p for p in make_processes(seed)}
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    extra = {}
    for name, (kind, sp, tgt, tm, s0w, aw, bw, ew) in _EXTRA_WINDOWS.items():
        s0 = float(math.exp(rng.uniform(math.log(s0w[0]), math.log(s0w[1]))))
        a = float(rng.uniform(*aw))
        b = float(rng.uniform(*bw))
        eth = float(rng.uniform(*ew))
        extra[name] = Process(name, sp, kind, tgt, eth, tm, power_law_table(s0, a, b, eth),
                              dict(sigma0=s0, a=a, b=b, e_th=eth))
    order = ["e-elastic", "e-vib", "e-diss6.4", "e-diss8.6", "e-ion", "e-att", "O2+-cx", "O--neut", "O--el",
             "O--dd", "O--ad"]
    return [base[n] if n in base else extra[n] for n in order]


# The remaining Table 1 channels with a collision partner other than a
# charged particle of the same kind (rows 1-6 are Coulomb scattering, not
# modelled), seeded with a third stream: Rydberg (11), a1Delta_g (14) and
# b1Sigma_g (15) excitation at the textbook excitation energies of O2 (the
# Rydberg window a guess), dissociative recombination (16, falling as 1/E) and
# electron-impact detachment of O- (22, above the electron affinity of O).
_FULL_WINDOWS = {
    "e-ryd": ("excite", ELECTRON, "O2", M_O2, (1e-21, 1e-20), (0.5, 2.0), (0.0, 0.5), (8.5, 9.5)),
    "e-a1": ("excite", ELECTRON, "O2", M_O2, (5e-22, 3e-21), (0.5, 2.0), (0.5, 1.5), (0.977, 0.977)),
    "e-b1": ("excite", ELECTRON, "O2", M_O2, (1e-22, 1e-21), (0.5, 2.0), (0.5, 1.5), (1.627, 1.627)),
    "e-recomb": ("recomb", ELECTRON, "grid+", M_O2PLUS, (1e-20, 1e-19), (0.0, 0.0), (1.0, 1.5), (0.0, 0.0)),
    "e-edet": ("edetach", ELECTRON, "grid-", M_OMINUS, (1e-20, 1e-19), (1.0, 2.0), (0.0, 0.5), (1.461, 1.461)),
}


def make_processes_full(seed: int = TABLE_SEED) -> List[Process]:
    """All sixteen channels of Table 1 that have a model here: e + O2 elastic (7),
    vibrational (10), Rydberg (11), dissociation at 6.4 eV (12) and 8.6 eV (13),
    a1Delta_g (14), b1Sigma_g (15), ionisation (21), attachment (18); e + O2+
    recombination (16); e + O- detachment (22); O2+ charge exchange (9); O-
    neutralisation (17), elastic (8), direct (19) and associative (20) detachment."""
    ext = {p.name: p for p in make_processes_extended(seed)}
    rng = np.random.Generator(np.random.PCG64(seed + 2))
    for name, (kind, sp, tgt, tm, s0w, aw, bw, ew) in _FULL_WINDOWS.items():
        s0 = float(math.exp(rng.uniform(math.log(s0w[0]), math.log(s0w[1]))))
        a = float(rng.uniform(*aw))
        b = float(rng.uniform(*bw))
        eth = float(rng.uniform(*ew))
        ext[name] = Process(name, sp, kind, tgt, eth, tm, power_law_table(s0, a, b, eth),
                            dict(sigma0=s0, a=a, b=b, e_th=eth))
    order = ["e-elastic", "e-vib", "e-ryd", "e-diss6.4", "e-diss8.6", "e-a1", "e-b1", "e-ion", "e-att",
             "e-recomb", "e-edet", "O2+-cx", "O--neut", "O--el", "O--dd", "O--ad"]
    return [ext[n] for n in order]


def constant_process(name, species, kind, target, sigma, e_th=0.0, target_mass=M_O2) -> Process:
    """A table with one constant cross section (test inputs)."""
    tab = np.full(TABLE_N, float(sigma))
    if e_th > 0:
        tab[energy_grid() <= e_th] = 0.0
    return Process(name, species, kind, target, e_th, target_mass, tab, dict(sigma0=sigma, a=0, b=0, e_th=e_th))


# --- the five workloads -----------------------------------------------------

def config(i: int, **over) -> Discharge:
    """Workload i (1-based).

    1: small FP64-checkable discharge, 128 cells, 30k superparticles.
    2: working size, 512 cells, 600k superparticles (parity case).
    3: large throughput discharge, 4096 cells, 4.8e7 superparticles.
    4: one member of the batched sweep (drawn by sweep_member()).
    """
    if i == 1:
        d = Discharge("cfg1-128cells-30k", L=0.025, ng=128, U=200.0, f=13.56e6, p=20.0,
                      steps_per_cycle=400, ksub=10, cycles=20, n_plus0=1e15, frac_minus=0.5,
                      n_total=30000, sort_every=20, diag_every=20, seed=1001)
    elif i == 2:
        d = Discharge("cfg2-512cells-600k", L=0.025, ng=512, U=400.0, f=13.56e6, p=40.0,
                      steps_per_cycle=2000, ksub=20, cycles=200, n_plus0=1e15, frac_minus=0.5,
                      n_total=600000, sort_every=20, diag_every=20, seed=2001)
    elif i == 3:
        d = Discharge("cfg3-4096cells-4.8e7", L=0.04, ng=4096, U=500.0, f=13.56e6, p=100.0,
                      steps_per_cycle=2000, ksub=20, cycles=50, n_plus0=1e15, frac_minus=2.0 / 3.0,
                      counts=(8_000_000, 24_000_000, 16_000_000), sort_every=20, diag_every=100,
                      seed=3001, capacities=(96_000_000, 96_000_000, 24_000_000))
    else:
        raise ValueError("workload index must be 1, 2 or 3 (use sweep_member for the batch)")
    return dataclasses.replace(d, **over)


def sweep_member(j: int, seed: int = 4000, **over) -> Discharge:
    """Member j of the batched sweep: U ~ U[100,600] V, p ~ logU[5,100] Pa,
    cells ~ U{256..1024}, superparticles per species ~ logU[5e4, 2e6]."""
    rng = np.random.Generator(np.random.PCG64(seed * 1000 + j))
    U = float(rng.uniform(100.0, 600.0))
    p = float(math.exp(rng.uniform(math.log(5.0), math.log(100.0))))
    ng = int(rng.integers(256, 1025))
    nps = float(math.exp(rng.uniform(math.log(5e4), math.log(2e6))))
    d = Discharge(f"sweep{j}", L=0.025, ng=ng, U=U, f=13.56e6, p=p, steps_per_cycle=2000,
                  ksub=20, cycles=1, n_plus0=1e15, frac_minus=0.5, n_total=int(3 * nps),
                  seed=seed + j)
    d = dataclasses.replace(d, **over)
    if "capacities" not in over:
        # electrons and O2+ multiply several-fold on the way from the uniform load
        # to the driven steady state; O- are lost to neutralisation and detachment
        c = d.species_counts()
        d = dataclasses.replace(d, capacities=(12 * c[0] + 4096, 12 * c[1] + 4096, 4 * c[2] + 4096))
    return d
