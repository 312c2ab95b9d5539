"""ctypes access to the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
baseline leg of the benchmark.  The product path never imports this module.
It imports nothing from the product package: callers pass the discharge,
species and process descriptions as plain objects.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "oracle.c")]

KIND = {"elastic": 0, "excite": 1, "ionize": 2, "attach": 3, "cx": 4, "neutralize": 5, "detach": 6,
        "ion_elastic": 7, "recomb": 8, "edetach": 9}
TARGET = {"O2": 0, "O2a": 1, "grid+": 2, "grid-": 3}
EV_EION = 3          # species field of the event records of the electron-ion test
F_EXT_FIELD, F_NO_COLL = 1, 2
CD_MAX, CD_CAP, NBIN = 32767, 0x8000, 256
# counters
C_PUSH, C_CAND, C_NULL, C_ABS0, C_ABSL, C_BORN, C_EVENT = 0, 3, 6, 9, 12, 15, 18
C_PAIRED, C_DEFICIT, C_CLAMP, C_REDRAW = 34, 35, 36, 37
C_EICAND, C_EINULL, C_PAIRED_NEG, C_DEFICIT_NEG, NCOUNT = 38, 39, 40, 41, 44


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no FMA contraction, no fast-math).  This build is the
    reference for stored values: other optimisation levels may call libm in other forms
    (sin and cos fused into sincos) and move a last bit."""
    if force or not os.path.exists(LIB_PATH) or any(
            os.path.getmtime(s) > os.path.getmtime(LIB_PATH) for s in SOURCES):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               *SOURCES, "-o", tmp, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Config(C.Structure):
    _fields_ = [("L", C.c_double), ("ng", C.c_int32), ("U", C.c_double), ("f", C.c_double),
                ("p", C.c_double), ("t_gas", C.c_double), ("steps_per_cycle", C.c_int32),
                ("ksub", C.c_int32), ("c_meta", C.c_double), ("seed", C.c_uint64),
                ("weight", C.c_double), ("diag_every", C.c_int32), ("flags", C.c_int32),
                ("e_ext0", C.c_double), ("e_ext1", C.c_double),
                ("table_emin", C.c_double), ("table_emax", C.c_double), ("table_n", C.c_int32)]


class _Species(C.Structure):
    _fields_ = [("charge", C.c_double), ("mass", C.c_double), ("t0_ev", C.c_double),
                ("count", C.c_int64), ("capacity", C.c_int64)]


class _Process(C.Structure):
    _fields_ = [("species", C.c_int32), ("kind", C.c_int32), ("target", C.c_int32),
                ("e_th", C.c_double), ("target_mass", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u32, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
        L.orc_create.restype = vp
        L.orc_create.argtypes = [C.POINTER(_Config), C.POINTER(_Species), i32, C.POINTER(_Process), vp]
        L.orc_destroy.argtypes = [vp]
        L.orc_load_uniform.argtypes = [vp]
        L.orc_load_profile.argtypes = [vp, i32, vp, vp, vp]
        L.orc_load_profile.restype = i32
        L.orc_get_current.argtypes = [vp, vp, vp, vp, vp]
        L.orc_set_particles.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, vp, vp, u32]
        L.orc_set_particles64.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, vp, u32]
        L.orc_count.restype = i64
        L.orc_count.argtypes = [vp, i32]
        L.orc_next_id.restype = u32
        L.orc_next_id.argtypes = [vp, i32]
        L.orc_get_particles.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp]
        L.orc_set_step.argtypes = [vp, i64]
        L.orc_get_step.restype = i64
        L.orc_get_step.argtypes = [vp]
        L.orc_prepare.argtypes = [vp, i32]
        L.orc_step.argtypes = [vp, i64]
        L.orc_get_hist.argtypes = [vp, vp]
        L.orc_get_field.argtypes = [vp, vp, vp]
        L.orc_set_hist.argtypes = [vp, vp]
        L.orc_get_counters.argtypes = [vp, vp]
        L.orc_nu_max.restype = dbl
        L.orc_nu_max.argtypes = [vp, i32]
        L.orc_info.argtypes = [vp, vp]
        L.orc_sigma.restype = dbl
        L.orc_sigma.argtypes = [vp, i32, dbl]
        L.orc_reset_moments.argtypes = [vp]
        L.orc_sample_moments.argtypes = [vp]
        L.orc_get_moments.restype = i64
        L.orc_get_moments.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_log_events.argtypes = [vp, i32]
        L.orc_get_events.restype = i64
        L.orc_get_events.argtypes = [vp, i64, vp]
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_poisson.argtypes = [i32, dbl, dbl, vp, vp, vp]
        L.orc_deposit_canonical.argtypes = [i32, i64, vp, vp, vp]
        L.orc_metastable_config.restype = i32
        L.orc_metastable_config.argtypes = [vp, i32, dbl, dbl, dbl]
        L.orc_metastable_update.restype = i32
        L.orc_metastable_update.argtypes = [vp, vp]
        L.orc_metastable_tally.argtypes = [vp, vp]
        L.orc_metastable_set.restype = i32
        L.orc_metastable_set.argtypes = [vp, vp]
        L.orc_metastable_solve.argtypes = [i32, dbl, dbl, dbl, dbl, vp, vp]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def metastable_solve(ng, dx, D, nu_q, h, prod):
    """Steady O2(a) profile on the nodes for a production rate per node [m^-3 s^-1]."""
    prod = np.ascontiguousarray(prod, dtype=np.float64)
    n = np.zeros(ng + 1)
    lib().orc_metastable_solve(int(ng), float(dx), float(D), float(nu_q), float(h), _p(prod), _p(n))
    return n


def philox(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def poisson(ng, dx, phi0, rho):
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    phi = np.zeros(ng + 1)
    E = np.zeros(ng + 1)
    lib().orc_poisson(ng, dx, phi0, _p(rho), _p(phi), _p(E))
    return phi, E


def deposit_canonical(ng, cell, off):
    cell = np.ascontiguousarray(cell, dtype=np.int32)
    off = np.ascontiguousarray(off, dtype=np.float32)
    Q = np.zeros(ng + 1, dtype=np.int64)
    lib().orc_deposit_canonical(ng, len(cell), _p(cell), _p(off), _p(Q))
    return Q


class Oracle:
    """One FP64 discharge.  `d` has the Discharge fields, `species` a list of 3
    objects with charge/mass/t0_ev/count/capacity, `procs` objects with
    species/kind/target/e_th/target_mass/sigma."""

    def __init__(self, d, species, procs, flags=0, e_ext=(0.0, 0.0), seed=None,
                 table=(1e-3, 1e3, 512)):
        self.d = d
        self.ng = d.ng
        cfg = _Config(L=d.L, ng=d.ng, U=d.U, f=d.f, p=d.p, t_gas=d.t_gas,
                      steps_per_cycle=d.steps_per_cycle, ksub=d.ksub, c_meta=d.c_meta,
                      seed=int(d.seed if seed is None else seed) & (2**64 - 1), weight=d.weight,
                      diag_every=d.diag_every, flags=flags,
                      e_ext0=e_ext[0], e_ext1=e_ext[1], table_emin=table[0], table_emax=table[1],
                      table_n=table[2])
        sp = (_Species * 3)(*[_Species(s.charge, s.mass, s.t0_ev, s.count, s.capacity) for s in species])
        pr = (_Process * max(1, len(procs)))(*[_Process(p.species, KIND[p.kind], TARGET[p.target], p.e_th,
                                                        p.target_mass) for p in procs])
        self.sigma = np.ascontiguousarray(np.stack([p.sigma for p in procs]) if procs else np.zeros((1, table[2])),
                                          dtype=np.float64)
        self.nproc = len(procs)
        self.h = lib().orc_create(C.byref(cfg), sp, len(procs), pr, _p(self.sigma))
        if not self.h:
            raise ValueError("oracle rejected the configuration")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def load_uniform(self):
        lib().orc_load_uniform(self.h)

    def load_profile(self, x, dens, mean_ev):
        """Warm-start loading from profiles (x / L, densities [3][n], mean energies [3][n])."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        dens = np.ascontiguousarray(dens, dtype=np.float64)
        mean_ev = np.ascontiguousarray(mean_ev, dtype=np.float64)
        if lib().orc_load_profile(self.h, len(x), _p(x), _p(dens), _p(mean_ev)) != 0:
            raise ValueError("invalid profile")

    def set_particles(self, s, st, next_id):
        n = len(st["id"])
        a = {k: np.ascontiguousarray(st[k], dtype=t) for k, t in
             (("cell", np.int32), ("off", np.float32), ("vx", np.float32), ("vy", np.float32),
              ("vz", np.float32), ("id", np.uint32), ("cd", np.int32))}
        lib().orc_set_particles(self.h, s, n, _p(a["cell"]), _p(a["off"]), _p(a["vx"]), _p(a["vy"]),
                                _p(a["vz"]), _p(a["id"]), _p(a["cd"]), int(next_id))

    def set_particles64(self, s, st, next_id):
        n = len(st["id"])
        a = {k: np.ascontiguousarray(st[k], dtype=t) for k, t in
             (("xi", np.float64), ("vx", np.float64), ("vy", np.float64), ("vz", np.float64),
              ("id", np.uint32), ("cd", np.int32))}
        lib().orc_set_particles64(self.h, s, n, _p(a["xi"]), _p(a["vx"]), _p(a["vy"]), _p(a["vz"]),
                                  _p(a["id"]), _p(a["cd"]), int(next_id))

    def count(self, s):
        return lib().orc_count(self.h, s)

    def next_id(self, s):
        return lib().orc_next_id(self.h, s)

    def get_particles(self, s):
        n = self.count(s)
        out = {"xi": np.zeros(n), "vx": np.zeros(n), "vy": np.zeros(n), "vz": np.zeros(n),
               "id": np.zeros(n, dtype=np.uint32), "cd": np.zeros(n, dtype=np.int32)}
        lib().orc_get_particles(self.h, s, _p(out["xi"]), _p(out["vx"]), _p(out["vy"]), _p(out["vz"]),
                                _p(out["id"]), _p(out["cd"]))
        return out

    def canonical(self, s):
        """The state rounded to the single-precision exchange record."""
        p = self.get_particles(s)
        cell = np.floor(p["xi"]).astype(np.int32)
        off = (p["xi"] - cell).astype(np.float32)
        # rounding may carry the offset to 1.0: move to the next cell
        carry = off >= np.float32(1.0)
        cell[carry] += 1
        off[carry] = np.float32(0.0)
        return {"cell": cell, "off": off, "vx": p["vx"].astype(np.float32), "vy": p["vy"].astype(np.float32),
                "vz": p["vz"].astype(np.float32), "id": p["id"], "cd": p["cd"]}

    def set_step(self, n):
        lib().orc_set_step(self.h, n)

    @property
    def step_index(self):
        return lib().orc_get_step(self.h)

    def prepare(self, shift=True):
        lib().orc_prepare(self.h, 1 if shift else 0)

    def step(self, n=1):
        lib().orc_step(self.h, n)

    def hist(self):
        Q = np.zeros((3, self.ng + 1), dtype=np.int64)
        lib().orc_get_hist(self.h, _p(Q))
        return Q

    def set_hist(self, Q):
        Q = np.ascontiguousarray(Q, dtype=np.int64)
        lib().orc_set_hist(self.h, _p(Q))

    def field(self):
        phi = np.zeros(self.ng + 1)
        E = np.zeros(self.ng + 1)
        lib().orc_get_field(self.h, _p(phi), _p(E))
        return phi, E

    def counters(self):
        c = np.zeros(NCOUNT, dtype=np.int64)
        lib().orc_get_counters(self.h, _p(c))
        return c

    def nu_max(self, s):
        return lib().orc_nu_max(self.h, s)

    def info(self):
        o = np.zeros(6)
        lib().orc_info(self.h, _p(o))
        return dict(dx=o[0], dt=o[1], n_o2=o[2], nu_max=tuple(o[3:6]))

    def sigma_at(self, p, e):
        return lib().orc_sigma(self.h, p, e)

    def reset_moments(self):
        lib().orc_reset_moments(self.h)

    def sample_moments(self):
        """Adds one sample of the energy moments of the state as it is."""
        lib().orc_sample_moments(self.h)

    def moments(self):
        ng = self.ng
        sumQ = np.zeros((3, ng + 1))
        sumphi = np.zeros(ng + 1)
        esum = np.zeros((3, ng), dtype=np.int64)
        ecnt = np.zeros((3, ng), dtype=np.int64)
        edf = np.zeros((3, NBIN), dtype=np.int64)
        iedf = np.zeros((3, 2, NBIN), dtype=np.int64)
        nd = np.zeros(1, dtype=np.int64)
        nacc = lib().orc_get_moments(self.h, _p(sumQ), _p(sumphi), _p(esum), _p(ecnt), _p(edf), _p(iedf), _p(nd))
        return dict(nacc=nacc, sumQ=sumQ, sumphi=sumphi, esum=esum, ecnt=ecnt, edf=edf, iedf=iedf,
                    ndiag=int(nd[0]))

    def current(self):
        """Current density at the driven electrode: per-phase sums and counts over
        the rf cycle, and the sum of U j over the samples with its count."""
        spc = self.d.steps_per_cycle
        js = np.zeros(spc)
        jc = np.zeros(spc, dtype=np.int64)
        ps = np.zeros(1)
        pn = np.zeros(1, dtype=np.int64)
        lib().orc_get_current(self.h, _p(js), _p(jc), _p(ps), _p(pn))
        return {"jsum": js, "jcnt": jc, "psum": float(ps[0]), "pn": int(pn[0])}

    def metastable_config(self, proc, D, nu_q, gamma):
        """Spatially resolved O2(a): production by process index proc, diffusion D
        [m^2/s], volume loss nu_q [1/s], surface loss probability gamma."""
        if lib().orc_metastable_config(self.h, int(proc), float(D), float(nu_q), float(gamma)) != 0:
            raise ValueError("invalid metastable configuration")

    def metastable_update(self):
        n = np.zeros(self.ng + 1)
        if lib().orc_metastable_update(self.h, _p(n)) != 0:
            raise ValueError("metastable update without configuration or tally window")
        return n

    def metastable_set(self, n):
        """Test hook: use the given O2(a) profile [ng + 1] (after metastable_config)."""
        n = np.ascontiguousarray(n, dtype=np.float64)
        if lib().orc_metastable_set(self.h, _p(n)) != 0:
            raise ValueError("metastable_set before metastable_config")

    def metastable_tally(self):
        q = np.zeros(self.ng + 1, dtype=np.int64)
        lib().orc_metastable_tally(self.h, _p(q))
        return q

    def log_events(self, on=True):
        lib().orc_log_events(self.h, 1 if on else 0)

    def events(self):
        n = lib().orc_get_events(self.h, 0, None)
        rec = np.zeros((max(n, 1), 6), dtype=np.int64)
        lib().orc_get_events(self.h, n, _p(rec))
        return rec[:n]
