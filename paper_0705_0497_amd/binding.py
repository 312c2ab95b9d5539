"""Thin ctypes binding of include/pic.h.

Argument marshalling only: every step of the method runs in the HIP kernels of
libpicmcc.so.  PyTorch supplies the device workspace and the stream.  There is
no fallback: if the library is missing or no gfx950 device is present, calls
raise.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpicmcc.so")

PIC_OK, PIC_EINVAL, PIC_ECAPACITY, PIC_EIDOVERFLOW, PIC_ENAN, PIC_EHIP, PIC_ENODEVICE = 0, -1, -2, -3, -5, -6, -7
PIC_EBUSY = -8
PIC_WFALLBACK = 1
TUNE_MAX = 32
KIND = {"elastic": 0, "excite": 1, "ionize": 2, "attach": 3, "cx": 4, "neutralize": 5, "detach": 6,
        "ion_elastic": 7, "recomb": 8, "edetach": 9}
TARGET = {"O2": 0, "O2a": 1, "grid+": 2, "grid-": 3}
EV_EION = 3          # species field of the event records of the electron-ion test
F_EXT_FIELD, F_NO_COLL = 1, 2
NBIN, NCOUNT = 256, 44
C_PUSH, C_CAND, C_NULL, C_ABS0, C_ABSL, C_BORN, C_EVENT = 0, 3, 6, 9, 12, 15, 18
C_PAIRED, C_DEFICIT, C_CLAMP, C_REDRAW = 34, 35, 36, 37
C_EICAND, C_EINULL, C_PAIRED_NEG, C_DEFICIT_NEG = 38, 39, 40, 41

EXPORTS = ("pic_version", "pic_query", "pic_create", "pic_destroy", "pic_load_uniform", "pic_load_profiles",
           "pic_set_particles",
           "pic_count", "pic_get_particles", "pic_prepare", "pic_set_step", "pic_get_step", "pic_step",
           "pic_sync", "pic_moments", "pic_get_hist", "pic_get_field", "pic_get_counters", "pic_get_events",
           "pic_nu_max", "pic_step_timed", "pic_strerror", "pic_last_error",
           "pic_batch_query", "pic_batch_create", "pic_batch_step_cycles", "pic_batch_sync",
           "pic_batch_set_config", "pic_batch_get_config", "pic_batch_autotune", "pic_batch_destroy",
           "pic_batch_last_error", "pic_ksub_select", "pic_metastable_config", "pic_metastable_update")
MLP_EXPORTS = ("mlp_query", "mlp_create", "mlp_destroy", "mlp_set_params", "mlp_get_params", "mlp_forward",
               "mlp_forward_static", "mlp_backward", "mlp_get_grads", "mlp_adam", "mlp_last_error")
MLP_NPARAM = 199942
MLP_STATIC_MAX_BATCH = 4096      # largest batch of mlp_forward_static


class PicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class pic_config(C.Structure):
    _fields_ = [("L", C.c_double), ("ng", C.c_int32), ("U", C.c_double), ("f", C.c_double), ("p", C.c_double),
                ("t_gas", C.c_double), ("steps_per_cycle", C.c_int32), ("ksub", C.c_int32), ("c_meta", C.c_double),
                ("seed", C.c_uint64), ("weight", C.c_double), ("diag_every", C.c_int32),
                ("sort_every", C.c_int32), ("flags", C.c_int32),
                ("e_ext0", C.c_double), ("e_ext1", C.c_double), ("table_emin", C.c_double),
                ("table_emax", C.c_double), ("table_n", C.c_int32), ("max_products", C.c_int32),
                ("event_capacity", C.c_int32), ("block", C.c_int32), ("grid", C.c_int32),
                ("sort_kind", C.c_int32)]


class pic_species(C.Structure):
    _fields_ = [("charge", C.c_double), ("mass", C.c_double), ("t0_ev", C.c_double), ("count", C.c_int64),
                ("capacity", C.c_int64)]


class pic_process(C.Structure):
    _fields_ = [("species", C.c_int32), ("kind", C.c_int32), ("target", C.c_int32), ("e_th", C.c_double),
                ("target_mass", C.c_double), ("sigma", C.POINTER(C.c_double))]


class pic_metastable(C.Structure):
    _fields_ = [("source_process", C.c_int32), ("diffusion", C.c_double), ("quench_rate", C.c_double),
                ("surface_loss", C.c_double)]


class pic_moments_out(C.Structure):
    _fields_ = [("sum_q", C.c_void_p), ("sum_phi", C.c_void_p), ("esum", C.c_void_p), ("ecnt", C.c_void_p),
                ("edf", C.c_void_p), ("iedf", C.c_void_p), ("nacc", C.c_int64), ("ndiag", C.c_int64),
                ("current", C.c_void_p), ("current_n", C.c_void_p), ("power_sum", C.c_double),
                ("power_n", C.c_int64)]


class pic_batch_config(C.Structure):
    _fields_ = [("block", C.c_int32), ("sort_every", C.c_int32), ("use_graph", C.c_int32), ("grid", C.c_int32)]


class pic_batch_tuning(C.Structure):
    _fields_ = [("n", C.c_int32), ("block", C.c_int32 * TUNE_MAX), ("sort_every", C.c_int32 * TUNE_MAX),
                ("ms_per_step", C.c_double * TUNE_MAX), ("best", C.c_int32)]


_lib = None


def lib():
    """The loaded libpicmcc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} missing (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u32, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
        P = C.POINTER
        L.pic_version.restype = i32
        L.pic_query.argtypes = [P(pic_config), P(pic_species), P(pic_process), i32, P(C.c_uint64)]
        L.pic_create.argtypes = [P(pic_config), P(pic_species), P(pic_process), i32, vp, C.c_uint64, vp, P(vp)]
        L.pic_destroy.argtypes = [vp]
        L.pic_load_uniform.argtypes = [vp]
        L.pic_load_profiles.argtypes = [vp, i32, vp, vp, vp]
        L.pic_set_particles.argtypes = [vp, i32, i64, vp, vp, vp, vp, vp, vp, vp, u32]
        L.pic_count.argtypes = [vp, i32, P(i64)]
        L.pic_get_particles.argtypes = [vp, i32, P(i64), vp, vp, vp, vp, vp, vp, vp, P(u32)]
        L.pic_prepare.argtypes = [vp, i32]
        L.pic_set_step.argtypes = [vp, i64]
        L.pic_get_step.argtypes = [vp, P(i64)]
        L.pic_step.argtypes = [vp, i64]
        L.pic_sync.argtypes = [vp]
        L.pic_moments.argtypes = [vp, P(pic_moments_out), i32]
        L.pic_get_hist.argtypes = [vp, vp]
        L.pic_get_field.argtypes = [vp, vp, vp]
        L.pic_get_counters.argtypes = [vp, vp]
        L.pic_get_events.argtypes = [vp, i64, vp, P(i64), i32]
        L.pic_nu_max.argtypes = [vp, i32, P(dbl)]
        L.pic_metastable_config.argtypes = [vp, P(pic_metastable)]
        L.pic_metastable_update.argtypes = [vp, vp]
        L.pic_step_timed.argtypes = [vp, i64, P(dbl), P(dbl), P(i64)]
        L.pic_strerror.restype = C.c_char_p
        L.pic_strerror.argtypes = [i32]
        L.pic_last_error.restype = C.c_char_p
        L.pic_last_error.argtypes = [vp]
        L.pic_batch_query.argtypes = [i32, P(C.c_uint64)]
        L.pic_batch_create.argtypes = [P(vp), i32, P(pic_batch_config), vp, C.c_uint64, vp, P(vp)]
        L.pic_batch_step_cycles.argtypes = [vp, i64]
        L.pic_batch_sync.argtypes = [vp]
        L.pic_batch_set_config.argtypes = [vp, P(pic_batch_config)]
        L.pic_batch_get_config.argtypes = [vp, P(pic_batch_config)]
        L.pic_batch_autotune.argtypes = [vp, i32, P(pic_batch_tuning)]
        L.pic_batch_destroy.argtypes = [vp]
        L.pic_batch_last_error.restype = C.c_char_p
        L.pic_batch_last_error.argtypes = [vp]
        L.pic_ksub_select.argtypes = [P(pic_config), P(pic_species), dbl, dbl, P(i32)]
        L.mlp_query.argtypes = [i32, P(C.c_uint64)]
        L.mlp_create.argtypes = [i32, vp, C.c_uint64, vp, P(vp)]
        L.mlp_destroy.argtypes = [vp]
        L.mlp_set_params.argtypes = [vp, vp]
        L.mlp_get_params.argtypes = [vp, vp]
        L.mlp_forward.argtypes = [vp, i32, vp, vp]
        L.mlp_forward_static.argtypes = [vp, i32, vp, vp]
        L.mlp_backward.argtypes = [vp, i32, vp, vp, vp]
        L.mlp_get_grads.argtypes = [vp, vp]
        L.mlp_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float]
        L.mlp_last_error.restype = C.c_char_p
        L.mlp_last_error.argtypes = [vp]
        _lib = L
    return _lib


def _check(code, h=None):
    if code != PIC_OK:
        msg = lib().pic_last_error(h).decode() or lib().pic_strerror(code).decode()
        raise PicError(code, msg)


def _bcheck(code, b=None):
    if code != PIC_OK:
        msg = lib().pic_batch_last_error(b).decode() or lib().pic_strerror(code).decode()
        raise PicError(code, msg)


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


# ---------------------------------------------------------------- struct builders
SORT_CELL, SORT_COMPACT = 0, 1


def make_config(d, flags=0, e_ext=(0.0, 0.0), seed=None, max_products=None, event_capacity=0, block=0, grid=0,
                sort_every=None, diag_every=None, table=(1e-3, 1e3, 512), sort_kind=None):
    if max_products is None:
        max_products = int(min(1 << 24, max(4096, sum(d.species_counts()) // 16)))
    return pic_config(L=d.L, ng=d.ng, U=d.U, f=d.f, p=d.p, t_gas=d.t_gas, steps_per_cycle=d.steps_per_cycle,
                      ksub=d.ksub, c_meta=d.c_meta, seed=int(d.seed if seed is None else seed) & (2 ** 64 - 1),
                      weight=d.weight, diag_every=d.diag_every if diag_every is None else diag_every,
                      sort_every=d.sort_every if sort_every is None else sort_every,
                      flags=flags, e_ext0=e_ext[0], e_ext1=e_ext[1], table_emin=table[0], table_emax=table[1],
                      table_n=table[2], max_products=max_products, event_capacity=event_capacity, block=block,
                      grid=grid, sort_kind=getattr(d, "sort_kind", SORT_CELL) if sort_kind is None else sort_kind)


def make_species(species):
    return (pic_species * 3)(*[pic_species(s.charge, s.mass, s.t0_ev, s.count, s.capacity) for s in species])


def make_processes(procs):
    tabs = [np.ascontiguousarray(p.sigma, dtype=np.float64) for p in procs]
    arr = (pic_process * max(1, len(procs)))(*[
        pic_process(p.species, KIND[p.kind], TARGET[p.target], p.e_th, p.target_mass,
                    t.ctypes.data_as(C.POINTER(C.c_double))) for p, t in zip(procs, tabs)])
    return arr, tabs


# ---------------------------------------------------------------- C ABI, same names
def pic_version():
    return lib().pic_version()


def pic_query(cfg, sp, pr, nproc):
    n = C.c_uint64(0)
    _check(lib().pic_query(C.byref(cfg), sp, pr, nproc, C.byref(n)))
    return n.value


def pic_create(cfg, sp, pr, nproc, workspace_ptr, nbytes, stream_ptr):
    h = C.c_void_p()
    _check(lib().pic_create(C.byref(cfg), sp, pr, nproc, C.c_void_p(workspace_ptr), nbytes,
                            C.c_void_p(stream_ptr), C.byref(h)))
    return h


def pic_destroy(h):
    _check(lib().pic_destroy(h))


def pic_load_uniform(h):
    _check(lib().pic_load_uniform(h), h)


def pic_load_profiles(h, x, dens, mean_ev):
    """Returns True if the profile was used, False after the uniform fallback."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    dens = np.ascontiguousarray(dens, dtype=np.float64)
    mean_ev = np.ascontiguousarray(mean_ev, dtype=np.float64)
    if dens.shape != (3, len(x)) or mean_ev.shape != (3, len(x)):
        raise ValueError("dens and mean_ev must be [3][n_pts]")
    code = lib().pic_load_profiles(h, len(x), _ptr(x), _ptr(dens), _ptr(mean_ev))
    if code == PIC_WFALLBACK:
        return False
    _check(code, h)
    return True


def pic_set_particles(h, s, st, next_id):
    n = len(st["id"])
    a = {k: np.ascontiguousarray(st[k], dtype=t) for k, t in
         (("cell", np.int32), ("off", np.float32), ("vx", np.float32), ("vy", np.float32), ("vz", np.float32),
          ("id", np.uint32), ("cd", np.int32))}
    _check(lib().pic_set_particles(h, s, n, _ptr(a["cell"]), _ptr(a["off"]), _ptr(a["vx"]), _ptr(a["vy"]),
                                   _ptr(a["vz"]), _ptr(a["id"]), _ptr(a["cd"]), int(next_id)), h)


def pic_count(h, s):
    n = C.c_int64(0)
    _check(lib().pic_count(h, s, C.byref(n)), h)
    return n.value


def pic_get_particles(h, s, cap=None):
    if cap is None:
        cap = pic_count(h, s)
    n = C.c_int64(cap)
    out = {"cell": np.zeros(cap, np.int32), "off": np.zeros(cap, np.float32), "vx": np.zeros(cap, np.float32),
           "vy": np.zeros(cap, np.float32), "vz": np.zeros(cap, np.float32), "id": np.zeros(cap, np.uint32),
           "cd": np.zeros(cap, np.int32)}
    nid = C.c_uint32(0)
    _check(lib().pic_get_particles(h, s, C.byref(n), _ptr(out["cell"]), _ptr(out["off"]), _ptr(out["vx"]),
                                   _ptr(out["vy"]), _ptr(out["vz"]), _ptr(out["id"]), _ptr(out["cd"]),
                                   C.byref(nid)), h)
    return {k: v[:n.value] for k, v in out.items()}, nid.value


def pic_prepare(h, shift):
    _check(lib().pic_prepare(h, 1 if shift else 0), h)


def pic_set_step(h, step):
    _check(lib().pic_set_step(h, int(step)), h)


def pic_get_step(h):
    n = C.c_int64(0)
    _check(lib().pic_get_step(h, C.byref(n)), h)
    return n.value


def pic_step(h, n_steps):
    _check(lib().pic_step(h, int(n_steps)), h)


def pic_sync(h):
    _check(lib().pic_sync(h), h)


def pic_moments(h, ng, reset=False, steps_per_cycle=1):
    m = {"sum_q": np.zeros((3, ng + 1)), "sum_phi": np.zeros(ng + 1), "esum": np.zeros((3, ng), np.int64),
         "ecnt": np.zeros((3, ng), np.int64), "edf": np.zeros((3, NBIN), np.int64),
         "iedf": np.zeros((3, 2, NBIN), np.int64), "current": np.zeros(steps_per_cycle),
         "current_n": np.zeros(steps_per_cycle, np.int64)}
    o = pic_moments_out(*[_ptr(m[k]) for k in ("sum_q", "sum_phi", "esum", "ecnt", "edf", "iedf")], 0, 0,
                        _ptr(m["current"]), _ptr(m["current_n"]), 0.0, 0)
    _check(lib().pic_moments(h, C.byref(o), 1 if reset else 0), h)
    m["nacc"], m["ndiag"] = o.nacc, o.ndiag
    m["power_sum"], m["power_n"] = o.power_sum, o.power_n
    return m


def pic_get_hist(h, ng):
    q = np.zeros((3, ng + 1), np.int64)
    _check(lib().pic_get_hist(h, _ptr(q)), h)
    return q


def pic_get_field(h, ng):
    phi = np.zeros(ng + 1)
    e = np.zeros(ng + 1, np.float32)
    _check(lib().pic_get_field(h, _ptr(phi), _ptr(e)), h)
    return phi, e


def pic_get_counters(h):
    c = np.zeros(NCOUNT, np.int64)
    _check(lib().pic_get_counters(h, _ptr(c)), h)
    return c


def pic_get_events(h, max_records, clear=False):
    rec = np.zeros((max(1, max_records), 4), np.int64)
    n = C.c_int64(0)
    _check(lib().pic_get_events(h, max_records, _ptr(rec), C.byref(n), 1 if clear else 0), h)
    return rec[:min(n.value, max_records)], n.value


def pic_metastable_config(h, source_process, diffusion, quench_rate, surface_loss):
    m = pic_metastable(int(source_process), float(diffusion), float(quench_rate), float(surface_loss))
    _check(lib().pic_metastable_config(h, C.byref(m)), h)


def pic_metastable_update(h, ng):
    n = np.zeros(ng + 1)
    _check(lib().pic_metastable_update(h, _ptr(n)), h)
    return n


def pic_nu_max(h, s):
    v = C.c_double(0)
    _check(lib().pic_nu_max(h, s, C.byref(v)), h)
    return v.value


def pic_step_timed(h, n_steps):
    a, b, c = C.c_double(0), C.c_double(0), C.c_int64(0)
    _check(lib().pic_step_timed(h, int(n_steps), C.byref(a), C.byref(b), C.byref(c)), h)
    return a.value, b.value, c.value


# ---------------------------------------------------------------- convenience owner of one discharge
class Discharge:
    """One discharge on the current GPU: builds the C structs from a workload
    description (see inputs.Discharge), allocates the workspace as a torch
    uint8 tensor and runs everything through the C ABI above."""

    def __init__(self, d, procs, species=None, flags=0, e_ext=(0.0, 0.0), seed=None, max_products=None,
                 event_capacity=0, block=0, grid=0, sort_every=None, diag_every=None, stream=None, sort_kind=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the PIC-MCC path runs only on a gfx950 device")
        self.d = d
        self.ng = d.ng
        self.cfg = make_config(d, flags, e_ext, seed, max_products, event_capacity, block, grid, sort_every,
                               diag_every, sort_kind=sort_kind)
        self.species = species if species is not None else d.species()
        self.sp = make_species(self.species)
        self.pr, self._tabs = make_processes(procs)
        self.nproc = len(procs)
        self.event_capacity = event_capacity
        nbytes = pic_query(self.cfg, self.sp, self.pr, self.nproc)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.h = pic_create(self.cfg, self.sp, self.pr, self.nproc, self.workspace.data_ptr(), nbytes,
                            self.stream.cuda_stream)

    def close(self):
        if getattr(self, "h", None):
            pic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_uniform(self):
        pic_load_uniform(self.h)

    def load_profiles(self, x, dens, mean_ev):
        return pic_load_profiles(self.h, x, dens, mean_ev)

    def set_particles(self, s, st, next_id):
        pic_set_particles(self.h, s, st, next_id)

    def get_particles(self, s):
        return pic_get_particles(self.h, s)

    def count(self, s):
        return pic_count(self.h, s)

    def prepare(self, shift=True):
        pic_prepare(self.h, shift)

    def set_step(self, n):
        pic_set_step(self.h, n)

    @property
    def step_index(self):
        return pic_get_step(self.h)

    def step(self, n=1):
        pic_step(self.h, n)

    def sync(self):
        pic_sync(self.h)

    def moments(self, reset=False):
        return pic_moments(self.h, self.ng, reset, self.d.steps_per_cycle)

    def hist(self):
        return pic_get_hist(self.h, self.ng)

    def field(self):
        return pic_get_field(self.h, self.ng)

    def counters(self):
        return pic_get_counters(self.h)

    def clear_events(self):
        pic_get_events(self.h, 0, True)

    def events(self, clear=True):
        rec, n = pic_get_events(self.h, self.event_capacity, clear)
        if n > self.event_capacity:
            raise RuntimeError(f"event log overflow: {n} > {self.event_capacity}")
        return rec

    def nu_max(self, s):
        return pic_nu_max(self.h, s)

    def metastable_config(self, source_process, diffusion, quench_rate, surface_loss):
        """Spatially resolved O2(a): production by process index source_process,
        diffusion [m^2/s], volume loss [1/s], surface loss probability."""
        pic_metastable_config(self.h, source_process, diffusion, quench_rate, surface_loss)

    def metastable_update(self):
        """Solve the O2(a) profile from the production since the last update; [ng + 1] m^-3."""
        return pic_metastable_update(self.h, self.ng)

    def step_timed(self, n):
        return pic_step_timed(self.h, n)


# ---------------------------------------------------------------- batches, same names
def pic_batch_query(n_members):
    n = C.c_uint64(0)
    _bcheck(lib().pic_batch_query(int(n_members), C.byref(n)))
    return n.value


def pic_batch_create(handles, cfg, workspace_ptr, nbytes, stream_ptr):
    arr = (C.c_void_p * len(handles))(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    b = C.c_void_p()
    _bcheck(lib().pic_batch_create(arr, len(handles), C.byref(cfg), C.c_void_p(workspace_ptr), nbytes,
                                   C.c_void_p(stream_ptr), C.byref(b)))
    return b


def pic_batch_step_cycles(b, cycles):
    _bcheck(lib().pic_batch_step_cycles(b, int(cycles)), b)


def pic_batch_sync(b):
    _bcheck(lib().pic_batch_sync(b), b)


def pic_batch_set_config(b, cfg):
    _bcheck(lib().pic_batch_set_config(b, C.byref(cfg)), b)


def pic_batch_get_config(b):
    c = pic_batch_config()
    _bcheck(lib().pic_batch_get_config(b, C.byref(c)), b)
    return c


def pic_batch_autotune(b, window):
    t = pic_batch_tuning()
    _bcheck(lib().pic_batch_autotune(b, int(window), C.byref(t)), b)
    return t


def pic_batch_destroy(b):
    _bcheck(lib().pic_batch_destroy(b))


def pic_ksub_select(cfg, sp, n_ion_max, phi_max):
    k = C.c_int32(0)
    _check(lib().pic_ksub_select(C.byref(cfg), sp, float(n_ion_max), float(phi_max), C.byref(k)))
    return k.value


class Batch:
    """Discharges advanced together (one launch per kernel per step, one HIP
    graph per rf cycle).  `members` are Discharge objects created on one
    non-default stream; they are handed back by sync()."""

    def __init__(self, members, block=0, sort_every=20, use_graph=True, grid=0):
        import torch
        self.members = list(members)
        self.stream = self.members[0].stream
        nbytes = pic_batch_query(len(self.members))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.cfg = pic_batch_config(block, sort_every, 1 if use_graph else 0, grid)
        self.b = pic_batch_create([m.h for m in self.members], self.cfg, self.workspace.data_ptr(), nbytes,
                                  self.stream.cuda_stream)

    def step_cycles(self, n=1):
        pic_batch_step_cycles(self.b, n)

    def sync(self):
        pic_batch_sync(self.b)

    def config(self):
        c = pic_batch_get_config(self.b)
        return {"block": c.block, "sort_every": c.sort_every, "use_graph": bool(c.use_graph), "grid": c.grid}

    def set_config(self, block=None, sort_every=None, use_graph=None, grid=None):
        c = pic_batch_get_config(self.b)
        if block is not None:
            c.block = block
        if sort_every is not None:
            c.sort_every = sort_every
        if use_graph is not None:
            c.use_graph = 1 if use_graph else 0
        if grid is not None:
            c.grid = grid
        pic_batch_set_config(self.b, c)

    def autotune(self, window=200):
        t = pic_batch_autotune(self.b, window)
        trials = [{"block": t.block[i], "sort_every": t.sort_every[i], "ms_per_step": t.ms_per_step[i]}
                  for i in range(t.n)]
        return {"trials": trials, "best": trials[t.best] if t.n else None}

    def close(self):
        if getattr(self, "b", None):
            pic_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- warm-start network, same names
def _mcheck(code, h=None):
    if code != PIC_OK:
        msg = lib().mlp_last_error(h).decode() or lib().pic_strerror(code).decode()
        raise PicError(code, msg)


def mlp_query(max_batch):
    n = C.c_uint64(0)
    _mcheck(lib().mlp_query(int(max_batch), C.byref(n)))
    return n.value


def mlp_create(max_batch, workspace_ptr, nbytes, stream_ptr):
    h = C.c_void_p()
    _mcheck(lib().mlp_create(int(max_batch), C.c_void_p(workspace_ptr), nbytes, C.c_void_p(stream_ptr), C.byref(h)))
    return h


def mlp_destroy(h):
    _mcheck(lib().mlp_destroy(h))


def mlp_set_params(h, p):
    a = np.ascontiguousarray(p, dtype=np.float32)
    if a.size != MLP_NPARAM:
        raise ValueError(f"need {MLP_NPARAM} parameters")
    _mcheck(lib().mlp_set_params(h, _ptr(a)), h)


def mlp_get_params(h):
    a = np.zeros(MLP_NPARAM, np.float32)
    _mcheck(lib().mlp_get_params(h, _ptr(a)), h)
    return a


def mlp_forward(h, batch, x_ptr, y_ptr):
    _mcheck(lib().mlp_forward(h, int(batch), C.c_void_p(x_ptr), C.c_void_p(y_ptr)), h)


def mlp_forward_static(h, batch, x_ptr, y_ptr):
    """Inference with the activations in the library's static per-device array
    (no allocation, no copy); batch <= MLP_STATIC_MAX_BATCH."""
    _mcheck(lib().mlp_forward_static(h, int(batch), C.c_void_p(x_ptr), C.c_void_p(y_ptr)), h)


def mlp_backward(h, batch, x_ptr, t_ptr, want_loss=True):
    loss = C.c_float(0.0)
    _mcheck(lib().mlp_backward(h, int(batch), C.c_void_p(x_ptr), C.c_void_p(t_ptr),
                               C.byref(loss) if want_loss else None), h)
    return loss.value if want_loss else None


def mlp_get_grads(h):
    a = np.zeros(MLP_NPARAM, np.float32)
    _mcheck(lib().mlp_get_grads(h, _ptr(a)), h)
    return a


def mlp_adam(h, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _mcheck(lib().mlp_adam(h, float(lr), float(beta1), float(beta2), float(eps)), h)


class Network:
    """The warm-start network on the current GPU (torch workspace and stream)."""

    def __init__(self, max_batch, params=None, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the network kernels run only on a gfx950 device")
        self.max_batch = int(max_batch)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        nbytes = mlp_query(self.max_batch)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        self.h = mlp_create(self.max_batch, self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)
        if params is not None:
            self.set_params(params)

    def set_params(self, p):
        mlp_set_params(self.h, p)

    def params(self):
        return mlp_get_params(self.h)

    def forward(self, x):
        """x: float32 CUDA tensor [B][3] -> float32 CUDA tensor [B][6]."""
        import torch
        x = x.contiguous()
        y = torch.empty((x.shape[0], 6), dtype=torch.float32, device=x.device)
        for b0 in range(0, x.shape[0], self.max_batch):
            b1 = min(x.shape[0], b0 + self.max_batch)
            mlp_forward(self.h, b1 - b0, x[b0:b1].data_ptr(), y[b0:b1].data_ptr())
        return y

    def backward(self, x, t, want_loss=True):
        x, t = x.contiguous(), t.contiguous()
        return mlp_backward(self.h, x.shape[0], x.data_ptr(), t.data_ptr(), want_loss)

    def grads(self):
        return mlp_get_grads(self.h)

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        mlp_adam(self.h, lr, beta1, beta2, eps)

    def close(self):
        if getattr(self, "h", None):
            mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
