"""The C-ABI library loads, exports every symbol include/pic.h declares, and
validates configurations on the host (no device call)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_0705_0497_amd import binding as B
from paper_0705_0497_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared(header="pic.h", prefix="pic_"):
    text = open(os.path.join(ROOT, "include", header)).read()
    return sorted(set(re.findall(r"\b(" + prefix + r"[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    names = declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTS)
    assert lib.pic_version() >= 10000
    mnames = declared("mlp.h", "mlp_")
    assert set(mnames) == set(B.MLP_EXPORTS)
    for n in mnames:
        assert hasattr(lib, n), n


def _args(d=None, procs=None, **kw):
    d = d or I.config(1)
    procs = I.make_processes() if procs is None else procs
    cfg = B.make_config(d, **kw)
    sp = B.make_species(d.species())
    pr, tabs = B.make_processes(procs)
    return cfg, sp, pr, len(procs), tabs


def test_query_reports_workspace_size():
    cfg, sp, pr, n, _ = _args()
    nbytes = B.pic_query(cfg, sp, pr, n)
    caps = sum(s.capacity for s in I.config(1).species())
    assert nbytes >= 48 * caps


@pytest.mark.parametrize("field,value", [("ng", 1), ("ng", 9000), ("L", 0.0), ("ksub", 0), ("weight", -1.0),
                                         ("table_n", 1), ("max_products", 0), ("max_products", (1 << 24) + 1),
                                         ("block", 300), ("c_meta", -0.5)])
def test_query_rejects_invalid_config(field, value):
    cfg, sp, pr, n, _ = _args()
    setattr(cfg, field, value)
    with pytest.raises(B.PicError) as e:
        B.pic_query(cfg, sp, pr, n)
    assert e.value.code == B.PIC_EINVAL


def test_query_rejects_bad_species_and_processes():
    cfg, sp, pr, n, tabs = _args()
    sp[0].charge = 1.0
    with pytest.raises(B.PicError):
        B.pic_query(cfg, sp, pr, n)
    cfg, sp, pr, n, tabs = _args()
    pr[0].kind = B.KIND["cx"]           # charge exchange is not an electron process
    with pytest.raises(B.PicError):
        B.pic_query(cfg, sp, pr, n)
    cfg, sp, pr, n, tabs = _args()
    tabs[0][3] = float("nan")
    with pytest.raises(B.PicError):
        B.pic_query(cfg, sp, pr, n)
    cfg, sp, pr, n, tabs = _args()
    sp[1].count = sp[1].capacity + 1
    with pytest.raises(B.PicError):
        B.pic_query(cfg, sp, pr, n)


def test_query_accepts_all_sixteen_channels_and_checks_electron_ion_targets():
    full = I.make_processes_full()
    cfg, sp, pr, n, tabs = _args(procs=full)
    assert n == 16 and B.pic_query(cfg, sp, pr, n) > 0
    names = [p.name for p in full]
    for name, bad in (("e-recomb", "grid-"), ("e-edet", "grid+"), ("e-recomb", "O2"), ("O--neut", "grid-")):
        cfg, sp, pr, n, tabs = _args(procs=full)
        pr[names.index(name)].target = B.TARGET[bad]
        with pytest.raises(B.PicError) as e:
            B.pic_query(cfg, sp, pr, n)
        assert e.value.code == B.PIC_EINVAL, (name, bad)
    cfg, sp, pr, n, tabs = _args(procs=full)
    pr[names.index("O2+-cx")].kind = B.KIND["recomb"]      # electron-ion kinds belong to electrons
    with pytest.raises(B.PicError):
        B.pic_query(cfg, sp, pr, n)


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", "/nonexistent/libpicmcc.so")
    with pytest.raises(RuntimeError):
        B.lib()


def test_batch_query_sizes_and_limits():
    assert B.pic_batch_query(1) > 0
    assert B.pic_batch_query(64) > B.pic_batch_query(1)
    for n in (0, 65):
        with pytest.raises(B.PicError):
            B.pic_batch_query(n)


def _ksub_expected(d, species, n_ion, phi):
    """Largest divisor k of the steps per cycle with omega_pi k dt <= 0.2 and
    sqrt(2 e phi / M) k dt <= dx for both ion species (host rule, restated)."""
    eps0, qe = 8.8541878128e-12, 1.602176634e-19
    dt, dx = 1.0 / (d.f * d.steps_per_cycle), d.L / d.ng
    best = 1
    for k in range(1, d.steps_per_cycle + 1):
        if d.steps_per_cycle % k:
            continue
        ok = all(np.sqrt(n_ion * qe * qe / (eps0 * s.mass)) * k * dt <= 0.2 and
                 np.sqrt(2 * qe * phi / s.mass) * k * dt <= dx for s in species[1:])
        if not ok:
            break
        best = k
    return best


def test_ksub_select_physics_valid_subcycling():
    d = I.config(2)
    sp = B.make_species(d.species())
    cfg = B.make_config(d)
    # nothing limits: every divisor is valid, the cycle itself is returned
    assert B.pic_ksub_select(cfg, sp, 0.0, 0.0) == d.steps_per_cycle
    ks = []
    for U in (50.0, 100.0, 200.0, 400.0, 600.0):
        k = B.pic_ksub_select(cfg, sp, 3e15, U)
        assert d.steps_per_cycle % k == 0
        assert k == _ksub_expected(d, d.species(), 3e15, U)
        ks.append(k)
    assert ks == sorted(ks, reverse=True) and ks[0] > ks[-1]      # harder drive, shorter ion steps
    # a finer grid never allows a longer ion step
    fine = B.make_config(I.config(2, ng=2048))
    assert B.pic_ksub_select(fine, sp, 3e15, 400.0) <= B.pic_ksub_select(cfg, sp, 3e15, 400.0)
    # plasma-frequency limit alone: omega_pi k dt <= 0.2 at a huge density forces k = 1
    assert B.pic_ksub_select(cfg, sp, 1e22, 0.0) == 1
    with pytest.raises(B.PicError):
        B.pic_ksub_select(cfg, sp, -1.0, 100.0)


def test_mlp_query_sizes_and_limits():
    small, big = B.mlp_query(1), B.mlp_query(4096)
    assert small >= 18 * B.MLP_NPARAM                      # FP32 params, grads, moments + bf16 copy
    assert big - small >= 4095 * (4 * 4 + 2 * 4) * 256     # pre-activations and activations per sample
    for n in (0, (1 << 20) + 1):
        with pytest.raises(B.PicError):
            B.mlp_query(n)
