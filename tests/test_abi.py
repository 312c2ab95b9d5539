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


def declared():
    text = open(os.path.join(ROOT, "include", "pic.h")).read()
    return sorted(set(re.findall(r"\b(pic_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    names = declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTS)
    assert lib.pic_version() >= 10000


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
                                         ("block", 300), ("pair_rounds", 0), ("c_meta", -0.5)])
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


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(B, "_lib", None)
    monkeypatch.setattr(B, "LIB_PATH", "/nonexistent/libpicmcc.so")
    with pytest.raises(RuntimeError):
        B.lib()
