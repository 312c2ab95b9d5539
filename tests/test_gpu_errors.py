"""Device-side errors forced from the host: a full species store, a full
per-step product buffer, 32-bit ids running out and a runaway field.  The
kernels meet each condition through their own bounds checks (a product beyond
the store or the buffer is dropped, a particle whose position is no longer
finite is removed) and every launch ends normally; the sticky flag comes back
at the next synchronising call as its documented code, and stays until the
handle is destroyed.  Products get their ids in the step after the one that
made them, so each case runs two steps."""
import dataclasses

import numpy as np
import pytest

from paper_0705_0497_amd import inputs as I
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _attaching():
    """The default channels with attachment at a constant 1e-18 m^2 from 0 eV:
    several hundred O- products in every step of the 128-cell discharge."""
    procs = I.make_processes()
    k = [p.name for p in procs].index("e-att")
    procs[k] = I.constant_process("e-att", 0, "attach", "O2", 1e-18)
    return procs


def _raises(g, code, steps=2):
    from paper_0705_0497_amd.binding import PicError
    with pytest.raises(PicError) as ei:
        g.step(steps)
        g.sync()
    assert ei.value.code == code, str(ei.value)
    with pytest.raises(PicError) as again:            # sticky
        g.sync()
    assert again.value.code == code
    return str(ei.value)


def _loaded(d, procs, species=None, **kw):
    from paper_0705_0497_amd.binding import Discharge
    g = Discharge(d, procs, species=species, **kw)
    g.load_uniform()
    return g


def test_control_run_has_no_error():
    from paper_0705_0497_amd import binding as B
    d = I.config(1)
    g = _loaded(d, _attaching())
    g.step(4)
    g.sync()
    c = g.counters()
    assert c[B.C_BORN + 2] > 400, "the forcing process must produce O- in every step"


def test_full_species_store_raises_capacity():
    from paper_0705_0497_amd import binding as B
    d = I.config(1)
    sp = d.species()
    sp[2] = dataclasses.replace(sp[2], capacity=sp[2].count + 5)
    g = _loaded(d, _attaching(), species=sp)
    msg = _raises(g, B.PIC_ECAPACITY)
    assert "full" in msg


def test_full_product_buffer_raises_capacity():
    from paper_0705_0497_amd import binding as B
    d = I.config(1)
    g = _loaded(d, _attaching(), max_products=16)
    _raises(g, B.PIC_ECAPACITY)


def test_exhausted_ids_raise_id_overflow():
    from paper_0705_0497_amd import binding as B
    d = I.config(1)
    procs = _attaching()
    st, nid, step = H.canonical_from_oracle(d, procs)
    nid = list(nid)
    nid[2] = (1 << 32) - 8                       # eight ids left for O-
    g = H.gpu_from_canonical(d, procs, st, nid, step)
    msg = _raises(g, B.PIC_EIDOVERFLOW)
    assert "ids" in msg


def test_runaway_field_raises_nan():
    from paper_0705_0497_amd import binding as B
    d = I.config(1)
    g = _loaded(d, I.make_processes(), flags=B.F_EXT_FIELD, e_ext=(1e30, 0.0))
    _raises(g, B.PIC_ENAN)
