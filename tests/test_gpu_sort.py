"""The cell sort (PIC_SORT_CELL): a store of particles that do not move (no
field, no velocity, no collisions) is sorted by the step-0 re-ordering and
read back in store order.  The cells must come back non-decreasing and every
particle record (position, velocity, id, countdown) unchanged, for stores whose
tiles span few cells (ordered with local disorder, one cell), and stores whose
tiles span more cells than one tile orders in LDS (random order, two far
cells), at 128, 2048 and 8192 cells with ragged particle counts."""
import numpy as np
import pytest

from paper_0705_0497_amd import inputs as I

pytestmark = pytest.mark.gpu


def _store(n, ng, kind, rng):
    if kind == "random":
        cell = rng.integers(0, ng, n)
    elif kind == "ordered":
        cell = np.sort(rng.integers(0, ng, n))
        j = rng.integers(0, n, n // 3)                # a third of the slots moved up to 40 cells
        cell[j] = np.clip(cell[j] + rng.integers(-40, 41, j.size), 0, ng - 1)
    elif kind == "one_cell":
        cell = np.full(n, ng // 2)
    else:                                             # two far cells
        cell = np.where(rng.random(n) < 0.5, 0, ng - 1)
    return {"cell": cell.astype(np.int32), "off": rng.random(n).astype(np.float32),
            "vx": np.zeros(n, np.float32), "vy": rng.standard_normal(n).astype(np.float32),
            "vz": rng.standard_normal(n).astype(np.float32),
            "id": rng.permutation(n).astype(np.uint32) + np.uint32(5),
            "cd": rng.integers(1, 2000, n).astype(np.int32)}


@pytest.mark.parametrize("ng,n,kind", [(128, 30001, "ordered"), (128, 7, "random"), (2048, 200003, "random"),
                                       (2048, 100001, "ordered"), (2048, 4099, "one_cell"),
                                       (8192, 50005, "two_cells"), (8192, 150001, "ordered")])
def test_cell_sort_orders_the_store_and_keeps_every_particle(ng, n, kind):
    from paper_0705_0497_amd.binding import Discharge, F_EXT_FIELD, F_NO_COLL, SORT_CELL
    rng = np.random.Generator(np.random.PCG64(ng * 7 + n))
    d = I.config(1, ng=ng, counts=(n, n, n), capacities=(n + 64, n + 64, n + 64), sort_every=1, diag_every=0)
    g = Discharge(d, [], flags=F_EXT_FIELD | F_NO_COLL, e_ext=(0.0, 0.0), sort_kind=SORT_CELL)
    stores = [_store(n, ng, kind, rng) for _ in range(3)]
    for s in range(3):
        g.set_particles(s, stores[s], n + 5)
    g.set_step(0)
    g.prepare(False)
    g.step(1)
    for s in range(3):
        got, nid = g.get_particles(s)
        assert nid == n + 5 and got["id"].size == n
        assert np.all(np.diff(got["cell"]) >= 0), f"species {s}: store not ordered by cell"
        a = np.argsort(stores[s]["id"])
        b = np.argsort(got["id"])
        for k in ("cell", "off", "vx", "vy", "vz", "id"):
            np.testing.assert_array_equal(got[k][b], stores[s][k][a], err_msg=f"species {s} field {k}")
        if s == 0:
            np.testing.assert_array_equal(got["cd"][b] & 0x7FFF, stores[s]["cd"][a])
