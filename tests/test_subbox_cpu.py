"""The sampled-cell oracle (tests/subbox.py) equals the whole-box oracle at its sampled cells.

This pins the locality argument the full-size GPU tests rest on: a step's new state at a cell
depends only on the fields and markers within the influence radius, so the oracle run on a
small periodic box cut around the cell gives the whole-box value (up to float64 round-off of
a different summation size). Cells near the wall, on the axis, next to the box faces (the
small box wraps across them) and next to the fringe centre are sampled.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from tests.subbox import oracle_cell


@pytest.fixture(autouse=True, scope="module")
def _threads():
    oracle.set_threads(8)
    yield


def _box(bext):
    w = W.pipe_workload("subbox", 7, 64, 38, 36, 13.0, 50.0, 10.0, 1e-2, bext_kind=bext, fringe_x0=32.0,
                        fringe_w=4.0, n_mag=2, noise=1e-2, rho_amp=1e-3, b_amp=1e-3)
    return w


# axis, wall points, near-wall, box corners (outside the pipe); x within the fringe's reach
CELLS = [(32, 19, 18), (25, 19 + 13, 18), (38, 19, 18 - 13), (28, 19 + 9, 18 + 9), (40, 0, 0), (22, 37, 35),
         (33, 6, 30)]


@pytest.mark.parametrize("bext", [W.BEXT_TANH_FRINGE_Y, W.BEXT_UNIFORM_Y])
@pytest.mark.parametrize("steps,n_mag", [(1, 2), (2, 1)])
def test_sampled_cells_equal_the_whole_box(bext, steps, n_mag):
    w = _box(bext)
    w.params.n_mag = n_mag
    p = oracle.make_params(w.nx, w.ny, w.nz, w.params)
    o = oracle.Oracle(p, w.markers, w.rho, w.u, w.b)
    o.step(steps)
    us, bs = np.abs(o.u).max(), np.abs(o.b).max()
    for cx, cy, cz in CELLS:
        r_, u_, b_ = oracle_cell(w, (cx, cy, cz), n_mag, steps)
        assert abs(r_ - o.rho[cz, cy, cx]) <= 1e-13, (cx, cy, cz)
        assert np.abs(u_ - o.u[:, cz, cy, cx]).max() <= 1e-12 * us, (cx, cy, cz)
        assert np.abs(b_ - o.b[:, cz, cy, cx]).max() <= 1e-12 * bs, (cx, cy, cz)


def test_too_small_a_box_is_detectably_wrong():
    """Control: cut the small box tighter than the influence radius and the wall cells differ,
    so the radius is doing real work."""
    from tests import subbox

    w = _box(W.BEXT_UNIFORM_Y)
    p = oracle.make_params(w.nx, w.ny, w.nz, w.params)
    o = oracle.Oracle(p, w.markers, w.rho, w.u, w.b)
    o.step(1)
    keep = subbox.influence_radius
    try:
        subbox.influence_radius = lambda n: 1
        _, u_, _ = oracle_cell(w, CELLS[1], 2, 1)
    finally:
        subbox.influence_radius = keep
    cx, cy, cz = CELLS[1]
    assert np.abs(u_ - o.u[:, cz, cy, cx]).max() > 1e-9 * np.abs(o.u).max()
