"""Oracle values at sampled cells of boxes too large for the oracle (test infrastructure).

One step of the method is local: with N_mag sweeps a cell's new state depends only on the
fields within a Chebyshev distance of about 4 N_mag + 5 cells (one cell per sweep and per
fluid gather, three per wall correction through the Lagrange taps of the markers whose taps
reach the cell, one for the Lorentz curl) and on the markers within one more cell (the row
sums d_j reach one tap stencil further). So the oracle run on a small periodic box cut around
a cell, holding the fields and markers found there, reproduces that cell's new state exactly:
the wrap of the small box only disturbs cells near its faces. `tests/test_subbox_cpu.py` pins
this against whole-box oracle runs; the full-size GPU tests use it to check sampled cells.
"""
from __future__ import annotations

import copy

import numpy as np

import oracle
import workloads as W


def influence_radius(n_mag: int) -> int:
    return 4 * n_mag + 5


def sub_box(w, center, n_mag: int, steps: int = 1, margin: int = 3):
    """(params, markers, rho, u, b, r) of the periodic box of side 2r + 1 centred on `center`
    (x, y, z) of workload `w`, in the small box's own coordinates (the centre at (r, r, r));
    r covers `steps` steps of `n_mag` sweeps."""
    r = influence_radius(n_mag) * steps + margin
    cx, cy, cz = center
    n = (w.nx, w.ny, w.nz)
    ix = (cx - r + np.arange(2 * r + 1)) % w.nx
    iy = (cy - r + np.arange(2 * r + 1)) % w.ny
    iz = (cz - r + np.arange(2 * r + 1)) % w.nz
    sel = np.ix_(iz, iy, ix)
    rho = w.rho[sel]
    u = np.stack([w.u[a][sel] for a in range(3)])
    b = np.stack([w.b[a][sel] for a in range(3)])
    p = copy.copy(w.params)
    p.n_mag = n_mag
    if p.bext_kind == W.BEXT_TANH_FRINGE_Y:
        # the fringe depends on x itself: the small box must not wrap around the seam at x = 0
        assert r <= cx <= w.nx - 1 - r, ("fringe field: sample too close to the x seam", cx, r)
        p.fringe_x0 = p.fringe_x0 - (cx - r)
    p.yc = p.yc - (cy - r)
    p.zc = p.zc - (cz - r)
    X = w.markers
    if X is not None and X.shape[1]:
        # minimum-image offsets of the markers from the centre, kept well inside the small box
        d = np.stack([((X[a] - c + n[a] / 2.0) % n[a]) - n[a] / 2.0 for a, c in enumerate(center)])
        keep = np.all(np.abs(d) <= r - 2, axis=0)
        Xs = d[:, keep] + r
    else:
        Xs = np.zeros((3, 0))
    return p, Xs, rho, u, b, r


def oracle_cell(w, center, n_mag: int, steps: int = 1, **over):
    """The oracle's (rho, u[3], b[3]) at `center` after `steps` steps of `n_mag` sweeps."""
    p, Xs, rho, u, b, r = sub_box(w, center, n_mag, steps)
    side = 2 * r + 1
    op = oracle.make_params(side, side, side, p, **over)
    o = oracle.Oracle(op, Xs if Xs.shape[1] else None, rho, u, b)
    o.step(steps)
    return o.rho[r, r, r], o.u[:, r, r, r].copy(), o.b[:, r, r, r].copy()
