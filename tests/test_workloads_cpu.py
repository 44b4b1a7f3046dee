"""The seeded inputs of the unsteady large-pipe case (CPU): a Poiseuille profile of bulk velocity
U0 plus a divergence-free perturbation of amplitude 5% of U0 confined to the pipe."""
import numpy as np

import workloads as W


def _d(f, axis):
    return 0.5 * (np.roll(f, -1, axis=axis) - np.roll(f, 1, axis=axis))


def test_perturbed_pipe_initial_state():
    nx, ny, nz, R, yc, zc = 64, 48, 48, 20.0, 24, 24
    rho, u, b = W.perturbed_pipe_fields(nx, ny, nz, R, yc, zc, key=6)
    assert np.all(rho == 1.0) and np.all(b == 0.0)
    y = np.arange(ny)[None, :] - yc
    z = np.arange(nz)[:, None] - zc
    s = (y * y + z * z) / R ** 2
    base = np.zeros_like(u)
    base[0] = np.where(s < 1.0, 2.0 * W.U0 * (1.0 - s), 0.0)[:, :, None]
    du = u - base
    assert abs(np.abs(du).max() - 0.05 * W.U0) <= 1e-15
    div = _d(du[0], 2) + _d(du[1], 1) + _d(du[2], 0)
    assert np.abs(div).max() <= 1e-14 * np.abs(du).max()
    assert np.abs(du[:, s >= 1.1, :]).max() == 0.0            # confined to the pipe
    assert np.abs(du[0]).max() > 0 and np.abs(du[1]).max() > 0 and np.abs(du[2]).max() > 0
    bulk = u[0][s < 1.0].mean()
    assert abs(bulk / W.U0 - 1.0) <= 0.02, bulk
    # seeded: the same bytes every call
    assert np.array_equal(u, W.perturbed_pipe_fields(nx, ny, nz, R, yc, zc, key=6)[1])
