"""Isotropic finite-difference operators on a periodic D3Q19 (default) or D3Q27 lattice, written
with numpy rolls.

Used by the tests to check fixed points and identities of the oracle from the operator side:
  grad_a phi = 3 sum_i w_i e_ia phi(x + e_i),   lap phi = 6 sum_i w_i (phi(x + e_i) - phi(x)).
Arrays are (nz, ny, nx); vectors are (3, nz, ny, nx).
"""
import itertools

import numpy as np

VEL = [(0, 0, 0)] + [v for v in itertools.product((-1, 0, 1), repeat=3)
                     if 0 < sum(abs(c) for c in v) <= 2]
WGT = [1.0 / 3.0] + [1.0 / 18.0 if sum(abs(c) for c in v) == 1 else 1.0 / 36.0 for v in VEL[1:]]
assert len(VEL) == 19 and abs(sum(WGT) - 1.0) < 1e-15
# D3Q27: all 27 offsets, weights the product of the 1D weights 2/3 (0) and 1/6 (+-1)
VEL27 = list(itertools.product((-1, 0, 1), repeat=3))
WGT27 = [float(np.prod([2.0 / 3.0 if c == 0 else 1.0 / 6.0 for c in v])) for v in VEL27]
assert len(VEL27) == 27 and abs(sum(WGT27) - 1.0) < 1e-15


def _set(lattice):
    return (VEL27, WGT27) if lattice == 27 else (VEL, WGT)


def shift(f, e):
    """phi(x + e) on the periodic grid (x fastest = last axis)."""
    ex, ey, ez = e
    return np.roll(f, shift=(-ez, -ey, -ex), axis=(-3, -2, -1))


def grad(f, lattice=19):
    g = np.zeros((3,) + f.shape)
    for e, w in zip(*_set(lattice)):
        if e == (0, 0, 0):
            continue
        s = shift(f, e)
        for a in range(3):
            if e[a]:
                g[a] += 3.0 * w * e[a] * s
    return g


def lap(f, lattice=19):
    out = np.zeros_like(f)
    for e, w in zip(*_set(lattice)):
        if e == (0, 0, 0):
            continue
        out += 6.0 * w * (shift(f, e) - f)
    return out


def div_flux(u, B, lattice=19):
    """[div(uB - Bu)]_a = sum_c d_c (u_c B_a - B_c u_a)."""
    out = np.zeros_like(u)
    for a in range(3):
        for c in range(3):
            out[a] += grad(u[c] * B[a] - B[c] * u[a], lattice)[c]
    return out


def curl(b):
    gx, gy, gz = grad(b[0]), grad(b[1]), grad(b[2])
    return np.stack([gz[1] - gy[2], gx[2] - gz[0], gy[0] - gx[1]])
