"""FP64 CPU oracle of the QS-MHD single-step lattice Boltzmann step (arXiv:2211.09370).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and by bench.py's CPU
baseline leg. The product package never imports it. The arithmetic lives in mhd_oracle.c
(plain literal loops in double precision); this module only marshals numpy arrays through ctypes.

Functions and the passage each follows:
  mag_sweep    - tau_m = 1 macroscopic magnetic update with c = 6 eta (Sec. 5.7)
  lagrange3    - three-point Lagrange kernel of the immersed boundary (Sec. 5.2)
  ib_rowsums   - d_j = sum_i (D D^T)_ji (Sec. 5.3)
  ib_correct   - explicit correction phi* + D^T diag(s) (phi_b - D phi*), s from Sec. 5.5 / 5.6
  lorentz      - G x + (curl b) x B with isotropic differences (Sec. 5.1)
  fluid        - single-step density / momentum update with GZS forcing and the lattice
                 discrete-effect term (Sec. 3.3, Sec. 5.1), with the time-step rescaling gamma
                 (Sec. 7); for tau >= 1 the macroscopic tau = 1 update with speed 6 nu (Sec. 5.7)
  fluid_tau    - tau = 3 nu / gamma + 1/2 (Sec. 7)
  Oracle.step  - whole step in the order of Sec. 5.7 (magnetic iteration, then velocity)
  budgets      - energy budget averages of Sec. 4 over r < R_omega (default R - 2), mass, flow
                 rate, and the Joule dissipation in lattice Dirichlet form
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

BUDGET_NAMES = ("E_k", "E_m", "E_b", "P_in", "P_p", "P_nu", "P_L", "M_eta", "M_adv", "joule",
                "mass", "Q", "u_max", "n_omega", "G", "nonfinite", "res_mag", "D_eta")


class OrcParams(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("nu", C.c_double), ("eta", C.c_double), ("n_mag", C.c_int),
                ("lambda_u", C.c_double), ("lambda_b", C.c_double),
                ("G0", C.c_double), ("G1", C.c_double), ("period", C.c_double),
                ("bext_kind", C.c_int), ("B0", C.c_double), ("fringe_x0", C.c_double),
                ("fringe_w", C.c_double), ("yc", C.c_double), ("zc", C.c_double),
                ("radius", C.c_double), ("flow_control", C.c_int), ("u_target", C.c_double),
                ("k_c", C.c_double), ("ib_u", C.c_int), ("ib_b", C.c_int),
                ("alpha", C.c_double), ("magnet_L", C.c_double), ("magnet_D", C.c_double),
                ("lattice", C.c_int), ("gamma", C.c_double), ("omega_radius", C.c_double)]


_D = C.POINTER(C.c_double)
_I64 = C.POINTER(C.c_int64)


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        P = C.POINTER(OrcParams)
        L.orc_mag_sweep.argtypes = [P, _D, _D, _D]
        L.orc_lagrange3.argtypes = [C.c_double, _D]
        L.orc_lagrange3.restype = C.c_int
        L.orc_marker_taps.argtypes = [P, _D, _I64, _D]
        L.orc_marker_taps.restype = C.c_int
        L.orc_ib_rowsums.argtypes = [P, C.c_int64, _D, _D]
        L.orc_ib_correct.argtypes = [P, C.c_int64, _D, _D, C.c_double, _D, _D]
        L.orc_lorentz.argtypes = [P, _D, C.c_double, _D]
        L.orc_fluid.argtypes = [P, _D, _D, _D, _D, _D]
        L.orc_fluid_tau.argtypes = [P]
        L.orc_fluid_tau.restype = C.c_double
        L.orc_create.argtypes = [P, C.c_int64, _D, _D, _D]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_get_rowsums.argtypes = [C.c_void_p, _D]
        L.orc_step.argtypes = [C.c_void_p, _D, _D, _D, C.c_int64, _I64, _D]
        L.orc_budgets.argtypes = [P, _D, _D, _D, C.c_double, _D]
        L.orc_bext.argtypes = [P, C.c_int, C.c_int, C.c_int, _D]
        L.orc_bext_at.argtypes = [P, C.c_double, C.c_double, C.c_double, _D]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _LIB = L
    return _LIB


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_params(nx, ny, nz, prm=None, *, ib_u=1, ib_b=1, **over) -> OrcParams:
    """Build OrcParams from a workloads.Params-like object (attribute names match) + overrides."""
    fields = dict(nu=0.1, eta=1.0, n_mag=1, lambda_u=1.0, lambda_b=0.0, G0=0.0, G1=0.0, period=0.0,
                  bext_kind=0, B0=0.0, fringe_x0=0.0, fringe_w=1.0, yc=0.0, zc=0.0, radius=0.0,
                  flow_control=0, u_target=0.0, k_c=0.1, alpha=1.0, magnet_L=0.0, magnet_D=0.0,
                  lattice=19, gamma=1.0, omega_radius=0.0)
    if prm is not None:
        for k in list(fields):
            src = {"radius": "avg_radius", "u_target": "u_bulk_target"}.get(k, k)
            if hasattr(prm, src):
                fields[k] = getattr(prm, src)
    fields.update(over)
    return OrcParams(nx=nx, ny=ny, nz=nz, ib_u=ib_u, ib_b=ib_b,
                     **{k: (int(v) if k in ("n_mag", "bext_kind", "flow_control", "lattice") else float(v))
                        for k, v in fields.items()})


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """OpenMP thread count of the oracle (tiny grids run faster on one thread)."""
    lib().orc_set_threads(int(n))


def bext(p: OrcParams, x, y, z):
    out = np.zeros(3)
    lib().orc_bext(C.byref(p), x, y, z, _ptr(out))
    return out


def bext_at(p: OrcParams, x: float, y: float, z: float):
    """Imposed field at real coordinates (the six-magnet field is continuous)."""
    out = np.zeros(3)
    lib().orc_bext_at(C.byref(p), float(x), float(y), float(z), _ptr(out))
    return out


def mag_sweep(p: OrcParams, u, b):
    u, b = _f64(u), _f64(b)
    out = np.empty_like(b)
    lib().orc_mag_sweep(C.byref(p), _ptr(u), _ptr(b), _ptr(out))
    return out


def lagrange3(X: float):
    w = np.zeros(3)
    base = lib().orc_lagrange3(float(X), _ptr(w))
    return base, w


def marker_taps(p: OrcParams, Xj):
    Xj = _f64(Xj)
    idx = np.zeros(27, dtype=np.int64)
    w = np.zeros(27)
    n = lib().orc_marker_taps(C.byref(p), _ptr(Xj), idx.ctypes.data_as(_I64), _ptr(w))
    return idx[:n].copy(), w[:n].copy()


def ib_rowsums(p: OrcParams, X):
    X = _f64(X)
    M = X.shape[1]
    d = np.zeros(M)
    lib().orc_ib_rowsums(C.byref(p), M, _ptr(X), _ptr(d))
    return d


def ib_correct(p: OrcParams, X, d, lam, phi, wall=None):
    X, d, phi = _f64(X), _f64(d), _f64(phi).copy()
    wall = None if wall is None else _f64(wall)
    lib().orc_ib_correct(C.byref(p), X.shape[1], _ptr(X), _ptr(d), float(lam), _ptr(wall),
                         _ptr(phi))
    return phi


def lorentz(p: OrcParams, b, G):
    b = _f64(b)
    F = np.empty_like(b)
    lib().orc_lorentz(C.byref(p), _ptr(b), float(G), _ptr(F))
    return F


def fluid_tau(p: OrcParams) -> float:
    return float(lib().orc_fluid_tau(C.byref(p)))


def fluid(p: OrcParams, rho, u, F):
    rho, u, F = _f64(rho), _f64(u), _f64(F)
    r2 = np.empty_like(rho)
    u2 = np.empty_like(u)
    lib().orc_fluid(C.byref(p), _ptr(rho), _ptr(u), _ptr(F), _ptr(r2), _ptr(u2))
    return r2, u2


def budgets(p: OrcParams, rho, u, b, G) -> dict:
    rho, u, b = _f64(rho), _f64(u), _f64(b)
    out = np.zeros(len(BUDGET_NAMES))
    lib().orc_budgets(C.byref(p), _ptr(rho), _ptr(u), _ptr(b), float(G), _ptr(out))
    return dict(zip(BUDGET_NAMES, out.tolist()))


class Oracle:
    """Whole-step oracle state: rho (nz,ny,nx), u and b (3,nz,ny,nx) in float64."""

    def __init__(self, p: OrcParams, markers=None, rho=None, u=None, b=None, u_wall=None,
                 b_wall=None):
        self.p = p
        shape = (p.nz, p.ny, p.nx)
        self.rho = _f64(rho).copy() if rho is not None else np.ones(shape)
        self.u = _f64(u).copy() if u is not None else np.zeros((3,) + shape)
        self.b = _f64(b).copy() if b is not None else np.zeros((3,) + shape)
        X = _f64(markers) if markers is not None else np.zeros((3, 0))
        self._X = X
        self._uw = None if u_wall is None else _f64(u_wall)
        self._bw = None if b_wall is None else _f64(b_wall)
        self.M = X.shape[1]
        self._ctx = lib().orc_create(C.byref(p), self.M, _ptr(X) if self.M else None,
                                     _ptr(self._uw), _ptr(self._bw))
        self.t = C.c_int64(0)
        self.G = C.c_double(p.G0)

    def rowsums(self):
        d = np.zeros(self.M)
        if self.M:
            lib().orc_get_rowsums(self._ctx, _ptr(d))
        return d

    def step(self, n: int = 1):
        lib().orc_step(self._ctx, _ptr(self.rho), _ptr(self.u), _ptr(self.b), int(n),
                       C.byref(self.t), C.byref(self.G))

    def budgets(self) -> dict:
        return budgets(self.p, self.rho, self.u, self.b, self.G.value)

    def close(self):
        if self._ctx:
            lib().orc_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
