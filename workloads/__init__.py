"""Seeded synthetic inputs for the QS-MHD pipe-flow step (geometry, parameters, initial fields).

This module holds no arithmetic of the lattice method itself: it only produces the inputs that
both the HIP path and the FP64 oracle consume (marker positions, lattice-unit parameters, initial
density/velocity/induced-field arrays). Everything is generated in float64 from numpy's
SeedSequence, keyed by a workload id, so every caller sees the same bytes.

Conventions (lattice units, dx = dt = 1):
  * box nx * ny * nz, periodic on every face, pipe axis along x;
  * fields are component-major, x fastest: u has shape (3, nz, ny, nx);
  * wall markers sit on integer x planes, on a circle of radius R around (yc, zc),
    m_slice = round(2 pi R) markers per plane (element size close to dx^2, Sec. 5.3 remark on
    element area), angle theta_j = 2 pi j / m_slice measured from +y towards +z.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED = 221109370
U0 = 0.05  # reference (bulk) velocity in lattice units

# bext_kind values shared by the C ABI, the oracle and the workloads
BEXT_NONE = 0
BEXT_UNIFORM_Y = 1
BEXT_TANH_FRINGE_Y = 2
BEXT_SIX_MAGNETS = 3


@dataclasses.dataclass
class Params:
    """Physical parameters in lattice units (mirrors the C `mhd_params` struct field by field)."""
    nu: float
    eta: float
    n_mag: int
    lambda_u: float = 1.0
    lambda_b: float = 0.0  # <= 0 selects the default eta/eta_ref with eta_ref = 1/6
    G0: float = 0.0
    G1: float = 0.0
    period: float = 0.0
    bext_kind: int = BEXT_NONE
    B0: float = 0.0
    fringe_x0: float = 0.0
    fringe_w: float = 1.0
    yc: float = 0.0
    zc: float = 0.0
    avg_radius: float = 0.0
    flow_control: int = 0
    u_bulk_target: float = 0.0
    k_c: float = 0.1
    alpha: float = 1.0  # accelerated magnetic iteration (1: plain sweep)
    magnet_L: float = 0.0  # six magnets: strip half-width (<= 0: R / 6)
    magnet_D: float = 0.0  # six magnets: distance of the strips from the axis (<= 0: outside the box)
    lattice: int = 19  # 19 or 27 (the paper's D3Q27)
    gamma: float = 1.0  # time-step rescaling of the fluid update (1: none)
    omega_radius: float = 0.0  # budget region r < omega_radius (<= 0: avg_radius - 2)


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    R: float
    params: Params
    markers: np.ndarray          # (3, M) float64
    rho: np.ndarray              # (nz, ny, nx)
    u: np.ndarray                # (3, nz, ny, nx)
    b: np.ndarray                # (3, nz, ny, nx)

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz


def rng_for(key: int) -> np.random.Generator:
    """numpy Generator from SeedSequence(SEED) spawned child `key`."""
    ss = np.random.SeedSequence(SEED)
    child = ss.spawn(key + 1)[key]
    return np.random.default_rng(child)


def n_mag_for(eta: float, cap: int = 270) -> int:
    """Sweeps per fluid step: ceil(1/dt) with dt = 1/(6 eta), capped at the effective count."""
    return int(max(1, min(math.ceil(6.0 * eta - 1e-9), cap)))


def map_params(Re: float, Ha: float, Rm: float, R: float, U0: float = U0):
    """(Re, Ha, Rm) -> (nu, eta, B0) with L = R and U = U0 (Ha = B0 R / sqrt(eta nu))."""
    nu = U0 * R / Re
    eta = U0 * R / Rm
    B0 = Ha * math.sqrt(eta * nu) / R
    return nu, eta, B0


def poiseuille_G(nu: float, R: float, U0: float = U0) -> float:
    """Body force giving bulk velocity U0 in a Poiseuille pipe of radius R: 8 nu U0 / R^2."""
    return 8.0 * nu * U0 / (R * R)


def pipe_markers(nx: int, R: float, yc: float, zc: float, m_slice: Optional[int] = None,
                 x_planes: Optional[np.ndarray] = None) -> np.ndarray:
    """Circle of markers of radius R on each integer x plane; returns (3, M) float64."""
    if m_slice is None:
        m_slice = int(round(2.0 * math.pi * R))
    if x_planes is None:
        x_planes = np.arange(nx, dtype=np.float64)
    th = 2.0 * math.pi * np.arange(m_slice, dtype=np.float64) / m_slice
    ys = yc + R * np.cos(th)
    zs = zc + R * np.sin(th)
    X = np.empty((3, len(x_planes) * m_slice), dtype=np.float64)
    for p, x in enumerate(x_planes):
        sl = slice(p * m_slice, (p + 1) * m_slice)
        X[0, sl] = x
        X[1, sl] = ys
        X[2, sl] = zs
    return X


def plane_wall_markers(nx: int, nz: int, y_wall: float) -> np.ndarray:
    """One marker on every (x, z) node of the plane y = y_wall; returns (3, nx*nz)."""
    xs, zs = np.meshgrid(np.arange(nx, dtype=np.float64), np.arange(nz, dtype=np.float64),
                         indexing="xy")
    X = np.empty((3, nx * nz), dtype=np.float64)
    X[0] = xs.ravel()
    X[1] = y_wall
    X[2] = zs.ravel()
    return X


def noise_fields(nx, ny, nz, key, amp=1e-4, rho_amp=0.0, b_amp=0.0):
    """rho = 1 (+ optional noise), u ~ U(-amp, amp) per cell and component, b (default 0)."""
    g = rng_for(key)
    u = g.uniform(-amp, amp, size=(3, nz, ny, nx))
    rho = np.ones((nz, ny, nx))
    if rho_amp:
        rho = rho + g.uniform(-rho_amp, rho_amp, size=(nz, ny, nx))
    b = np.zeros((3, nz, ny, nx))
    if b_amp:
        b = g.uniform(-b_amp, b_amp, size=(3, nz, ny, nx))
    return rho, u, b


def pipe_workload(name, key, nx, ny, nz, R, Re, Ha, Rm, *, bext_kind=BEXT_UNIFORM_Y,
                  fringe_x0=0.0, fringe_w=8.0, n_mag_cap=270, n_mag=None, noise=1e-4,
                  rho_amp=0.0, b_amp=0.0, G=None) -> Workload:
    nu, eta, B0 = map_params(Re, Ha, Rm, R)
    yc, zc = ny // 2, nz // 2
    p = Params(nu=nu, eta=eta, n_mag=n_mag if n_mag is not None else n_mag_for(eta, n_mag_cap),
               G0=poiseuille_G(nu, R) if G is None else G, bext_kind=bext_kind, B0=B0,
               fringe_x0=fringe_x0, fringe_w=fringe_w, yc=float(yc), zc=float(zc),
               avg_radius=float(R), u_bulk_target=U0)
    X = pipe_markers(nx, R, yc, zc)
    rho, u, b = noise_fields(nx, ny, nz, key, amp=noise, rho_amp=rho_amp, b_amp=b_amp)
    return Workload(name, nx, ny, nz, float(R), p, X, rho, u, b)


def small_pipe(**kw) -> Workload:
    """8 x 32 x 32 box, R = 14, 88 markers per plane, uniform B0 along y,
    Ha = 5, Re = 10, Rm = 1e-3 (nu = 0.07, eta = 700, B0 = 2.5, 270 sweeps per step)."""
    return pipe_workload("pipe8x32x32_R14_Ha5", 1, 8, 32, 32, 14.0, 10.0, 5.0, 1e-3, **kw)


def fringe_pipe(**kw) -> Workload:
    """128^3 box, R = 60, 377 markers per plane, fringe field B0 (1 + tanh((x - 64)/8))/2 along y,
    Ha = 20, Re = 500, Rm = 1e-2 (nu = 0.006, eta = 300, 270 sweeps per step)."""
    return pipe_workload("pipe128x128x128_R60_fringe_Ha20", 2, 128, 128, 128, 60.0, 500.0, 20.0,
                         1e-2, bext_kind=BEXT_TANH_FRINGE_Y, fringe_x0=64.0, fringe_w=8.0, **kw)


def quarter_fringe_pipe(**kw) -> Workload:
    """1/4 linear scale of the 128^3 fringe pipe: 32^3 box, R = 15 (94 markers per plane)."""
    return pipe_workload("pipe32x32x32_R15_fringe_Ha20", 3, 32, 32, 32, 15.0, 500.0, 20.0, 1e-2,
                         bext_kind=BEXT_TANH_FRINGE_Y, fringe_x0=16.0, fringe_w=2.0, **kw)


def large_pipe(Rm=1e-2, **kw) -> Workload:
    """512 x 256 x 256 box, R = 120, 754 markers per plane, uniform B0, Ha = 30, Re = 5000."""
    return pipe_workload(f"pipe512x256x256_R120_Ha30_Rm{Rm:g}", 5, 512, 256, 256, 120.0, 5000.0,
                         30.0, Rm, **kw)


def pipe_slab(nx: int) -> Workload:
    """One axial slab of the 512 x 256 x 256 pipe: the same cross-section, physics and ring,
    nx planes long (64 = one GPU's share of eight, 128 = of four), periodic in x."""
    return pipe_workload(f"pipe512x256x256_R120_Ha30_Rm0.01_slab{nx}", 5, nx, 256, 256, 120.0, 5000.0,
                         30.0, 1e-2)


def batch_pipes(n: int = 64, key: int = 4, R_range=(16.0, 64.0), lengths=(32, 64, 128, 256),
                Ha_range=(1.0, 50.0), Rm_range=(1e-4, 1.0), Re_range=(50.0, 1000.0),
                noise: float = 1e-4, n_mag_cap: int = 270):
    """Independent pipes of uneven size and physics for the batched form.

    Pipe i: R ~ U(R_range), length L drawn from `lengths`, box L x (2 ceil(R) + 4)^2 with the axis
    at the box centre, markers L * round(2 pi R); Ha and Rm log-uniform, Re uniform, mapped to
    (nu, eta, B0) with L = R, U = U0; n_mag = min(ceil(6 eta), cap); the imposed field is uniform
    or (probability 1/2) a tanh fringe centred at L/2 with width 8. The fields are not generated
    here (a 64-pipe batch holds ~60 M cells): `batch_fields(w)` gives rho = 1, u ~ U(+-noise),
    b = 0 for one of them.
    """
    g = rng_for(key)
    out = []
    for i in range(n):
        R = float(g.uniform(*R_range))
        L = int(g.choice(lengths))
        Ha = float(math.exp(g.uniform(math.log(Ha_range[0]), math.log(Ha_range[1]))))
        Rm = float(math.exp(g.uniform(math.log(Rm_range[0]), math.log(Rm_range[1]))))
        Re = float(g.uniform(*Re_range))
        fringe = bool(g.uniform() < 0.5)
        field_seed = int(g.integers(0, 2**62))
        side = 2 * int(math.ceil(R)) + 4
        nu, eta, B0 = map_params(Re, Ha, Rm, R)
        yc = zc = side // 2
        p = Params(nu=nu, eta=eta, n_mag=n_mag_for(eta, n_mag_cap), G0=poiseuille_G(nu, R),
                   bext_kind=BEXT_TANH_FRINGE_Y if fringe else BEXT_UNIFORM_Y, B0=B0,
                   fringe_x0=L / 2.0, fringe_w=8.0, yc=float(yc), zc=float(zc), avg_radius=R,
                   u_bulk_target=U0)
        X = pipe_markers(L, R, yc, zc)
        w = Workload(f"batch{i}_L{L}_R{R:.1f}_Ha{Ha:.2g}_Rm{Rm:.2g}_Re{Re:.0f}", L, side, side, R,
                     p, X, None, None, None)
        w.field_seed = field_seed
        w.noise = noise
        out.append(w)
    return out


def batch_fields(w: Workload):
    """(rho, u, b) of a pipe from `batch_pipes`: rho = 1, u ~ U(+-noise) per component, b = 0."""
    g = np.random.default_rng(w.field_seed)
    u = g.uniform(-w.noise, w.noise, size=(3, w.nz, w.ny, w.nx))
    return np.ones((w.nz, w.ny, w.nx)), u, np.zeros((3, w.nz, w.ny, w.nx))


def perturbed_pipe_fields(nx, ny, nz, R, yc, zc, key, amp=0.05 * U0, n_modes=8, kx_max=4,
                          U=U0):
    """Initial state of the unsteady large-pipe case: rho = 1, b = 0, u = the Poiseuille profile of
    bulk velocity U inside r < R (2 U (1 - r^2/R^2), zero outside) plus a divergence-free
    perturbation: the curl, by central differences, of a seeded smooth vector potential
    A_c = env(r) sum_q a_cq cos(2 pi (m_q x / nx + (l_q y + n_q z) / (2R)) + phi_cq) with axial
    wave numbers |m_q| <= kx_max, cross-section wave numbers l, n in 0..3 and the envelope
    env = (1 - r^2/R^2)^2 inside r < R (zero outside), scaled so that max |du| = amp. Central
    differences commute, so the discrete divergence of the perturbation vanishes to round-off.
    Returns (rho, u, b) in float64, u of shape (3, nz, ny, nx)."""
    g = rng_for(key)
    y = np.arange(ny, dtype=np.float64)[:, None] - yc
    z = np.arange(nz, dtype=np.float64)[None, :] - zc
    r2 = (y * y + z * z).T  # (nz, ny)
    s = r2 / (R * R)
    env = np.where(s < 1.0, (1.0 - s) ** 2, 0.0)
    xs = np.arange(nx, dtype=np.float64)
    Y = np.broadcast_to(np.arange(ny, dtype=np.float64)[None, :], (nz, ny))
    Z = np.broadcast_to(np.arange(nz, dtype=np.float64)[:, None], (nz, ny))
    A = np.zeros((3, nz, ny, nx))
    for c in range(3):
        for _ in range(n_modes):
            m = int(g.integers(-kx_max, kx_max + 1))
            l, n = int(g.integers(0, 4)), int(g.integers(0, 4))
            a, ph = float(g.normal()), float(g.uniform(0.0, 2.0 * math.pi))
            beta = 2.0 * math.pi * (l * Y + n * Z) / (2.0 * R) + ph  # (nz, ny)
            ax = 2.0 * math.pi * m * xs / nx                          # (nx,)
            # cos(ax + beta) = cos(ax) cos(beta) - sin(ax) sin(beta), built plane by plane
            A[c] += a * (np.cos(beta)[:, :, None] * np.cos(ax)[None, None, :]
                         - np.sin(beta)[:, :, None] * np.sin(ax)[None, None, :])
        A[c] *= env[:, :, None]

    def d(f, axis):  # central difference along x (axis 2), y (1) or z (0), periodic
        return 0.5 * (np.roll(f, -1, axis=axis) - np.roll(f, 1, axis=axis))

    du = np.empty_like(A)
    du[0] = d(A[2], 1) - d(A[1], 0)
    du[1] = d(A[0], 0) - d(A[2], 2)
    du[2] = d(A[1], 2) - d(A[0], 1)
    del A
    du *= amp / np.abs(du).max()
    u = du
    u[0] += np.where(s < 1.0, 2.0 * U * (1.0 - s), 0.0)[:, :, None]
    return np.ones((nz, ny, nx)), u, np.zeros((3, nz, ny, nx))


def large_pipe_perturbed(Rm=1e-2, nx=512, ny=256, nz=256, R=120.0, **kw) -> Workload:
    """The unsteady large-pipe case: 512 x 256 x 256 box, R = 120 (754 markers per plane), uniform
    B0 along y, Re = 5000, Ha = 30 (nu = 0.0012, tau = 0.5036), the given Rm (1e-3 .. 1 gives
    eta = 6000 .. 6 and 270 .. 36 sweeps per step), started from the Poiseuille profile with a
    divergence-free 5% perturbation (perturbed_pipe_fields)."""
    w = pipe_workload(f"pipe{nx}x{ny}x{nz}_R{R:g}_Ha30_Rm{Rm:g}_perturbed", 6, nx, ny, nz, R, 5000.0,
                      30.0, Rm, noise=0.0, **kw)
    w.rho, w.u, w.b = perturbed_pipe_fields(nx, ny, nz, R, w.params.yc, w.params.zc, key=6)
    return w
