"""More pins of the FP64 oracle (CPU only): the lambda-scaled wall correction on markers whose
row sums d_j differ from 1, the fixed point of the magnetic iteration with the wall correction
solved directly, and the steady power balance (injected work = viscous + Joule dissipation).

None of these re-types an oracle formula:
  * the wall correction is checked against the implicit equation of Sec. 5.5 (eq. "IMB scaling
    for Lagrangian correction", with the paper's approximation D D^+ ~ D D^T) built from a dense
    interpolation matrix of the textbook Lagrange basis and numpy's pseudo-inverse; for markers
    whose supports are disjoint, A = D D^T is diagonal and the paper's explicit scaling solves
    that equation exactly, whatever lambda and d_j are;
  * the fixed point of sweep + correction is found by a direct linear solve of the affine map
    probed column by column, and checked off the wall band against the quasi-static induction
    equation written with independent numpy operators;
  * the power balance is a consequence of the steady equations (summation by parts), checked on
    the plane Hartmann flow, whose walls sit on lattice nodes, and on the pipe.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from tests import fdops
from tests.test_oracle_pins import _dense_D, _hartmann_run


@pytest.fixture(autouse=True, scope="module")
def _threads():
    oracle.set_threads(8)
    yield


# --------------------------------------------------------------------------------------------
# lambda-scaled explicit correction (Sec. 5.5 velocity, Sec. 5.6 magnetic field)
# --------------------------------------------------------------------------------------------

NX, NY, NZ = 10, 26, 26


def _isolated_curved_markers():
    """Markers on a circle of radius 8 around (13, 13), at angles and x positions off the lattice
    nodes, spaced so that no two 3 x 3 x 3 supports share a node."""
    th = 2 * math.pi * (np.arange(6) + 0.23) / 6
    X = np.stack([np.array([1.3, 4.6, 7.4, 2.8, 6.2, 8.7]),
                  13.0 + 8.0 * np.cos(th), 13.0 + 8.0 * np.sin(th)])
    return X


def _recover_delta(D, phi_star, phi):
    """Lagrangian corrections delta (3 x M) from phi - phi* = D^T delta (least squares)."""
    diff = (phi - phi_star).reshape(3, -1)
    return np.linalg.lstsq(D.T, diff.T, rcond=None)[0].T


def _check_scaling_equation(D, phi_star, delta, lam, wall):
    """delta = lam A^+ (U_b - D phi*) + (1 - lam) A delta with A = D D^T (Sec. 5.5)."""
    A = D @ D.T
    b = wall - (D @ phi_star.reshape(3, -1).T).T          # (3, M)
    t1 = lam * (np.linalg.pinv(A) @ b.T).T
    t2 = (1.0 - lam) * (A @ delta.T).T
    scale = max(np.abs(t1).max(), np.abs(t2).max(), np.abs(delta).max())
    assert np.abs(delta - (t1 + t2)).max() <= 1e-13 * scale, (lam, np.abs(delta - (t1 + t2)).max(), scale)


def test_isolated_curved_markers_have_diagonal_A_and_row_sums_below_one():
    X = _isolated_curved_markers()
    D = _dense_D(NX, NY, NZ, X)
    A = D @ D.T
    assert np.count_nonzero(A - np.diag(np.diag(A))) == 0
    d = oracle.ib_rowsums(oracle.make_params(NX, NY, NZ), X)
    np.testing.assert_allclose(d, np.diag(A), rtol=1e-14)
    assert d.max() < 0.95 and d.min() > 0.3, d


@pytest.mark.parametrize("lam", [0.7, 1.0, 36.0, 4200.0])
def test_scaled_correction_solves_the_scaling_equation(lam):
    X = _isolated_curved_markers()
    p = oracle.make_params(NX, NY, NZ)
    D = _dense_D(NX, NY, NZ, X)
    g = W.rng_for(110)
    phi_star = g.normal(size=(3, NZ, NY, NX))
    wall = g.normal(size=(3, X.shape[1]))
    d = oracle.ib_rowsums(p, X)
    phi = oracle.ib_correct(p, X, d, lam, phi_star, wall)
    delta = _recover_delta(D, phi_star, phi)
    # the correction lies in the range of D^T (nothing else changed)
    resid = (phi - phi_star).reshape(3, -1) - (D.T @ delta.T).T
    assert np.abs(resid).max() <= 1e-13 * np.abs(delta).max()
    _check_scaling_equation(D, phi_star, delta, lam, wall)
    # lambda = 1 is the least-squares solve: the corrected field interpolates to the wall value
    if lam == 1.0:
        np.testing.assert_allclose((D @ phi.reshape(3, -1).T).T, wall, rtol=0, atol=1e-13)


def test_scaled_corrections_of_a_whole_step_use_lambda_u_for_u_and_lambda_b_for_b():
    # One step with one sweep: b = b* + correction(lambda_b) with b* the sweep of (u, b) and
    # u = u* + correction(lambda_u) with u* the fluid update under the Lorentz force of the new b.
    X = _isolated_curved_markers()
    lam_u, lam_b = 0.7, 36.0
    p = oracle.make_params(NX, NY, NZ, nu=0.05, eta=2.0, n_mag=1, lambda_u=lam_u, lambda_b=lam_b,
                           G0=1e-5, bext_kind=W.BEXT_UNIFORM_Y, B0=0.3, yc=13.0, zc=13.0, radius=8.0)
    D = _dense_D(NX, NY, NZ, X)
    g = W.rng_for(111)
    rho0 = 1.0 + g.uniform(-1e-3, 1e-3, size=(NZ, NY, NX))
    u0 = g.uniform(-1e-2, 1e-2, size=(3, NZ, NY, NX))
    b0 = g.uniform(-1e-2, 1e-2, size=(3, NZ, NY, NX))
    uw = g.uniform(-1e-2, 1e-2, size=(3, X.shape[1]))
    bw = g.uniform(-1e-2, 1e-2, size=(3, X.shape[1]))
    o = oracle.Oracle(p, X, rho0, u0, b0, u_wall=uw, b_wall=bw)
    o.step(1)
    b_star = oracle.mag_sweep(p, u0, b0)
    _check_scaling_equation(D, b_star, _recover_delta(D, b_star, o.b), lam_b, bw)
    _, u_star = oracle.fluid(p, rho0, u0, oracle.lorentz(p, o.b, p.G0))
    _check_scaling_equation(D, u_star, _recover_delta(D, u_star, o.u), lam_u, uw)
    # and the two ratios are not interchangeable
    with pytest.raises(AssertionError):
        _check_scaling_equation(D, u_star, _recover_delta(D, u_star, o.u), lam_b, uw)


# --------------------------------------------------------------------------------------------
# Fixed point of the magnetic iteration with the wall correction (Sec. 5.6, 5.7), solved directly
# --------------------------------------------------------------------------------------------

def test_sweep_and_correction_fixed_point_is_the_direct_solve():
    nx, ny, nz, R, eta = 4, 16, 16, 5.0, 1.5
    p = oracle.make_params(nx, ny, nz, eta=eta, bext_kind=W.BEXT_UNIFORM_Y, B0=0.4, yc=8.0, zc=8.0,
                           radius=R)
    X = W.pipe_markers(nx, R, 8, 8)
    d = oracle.ib_rowsums(p, X)
    lam_b = 6.0 * eta  # the default resistivity ratio
    g = W.rng_for(112)
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    z = np.arange(nz)[:, None, None]
    u = np.stack([0.04 * np.cos(2 * np.pi * y / ny) * np.cos(2 * np.pi * z / nz) + 0 * x,
                  0.01 * np.sin(2 * np.pi * x / nx) + 0 * y * z,
                  0.01 * np.sin(2 * np.pi * (y + z) / ny) + 0 * x])
    bw = g.uniform(-1e-3, 1e-3, size=(3, X.shape[1]))

    def T(b):
        return oracle.ib_correct(p, X, d, lam_b, oracle.mag_sweep(p, u, b), bw)

    n = 3 * nx * ny * nz
    c = T(np.zeros((3, nz, ny, nx))).ravel()
    L = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        L[:, k] = T(e.reshape(3, nz, ny, nx)).ravel() - c
    assert np.abs(np.linalg.eigvals(L)).max() < 1.0  # a contraction
    b_fix = np.linalg.solve(np.eye(n) - L, c).reshape(3, nz, ny, nx)
    b = np.zeros((3, nz, ny, nx))
    for _ in range(3000):
        b = T(b)
    assert np.abs(b - b_fix).max() <= 1e-10 * np.abs(b_fix).max()
    # off the wall band the fixed point solves eta lap b = div(u B - B u) (lattice operators)
    band = np.zeros(nx * ny * nz, bool)
    for j in range(X.shape[1]):
        band[oracle.marker_taps(p, X[:, j])[0]] = True
    band = band.reshape(nz, ny, nx)
    near = band.copy()
    for e in fdops.VEL[1:]:
        near |= fdops.shift(band, e)
    B = b_fix.copy()
    B[1] += 0.4
    lap_b = np.stack([fdops.lap(b_fix[a]) for a in range(3)])
    div = np.zeros_like(b_fix)
    for a in range(3):
        for cc in range(3):
            div[a] += fdops.grad(u[cc] * B[a] - B[cc] * u[a])[cc]
    res = eta * lap_b - div
    assert np.abs(res[:, ~near]).max() <= 1e-10 * np.abs(div).max()
    assert np.abs(res[:, band]).max() > 1e-4 * np.abs(div).max()  # the wall acts in the band


# --------------------------------------------------------------------------------------------
# Steady power balance: injected work = viscous + Joule dissipation (Sec. 4 energy balance)
# --------------------------------------------------------------------------------------------

@pytest.mark.parametrize("a, steps", [(8, 3000), (16, 8000)])
def test_plane_hartmann_power_balance_closes(a, steps):
    # Walls on nodes hold u = b = 0 exactly, so over the slab between them the steady equations
    # summed by parts give P_in = -P_nu + D_eta and -P_L = D_eta (Lorentz work = Joule heat).
    oracle.set_threads(1)
    o, y, inside, (nu, eta, B0, G) = _hartmann_run(a, 4.0, steps)
    p = oracle.OrcParams.from_buffer_copy(o.p)
    p.omega_radius = float(a)  # Omega = the nodes strictly between the walls
    bud = oracle.budgets(p, o.rho, o.u, o.b, G)
    assert bud["n_omega"] == 2 * a - 1
    visc, joule = -bud["P_nu"], bud["D_eta"]
    assert visc > 0 and joule > 0
    assert abs(bud["P_in"] - (visc + joule)) <= 1e-5 * bud["P_in"], bud
    assert abs(-bud["P_L"] - joule) <= 1e-5 * joule, bud
    assert abs(bud["P_p"]) <= 1e-6 * bud["P_in"]
    # D_eta is the lattice form of eta <|J|^2>: the two differ by the wall layer only (first order)
    assert 0.5 * joule < bud["joule"] < joule
    oracle.set_threads(8)
