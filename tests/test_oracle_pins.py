"""Pins of the FP64 oracle against what the paper and the mathematics fix (CPU only).

Each test names the passage it pins. None of them re-types an oracle formula: they check the
oracle against closed forms (Poiseuille, Hartmann, Gold), exact identities (mass, momentum
bookkeeping, symmetry), textbook definitions (Lagrange interpolation, Fourier symbols) and fixed
points written with independent numpy finite-difference operators.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W
from oracle import gold
from tests import fdops


@pytest.fixture(autouse=True, scope="module")
def _threads():
    oracle.set_threads(8)
    yield


# --------------------------------------------------------------------------------------------
# Immersed boundary kernel and row sums (Sec. 5.2, Sec. 5.3)
# --------------------------------------------------------------------------------------------

def lagrange_basis(X):
    """Textbook quadratic Lagrange basis on the three nodes nearest to X."""
    n0 = math.floor(X + 0.5)
    nodes = [n0 - 1, n0, n0 + 1]
    w = []
    for t, nt in enumerate(nodes):
        v = 1.0
        for s, ns in enumerate(nodes):
            if s != t:
                v *= (X - ns) / (nt - ns)
        w.append(v)
    return n0 - 1, np.array(w)


@pytest.mark.parametrize("X", [3.0, 3.3, 3.49, 2.5, 7.77, 0.5, 10.25, 5.999])
def test_lagrange_kernel_is_quadratic_lagrange_interpolation(X):
    base, w = oracle.lagrange3(X)
    base_ref, w_ref = lagrange_basis(X)
    assert base == base_ref
    np.testing.assert_allclose(w, w_ref, rtol=0, atol=1e-15)
    nodes = base + np.arange(3)
    # exact on polynomials of degree <= 2
    for coef in ([1, 0, 0], [0.3, -1.7, 0], [2.0, 0.5, -0.25]):
        f = lambda x: coef[0] + coef[1] * x + coef[2] * x * x
        assert abs(np.dot(w, f(nodes.astype(float))) - f(X)) < 1e-12


def test_lagrange_kernel_on_a_node_is_a_delta():
    base, w = oracle.lagrange3(6.0)
    assert base == 5 and list(w) == [0.0, 1.0, 0.0]


def _dense_D(nx, ny, nz, X):
    """Dense interpolation matrix D (M x N) from the textbook basis (periodic indexing)."""
    M = X.shape[1]
    D = np.zeros((M, nx * ny * nz))
    for j in range(M):
        bx, wx = lagrange_basis(X[0, j])
        by, wy = lagrange_basis(X[1, j])
        bz, wz = lagrange_basis(X[2, j])
        for c in range(3):
            for b in range(3):
                for a in range(3):
                    k = ((bx + a) % nx) + nx * (((by + b) % ny) + ny * ((bz + c) % nz))
                    D[j, k] += wx[a] * wy[b] * wz[c]
    return D


def test_rowsums_match_dense_DDt():
    nx, ny, nz = 3, 14, 14
    p = oracle.make_params(nx, ny, nz)
    X = W.pipe_markers(nx, 4.3, 7.0, 7.0, m_slice=27)
    X[0] += np.array([0.0, 0.25, 0.5])[np.arange(X.shape[1]) % 3]  # some off-plane markers too
    D = _dense_D(nx, ny, nz, X)
    d_ref = (D @ D.T).sum(axis=1)
    np.testing.assert_allclose(oracle.ib_rowsums(p, X), d_ref, rtol=1e-13)


def test_isolated_markers_enforce_wall_value_exactly():
    # For a marker whose support meets no other marker, A = D D^T is diagonal, the explicit
    # correction with lambda = 1 is the exact least-squares solve and D u = U_b afterwards.
    nx, ny, nz = 12, 12, 12
    p = oracle.make_params(nx, ny, nz)
    X = np.array([[2.3, 8.1], [3.7, 8.6], [4.45, 2.2]])
    g = W.rng_for(100)
    phi = g.normal(size=(3, nz, ny, nx))
    wall = g.normal(size=(3, 2))
    d = oracle.ib_rowsums(p, X)
    out = oracle.ib_correct(p, X, d, 1.0, phi, wall)
    D = _dense_D(nx, ny, nz, X)
    np.testing.assert_allclose(D @ out.reshape(3, -1).T, wall.T, rtol=0, atol=1e-13)


@pytest.mark.parametrize("lam", [1.0, 0.7, 36.0])
def test_markers_on_nodes_are_exact_for_any_lambda(lam):
    nx, ny, nz = 4, 10, 3
    p = oracle.make_params(nx, ny, nz)
    X = W.plane_wall_markers(nx, nz, 6.0)
    d = oracle.ib_rowsums(p, X)
    np.testing.assert_array_equal(d, np.ones(X.shape[1]))
    phi = W.rng_for(101).normal(size=(3, nz, ny, nx))
    out = oracle.ib_correct(p, X, d, lam, phi)
    np.testing.assert_array_equal(out[:, :, 6, :], 0.0)
    keep = np.ones(ny, bool)
    keep[6] = False
    np.testing.assert_array_equal(out[:, :, keep, :], phi[:, :, keep, :])


# --------------------------------------------------------------------------------------------
# Magnetic iteration (Sec. 5.7)
# --------------------------------------------------------------------------------------------

def test_magnetic_sweep_symbol_is_the_lattice_average():
    # u = 0: one tau_m = 1 sweep multiplies a lattice Fourier mode by sum_i w_i cos(k.e_i),
    # the D3Q19 averaging symbol, whose minimum 1/9 makes the plain sweep a contraction.
    n = 8
    p = oracle.make_params(n, n, n, eta=3.0)
    x = np.arange(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.zeros((3, n, n, n))
    for (kx, ky, kz) in [(1, 0, 0), (2, 3, 0), (4, 4, 0), (1, 2, 3), (4, 4, 4), (0, 4, 4)]:
        k = 2 * np.pi * np.array([kx, ky, kz]) / n
        mode = np.cos(k[0] * X + k[1] * Y + k[2] * Z)
        b = np.stack([mode, 0.5 * mode, -mode])
        out = oracle.mag_sweep(p, u, b)
        cx, cy, cz = np.cos(k)
        symbol = 1 / 3 + (cx + cy + cz) / 9 + (cx * cy + cx * cz + cy * cz) / 9
        np.testing.assert_allclose(out, symbol * b, atol=1e-14)
        assert symbol >= 1 / 9 - 1e-15


@pytest.mark.parametrize("lattice", [19, 27])
def test_magnetic_fixed_point_solves_qs_poisson_equation(lattice):
    # The iteration's steady state satisfies eta lap b = div(u B - B u), B = B_ext + b
    # (asymptotic limit stated in Sec. 5.7), with the isotropic operators of the lattice.
    n = 8
    eta = 2.0
    p = oracle.make_params(n, n, n, eta=eta, bext_kind=W.BEXT_UNIFORM_Y, B0=1.0, lattice=lattice)
    x = 2 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = 0.05 * np.stack([np.sin(Y) * np.cos(Z), np.cos(X + 2 * Z), np.sin(X - Y)])
    b = np.zeros((3, n, n, n))
    for _ in range(600):
        b = oracle.mag_sweep(p, u, b)
    B = b.copy()
    B[1] += 1.0
    res = eta * np.stack([fdops.lap(b[a], lattice) for a in range(3)]) - fdops.div_flux(u, B, lattice)
    scale = np.abs(fdops.div_flux(u, B, lattice)).max()
    assert np.abs(res).max() <= 1e-10 * scale


def test_magnetic_sweep_conserves_the_mean_field():
    n = 6
    p = oracle.make_params(n, n, n, eta=1.5, bext_kind=W.BEXT_UNIFORM_Y, B0=0.7)
    g = W.rng_for(102)
    u = 0.05 * g.normal(size=(3, n, n, n))
    b = 0.01 * g.normal(size=(3, n, n, n))
    out = oracle.mag_sweep(p, u, b)
    np.testing.assert_allclose(out.sum(axis=(1, 2, 3)), b.sum(axis=(1, 2, 3)), atol=1e-14)


# --------------------------------------------------------------------------------------------
# Fluid update (Sec. 3.3, Sec. 5.1): conservation and the discrete-effect term
# --------------------------------------------------------------------------------------------

# --------------------------------------------------------------------------------------------
# Accelerated magnetic iteration and the induction residual (Sec. 5.8)
# --------------------------------------------------------------------------------------------

def _symbol(k):
    cx, cy, cz = np.cos(k)
    return 1 / 3 + (cx + cy + cz) / 9 + (cx * cy + cx * cz + cy * cz) / 9


def test_d3q27_sweep_symbol_is_the_tensor_product_average():
    # D3Q27 weights are the product of the 1D weights (2/3, 1/6, 1/6), so for u = 0 one sweep
    # multiplies a mode by prod_a (2/3 + cos(k_a)/3), whose minimum 1/27 at k = (pi, pi, pi)
    # puts the accelerated iteration's stability edge at alpha = 13/27 (the paper reports
    # instability below about 1/2 for its D3Q27 scheme).
    n = 8
    x = np.arange(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.zeros((3, n, n, n))
    for alpha in (1.0, 13 / 27):
        p = oracle.make_params(n, n, n, eta=3.0, lattice=27, alpha=alpha)
        for (kx, ky, kz) in [(1, 0, 0), (2, 3, 0), (4, 4, 0), (1, 2, 3), (4, 4, 4), (0, 4, 4)]:
            k = 2 * np.pi * np.array([kx, ky, kz]) / n
            mode = np.cos(k[0] * X + k[1] * Y + k[2] * Z)
            b = np.stack([mode, 0.5 * mode, -mode])
            sigma = float(np.prod(2 / 3 + np.cos(k) / 3))
            out = oracle.mag_sweep(p, u, b)
            np.testing.assert_allclose(out, (1 + (sigma - 1) / alpha) * b, atol=1e-13)
            assert sigma >= 1 / 27 - 1e-15
            if (kx, ky, kz) == (4, 4, 4) and alpha < 1:
                assert abs(1 + (sigma - 1) / alpha + 1) < 1e-12


@pytest.mark.parametrize("alpha", [0.5, 4 / 9, 0.75, 1.7])
def test_accelerated_sweep_over_relaxes_each_mode_by_one_over_alpha(alpha):
    # Rest population (w_0 - 1 + alpha) b and the sum divided by alpha give, for u = 0, the mode
    # factor 1 + (sigma(k) - 1) / alpha with sigma the averaging symbol; at k = (pi, pi, 0),
    # sigma = 1/9 and the factor 1 - 8 / (9 alpha) reaches -1 at alpha = 4/9 (stability edge).
    n = 8
    p = oracle.make_params(n, n, n, eta=3.0, alpha=alpha)
    x = np.arange(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = np.zeros((3, n, n, n))
    for (kx, ky, kz) in [(1, 0, 0), (2, 3, 0), (4, 4, 0), (1, 2, 3), (0, 4, 4)]:
        k = 2 * np.pi * np.array([kx, ky, kz]) / n
        mode = np.cos(k[0] * X + k[1] * Y + k[2] * Z)
        b = np.stack([mode, -0.3 * mode, 2.0 * mode])
        out = oracle.mag_sweep(p, u, b)
        np.testing.assert_allclose(out, (1 + (_symbol(k) - 1) / alpha) * b, atol=1e-13)
    k = np.array([np.pi, np.pi, 0.0])
    assert abs(_symbol(k) - 1 / 9) < 1e-15
    factor = 1 - 8 / (9 * alpha)
    assert abs(factor) <= 1 + 1e-12  # every alpha >= 4/9 is stable on D3Q19
    if abs(alpha - 4 / 9) < 1e-12:
        assert abs(factor + 1) < 1e-12


def test_accelerated_sweep_has_the_plain_fixed_point():
    # The accelerated iteration only rescales the increment, so both converge to the same b.
    n = 8
    x = 2 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = 0.05 * np.stack([np.sin(Y) * np.cos(Z), np.cos(X + 2 * Z), np.sin(X - Y)])
    out = []
    for alpha, iters in ((1.0, 800), (0.5, 400)):
        p = oracle.make_params(n, n, n, eta=2.0, bext_kind=W.BEXT_UNIFORM_Y, B0=1.0, alpha=alpha)
        b = np.zeros((3, n, n, n))
        for _ in range(iters):
            b = oracle.mag_sweep(p, u, b)
        out.append(b)
    scale = np.abs(out[0]).max()
    assert scale > 1e-4
    assert np.abs(out[1] - out[0]).max() <= 1e-10 * scale


def test_accelerated_sweep_halves_the_sweeps_for_a_given_residual():
    # With alpha = 1/2 the slow modes contract twice as fast per sweep (mode factor above), so
    # N/2 accelerated sweeps leave about the error N plain sweeps leave (Sec. 5.8: N = 9 vs 18).
    n = 16
    x = 2 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = 0.05 * np.stack([np.sin(Y), np.cos(Z), np.sin(X)])
    ref = None
    errs = {}
    for alpha, iters in ((1.0, 3000), (1.0, 40), (0.5, 20)):
        p = oracle.make_params(n, n, n, eta=2.0, bext_kind=W.BEXT_UNIFORM_Y, B0=1.0, alpha=alpha)
        b = np.zeros((3, n, n, n))
        for _ in range(iters):
            b = oracle.mag_sweep(p, u, b)
        if ref is None:
            ref = b
        else:
            errs[alpha] = np.abs(b - ref).max()
    # the slowest mode's factors: plain (1 - e)^40 vs accelerated (1 - 2e)^20, equal to O(e^2)
    assert 0.8 < errs[0.5] / errs[1.0] < 1.05, errs


def test_induction_residual_of_a_mode_is_its_closed_form():
    # u = 0, B_ext = 0, b = cos(k.x) in one component: eta lap_h b = -6 eta (1 - sigma(k)) b, so
    # the root mean square over Omega (the whole box here) is 6 eta (1 - sigma) / sqrt(2).
    n = 8
    eta = 3.0
    p = oracle.make_params(n, n, n, eta=eta, radius=40.0, yc=n / 2, zc=n / 2)
    x = np.arange(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    k = 2 * np.pi * np.array([1, 2, 0]) / n
    b = np.zeros((3, n, n, n))
    b[2] = np.cos(k[0] * X + k[1] * Y + k[2] * Z)
    rec = oracle.budgets(p, np.ones((n, n, n)), np.zeros((3, n, n, n)), b, 0.0)
    assert rec["n_omega"] == n ** 3
    assert abs(rec["res_mag"] - 6 * eta * (1 - _symbol(k)) / math.sqrt(2)) < 1e-12


def test_induction_residual_vanishes_at_the_sweep_fixed_point():
    n = 8
    x = 2 * np.pi * np.arange(n) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = 0.05 * np.stack([np.sin(Y) * np.cos(Z), np.cos(X + 2 * Z), np.sin(X - Y)])
    p = oracle.make_params(n, n, n, eta=2.0, bext_kind=W.BEXT_UNIFORM_Y, B0=1.0, alpha=0.5,
                           radius=40.0, yc=n / 2, zc=n / 2)
    b = np.zeros((3, n, n, n))
    rho = np.ones((n, n, n))
    first = oracle.budgets(p, rho, u, oracle.mag_sweep(p, u, b), 0.0)["res_mag"]
    for _ in range(400):
        b = oracle.mag_sweep(p, u, b)
    last = oracle.budgets(p, rho, u, b, 0.0)["res_mag"]
    assert first > 0 and last < 1e-9 * first


def _random_state(n, key, F_mean=1e-4):
    g = W.rng_for(key)
    rho = 1.0 + 0.01 * g.uniform(-1, 1, size=(n, n, n))
    u = 0.05 * g.uniform(-1, 1, size=(3, n, n, n))
    F = F_mean * (1.0 + g.uniform(-1, 1, size=(3, n, n, n)))
    return rho, u, F


@pytest.mark.parametrize("lattice", [19, 27])
def test_lorentz_force_of_a_shear_mode_is_its_closed_form(lattice):
    """Sec. 5.1: J = curl_h b with the isotropic difference d_a f = 3 sum_i w_i e_ia f(x + e_i),
    which for a field varying along one axis is the central difference on both lattices (the
    weights of the velocities with e_a = 1 sum to 1/6), so d sin(k s) = sin(k) cos(k s) exactly;
    F = G x + J x (B_ext + b). With B_ext = B0 y: b = (0, 0, A sin(k y)) gives J = (A sin(k) cos(k y),
    0, 0) and F = (G, -J_x A sin(k y), J_x B0); b = (A sin(k z), 0, 0) gives J = (0, A sin(k) cos(k z), 0)
    and F = (G, 0, -J_y A sin(k z))."""
    n, A, B0, G = 12, 0.3, 0.8, 1e-4
    k = 2 * math.pi / n
    p = oracle.make_params(n, n, n, bext_kind=W.BEXT_UNIFORM_Y, B0=B0, lattice=lattice)
    s = np.sin(k * np.arange(n)); c = np.cos(k * np.arange(n))
    b = np.zeros((3, n, n, n))
    b[2] = A * s[None, :, None]                      # b_z(y)
    F = oracle.lorentz(p, b, G)
    Jx = A * math.sin(k) * c[None, :, None]
    assert np.abs(F[0] - G).max() < 1e-15
    assert np.abs(F[1] - (-Jx * A * s[None, :, None])).max() < 1e-14
    assert np.abs(F[2] - Jx * B0).max() < 1e-14
    b = np.zeros((3, n, n, n))
    b[0] = A * s[:, None, None]                      # b_x(z)
    F = oracle.lorentz(p, b, G)
    Jy = A * math.sin(k) * c[:, None, None]
    assert np.abs(F[0] - G).max() < 1e-15
    assert np.abs(F[1]).max() < 1e-15
    assert np.abs(F[2] - (-Jy * A * s[:, None, None])).max() < 1e-14


@pytest.mark.parametrize("lattice", [19, 27])
def test_budget_terms_of_shear_modes_are_their_closed_forms(lattice):
    """Sec. 4: every budget term on fields that vary along y only, averaged over a region Omega
    that holds the whole box (large radius). On such fields the isotropic gradient is the
    central difference (d sin ky = sin k cos ky) and the isotropic Laplacian the 1D second
    difference (2 (cos k - 1) sin ky) on both lattices, so each average is a closed form:
    with u = (U0 + A sin ky, 0, C cos ky), b = (0, 0, Bb sin ky), B_ext = B0 y, rho = 1,
      E_k = (U0^2 + A^2/2 + C^2/2)/2, E_m = (B0^2 + Bb^2/2)/2, E_b = Bb^2/4, P_in = G U0,
      P_nu = nu (cos k - 1)(A^2 + C^2), P_L = C Bb B0 sin(k)/2 = -M_adv,
      M_eta = eta (cos k - 1) Bb^2, joule = eta Bb^2 sin(k)^2/2, P_p = 0,
      residual^2 = ([2 eta (cos k - 1) Bb - B0 C sin k]^2 + (B0 A sin k)^2)/2;
    and with rho = 1 + e sin ky, u = (0, D cos ky, 0), b = 0: P_p = -D e sin(k)/6 (c_s^2 = 1/3)."""
    n, U0, A, C, Bb, B0, G, nu, eta = 12, 0.03, 0.02, 0.015, 0.01, 0.7, 2e-5, 0.05, 1.3
    k = 2 * math.pi / n
    sy = np.sin(k * np.arange(n))[None, :, None] * np.ones((n, n, n))
    cy = np.cos(k * np.arange(n))[None, :, None] * np.ones((n, n, n))
    p = oracle.make_params(n, n, n, nu=nu, eta=eta, bext_kind=W.BEXT_UNIFORM_Y, B0=B0, lattice=lattice,
                           yc=n / 2, zc=n / 2, radius=100.0)
    rho = np.ones((n, n, n))
    u = np.stack([U0 + A * sy, 0 * sy, C * cy])
    b = np.stack([0 * sy, 0 * sy, Bb * sy])
    r = oracle.budgets(p, rho, u, b, G)
    cm, sk = math.cos(k) - 1.0, math.sin(k)
    want = {"E_k": (U0 ** 2 + A ** 2 / 2 + C ** 2 / 2) / 2, "E_m": (B0 ** 2 + Bb ** 2 / 2) / 2, "E_b": Bb ** 2 / 4,
            "P_in": G * U0, "P_p": 0.0, "P_nu": nu * cm * (A ** 2 + C ** 2), "P_L": C * Bb * B0 * sk / 2,
            "M_eta": eta * cm * Bb ** 2, "M_adv": -C * Bb * B0 * sk / 2, "joule": eta * Bb ** 2 * sk ** 2 / 2,
            "mass": float(n ** 3), "Q": n * n * U0,
            "res_mag": math.sqrt(((2 * eta * cm * Bb - B0 * C * sk) ** 2 + (B0 * A * sk) ** 2) / 2)}
    assert r["n_omega"] == n ** 3
    for key, v in want.items():
        assert abs(r[key] - v) <= 1e-13 * max(1.0, abs(v)), (key, r[key], v)
    e, D = 1e-3, 0.02
    r = oracle.budgets(p, 1.0 + e * sy, np.stack([0 * sy, D * cy, 0 * sy]), np.zeros((3, n, n, n)), 0.0)
    assert abs(r["P_p"] - (-D * e * sk / 6)) <= 1e-15, r["P_p"]
    assert abs(r["E_k"] - D ** 2 / 4) <= 1e-15


@pytest.mark.parametrize("lattice", [19, 27])
def test_density_update_conserves_mass_exactly(lattice):
    rho, u, F = _random_state(7, 103)
    p = oracle.make_params(7, 7, 7, nu=0.05, lattice=lattice)
    r2, _ = oracle.fluid(p, rho, u, F)
    assert abs(r2.sum() - rho.sum()) <= 1e-13 * rho.sum()


@pytest.mark.parametrize("lattice", [19, 27])
def test_momentum_update_adds_exactly_the_body_force(lattice):
    # Without walls every gathered term telescopes on the periodic grid:
    # sum rho' u* - sum rho u = sum F.
    rho, u, F = _random_state(7, 104)
    for nu in (0.01, 0.1, 0.15):
        p = oracle.make_params(7, 7, 7, nu=nu, lattice=lattice)
        r2, u2 = oracle.fluid(p, rho, u, F)
        lhs = (r2 * u2).sum(axis=(1, 2, 3)) - (rho * u).sum(axis=(1, 2, 3))
        np.testing.assert_allclose(lhs, F.sum(axis=(1, 2, 3)), rtol=1e-12)


@pytest.mark.parametrize("lattice", [19, 27])
@pytest.mark.parametrize("gamma", [0.5, 2.0, 4.0])
def test_rescaled_update_conserves_mass_and_adds_the_force_over_gamma(lattice, gamma):
    # With the rescaled step dt / gamma (Sec. 7) the explicit force term is F / gamma and the
    # gathered terms still telescope: sum rho' = sum rho, sum rho' u* - sum rho u = sum F / gamma.
    rho, u, F = _random_state(7, 105)
    p = oracle.make_params(7, 7, 7, nu=0.04, lattice=lattice, gamma=gamma)
    r2, u2 = oracle.fluid(p, rho, u, F)
    assert abs(r2.sum() - rho.sum()) <= 1e-13 * rho.sum()
    lhs = (r2 * u2).sum(axis=(1, 2, 3)) - (rho * u).sum(axis=(1, 2, 3))
    np.testing.assert_allclose(lhs, F.sum(axis=(1, 2, 3)) / gamma, rtol=1e-12)


def _shear_state(n, ny, A, F0, m=1):
    """u = (A sin k y, 0, 0), F = (F0 sin k y, 0, 0), rho = 1 on an n x ny x n box."""
    k = 2 * np.pi * m / ny
    s = np.sin(k * np.arange(ny))[None, :, None]
    u = np.zeros((3, n, ny, n))
    F = np.zeros((3, n, ny, n))
    u[0] = A * s
    F[0] = F0 * s
    return np.ones((n, ny, n)), u, F, k, s


def _march_shear(p, rho, u, F, steps):
    for _ in range(steps):
        rho, u = oracle.fluid(p, rho, u, F)
    return rho, u


@pytest.mark.parametrize("lattice", [19, 27])
@pytest.mark.parametrize("gamma", [0.5, 1.0, 2.0, 4.0])
def test_rescaled_shear_wave_keeps_its_steady_state_and_slows_by_gamma(lattice, gamma):
    # Shear flow u = (A(y), 0, 0) under F = (F(y), 0, 0): within each group of directions with the
    # same e_y the quadratic equilibrium terms and the velocity-dependent forcing terms cancel, so
    # rho stays 1, u_y = u_z = 0, and each Fourier mode of u_x obeys
    #   A' = r A + F0 / gamma,  r = 1 - (2 tau - 1)(1 - cos k)/3 = 1 - 2 nu (1 - cos k) / gamma
    # (the single-step symbol with lambda = 2/3 + cos(k)/3 on both lattices). The steady amplitude
    # F0 / (2 nu (1 - cos k)) does not depend on gamma; the approach to it is slowed by gamma.
    oracle.set_threads(1)
    nu, A0, F0, steps = 0.04, 0.02, 2e-5, 40
    rho, u, F, k, s = _shear_state(3, 16, A0, F0)
    p = oracle.make_params(3, 16, 3, nu=nu, lattice=lattice, gamma=gamma)
    rho, u = _march_shear(p, rho, u, F, steps)
    r = 1.0 - 2.0 * nu * (1.0 - math.cos(k)) / gamma
    A_ss = F0 / (2.0 * nu * (1.0 - math.cos(k)))
    A_n = A_ss + (A0 - A_ss) * r ** steps
    np.testing.assert_allclose(u[0], A_n * np.broadcast_to(s, u[0].shape), rtol=0, atol=1e-13)
    assert np.abs(u[1:]).max() <= 1e-14 and np.abs(rho - 1.0).max() <= 1e-14
    oracle.set_threads(8)


@pytest.mark.parametrize("lattice", [19, 27])
@pytest.mark.parametrize("nu", [1.0 / 6.0, 0.3, 1.0])
def test_macroscopic_branch_shear_wave_is_its_closed_form(lattice, nu):
    # tau = 3 nu + 1/2 >= 1: the tau = 1 update with speed c = 6 nu (Sec. 5.7). For the same shear
    # flow each mode obeys A' = lambda A + (1 + lambda) F0 / (2 c), lambda = 2/3 + cos(k)/3, from
    # the gathered equilibria, the gathered GZS populations and the half-force term. The steady
    # amplitude (1 + lambda) F0 / (2 c (1 - lambda)) tends to F0 / (nu k^2) for small k.
    oracle.set_threads(1)
    A0, F0, steps = 0.05, 1e-3, 30
    rho, u, F, k, s = _shear_state(3, 24, A0, F0)
    p = oracle.make_params(3, 24, 3, nu=nu, lattice=lattice)
    assert oracle.fluid_tau(p) >= 1.0
    rho, u = _march_shear(p, rho, u, F, steps)
    c = 6.0 * nu
    lam = 2.0 / 3.0 + math.cos(k) / 3.0
    A_ss = (1.0 + lam) * F0 / (2.0 * c * (1.0 - lam))
    A_n = A_ss + (A0 - A_ss) * lam ** steps
    np.testing.assert_allclose(u[0], A_n * np.broadcast_to(s, u[0].shape), rtol=0, atol=1e-13)
    assert np.abs(u[1:]).max() <= 1e-14 and np.abs(rho - 1.0).max() <= 1e-14
    # the continuum limit of the steady amplitude
    assert abs(A_ss * nu * k * k / F0 - 1.0) < 0.02
    oracle.set_threads(8)


@pytest.mark.parametrize("lattice", [19, 27])
def test_macroscopic_branch_conserves_mass_and_adds_force_times_its_step(lattice):
    # sum_x sum_i f_i^eq(x - e_i) = sum rho and sum_i F_i = 0; sum_i c_i f_i^eq = rho u and
    # sum_i c_i F_i = F / 2, so with the half-force term sum rho' u' - sum rho u = dt sum F,
    # dt = 1 / (6 nu).
    rho, u, F = _random_state(7, 106, F_mean=1e-3)
    for nu in (0.2, 0.5):
        p = oracle.make_params(7, 7, 7, nu=nu, lattice=lattice)
        r2, u2 = oracle.fluid(p, rho, u, F)
        assert abs(r2.sum() - rho.sum()) <= 1e-13 * rho.sum()
        lhs = (r2 * u2).sum(axis=(1, 2, 3)) - (rho * u).sum(axis=(1, 2, 3))
        np.testing.assert_allclose(lhs, F.sum(axis=(1, 2, 3)) / (6.0 * nu), rtol=1e-12)


def test_macroscopic_branch_rejects_rescaling():
    rho, u, F = _random_state(5, 107)
    p = oracle.make_params(5, 5, 5, nu=0.5, gamma=2.0)  # tau = 3 nu / gamma + 1/2 = 1.25
    r2, u2 = oracle.fluid(p, rho, u, F)
    assert np.isnan(r2).all() and np.isnan(u2).all()


def _smooth_fields(n):
    h = 2 * np.pi / n
    x = h * np.arange(n)
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    u = 0.05 * np.stack([np.sin(Y + Z), np.cos(X) * np.sin(Z), np.sin(X + Y)])
    F = 1e-3 * np.stack([np.cos(Z), np.sin(X), np.cos(Y + X)])
    return h, u, F


def _spectral_div(n, h, T):
    """div of the tensor T[a][c] (row a, derivative along c), in lattice units."""
    k = np.fft.fftfreq(n, d=1.0 / n)

    def d(f, axis):
        shape = [1, 1, 1]
        shape[axis] = n
        return np.real(np.fft.ifftn(1j * k.reshape(shape) * np.fft.fftn(f))) * h

    axes = {0: 2, 1: 1, 2: 0}  # component index -> array axis
    out = np.zeros((3, n, n, n))
    for a in range(3):
        for c in range(3):
            out[a] += d(T[a][c], axes[c])
    return out


def test_rescaled_equilibrium_divides_the_momentum_flux_by_gamma():
    # At a fixed tau (nu proportional to gamma) the rescaled update differs only by the quadratic
    # equilibrium part divided by gamma, so without force rho' u* is affine in 1/gamma, and its
    # slope, the gathered quadratic part, tends to -div(u u) (the Euler momentum flux) at second
    # order.
    errs = []
    for n in (16, 32, 64):
        h, u, _ = _smooth_fields(n)
        rho = np.ones((n, n, n))
        M = {}
        for g in (1.0, 2.0, 4.0):
            p = oracle.make_params(n, n, n, nu=0.05 * g, gamma=g)
            r2, u2 = oracle.fluid(p, rho, u, np.zeros_like(u))
            M[g] = r2 * u2
        slope = (M[1.0] - M[2.0]) / (1.0 - 0.5)
        np.testing.assert_allclose(M[4.0], M[2.0] - slope * (0.5 - 0.25), rtol=0, atol=1e-14)
        cont = -_spectral_div(n, h, [[u[a] * u[c] for c in range(3)] for a in range(3)])
        errs.append(np.abs(slope - cont).max() / np.abs(cont).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 1.9, (errs, orders)


@pytest.mark.parametrize("gamma", [1.0, 2.5])
def test_discrete_effect_term_converges_to_its_continuum_form(gamma):
    # -(tau/2) sum_i e_i [F_i(x+e_i) - F_i(x-e_i)] -> -(tau - 1/2) div(u F + F u) / gamma^2,
    # second order; tau = 3 nu / gamma + 1/2 and the rescaled F_i of Sec. 7 (its velocity terms
    # carry 1/gamma^2).
    nu = 0.05
    tau = 3 * nu / gamma + 0.5
    errs = []
    for n in (16, 32, 64):
        h, u, F = _smooth_fields(n)
        rho = np.ones((n, n, n))
        p = oracle.make_params(n, n, n, nu=nu, gamma=gamma)
        r_F, u_F = oracle.fluid(p, rho, u, F)
        r_0, u_0 = oracle.fluid(p, rho, u, np.zeros_like(F))
        term = r_F * u_F - r_0 * u_0 - F / gamma
        # continuum value with spectral derivatives of the smooth products
        cont = _spectral_div(n, h, [[u[a] * F[c] + F[a] * u[c] for c in range(3)] for a in range(3)])
        cont *= -(tau - 0.5) / gamma**2
        errs.append(np.abs(term - cont).max() / np.abs(cont).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 1.9, (errs, orders)


# --------------------------------------------------------------------------------------------
# Closed forms: plane Poiseuille (B = 0) and plane Hartmann (uniform B normal to the walls)
# --------------------------------------------------------------------------------------------

def _plane_channel(ny, yc, a, **kw):
    X = np.concatenate([W.plane_wall_markers(1, 1, yc - a), W.plane_wall_markers(1, 1, yc + a)], 1)
    p = oracle.make_params(1, ny, 1, yc=float(yc), zc=0.0, radius=float(a), **kw)
    return p, X


@pytest.mark.parametrize("lattice", [19, 27])
def test_plane_poiseuille_is_exact(lattice):
    # Walls on lattice nodes (D = delta, d = 1): the steady discrete state is the parabola
    # G (a^2 - y^2) / (2 nu), exactly.
    oracle.set_threads(1)
    ny, yc, a, nu, G = 24, 12, 8, 0.1, 1e-5
    p, X = _plane_channel(ny, yc, a, nu=nu, eta=1.0, n_mag=1, G0=G, lattice=lattice)
    y = np.arange(ny) - yc
    u0 = np.zeros((3, 1, ny, 1))
    u0[0, 0, :, 0] = gold.plane_poiseuille_u(y, a, nu, G) * 0.9
    o = oracle.Oracle(p, X, u=u0)
    o.step(6000)
    inside = np.abs(y) <= a
    ref = gold.plane_poiseuille_u(y[inside], a, nu, G)
    got = o.u[0, 0, inside, 0]
    assert np.abs(got - ref).max() <= 1e-10 * ref.max()
    assert np.abs(o.u[1:]).max() <= 1e-14
    assert np.abs(o.rho - 1.0).max() <= 1e-12  # 6000 steps of round-off
    oracle.set_threads(8)


def _hartmann_fd(a, nu, eta, B0, G):
    """Steady 3-point finite-difference system nu u'' + B0 b' + G = 0, eta b'' + B0 u' = 0,
    u = b = 0 at y = +-a (central differences)."""
    n = 2 * a - 1
    A = np.zeros((2 * n, 2 * n))
    rhs = np.zeros(2 * n)
    for i in range(n):
        for (off, cu, cb) in ((-1, nu, -0.5 * B0), (0, -2 * nu, 0.0), (1, nu, 0.5 * B0)):
            j = i + off
            if 0 <= j < n:
                A[i, j] += cu
                A[i, n + j] += cb
        for (off, cb, cu) in ((-1, eta, -0.5 * B0), (0, -2 * eta, 0.0), (1, eta, 0.5 * B0)):
            j = i + off
            if 0 <= j < n:
                A[n + i, n + j] += cb
                A[n + i, j] += cu
        rhs[i] = -G
    sol = np.linalg.solve(A, rhs)
    return sol[:n], sol[n:]


def _hartmann_run(a, Ha, steps):
    ny = 2 * a + 8
    yc = ny // 2
    nu, eta, G = 0.1, 4.0, 1e-5
    B0 = Ha * math.sqrt(eta * nu) / a
    p, X = _plane_channel(ny, yc, a, nu=nu, eta=eta, n_mag=24, G0=G,
                          bext_kind=W.BEXT_UNIFORM_Y, B0=B0)
    y = (np.arange(ny) - yc).astype(float)
    uc, bc = gold.plane_hartmann(np.clip(y, -a, a), a, nu, eta, B0, G)
    u0 = np.zeros((3, 1, ny, 1))
    b0 = np.zeros((3, 1, ny, 1))
    inside = np.abs(y) < a
    u0[0, 0, inside, 0] = uc[inside]
    b0[0, 0, inside, 0] = bc[inside]
    o = oracle.Oracle(p, X, u=u0, b=b0)
    o.step(steps)
    prev = o.u.copy()
    o.step(200)
    assert np.abs(o.u - prev).max() <= 1e-9 * np.abs(o.u).max(), "not converged"
    return o, y, inside, (nu, eta, B0, G)


def test_plane_hartmann_matches_fd_system_and_closed_form():
    oracle.set_threads(1)
    errs = []
    for a in (8, 16):
        o, y, inside, (nu, eta, B0, G) = _hartmann_run(a, 4.0, 3000 if a == 8 else 8000)
        uf, bf = _hartmann_fd(a, nu, eta, B0, G)
        u = o.u[0, 0, inside, 0]
        b = o.b[0, 0, inside, 0]
        assert np.abs(u - uf).max() <= 1e-4 * np.abs(uf).max()
        assert np.abs(b - bf).max() <= 1e-4 * np.abs(bf).max()
        uc, bc = gold.plane_hartmann(y[inside], a, nu, eta, B0, G)
        errs.append(np.abs(u - uc).max() / np.abs(uc).max())
    order = math.log2(errs[0] / errs[1])
    assert order >= 1.9, (errs, order)
    oracle.set_threads(8)


# --------------------------------------------------------------------------------------------
# Pipe: conservation and symmetry of the whole step
# --------------------------------------------------------------------------------------------

def test_pipe_step_conserves_mass_to_roundoff():
    w = W.small_pipe(rho_amp=1e-3)
    p = oracle.make_params(w.nx, w.ny, w.nz, w.params, n_mag=40)
    o = oracle.Oracle(p, w.markers, w.rho, w.u, w.b)
    m0 = o.rho.sum()
    o.step(20)
    assert abs(o.rho.sum() - m0) <= 1e-13 * m0


def test_pipe_step_keeps_the_mirror_symmetries():
    # Uniform field along y, 88 markers per plane (a multiple of 4), integer centre:
    # u_x is even in y and z, b_x is odd in y and even in z.
    w = W.small_pipe(noise=0.0)
    p = oracle.make_params(w.nx, w.ny, w.nz, w.params, n_mag=60)
    o = oracle.Oracle(p, w.markers, w.rho, w.u, w.b)
    o.step(4)
    yc, zc, n = int(w.params.yc), int(w.params.zc), w.ny
    iy = (2 * yc - np.arange(n)) % n
    iz = (2 * zc - np.arange(w.nz)) % w.nz
    ux, bx = o.u[0], o.b[0]
    assert np.abs(ux).max() > 0 and np.abs(bx).max() > 0
    assert np.abs(ux - ux[:, iy, :]).max() <= 1e-12 * np.abs(ux).max()
    assert np.abs(ux - ux[iz, :, :]).max() <= 1e-12 * np.abs(ux).max()
    assert np.abs(bx + bx[:, iy, :]).max() <= 1e-12 * np.abs(bx).max()
    assert np.abs(bx - bx[iz, :, :]).max() <= 1e-12 * np.abs(bx).max()


# --------------------------------------------------------------------------------------------
# Gold's solution itself (Sec. 4)
# --------------------------------------------------------------------------------------------

def test_gold_series_solves_the_pipe_equations():
    R, nu, eta, G, Ha = 1.0, 1.0, 1.0, 1.0, 6.0
    B0 = Ha * math.sqrt(eta * nu) / R
    h = 2e-3
    pts = [(0.3, 0.2), (-0.5, 0.1), (0.1, -0.6), (0.0, 0.0), (0.55, 0.55)]
    for (yy, zz) in pts:
        def U(y, z):
            return gold.gold_u(np.hypot(y, z) / R, np.arctan2(z, y), Ha, R, nu, G)

        def Bx(y, z):
            return gold.gold_b(np.hypot(y, z) / R, np.arctan2(z, y), Ha, R, nu, eta, G)

        def lap(f):
            return (f(yy + h, zz) + f(yy - h, zz) + f(yy, zz + h) + f(yy, zz - h) - 4 * f(yy, zz)) / h**2

        def dy(f):
            return (f(yy + h, zz) - f(yy - h, zz)) / (2 * h)

        r1 = nu * lap(U) + B0 * dy(Bx) + G
        r2 = eta * lap(Bx) + B0 * dy(U)
        assert abs(r1) < 1e-4 * G and abs(r2) < 1e-4 * G * R * R / math.sqrt(eta * nu)
    th = np.linspace(0, 2 * np.pi, 37)
    umax = gold.gold_u(0.0, 0.0, Ha, R, nu, G)
    assert np.abs(gold.gold_u(1.0, th, Ha, R, nu, G)).max() < 1e-10 * umax
    assert np.abs(gold.gold_b(1.0, th, Ha, R, nu, eta, G)).max() < 1e-10 * umax


def test_gold_series_tends_to_poiseuille():
    r = np.linspace(0, 1, 7)
    for th in (0.0, 0.7, np.pi / 2):
        u = gold.gold_u(r, th, 0.05, 1.0, 1.0, 1.0)
        np.testing.assert_allclose(u, gold.poiseuille_pipe_u(r, 1.0, 1.0, 1.0), rtol=2e-4, atol=1e-9)


def test_plane_hartmann_closed_form_solves_its_ode():
    a, nu, eta, B0, G = 1.0, 0.3, 2.0, 3.0, 0.7
    y = np.linspace(-0.9, 0.9, 13)
    h = 1e-4
    u = lambda s: gold.plane_hartmann(s, a, nu, eta, B0, G)[0]
    b = lambda s: gold.plane_hartmann(s, a, nu, eta, B0, G)[1]
    d2 = lambda f: (f(y + h) - 2 * f(y) + f(y - h)) / h**2
    d1 = lambda f: (f(y + h) - f(y - h)) / (2 * h)
    np.testing.assert_allclose(nu * d2(u) + B0 * d1(b) + G, 0.0, atol=1e-5)
    np.testing.assert_allclose(eta * d2(b) + B0 * d1(u), 0.0, atol=1e-5)
    ua, ba = gold.plane_hartmann(np.array([-a, a]), a, nu, eta, B0, G)
    np.testing.assert_allclose(ua, 0.0, atol=1e-12)
    np.testing.assert_allclose(ba, 0.0, atol=1e-12)


def test_unsteady_kinetic_energy_balance_holds_step_by_step():
    # Sec. 4 energy balance under the variable force G(t) = G1 cos(2 pi t / T): the central
    # difference of the recorded E_k equals P_in + P_p + P_nu + P_L to the scheme's accuracy.
    w = W.small_pipe()
    p = oracle.make_params(w.nx, w.ny, w.nz, w.params, G0=0.0, G1=-3 * w.params.G0, period=200.0,
                           n_mag=60)
    o = oracle.Oracle(p, w.markers, w.rho, w.u, w.b)
    rec = []
    for _ in range(120):
        o.step(1)
        rec.append(o.budgets())
    E = np.array([r["E_k"] for r in rec])
    P = np.array([r["P_in"] + r["P_p"] + r["P_nu"] + r["P_L"] for r in rec])
    dE = (E[2:] - E[:-2]) / 2
    assert np.abs(dE).max() > 0.5 * max(abs(r["P_in"]) for r in rec)  # really unsteady
    assert np.abs(dE - P[1:-1]).max() <= 0.05 * np.abs(P).max()


# --------------------------------------------------------------------------------------------
# Six-magnet imposed field (Sec. 6)
# --------------------------------------------------------------------------------------------

def _magnet_params(n=40, R=14.0, B0=0.3):
    return oracle.make_params(8, n, n, bext_kind=W.BEXT_SIX_MAGNETS, B0=B0, radius=R, yc=n // 2,
                              zc=n // 2)


def test_six_magnet_field_is_harmonic_in_the_box():
    # Biot-Savart field outside its sources: divergence- and curl-free (central differences,
    # h = 1e-4, at seeded points of the box); this also makes the induced-field iteration exact
    # (reading of the unknown: lap B_ext = 0).
    p = _magnet_params()
    g = W.rng_for(120)
    h = 1e-4
    for y, z in g.uniform(0, 39, size=(25, 2)):
        def B(yy, zz):
            return oracle.bext_at(p, 0.0, yy, zz)
        dBdy = (B(y + h, z) - B(y - h, z)) / (2 * h)
        dBdz = (B(y, z + h) - B(y, z - h)) / (2 * h)
        scale = np.abs(dBdy).max() + np.abs(dBdz).max()
        assert abs(dBdy[1] + dBdz[2]) <= 1e-6 * scale
        assert abs(dBdy[2] - dBdz[1]) <= 1e-6 * scale
        assert B(y, z)[0] == 0.0


def test_six_magnet_field_alternates_under_a_sixth_turn_and_is_scaled_to_B0():
    p = _magnet_params()
    yc = zc = 20.0
    c, s = math.cos(math.pi / 3), math.sin(math.pi / 3)
    g = W.rng_for(121)
    for y, z in g.uniform(8, 32, size=(20, 2)):
        ry, rz = y - yc, z - zc
        B = oracle.bext_at(p, 0.0, y, z)
        Br = oracle.bext_at(p, 0.0, yc + c * ry - s * rz, zc + s * ry + c * rz)
        rot = np.array([c * B[1] - s * B[2], s * B[1] + c * B[2]])
        np.testing.assert_allclose(Br[1:], -rot, atol=1e-12 * np.abs(B).max())
    wall = oracle.bext_at(p, 0.0, yc + 14.0, zc)
    assert abs(np.linalg.norm(wall) - 0.3) < 1e-14
    # finite everywhere in the box: the strips lie outside it
    field = np.array([[oracle.bext(p, 0, y, z) for z in range(40)] for y in range(40)])
    assert np.isfinite(field).all() and np.abs(field).max() < 10 * 0.3


def test_six_magnet_flow_keeps_the_mirror_symmetries():
    # Odd box centred on the axis (the mirrors map the periodic box onto itself without using
    # the seam, where the non-periodic field jumps) and a ring of 88 markers: the hexapole is
    # symmetric under z -> -z and antisymmetric (alternating poles) under y -> -y, so u_x is
    # even in both and b_x odd in z, even in y.
    n = 33
    w = W.pipe_workload("six_magnets", 7, 8, n, n, 14.0, 50.0, 10.0, 1e-2,
                        bext_kind=W.BEXT_SIX_MAGNETS, noise=0.0)
    assert w.params.yc == (n - 1) / 2 and w.markers.shape[1] == 8 * 88
    p = oracle.make_params(w.nx, w.ny, w.nz, w.params, n_mag=20)
    o = oracle.Oracle(p, w.markers, w.rho, w.u, w.b)
    o.step(15)
    ux, bx = o.u[0], o.b[0]
    assert np.abs(ux).max() > 1e-4 and np.abs(bx).max() > 1e-6
    for f, sz, sy in ((ux, 1, 1), (bx, -1, 1)):
        s = np.abs(f).max()
        assert np.abs(np.flip(f, axis=0) - sz * f).max() <= 1e-11 * s
        assert np.abs(np.flip(f, axis=1) - sy * f).max() <= 1e-11 * s


def test_flow_rate_control_reaches_its_target():
    # Integral control of G on the bulk velocity over the flow region: at steady state the
    # plane channel carries the parabola whose node average equals the target, so
    # G = 2 nu U_t (2a + 1) / sum_{|y| <= a} (a^2 - y^2).
    oracle.set_threads(1)
    ny, yc, a, nu, Ut = 24, 12, 8, 0.1, 0.01
    p, X = _plane_channel(ny, yc, a, nu=nu, eta=1.0, n_mag=1, G0=0.0, flow_control=1,
                          u_target=Ut, k_c=1.0)
    o = oracle.Oracle(p, X)
    o.step(20000)
    y = np.arange(-a, a + 1)
    G_ss = 2 * nu * Ut * (2 * a + 1) / np.sum(a * a - y * y)
    assert abs(o.G.value - G_ss) <= 1e-6 * G_ss, (o.G.value, G_ss)
    ub = o.u[0, 0, yc - a:yc + a + 1, 0].mean()
    assert abs(ub - Ut) <= 1e-6 * Ut
    oracle.set_threads(8)
