"""Gold's closed-form solution for fully developed pipe flow under a uniform transverse field
(Sec. 4, the velocity and magnetic Gold solutions), plus plane Poiseuille / Hartmann forms.

TEST INFRASTRUCTURE ONLY (part of the oracle).

Conventions: lattice units; the pipe of radius R has its axis along x, the imposed field B0 points
along y and theta is measured from +y (the series carries cosh(alpha r cos theta), so r cos theta
is the coordinate along the field). r is normalised by R inside the series, alpha = Ha / 2, and
the pressure gradient dp/dx = -G. Ha = B0 R / sqrt(eta nu).
"""
from __future__ import annotations

import numpy as np
from scipy import special


def _ratio(n, a):
    """I'_n(a) / I_n(a)."""
    return special.ivp(n, a) / special.iv(n, a)


def _usable(n, a):
    """False once I_n(a) underflows (the remaining terms are below double precision)."""
    v = special.iv(n, a)
    return bool(np.isfinite(v) and v > 0.0)


def gold_u(rn, th, Ha, R, nu, G, nterms=60):
    """Axial velocity U_x(r, theta); rn = r / R in [0, 1]."""
    rn = np.asarray(rn, dtype=np.float64)
    th = np.asarray(th, dtype=np.float64)
    a = 0.5 * Ha
    even = np.zeros(np.broadcast(rn, th).shape)
    odd = np.zeros_like(even)
    for n in range(nterms):
        if not _usable(2 * n + 1, a):
            break
        eps = 1.0 if n == 0 else 2.0
        even = even + eps * _ratio(2 * n, a) * special.iv(2 * n, a * rn) * np.cos(2 * n * th)
        odd = odd + 2.0 * _ratio(2 * n + 1, a) * special.iv(2 * n + 1, a * rn) * np.cos((2 * n + 1) * th)
    arg = a * rn * np.cos(th)
    bracket = np.cosh(arg) * even - np.sinh(arg) * odd
    return -(R * R / (nu * Ha)) * (-G) * bracket


def gold_b(rn, th, Ha, R, nu, eta, G, nterms=60):
    """Induced axial field B_x(r, theta); rn = r / R in [0, 1]."""
    rn = np.asarray(rn, dtype=np.float64)
    th = np.asarray(th, dtype=np.float64)
    a = 0.5 * Ha
    arg = a * rn * np.cos(th)
    s = np.zeros(np.broadcast(rn, th).shape)
    for n in range(nterms):
        if not _usable(n, a):
            break
        # the n and -n terms of the exp(i n theta) series combine into eps_n cos(n theta)
        eps = 1.0 if n == 0 else 2.0
        term = (np.exp(-arg) - (-1.0) ** n * np.exp(arg)) * _ratio(n, a) * special.iv(n, a * rn)
        s = s + eps * term * np.cos(n * th)
    bracket = s - 2.0 * rn * np.cos(th)
    return -(1.0 / np.sqrt(eta * nu)) * (R * R / (2.0 * Ha)) * (-G) * bracket


def poiseuille_pipe_u(r, R, nu, G):
    """Ha = 0 limit: G (R^2 - r^2) / (4 nu)."""
    return G * (R * R - np.asarray(r) ** 2) / (4.0 * nu)


def plane_poiseuille_u(y, a, nu, G):
    """Plane channel |y| <= a: G (a^2 - y^2) / (2 nu)."""
    return G * (a * a - np.asarray(y) ** 2) / (2.0 * nu)


def plane_hartmann(y, a, nu, eta, B0, G):
    """Textbook Hartmann channel with insulating walls at |y| = a, field B0 along y.
    Returns (u, b) solving nu u'' + B0 b' + G = 0, eta b'' + B0 u' = 0, u = b = 0 at |y| = a."""
    y = np.asarray(y, dtype=np.float64)
    Ha = B0 * a / np.sqrt(eta * nu)
    u = (G * a * a / (nu * Ha)) * (np.cosh(Ha) - np.cosh(Ha * y / a)) / np.sinh(Ha)
    K = G * a * a / (nu * Ha * np.tanh(Ha))
    ubar = (G * a * a / (nu * Ha * Ha)) * (Ha / np.tanh(Ha) - 1.0)
    b = (B0 / eta) * ((ubar - K) * y + K * a * np.sinh(Ha * y / a) / (Ha * np.cosh(Ha)))
    return u, b
