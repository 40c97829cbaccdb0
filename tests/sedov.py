"""Sedov-Taylor point blast in 3-D: the self-similar solution, integrated from
the Euler equations (test infrastructure for the blast-wave workload of
Sec. V, Test 3).

With the shock at R(t) = xi0 (E t^2 / rho0)^(1/5) and eta = r / R, write
    u = R' f(eta),   rho = rho0 g(eta),   p = rho0 R'^2 h(eta).
Because R'' = -(3/2) R'^2 / R, mass, momentum and entropy conservation become
    g f' + (f - eta) g'                      = -2 g f / eta
    (f - eta) f' + h' / g                    = (3/2) f
    -gamma (f - eta) g' / g + (f - eta) h'/h = 3
with the strong-shock values f = 2/(gamma+1), g = (gamma+1)/(gamma-1),
h = 2/(gamma+1) at eta = 1.  The blast energy fixes xi0:
    E = 4 pi R^3 rho0 R'^2 I,  I = int_0^1 (g f^2 / 2 + h / (gamma-1)) eta^2 d eta,
and R^3 R'^2 = (4/25) xi0^5 E / rho0, so xi0 = (25 / (16 pi I))^(1/5).
"""
from __future__ import annotations

import functools

import numpy as np
from scipy.integrate import solve_ivp


def _rhs(eta, y, gamma):
    f, g, h = y
    a = f - eta
    # [ g        a         0   ] [f']   [ -2 g f / eta ]
    # [ a        0       1/g   ] [g'] = [ 1.5 f        ]
    # [ 0  -gamma a/g    a/h   ] [h']   [ 3            ]
    M = np.array([[g, a, 0.0],
                  [a, 0.0, 1.0 / g],
                  [0.0, -gamma * a / g, a / h]])
    b = np.array([-2.0 * g * f / eta, 1.5 * f, 3.0])
    return np.linalg.solve(M, b)


@functools.lru_cache(maxsize=8)
def profile(gamma: float, eta_min: float = 1e-3, n: int = 4001):
    """(eta, f, g, h) on a grid from 1 down to eta_min, and xi0."""
    y0 = [2.0 / (gamma + 1.0), (gamma + 1.0) / (gamma - 1.0), 2.0 / (gamma + 1.0)]
    etas = np.linspace(1.0, eta_min, n)
    sol = solve_ivp(_rhs, (1.0, eta_min), y0, t_eval=etas, args=(gamma,),
                    rtol=1e-11, atol=1e-14, method="DOP853")
    assert sol.success, sol.message
    eta = sol.t[::-1]
    f, g, h = (v[::-1] for v in sol.y)
    integrand = (0.5 * g * f * f + h / (gamma - 1.0)) * eta * eta
    I = float(np.trapezoid(integrand, eta))
    xi0 = (25.0 / (16.0 * np.pi * I)) ** 0.2
    return eta, f, g, h, xi0


def xi0(gamma: float) -> float:
    return profile(gamma)[4]


def shock_radius(t, E, rho0, gamma):
    return xi0(gamma) * (E * t * t / rho0) ** 0.2


def density(r, t, E, rho0, gamma):
    """Exact density at radius r (ambient rho0 outside the shock)."""
    eta, f, g, h, x0 = profile(gamma)
    R = shock_radius(t, E, rho0, gamma)
    x = np.asarray(r, dtype=np.float64) / R
    out = np.full_like(x, rho0)
    inside = x < 1.0
    out[inside] = rho0 * np.interp(x[inside], eta, g, left=0.0)
    return out
