"""Exact solution of the 1-D Riemann problem for an ideal gas.

Independent of the oracle: the pressure in the star region is the root of
the textbook pressure function (Toro, "Riemann Solvers and Numerical Methods
for Fluid Dynamics", ch. 4: shock branch from the Rankine-Hugoniot
conditions, rarefaction branch from the isentropic relations), found here
with a bracketed Brent iteration; the solution is then sampled on x/t.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def _f_and_speed(p, rho_k, p_k, gamma):
    """Velocity jump across the wave of side k as a function of star pressure."""
    c_k = math.sqrt(gamma * p_k / rho_k)
    if p > p_k:  # shock
        A = 2.0 / ((gamma + 1.0) * rho_k)
        B = (gamma - 1.0) / (gamma + 1.0) * p_k
        return (p - p_k) * math.sqrt(A / (p + B))
    # rarefaction
    return 2.0 * c_k / (gamma - 1.0) * ((p / p_k) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def star_state(rhoL, uL, pL, rhoR, uR, pR, gamma):
    def g(p):
        return _f_and_speed(p, rhoL, pL, gamma) + _f_and_speed(p, rhoR, pR, gamma) + (uR - uL)

    lo, hi = 1e-14, max(pL, pR)
    while g(hi) < 0.0:
        hi *= 2.0
    p_star = brentq(g, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    u_star = 0.5 * (uL + uR) + 0.5 * (_f_and_speed(p_star, rhoR, pR, gamma)
                                      - _f_and_speed(p_star, rhoL, pL, gamma))
    return p_star, u_star


def sample(xi, rhoL, uL, pL, rhoR, uR, pR, gamma):
    """(rho, u, p) at similarity coordinate xi = (x - x0)/t."""
    p_s, u_s = star_state(rhoL, uL, pL, rhoR, uR, pR, gamma)
    gm, gp = gamma - 1.0, gamma + 1.0
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    cL = math.sqrt(gamma * pL / rhoL)
    cR = math.sqrt(gamma * pR / rhoR)
    for n, s in enumerate(xi.flat):
        if s <= u_s:  # left of the contact
            if p_s > pL:  # left shock
                rho_sL = rhoL * ((p_s / pL + gm / gp) / (gm / gp * p_s / pL + 1.0))
                S = uL - cL * math.sqrt(gp / (2 * gamma) * p_s / pL + gm / (2 * gamma))
                vals = (rhoL, uL, pL) if s <= S else (rho_sL, u_s, p_s)
            else:  # left rarefaction
                rho_sL = rhoL * (p_s / pL) ** (1.0 / gamma)
                c_sL = cL * (p_s / pL) ** (gm / (2 * gamma))
                head, tail = uL - cL, u_s - c_sL
                if s <= head:
                    vals = (rhoL, uL, pL)
                elif s >= tail:
                    vals = (rho_sL, u_s, p_s)
                else:
                    uu = 2.0 / gp * (cL + gm / 2.0 * uL + s)
                    cc = 2.0 / gp * (cL + gm / 2.0 * (uL - s))
                    rr = rhoL * (cc / cL) ** (2.0 / gm)
                    vals = (rr, uu, pL * (cc / cL) ** (2.0 * gamma / gm))
        else:  # right of the contact
            if p_s > pR:  # right shock
                rho_sR = rhoR * ((p_s / pR + gm / gp) / (gm / gp * p_s / pR + 1.0))
                S = uR + cR * math.sqrt(gp / (2 * gamma) * p_s / pR + gm / (2 * gamma))
                vals = (rhoR, uR, pR) if s >= S else (rho_sR, u_s, p_s)
            else:  # right rarefaction
                rho_sR = rhoR * (p_s / pR) ** (1.0 / gamma)
                c_sR = cR * (p_s / pR) ** (gm / (2 * gamma))
                head, tail = uR + cR, u_s + c_sR
                if s >= head:
                    vals = (rhoR, uR, pR)
                elif s <= tail:
                    vals = (rho_sR, u_s, p_s)
                else:
                    uu = 2.0 / gp * (-cR + gm / 2.0 * uR + s)
                    cc = 2.0 / gp * (cR - gm / 2.0 * (uR - s))
                    rr = rhoR * (cc / cR) ** (2.0 / gm)
                    vals = (rr, uu, pR * (cc / cR) ** (2.0 * gamma / gm))
        rho.flat[n], u.flat[n], p.flat[n] = vals
    return rho, u, p


def cell_average_density(x_edges, t, x0, left, right, gamma, sub=64):
    """Exact cell averages of rho on [x_edges[i], x_edges[i+1]] at time t."""
    rhoL, uL, pL = left
    rhoR, uR, pR = right
    out = np.empty(len(x_edges) - 1)
    for i in range(len(out)):
        xs = np.linspace(x_edges[i], x_edges[i + 1], sub + 1)
        xm = 0.5 * (xs[1:] + xs[:-1])
        r, _, _ = sample((xm - x0) / t, rhoL, uL, pL, rhoR, uR, pR, gamma)
        out[i] = r.mean()
    return out
