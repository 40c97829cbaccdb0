"""Test-side time integration around a single-stage step function.

SSP-RK3 (Shu-Osher): U1 = U + dt L(U); U2 = 3/4 U + 1/4 (U1 + dt L(U1));
U3 = 1/3 U + 2/3 (U2 + dt L(U2)); ghosts refilled before every stage;
dt = C min_s(h_s / amax_s) with C = 0.4.  `step(U, dt) -> (U_out, amax)` is
either the oracle or the GPU library, so the same driver serves both.
"""
from __future__ import annotations

import numpy as np

from paper_2210_06439_amd import inputs


def rk3_evolve(batch, step, t_end, refill, C=0.4, max_steps=100000):
    """SSP-RK3 to t_end; the last step is cut to land exactly on t_end."""
    U = batch.U.copy()
    refill(U)
    t = 0.0
    nsteps = 0
    while t < t_end and nsteps < max_steps:
        _, amax = step(U, 0.0)
        dt = C * float(np.min(batch.h / amax))
        if dt < t_end - t:
            t_next = t + dt
        else:
            dt = t_end - t
            t_next = t_end
        U1, _ = step(U, dt)
        refill(U1)
        S1, _ = step(U1, dt)
        U2 = 0.75 * U + 0.25 * S1
        refill(U2)
        S2, _ = step(U2, dt)
        U = (1.0 / 3.0) * U + (2.0 / 3.0) * S2
        refill(U)
        t = t_next
        nsteps += 1
    return U, nsteps


def density_profile(batch, U, axis):
    """rho along the chain axis from the first transverse row of each subgrid."""
    vals = []
    for s in range(batch.n_sub):
        blk = batch.interior(s, U)[0]            # [z, y, x]
        if axis == 0:
            vals.append(blk[0, 0, :])
        elif axis == 1:
            vals.append(blk[0, :, 0])
        else:
            vals.append(blk[:, 0, 0])
    return np.concatenate(vals)


def sod_refill(batch, axis):
    def refill(U):
        inputs.fill_ghosts_periodic_chain(batch, U, axis, outflow=True)
    return refill
