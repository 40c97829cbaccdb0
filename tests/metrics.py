"""Error metrics shared by the parity tests.

Mixed relative error per cell (the parity bar): for field f of subgrid s,

    err = |g - o| / max(|o|, S_f)

where S_f is a per-subgrid scale of the *input*: max |U_f| over the 14^3
block for rho, egas, tau and the species, and max(|s| + sqrt(rho*egas)) for
the three momenta (a momentum scale that stays O(1) where the velocity is
zero, as in the Sod-like data).  Face fluxes use max|F_f| + amax * S_f.
"""
from __future__ import annotations

import numpy as np

NB = 14


def field_scales(block: np.ndarray) -> np.ndarray:
    """S_f for one [nf,14,14,14] input block."""
    nf = block.shape[0]
    S = np.max(np.abs(block.reshape(nf, -1)), axis=1)
    rho, sx, sy, sz, E = block[0], block[1], block[2], block[3], block[4]
    mom = np.sqrt(sx * sx + sy * sy + sz * sz) + np.sqrt(np.abs(rho * E))
    S[1:4] = np.max(mom)
    return np.where(S > 0, S, 1.0)


def mixed_rel(g: np.ndarray, o: np.ndarray, scale) -> np.ndarray:
    """|g-o| / max(|o|, scale), scale broadcast along the leading field axis."""
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    sc = np.asarray(scale, dtype=np.float64).reshape((-1,) + (1,) * (o.ndim - 1))
    den = np.maximum(np.abs(o), sc)
    err = np.abs(g - o) / den
    both_nan = np.isnan(g) & np.isnan(o)
    return np.where(both_nan, 0.0, err)


def max_err_step(batch, U_gpu, U_ref) -> float:
    """Largest mixed-relative error over the interiors of all subgrids."""
    worst = 0.0
    for s in range(batch.n_sub):
        S = field_scales(np.asarray(batch.block(s)))
        e = mixed_rel(batch.interior(s, U_gpu), batch.interior(s, U_ref), S)
        worst = max(worst, float(np.max(e)))
    return worst
