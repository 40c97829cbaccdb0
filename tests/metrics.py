"""Error metrics shared by the parity tests.

The parity bar is a relative error per cell (`cell_rel`):

- density, total energy and the entropy tracer are strictly positive, so
  they take the plain relative error |g - o| / |o|, cell by cell;
- the momenta and the species can be zero (a fluid at rest, a species
  absent from a region), so they take a mixed relative error
  |g - o| / max(|o|, S_f), where S_f is a per-subgrid scale of the *input*:
  max |U_f| over the 14^3 block for a species, and max(|s| + sqrt(rho*egas))
  for the three momenta (a momentum scale that stays O(1) where the velocity
  is zero, as in the Sod-like data).

`mixed_rel` applies the scale floor to every field (the weaker, older
measure; reported beside the per-cell one).  Face fluxes use max|F_f| +
amax * S_f.
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


POSITIVE = (0, 4, 5)     # rho, egas, tau


def cell_rel(g: np.ndarray, o: np.ndarray, scale) -> np.ndarray:
    """The per-cell parity error of an [nf, ...] field array: plain relative
    error for the positive fields, mixed relative error for the others."""
    g = np.asarray(g, dtype=np.float64)
    o = np.asarray(o, dtype=np.float64)
    err = mixed_rel(g, o, scale)
    for f in POSITIVE:
        if f < o.shape[0]:
            d = np.abs(g[f] - o[f])
            pure = np.where(d == 0.0, 0.0, d / np.maximum(np.abs(o[f]), 1e-300))
            both_nan = np.isnan(g[f]) & np.isnan(o[f])
            err[f] = np.where(both_nan, 0.0, pure)
    return err


def max_err_step(batch, U_gpu, U_ref, idx=None, ref_batch=None) -> float:
    """Largest per-cell error (`cell_rel`) over the interiors of the
    subgrids idx (all by default); U_ref may be laid out as ref_batch."""
    return max_err_both(batch, U_gpu, U_ref, idx, ref_batch)[0]


def max_err_step_mixed(batch, U_gpu, U_ref, idx=None, ref_batch=None) -> float:
    """Largest mixed-relative error (`mixed_rel` on every field)."""
    return max_err_both(batch, U_gpu, U_ref, idx, ref_batch)[1]


def max_err_both(batch, U_gpu, U_ref, idx=None, ref_batch=None):
    """(largest per-cell error, largest mixed-relative error)."""
    idx = range(batch.n_sub) if idx is None else idx
    rb = batch if ref_batch is None else ref_batch
    worst = [0.0, 0.0]
    for n, s in enumerate(idx):
        S = field_scales(np.asarray(batch.block(s)))
        g = batch.interior(s, U_gpu)
        o = rb.interior(n if ref_batch is not None else s, U_ref)
        worst[0] = max(worst[0], float(np.max(cell_rel(g, o, S))))
        worst[1] = max(worst[1], float(np.max(mixed_rel(g, o, S))))
    return tuple(worst)
