"""Test-side mesh helpers: cut a global field into subgrid blocks with ghosts
from periodic wrap or zero-gradient padding, and put interiors back."""
from __future__ import annotations

import numpy as np

from paper_2210_06439_amd import inputs

NB, NI, NG = 14, 8, 3


def padded(G, periodic):
    """G[nf, Z, Y, X] with 3 ghost layers per side: wrap along periodic axes
    (given in x, y, z order), edge copy along the others."""
    out = G
    for a, per in enumerate(periodic):
        ax = 3 - a
        pad = [(0, 0)] * 4
        pad[ax] = (NG, NG)
        out = np.pad(out, pad, mode="wrap" if per else "edge")
    return out


def box_batch(G, nsub, h, periodic, dt=0.0):
    """Subgrids (x fastest) of the padded global field."""
    P = padded(G, periodic)
    nx, ny, nz = nsub
    blocks = []
    for bz in range(nz):
        for by in range(ny):
            for bx in range(nx):
                blocks.append(P[:, bz * NI:bz * NI + NB, by * NI:by * NI + NB,
                                bx * NI:bx * NI + NB].copy())
    return inputs.pack_blocks(blocks, [h] * len(blocks), dt=dt)


def interiors_to_global(batch, U, nsub):
    nx, ny, nz = nsub
    nf = 6 + int(batch.n_species[0])
    G = np.zeros((nf, nz * NI, ny * NI, nx * NI))
    for s in range(batch.n_sub):
        bx, by, bz = s % nx, (s // nx) % ny, s // (nx * ny)
        G[:, bz * NI:(bz + 1) * NI, by * NI:(by + 1) * NI, bx * NI:(bx + 1) * NI] = \
            batch.interior(s, U)
    return G


def refill(batch, nsub, periodic):
    """Ghost refill of a packed batch in place, from its own interiors."""
    def fill(U):
        ref = box_batch(interiors_to_global(batch, U, nsub), nsub, 1.0, periodic)
        for s in range(batch.n_sub):
            o = int(batch.offset[s])
            nf = 6 + int(batch.n_species[s])
            U[o:o + nf * batch.fstride] = ref.U[int(ref.offset[s]):int(ref.offset[s]) + nf * batch.fstride]
    return fill


def apply_map(batch, U, src, mode):
    """The ghost map's meaning, cell by cell (slow; small batches only)."""
    out = U.copy()
    for s in range(batch.n_sub):
        blk = batch.block(s, out)
        for k in range(NB):
            for j in range(NB):
                for i in range(NB):
                    d = [(-1 if x < NG else (1 if x >= NG + NI else 0)) for x in (i, j, k)]
                    if d == [0, 0, 0]:
                        continue
                    n = 9 * (d[2] + 1) + 3 * (d[1] + 1) + (d[0] + 1)
                    sb, m = int(src[s * 27 + n]), int(mode[s * 27 + n])
                    sidx = []
                    for a, x in enumerate((i, j, k)):
                        if d[a] == 0:
                            sidx.append(x)
                        elif m & (1 << a):
                            sidx.append(NG if x < NG else NG + NI - 1)
                        else:
                            sidx.append(x - NI * d[a])
                    sblk = batch.block(sb, U)
                    blk[:, k, j, i] = sblk[:, sidx[2], sidx[1], sidx[0]]
    return out


def generic_periodic_box(seed=97, n=16):
    """A periodic n^3 box (8^3 subgrids) of generic flow: smooth random
    velocity modes with cell noise, density and pressure jumps across
    different planes.  Unlike the rigidly rotating binary star, whose velocity
    has exactly zero divergence (so the sign of u_{j-1} - u_{j+1} on a line is
    decided by rounding), no Colella-Woodward detector sits on its threshold
    here."""
    rng = np.random.default_rng(seed)
    x = (np.arange(n) + 0.5) / n
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    rho = (1.0 + 0.3 * np.sin(2 * np.pi * (X + 0.3 * Y)) + np.where(Y > 0.5, 0.8, 0.0)
           + rng.uniform(0.0, 0.05, X.shape))
    p = (1.0 + 0.4 * np.cos(2 * np.pi * Z) + np.where(X > 0.5, 2.0, 0.0)
         + rng.uniform(0.0, 0.05, X.shape))
    v = [0.3 * np.sin(2 * np.pi * (X * a + Y * b + Z * c) + ph) + rng.normal(0.0, 0.02, X.shape)
         for a, b, c, ph in ((1, 0, 1, 0.1), (0, 1, 1, 0.7), (1, 1, 0, 1.3))]
    sp = [rho * w for w in rng.uniform(0.0, 0.2, (5,) + X.shape)]
    G = inputs.conserved_from_primitive(rho, v[0], v[1], v[2], p, sp)
    dt = inputs.cfl_dt(rho, v[0], v[1], v[2], p, 1.0 / n)
    return box_batch(G, (n // NI,) * 3, 1.0 / n, (True, True, True), dt=dt)
