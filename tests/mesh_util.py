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
