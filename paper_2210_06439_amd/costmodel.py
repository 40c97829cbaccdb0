"""Algorithmic cost of one hydro stage on one subgrid (for roofline reports).

Bytes: the stage must read each subgrid's 14^3 block of nf fields and write
its 8^3 interior: nf * 8 * (2744 + 512) bytes (plus 24 B of metadata and
8 B of amax, ignored).

FLOPs: the method's FP64 operations with every quantity that the definition
computes more than once counted once (a slope, an interface value or a
difference along a line is shared by neighbouring cells of that line; a
point state is shared by the faces it lies on).  Each +, -, *, /, sqrt, pow,
min, max and comparison counts 1; |x|, copysign and negation count 0.

  PPM per line (Colella-Woodward with MC slopes), per field:
    difference        1   (u_{m+1} - u_m)
    limited slope     8   (sum, *0.5, product test: *, cmp, 2|.| x2: *, *, min, min)
    interface value   5   (+, *0.5, -, *1/6, -)
    monotonicity     16   (2 -, *, cmp; dq, m6: -, +, *, -, *; dq*m6, dq*dq, 2 cmp; 3u-2q: *, *, -)
  point state        17   (1/rho; 3 velocities; e_k: 3 *, 2 +, *; e_i; switch: *, cmp;
                           p; c = sqrt(gamma p / rho): *, *, sqrt)
  face, per point and side: physical flux nf + 2; speeds u +- c: 2 +, 2 max/min
  face, per field: central-upwind point flux 6 x 9 points; Simpson 16
  face constants: a+, a-, a+ - a-, 1/(.), a+ a-, max(a+, -a-): 6 (+ 2 per point for the
                  speed reductions over the two sides)
  divergence, per cell and field: 3 -, 2 +, *, -  = 7
"""
from __future__ import annotations

import functools

NB, NI = 14, 8
CELLS = NI ** 3


def bytes_per_subgrid(nf: int) -> int:
    return nf * 8 * (NB ** 3 + NI ** 3)


def _lines():
    out = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                n = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)
                if n > 13:
                    out.append((dx, dy, dz))
    return out


def _needed_cells(d):
    """Cells whose values at c +- d/2 some face flux uses."""
    need = set()
    for k in range(3, 11):
        for j in range(3, 11):
            for i in range(3, 11):
                need.add((i, j, k))
    for axis in range(3):
        if d[axis] == 0:
            continue
        for a in range(3, 11):
            for b in range(3, 11):
                for layer in (2, 11):
                    c = [0, 0, 0]
                    c[axis] = layer
                    others = [x for x in range(3) if x != axis]
                    c[others[0]], c[others[1]] = a, b
                    need.add(tuple(c))
    return need


@functools.lru_cache(maxsize=None)
def ppm_flops_per_field() -> int:
    total = 0
    for d in _lines():
        M = _needed_cells(d)
        add = lambda c, m: (c[0] + m * d[0], c[1] + m * d[1], c[2] + m * d[2])
        I = set()                     # interfaces keyed by their left cell
        for c in M:
            I.add(add(c, -1))
            I.add(c)
        S = set()
        for c in I:
            S.add(c)
            S.add(add(c, 1))
        D = set()
        for c in S:
            D.add(add(c, -1))
            D.add(c)
        total += len(D) * 1 + len(S) * 8 + len(I) * 5 + len(M) * 16
    return total


def flops_per_subgrid(nf: int) -> int:
    ppm = ppm_flops_per_field() * nf
    points = CELLS * 26 + 6 * 64 * 9        # interior cells: 26; face-layer cells: 9
    states = points * 17
    faces = 3 * 576
    per_face = 9 * 2 * ((nf + 2) + 4) + 9 * 6 * nf + 16 * nf + 6 + 9 * 2
    div = CELLS * nf * 7 + 1
    return ppm + states + faces * per_face + div


def cost(n_species) -> tuple[int, int]:
    """(flops, bytes) of one stage over subgrids with these species counts."""
    fl = by = 0
    for ns in n_species:
        nf = 6 + int(ns)
        fl += flops_per_subgrid(nf)
        by += bytes_per_subgrid(nf)
    return fl, by
