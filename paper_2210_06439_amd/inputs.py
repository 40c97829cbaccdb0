"""Seeded synthetic inputs for the hydro step.

This module only builds input data: subgrid blocks of conserved fields with
their ghost layers filled, the per-subgrid metadata arrays, and request
streams for the serving loop.  It contains none of the hydro method's
arithmetic and imports neither the GPU library nor the CPU oracle, so both
sides of every parity test draw identical inputs from it.

Layout (one subgrid, field-major SoA): 8^3 interior cells plus 3 ghost
layers per side, 14^3 = 2744 cells per field, x fastest; field f of subgrid
s starts at ``offset[s] + f * fstride``.  Fields, in order:
rho, sx, sy, sz, egas, tau, spc_1..spc_ns (ns = 0 or 5).

The paper's workloads (a rotating star and a Sedov blast, both on 512 leaf
subgrids of 8^3 cells, Sec. V) need Octo-Tiger's own generators; the
workloads here are synthetic stand-ins with the same subgrid shape:

  config 1  one subgrid of i.i.d. random states
  config 2  64^3 periodic mesh (512 subgrids), perturbed planar Sod-like jump
  config 3  128^3 mesh (4096 subgrids), two Gaussian "stars" in rigid rotation
  config 4  uneven AMR-like batches of subgrids from levels 0-4 of config 3's field
  config 5  a Poisson stream of requests drawn from config 3's subgrids
"""
from __future__ import annotations

import dataclasses

import numpy as np

NB = 14                 # cells per dimension incl. ghosts
NG = 3                  # ghost layers
NI = 8                  # interior cells per dimension
NC = NB ** 3            # 2744 cells per field
FSTRIDE = 2752          # field stride in elements (2744 rounded up to 16 doubles)
GAMMA = 5.0 / 3.0


@dataclasses.dataclass
class SubgridBatch:
    """A packed batch of subgrids and its metadata arrays."""
    U: np.ndarray            # float64, flat
    offset: np.ndarray       # int64 [n_sub]
    h: np.ndarray            # float64 [n_sub]
    n_species: np.ndarray    # int32 [n_sub]
    fstride: int = FSTRIDE
    dt: float = 0.0          # a CFL-limited step size for this input (C = 0.4)
    name: str = ""

    @property
    def n_sub(self) -> int:
        return int(len(self.offset))

    def nf(self, s: int) -> int:
        return 6 + int(self.n_species[s])

    def block(self, s: int, U: np.ndarray | None = None) -> np.ndarray:
        """View [nf, 14, 14, 14] (z, y, x) of subgrid s."""
        U = self.U if U is None else U
        nf = self.nf(s)
        o = int(self.offset[s])
        return np.lib.stride_tricks.as_strided(
            U[o:], shape=(nf, NB, NB, NB),
            strides=(self.fstride * 8, NB * NB * 8, NB * 8, 8))

    def interior(self, s: int, U: np.ndarray | None = None) -> np.ndarray:
        return self.block(s, U)[:, NG:NG + NI, NG:NG + NI, NG:NG + NI]

    def subset(self, idx) -> "SubgridBatch":
        """A new packed batch holding the subgrids idx (copied)."""
        idx = np.asarray(idx, dtype=np.int64)
        blocks = [np.array(self.block(int(s))) for s in idx]
        return pack_blocks(blocks, self.h[idx], self.fstride, dt=self.dt,
                           name=f"{self.name}[subset]")

    @property
    def cell_updates(self) -> int:
        return self.n_sub * NI ** 3

    @property
    def bytes_algorithmic(self) -> int:
        """Bytes the step must move: read each 14^3 block, write its 8^3 interior."""
        nf = 6 + self.n_species.astype(np.int64)
        return int(np.sum(nf * 8 * (NC + NI ** 3)))


def packed_offsets(nfs, fstride=FSTRIDE) -> np.ndarray:
    sizes = np.asarray(nfs, dtype=np.int64) * fstride
    off = np.zeros(len(sizes), dtype=np.int64)
    if len(sizes) > 1:
        off[1:] = np.cumsum(sizes[:-1])
    return off


def pack_blocks(blocks, h, fstride=FSTRIDE, dt=0.0, name="") -> SubgridBatch:
    """Pack a list of [nf,14,14,14] blocks (nf = 6 or 11) into one flat buffer."""
    nfs = [b.shape[0] for b in blocks]
    for nf in nfs:
        assert nf in (6, 11), nf
    offset = packed_offsets(nfs, fstride)
    total = int(offset[-1] + nfs[-1] * fstride) if blocks else 0
    U = np.zeros(total, dtype=np.float64)
    for s, b in enumerate(blocks):
        o = int(offset[s])
        for f in range(b.shape[0]):
            U[o + f * fstride:o + f * fstride + NC] = b[f].reshape(-1)
    return SubgridBatch(U=U, offset=offset, h=np.asarray(h, dtype=np.float64).copy(),
                        n_species=np.asarray([nf - 6 for nf in nfs], dtype=np.int32),
                        fstride=fstride, dt=float(dt), name=name)


def conserved_from_primitive(rho, vx, vy, vz, p, species):
    """Conserved fields of an ideal gas (gamma = 5/3) from primitive samples.

    E = p/(gamma-1) + |s|^2/(2 rho), tau = (p/(gamma-1))^(1/gamma)."""
    sx, sy, sz = rho * vx, rho * vy, rho * vz
    eint = p / (GAMMA - 1.0)
    E = eint + 0.5 * (sx * sx + sy * sy + sz * sz) / rho
    tau = eint ** (1.0 / GAMMA)
    return np.stack([rho, sx, sy, sz, E, tau, *species])


def cfl_dt(rho, vx, vy, vz, p, h, C=0.4) -> float:
    """A step size C*h/max(|v|_inf + c) computed from the sampled primitives."""
    c = np.sqrt(GAMMA * p / rho)
    speed = np.maximum(np.maximum(np.abs(vx), np.abs(vy)), np.abs(vz)) + c
    return float(C * h / np.max(speed))


# ---------------------------------------------------------------- config 1 --

def config1(seed: int = 1001, n_species: int = 5) -> SubgridBatch:
    """One subgrid, h = 1/8, every cell (ghosts included) an i.i.d. state:
    rho ~ U[0.5,2], s ~ N(0, 0.1) per component, p ~ U[0.5,2], species
    weights w ~ U(0,1) with spc_k = rho w_k / sum(w)."""
    rng = np.random.default_rng(seed)
    shape = (NB, NB, NB)
    rho = rng.uniform(0.5, 2.0, shape)
    s = rng.normal(0.0, 0.1, (3,) + shape)
    p = rng.uniform(0.5, 2.0, shape)
    w = rng.uniform(0.0, 1.0, (5,) + shape)
    spc = [rho * w[k] / w.sum(axis=0) for k in range(n_species)]
    vx, vy, vz = s[0] / rho, s[1] / rho, s[2] / rho
    blk = conserved_from_primitive(rho, vx, vy, vz, p, spc)
    h = 1.0 / 8.0
    return pack_blocks([blk], [h], dt=cfl_dt(rho, vx, vy, vz, p, h), name="config1")


def random_batch(n_sub: int, seed: int, species=(5,)) -> SubgridBatch:
    """n_sub independent config-1-like subgrids; n_species drawn from `species`."""
    rng = np.random.default_rng(seed)
    blocks, hs, dts = [], [], []
    for s in range(n_sub):
        ns = int(rng.choice(np.asarray(species)))
        b = config1(seed=int(rng.integers(1 << 30)), n_species=ns)
        blocks.append(b.block(0).copy())
        hs.append(float(2.0 ** -int(rng.integers(3, 8))))
        dts.append(b.dt * hs[-1] / 0.125)
    return pack_blocks(blocks, hs, dt=min(dts), name=f"random{n_sub}")


# ------------------------------------------------------- mesh helpers -------

def _subgrids_from_global(G, nsub_per_dim, h, dt, name) -> SubgridBatch:
    """Cut a global array G[nf, Z, Y, X] that already holds 3 ghost layers on
    every side of an (8*nsub)^3 interior into 14^3 subgrid blocks."""
    blocks, hs = [], []
    n = nsub_per_dim
    for bz in range(n):
        for by in range(n):
            for bx in range(n):
                blocks.append(G[:, bz * NI:bz * NI + NB, by * NI:by * NI + NB,
                                bx * NI:bx * NI + NB])
                hs.append(h)
    return pack_blocks(blocks, hs, dt=dt, name=name)


def periodic_extend(G):
    """Add 3 periodic ghost layers on every side of G[nf, Z, Y, X]."""
    return np.pad(G, ((0, 0), (NG, NG), (NG, NG), (NG, NG)), mode="wrap")


# ---------------------------------------------------------------- config 2 --

def config2_fields(seed: int = 1002, N: int = 64):
    """Primitive fields of config 2 on the N^3 interior of the periodic box."""
    rng = np.random.default_rng(seed)
    nvec = rng.normal(size=3)
    nvec /= np.linalg.norm(nvec)
    ks = [k for k in np.ndindex(7, 7, 7) if k != (3, 3, 3)]
    k_rho = np.asarray(ks[rng.integers(len(ks))]) - 3
    k_p = np.asarray(ks[rng.integers(len(ks))]) - 3
    ph_rho, ph_p = rng.uniform(0, 2 * np.pi, 2)
    h = 1.0 / N
    c = (np.arange(N) + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    left = (nvec[0] * (X - 0.5) + nvec[1] * (Y - 0.5) + nvec[2] * (Z - 0.5)) < 0.0
    pert_r = 1.0 + 1e-3 * np.sin(2 * np.pi * (k_rho[0] * X + k_rho[1] * Y + k_rho[2] * Z) + ph_rho)
    pert_p = 1.0 + 1e-3 * np.sin(2 * np.pi * (k_p[0] * X + k_p[1] * Y + k_p[2] * Z) + ph_p)
    rho = np.where(left, 1.0, 0.125) * pert_r
    p = np.where(left, 1.0, 0.1) * pert_p
    zero = np.zeros_like(rho)
    fl = left.astype(np.float64)
    species = [0.6 * fl * rho, 0.6 * (1.0 - fl) * rho, 0.2 * rho, 0.1 * rho, 0.1 * rho]
    return rho, zero, zero, zero, p, species, h


def config2(seed: int = 1002, N: int = 64) -> SubgridBatch:
    """N^3 periodic mesh (N = 64: 512 subgrids), h = 1/N: a planar jump
    (rho, p) = (1, 1) | (0.125, 0.1) through the box centre with a seeded
    normal, each multiplied by 1 + 1e-3 sin(2 pi k.x + phi) with seeded
    integer k, zero velocity, 5 species.  Ghosts are periodic copies."""
    rho, vx, vy, vz, p, species, h = config2_fields(seed, N)
    G = periodic_extend(conserved_from_primitive(rho, vx, vy, vz, p, species))
    return _subgrids_from_global(G, N // NI, h, cfl_dt(rho, vx, vy, vz, p, h), "config2")


# ---------------------------------------------------------------- config 3 --

@dataclasses.dataclass
class BinaryStar:
    """Two Gaussian stars (sigma = 0.08, peaks 1 and 0.6, separation 0.4)
    over a 1e-10 floor, rigid rotation about z (Omega = 1), polytrope
    p = K rho^(5/3) with K = 1; species tag each star's core and envelope."""
    phi: float
    sigma: float = 0.08
    A1: float = 1.0
    A2: float = 0.6
    sep: float = 0.4
    floor: float = 1e-10
    omega: float = 1.0
    K: float = 1.0

    @classmethod
    def seeded(cls, seed: int = 1003) -> "BinaryStar":
        rng = np.random.default_rng(seed)
        return cls(phi=float(rng.uniform(0, 2 * np.pi)))

    def centres(self):
        e = np.array([np.cos(self.phi), np.sin(self.phi), 0.0])
        C = np.array([0.5, 0.5, 0.5])
        q = self.A2 / self.A1
        c1 = C - (q / (1 + q)) * self.sep * e
        c2 = C + (1 / (1 + q)) * self.sep * e
        return c1, c2

    def conserved(self, X, Y, Z):
        c1, c2 = self.centres()
        r1 = (X - c1[0]) ** 2 + (Y - c1[1]) ** 2 + (Z - c1[2]) ** 2
        r2 = (X - c2[0]) ** 2 + (Y - c2[1]) ** 2 + (Z - c2[2]) ** 2
        chi1 = np.exp(-r1 / (2 * self.sigma ** 2))
        chi2 = np.exp(-r2 / (2 * self.sigma ** 2))
        g1, g2 = self.A1 * chi1, self.A2 * chi2
        rho = g1 + g2 + self.floor
        vx = -self.omega * (Y - 0.5)
        vy = self.omega * (X - 0.5)
        vz = np.zeros_like(rho)
        p = self.K * rho ** (5.0 / 3.0)
        species = [g1 * chi1, g1 * (1 - chi1), g2 * chi2, g2 * (1 - chi2),
                   np.full_like(rho, self.floor)]
        return conserved_from_primitive(rho, vx, vy, vz, p, species), (rho, vx, vy, vz, p)

    def subgrid(self, origin, h, n_species=5):
        """One 14^3 block with lower interior corner at `origin`, ghosts evaluated
        analytically at their cell centres."""
        c = (np.arange(NB) - NG + 0.5) * h
        Z, Y, X = np.meshgrid(origin[2] + c, origin[1] + c, origin[0] + c, indexing="ij")
        U, prim = self.conserved(X, Y, Z)
        return U[:6 + n_species], prim


def config3(seed: int = 1003, N: int = 128) -> SubgridBatch:
    """128^3 uniform mesh = 4096 subgrids (h = 1/128) of the binary star field;
    ghosts evaluated analytically (so a ghost equals its neighbour's interior)."""
    star = BinaryStar.seeded(seed)
    h = 1.0 / N
    c = (np.arange(N + 2 * NG) - NG + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    G, (rho, vx, vy, vz, p) = star.conserved(X, Y, Z)
    del X, Y, Z
    dt = cfl_dt(rho, vx, vy, vz, p, h)
    return _subgrids_from_global(G, N // NI, h, dt, "config3")


def config3_subgrid16(seed: int = 1003, N: int = 128):
    """Config 3's field cut into 16^3 subgrids (22^3 cells per field with the
    ghosts, field stride 10656) for the library built for that size: 512
    subgrids at N = 128.  Returns (U, offset, h, n_species, fstride, dt)."""
    n, nb = 16, 22
    fstride = (nb ** 3 + 15) // 16 * 16
    star = BinaryStar.seeded(seed)
    h = 1.0 / N
    c = (np.arange(N + 2 * NG) - NG + 0.5) * h
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    G, (rho, vx, vy, vz, p) = star.conserved(X, Y, Z)
    del X, Y, Z
    dt = cfl_dt(rho, vx, vy, vz, p, h)
    m = N // n
    nf = G.shape[0]
    U = np.zeros(m ** 3 * nf * fstride)
    offset = np.arange(m ** 3, dtype=np.int64) * nf * fstride
    s = 0
    for bz in range(m):
        for by in range(m):
            for bx in range(m):
                blk = G[:, bz * n:bz * n + nb, by * n:by * n + nb, bx * n:bx * n + nb]
                o = int(offset[s])
                for f in range(nf):
                    U[o + f * fstride:o + f * fstride + nb ** 3] = blk[f].reshape(-1)
                s += 1
    return (U, offset, np.full(m ** 3, h), np.full(m ** 3, nf - 6, dtype=np.int32), fstride,
            dt)


# ---------------------------------------------------------------- config 4 --

def config4(seed: int = 1004, launch: int = 0, max_sub: int = 8192,
            n_override: int | None = None) -> SubgridBatch:
    """One uneven AMR-like batch: n = clip(round(lognormal(ln 256, 1.5)), 1, 8192)
    subgrids; level l in 0..4 with P(l) ~ 2^l and h_l = 2^-(4+l); origins on
    the level-l lattice (uniform for l <= 1, near a star centre for l >= 2,
    chosen in proportion to mass); n_species 0 or 5 with probability 1/2."""
    rng = np.random.default_rng([seed, launch])
    star = BinaryStar.seeded(1003)
    n = int(np.clip(round(float(np.exp(rng.normal(np.log(256), 1.5)))), 1, max_sub))
    if n_override is not None:
        n = int(n_override)
    levels = np.arange(5)
    pl = 2.0 ** levels / np.sum(2.0 ** levels)
    c1, c2 = star.centres()
    mass = np.array([star.A1, star.A2]) / (star.A1 + star.A2)
    blocks, hs, dts = [], [], []
    for _ in range(n):
        lev = int(rng.choice(levels, p=pl))
        h = 2.0 ** -(4 + lev)
        step = NI * h
        nblk = int(round(1.0 / step))
        if lev <= 1:
            o = rng.integers(0, nblk, 3) * step
        else:
            cc = c1 if rng.uniform() < mass[0] else c2
            x = cc + rng.normal(0.0, 1.5 * star.sigma, 3)
            o = np.clip(np.floor(x / step), 0, nblk - 1) * step
        ns = 5 if rng.uniform() < 0.5 else 0
        blk, (rho, vx, vy, vz, p) = star.subgrid(o, h, ns)
        blocks.append(blk)
        hs.append(h)
        dts.append(cfl_dt(rho, vx, vy, vz, p, h))
    return pack_blocks(blocks, hs, dt=min(dts), name=f"config4[{launch}]")


# ---------------------------------------------------------------- config 5 --

def config5_requests(n_requests: int, rate: float, seed: int = 1005, pool: int = 4096,
                     max_sub: int = 4096, median_n: float = 128.0, sigma: float = 1.5,
                     steps=(1, 2, 4)):
    """Request stream: Poisson(rate) arrivals; sizes
    clip(round(lognormal(ln median_n, sigma)), 1, min(max_sub, pool)) subgrids
    drawn without replacement from a pool of subgrids; session length S
    uniform over `steps`.  Returns (arrival seconds, subgrid indices, S) per
    request."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n_requests))
    out = []
    for i in range(n_requests):
        n = int(np.clip(np.round(np.exp(rng.normal(np.log(median_n), sigma))), 1,
                        min(max_sub, pool)))
        idx = np.sort(rng.choice(pool, size=n, replace=False))
        out.append((float(t[i]), idx, int(rng.choice(steps))))
    return out


# ------------------------------------------------------------- Sedov blast --

def sedov(N: int = 64, E0: float = 1.0, r0_cells: float = 3.5, p_amb: float = 1e-5,
          n_species: int = 0) -> SubgridBatch:
    """Point blast in the periodic unit box (N = 64: 512 subgrids, the
    paper's hydro-only blast-wave grid): rho = 1, v = 0, pressure p_amb, plus
    the energy E0 spread evenly as internal energy over the cells whose
    centres lie within r0_cells cells of the box centre (a cell corner).
    Species, if any, are fixed fractions (0.3, 0.25, 0.2, 0.15, 0.1) of rho.
    The batch's dt is left 0: the step size comes from the CFL condition."""
    h = 1.0 / N
    c = (np.arange(N) + 0.5) * h - 0.5
    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    hot = (X * X + Y * Y + Z * Z) <= (r0_cells * h) ** 2
    n_hot = int(np.count_nonzero(hot))
    eint = np.where(hot, E0 / (n_hot * h ** 3), 0.0) + p_amb / (GAMMA - 1.0)
    rho = np.ones_like(X)
    p = (GAMMA - 1.0) * eint
    zero = np.zeros_like(rho)
    frac = (0.3, 0.25, 0.2, 0.15, 0.1)
    species = [frac[k] * rho for k in range(n_species)]
    G = periodic_extend(conserved_from_primitive(rho, zero, zero, zero, p, species))
    return _subgrids_from_global(G, N // NI, h, 0.0, f"sedov{N}")


def sedov_energy(batch: SubgridBatch, U: np.ndarray | None = None) -> float:
    """Total energy sum(E) h^3 over the interiors."""
    tot = 0.0
    for s in range(batch.n_sub):
        tot += float(np.sum(batch.interior(s, U)[4])) * float(batch.h[s]) ** 3
    return tot


# ------------------------------------------------------------ ghost fills --

def fill_ghosts_periodic_chain(batch: SubgridBatch, U: np.ndarray, axis: int,
                               outflow: bool) -> None:
    """Refill ghosts of a chain of subgrids laid end to end along `axis`
    (subgrid s is followed by s+1), uniform transversally.  Along `axis`,
    ghosts come from the neighbour's interior; the chain ends get a
    zero-gradient copy (outflow=True) or wrap around (periodic).  The two
    transverse directions are periodic within each subgrid."""
    n = batch.n_sub
    ax = 3 - axis            # block axes are (f, z, y, x)
    blocks = [batch.block(s, U) for s in range(n)]
    lo_g, hi_g = slice(0, NG), slice(NG + NI, NB)
    for s in range(n):
        b = blocks[s]
        prev = blocks[s - 1] if s > 0 else (None if outflow else blocks[n - 1])
        nxt = blocks[s + 1] if s < n - 1 else (None if outflow else blocks[0])

        def sl(a, idx):
            out = [slice(None)] * 4
            out[a] = idx
            return tuple(out)

        if prev is None:
            edge = b[sl(ax, slice(NG, NG + 1))]
            b[sl(ax, lo_g)] = np.repeat(edge, NG, axis=ax)
        else:
            b[sl(ax, lo_g)] = prev[sl(ax, slice(NI, NI + NG))]
        if nxt is None:
            edge = b[sl(ax, slice(NG + NI - 1, NG + NI))]
            b[sl(ax, hi_g)] = np.repeat(edge, NG, axis=ax)
        else:
            b[sl(ax, hi_g)] = nxt[sl(ax, slice(NG, 2 * NG))]
    # transverse: periodic within each subgrid (data is uniform transversally)
    for s in range(n):
        b = blocks[s]
        for t_ax in (1, 2, 3):
            if t_ax == ax:
                continue

            def sl2(idx):
                out = [slice(None)] * 4
                out[t_ax] = idx
                return tuple(out)

            b[sl2(lo_g)] = b[sl2(slice(NI, NI + NG))]
            b[sl2(hi_g)] = b[sl2(slice(NG, 2 * NG))]


def sod_chain(N: int, axis: int = 0, n_species: int = 0):
    """A 1-D Sod tube of N cells along `axis` as a chain of N/8 subgrids:
    (rho, u, p) = (1, 0, 1) for x < 0.5 and (0.125, 0, 0.1) beyond, uniform
    in the transverse directions, outflow ghosts at both ends."""
    assert N % NI == 0
    h = 1.0 / N
    nsub = N // NI
    blocks = []
    for s in range(nsub):
        x = (s * NI + np.arange(NB) - NG + 0.5) * h
        rho1 = np.where(x < 0.5, 1.0, 0.125)
        p1 = np.where(x < 0.5, 1.0, 0.1)
        shape = [1, 1, 1]
        shape[2 - axis] = NB
        rho = np.broadcast_to(rho1.reshape(shape), (NB, NB, NB)).copy()
        p = np.broadcast_to(p1.reshape(shape), (NB, NB, NB)).copy()
        zero = np.zeros_like(rho)
        spc = [rho * (0.2 if k else 0.2) for k in range(n_species)]
        blocks.append(conserved_from_primitive(rho, zero, zero, zero, p, spc))
    b = pack_blocks(blocks, [h] * nsub, name=f"sod{N}")
    fill_ghosts_periodic_chain(b, b.U, axis, outflow=True)
    return b
