"""The library built for 16^3 subgrids (libhydro_n16.so; the subgrid size is
a compile-time choice, Sec. II "Data-Structure") against the oracle built for
the same size: the plain stages bitwise, with every method option; the
fused step, which runs each subgrid's eight 8^3 tiles through the 8^3 fused
kernel (bitwise the 8^3 library on those tiles, and within the parity
tolerance of the 16^3 oracle); the entropy-tracer re-sync, the ghost fill and
the stage combination; and the refusal of the other fused entry points."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_util import gpu_step, torch
from metrics import max_err_step
from paper_2210_06439_amd import hydro, inputs
from test_oracle_subgrid16 import _interior, _pack, _padded_field

pytestmark = pytest.mark.gpu

N = 16
NB = N + 6
SYM, VEL, ST, FL = hydro.KT_SYMMETRIC, hydro.VELOCITY, hydro.STEEPEN, hydro.FLATTEN
EINVAL = -1


def _batch(seeds=(80, 81), species=(5, 0), h=1.0 / 64):
    blocks = []
    for seed, ns in zip(seeds, species):
        P = _padded_field(seed)
        blocks.append(np.concatenate([P[:6], P[6:6 + ns]]))
    # _pack takes one nf for all blocks: pack each and concatenate
    parts = [_pack([b], N, h, 0.0) for b in blocks]
    U = np.concatenate([p[0] for p in parts])
    sizes = np.array([len(p[0]) for p in parts], dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
    fs = parts[0][4]
    return U, off, np.full(len(blocks), h), np.array(species, np.int32), fs


def _device(U, off, h, ns, fs):
    return hydro.DeviceBatch(U, off, h, ns, fs, n=N)


def _plain(db, dt, flags):
    T = torch()
    prm = hydro.params(dt=dt, flags=flags)
    qo, qn = db.q_layout()
    fo, fn = db.f_layout()
    Q = T.zeros(qn, dtype=T.float64, device="cuda")
    F = T.zeros(fn, dtype=T.float64, device="cuda")
    amax = T.zeros(db.n_sub, dtype=T.float64, device="cuda")
    status = T.zeros(db.n_sub, dtype=T.int32, device="cuda")
    U_out = db.U.clone()
    hydro.reconstruct(prm, db.struct, db.U, Q, qo, n=N)
    hydro.flux(prm, db.struct, Q, qo, F, fo, amax, status, n=N)
    hydro.divergence(prm, db.struct, F, fo, db.U, U_out, n=N)
    T.cuda.synchronize()
    return (Q.cpu().numpy(), F.cpu().numpy(), U_out.cpu().numpy(), amax.cpu().numpy(),
            status.cpu().numpy())


@pytest.mark.parametrize("flags", [0, SYM, VEL, ST | FL, VEL | ST | FL])
def test_plain_stages_bitwise(flags):
    U, off, h, ns, fs = _batch()
    dt = 2e-4
    Qg, Fg, Ug, ag, sg = _plain(_device(U, off, h, ns, fs), dt, flags)
    Q, qo = oracle.reconstruct(U, off, h, ns, fs, flags=flags, n=N)
    assert np.array_equal(Qg, Q)
    F, fo, a, st = oracle.flux(Q, qo, off, h, ns, fs, flags=flags, n=N)
    assert np.array_equal(Fg, F) and np.array_equal(ag, a) and np.array_equal(sg, st)
    Ur, ar, sr = oracle.step(U, off, h, ns, fs, dt, flags=flags, n=N)
    for s in range(len(off)):
        nf = 6 + int(ns[s])
        assert np.array_equal(_interior(Ug, off, fs, nf, N, s), _interior(Ur, off, fs, nf, N, s))
    assert np.array_equal(ag, ar)


def _fused16(db, dt, flags=0):
    T = torch()
    L = hydro.lib(N)
    out = db.U.clone()
    amax = T.zeros(db.n_sub, dtype=T.float64, device="cuda")
    status = T.zeros(db.n_sub, dtype=T.int32, device="cuda")
    prm = hydro.params(dt=dt, flags=flags)
    assert L.hydro_step(ctypes.byref(prm), ctypes.byref(db.struct), hydro._ptr(db.U),
                        hydro._ptr(out), hydro._ptr(amax), hydro._ptr(status), None) == 0
    T.cuda.synchronize()
    return out.cpu().numpy(), amax.cpu().numpy(), status.cpu().numpy()


@pytest.mark.parametrize("flags", [0, SYM | VEL, ST | FL])
def test_fused_step_16_is_its_tiles_step(flags):
    """The 16^3 fused step against the 8^3 library on the eight tiles of each
    subgrid (bitwise: interiors, the largest speed over the tiles, status),
    and against the 16^3 oracle within the parity tolerance."""
    U, off, h, ns, fs = _batch()
    dt = 2e-4
    Ug, ag, sg = _fused16(_device(U, off, h, ns, fs), dt, flags)
    tiles, th = [], []
    for s in range(len(off)):
        nf = 6 + int(ns[s])
        blk = np.stack([U[off[s] + f * fs:off[s] + f * fs + NB ** 3].reshape(NB, NB, NB)
                        for f in range(nf)])
        for bz in (0, 1):
            for by in (0, 1):
                for bx in (0, 1):
                    tiles.append(blk[:, bz * 8:bz * 8 + 14, by * 8:by * 8 + 14,
                                     bx * 8:bx * 8 + 14].copy())
                    th.append(h[s])
    tb = inputs.pack_blocks(tiles, th, dt=dt)
    Ut, at, st = gpu_step(tb, flags=flags)
    Ur, ar, sr = oracle.step(U, off, h, ns, fs, dt, flags=flags, n=N)
    Urt, art, srt = oracle.step(tb.U, tb.offset, tb.h, tb.n_species, tb.fstride, dt, flags=flags)
    for s in range(len(off)):
        nf = 6 + int(ns[s])
        g = _interior(Ug, off, fs, nf, N, s)
        r = _interior(Ur, off, fs, nf, N, s)
        for q in range(8):
            bz, by, bx = q >> 2, (q >> 1) & 1, q & 1
            sl = np.s_[:, bz * 8:bz * 8 + 8, by * 8:by * 8 + 8, bx * 8:bx * 8 + 8]
            assert np.array_equal(g[sl], tb.interior(8 * s + q, Ut)), (s, q)
            # the 16^3 oracle is its tiles' 8^3 oracle (the locality pin)
            assert np.array_equal(r[sl], tb.interior(8 * s + q, Urt)), (s, q)
        assert ag[s] == np.max(at[8 * s:8 * s + 8])
        assert sg[s] == np.bitwise_or.reduce(st[8 * s:8 * s + 8])
    assert max_err_step(tb, Ut, Urt) <= 1e-12
    assert np.max(np.abs(ag - ar) / ar) <= 1e-13 and np.array_equal(sg, sr)


def test_fused_step_16_flags_each_subgrid_alone():
    """Invalid metadata in one subgrid: its status is the bad-metadata bit and
    its output block is left as it was.  A NaN in another's interior: that
    subgrid gets the 16^3 oracle's status word (the non-finite bit among
    them).  The clean subgrid's results are those it has alone."""
    T = torch()
    U, off, h, ns, fs = _batch(seeds=(80, 81, 82), species=(5, 0, 5))
    U = U.copy()
    U[off[2] + (5 * NB + 7) * NB + 9] = np.nan       # density of interior cell (9, 7, 5)
    dt = 2e-4
    db = _device(U, off, h, ns, fs)
    db.n_species[1] = 9
    Ug, ag, sg = _fused16(db, dt)
    assert sg[1] == hydro.STATUS_BADMETA
    assert np.array_equal(Ug[off[1]:off[2]], U[off[1]:off[2]])
    Ur, ar, sr = oracle.step(U, off, h, ns, fs, dt, n=N)
    assert sg[2] == sr[2] and sg[2] & hydro.STATUS_NONFINITE
    Ua, aa, sa = _fused16(_device(U[:off[1]].copy(), off[:1], h[:1], ns[:1], fs), dt)
    assert np.array_equal(_interior(Ug, off, fs, 11, N, 0), _interior(Ua, off[:1], fs, 11, N, 0))
    assert ag[0] == aa[0] and sg[0] == sa[0] == 0 == sr[0]
    T.cuda.synchronize()


def test_other_fused_entry_points_refuse_the_16_build():
    T = torch()
    U, off, h, ns, fs = _batch()
    db = _device(U, off, h, ns, fs)
    L = hydro.lib(N)
    out = db.U.clone()
    amax = T.zeros(db.n_sub, dtype=T.float64, device="cuda")
    prm = hydro.params(dt=1e-4)
    assert L.hydro_step_variant(ctypes.byref(prm), ctypes.byref(db.struct), hydro._ptr(db.U),
                                hydro._ptr(out), hydro._ptr(amax), None, 1, None) == EINVAL
    assert L.hydro_rate(ctypes.byref(prm), ctypes.byref(db.struct), hydro._ptr(db.U),
                        hydro._ptr(out), hydro._ptr(amax), None, None) == EINVAL
    T.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), U)


def test_tau_resync_16():
    T = torch()
    U, off, h, ns, fs = _batch()
    # cold cells: lower the total energy of a slab of every subgrid
    for s in range(len(off)):
        e = U[off[s] + 4 * fs:off[s] + 4 * fs + NB ** 3].reshape(NB, NB, NB)
        rho = U[off[s]:off[s] + NB ** 3].reshape(NB, NB, NB)
        sx = U[off[s] + fs:off[s] + fs + NB ** 3].reshape(NB, NB, NB)
        e[:, :, :8] = 0.5 * sx[:, :, :8] ** 2 / rho[:, :, :8] * (1.0 + 1e-5)
    db = _device(U, off, h, ns, fs)
    hydro.tau_resync(hydro.params(), db.struct, db.U, n=N)
    T.cuda.synchronize()
    Ug = db.U.cpu().numpy()
    Ur = oracle.tau_resync(U, off, h, ns, fs, n=N)
    changed = 0
    for s in range(len(off)):
        nf = 6 + int(ns[s])
        g, r, i0 = (_interior(x, off, fs, nf, N, s) for x in (Ug, Ur, U))
        assert np.array_equal(np.delete(g, 5, axis=0), np.delete(r, 5, axis=0))
        assert np.all(np.abs(g[5] - r[5]) <= 4 * 2.0 ** -52 * np.abs(r[5]))
        changed += int(np.count_nonzero(r[5] != i0[5]))
        assert np.array_equal(r[5][:, :, :5], i0[5][:, :, :5])   # the cold slab keeps tau
    # the initial tau is e_i^(1/gamma) already, so only cells whose pow rounds
    # differently from the packing's change
    assert changed > 100
    # ghosts untouched
    assert np.array_equal(Ug[off[0]:off[0] + NB ** 2], U[off[0]:off[0] + NB ** 2])


def test_fill_ghosts_16_periodic_box():
    """A 2 x 2 x 1 periodic box of 16^3 subgrids: after the fill every block
    equals the wrap-padded global field cut at its position."""
    T = torch()
    rng = np.random.default_rng(95)
    nx, ny, nz, nf = 2, 2, 1, 6
    G = rng.normal(size=(nf, nz * N, ny * N, nx * N))
    P = np.pad(G, [(0, 0), (3, 3), (3, 3), (3, 3)], mode="wrap")
    want, start = [], []
    for bz in range(nz):
        for by in range(ny):
            for bx in range(nx):
                blk = P[:, bz * N:bz * N + NB, by * N:by * N + NB, bx * N:bx * N + NB].copy()
                want.append(blk)
                garbage = blk.copy()
                garbage[:, :3] = garbage[:, -3:] = 7.5               # ghosts to be refilled
                garbage[:, :, :3] = garbage[:, :, -3:] = 7.5
                garbage[:, :, :, :3] = garbage[:, :, :, -3:] = 7.5
                start.append(garbage)
    U, off, h, ns, fs = _pack(start, N, 0.1, 0.0)
    db = _device(U, off, h, ns, fs)
    gm = hydro.DeviceGhostMap(*hydro.box_ghost_map(nx, ny, nz))
    status = T.zeros(db.n_sub, dtype=T.int32, device="cuda")
    hydro.fill_ghosts(db.struct, gm, db.U, status, n=N)
    T.cuda.synchronize()
    Ug = db.U.cpu().numpy()
    assert not status.any().item()
    for s, blk in enumerate(want):
        got = np.stack([Ug[off[s] + f * fs:off[s] + f * fs + NB ** 3].reshape(NB, NB, NB)
                        for f in range(nf)])
        assert np.array_equal(got, blk), s


def test_rk_update_16():
    T = torch()
    U, off, h, ns, fs = _batch()
    db = _device(U, off, h, ns, fs)
    rng = np.random.default_rng(96)
    Uk = T.as_tensor(rng.normal(size=U.shape)).cuda()
    R = T.as_tensor(rng.normal(size=U.shape)).cuda()
    out = T.full_like(db.U, 3.25)
    clock = T.as_tensor(np.array([0.0, 0.01, 0.0])).cuda()
    hydro.rk_update(db.struct, 0.75, db.U, 0.25, Uk, R, clock, out, n=N)
    T.cuda.synchronize()
    o, uk, r = (x.cpu().numpy() for x in (out, Uk, R))
    for s in range(len(off)):
        nf = 6 + int(ns[s])
        a0, ak, ar = (_interior(x, off, fs, nf, N, s) for x in (U, uk, r))
        want = 0.75 * a0 + 0.25 * (ak + 0.01 * ar)
        size = 0.75 * np.abs(a0) + 0.25 * (np.abs(ak) + 0.01 * np.abs(ar))
        assert np.all(np.abs(_interior(o, off, fs, nf, N, s) - want) <= 4 * 2.0 ** -52 * size)
    assert np.all(o[off[0]:off[0] + NB ** 2] == 3.25)            # ghosts untouched
