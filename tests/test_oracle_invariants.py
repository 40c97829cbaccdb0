"""Invariants that pin the oracle's whole step: exactness on uniform and
linear data, mirror and axis-permutation symmetry, species independence,
periodic conservation, argument checks."""
import numpy as np
import pytest

import oracle
from paper_2210_06439_amd import inputs
from metrics import field_scales, mixed_rel

NB = 14


def run_step(batch, dt=None):
    dt = batch.dt if dt is None else dt
    return oracle.step(batch.U, batch.offset, batch.h, batch.n_species, batch.fstride, dt)


def one(block, h=0.125, dt=0.0):
    return inputs.pack_blocks([block], [h], dt=dt)


def slot(dx, dy, dz):
    n = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1)
    return n if n < 13 else n - 1


DIRS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
        if (dx, dy, dz) != (0, 0, 0)]


def test_uniform_state_is_unchanged_bitwise():
    V = np.array([1.3, 0.2, -0.1, 0.05, 2.7, 1.1, 0.2, 0.3, 0.4, 0.2, 0.2])
    blk = np.broadcast_to(V[:, None, None, None], (11, NB, NB, NB)).copy()
    b = one(blk, dt=0.01)
    Q, _ = oracle.reconstruct(b.U, b.offset, b.h, b.n_species, b.fstride)
    assert np.array_equal(np.unique(Q.reshape(11, -1), axis=1).ravel(), V)
    Uo, amax, st = run_step(b)
    assert np.array_equal(Uo, b.U)
    assert st[0] == 0 and amax[0] > 0


def test_linear_data_reconstructed_exactly():
    """U_f = a_f + beta_f . (i, j, k) with dyadic coefficients: every PPM
    intermediate is exact, so Q_f(c, d) = U_f(c) + (beta_f . d)/2 bitwise."""
    rng = np.random.default_rng(0)
    nf = 11
    a = rng.integers(-8, 9, nf) / 4.0
    beta = rng.integers(-8, 9, (nf, 3)) / 8.0
    k, j, i = np.meshgrid(np.arange(NB), np.arange(NB), np.arange(NB), indexing="ij")
    blk = np.stack([a[f] + beta[f, 0] * i + beta[f, 1] * j + beta[f, 2] * k for f in range(nf)])
    b = one(blk)
    Q, _ = oracle.reconstruct(b.U, b.offset, b.h, b.n_species, b.fstride)
    Q = Q.reshape(nf, 26, 10, 10, 10)
    for d in DIRS:
        for f in range(nf):
            expect = blk[f, 2:12, 2:12, 2:12] + 0.5 * (beta[f] @ np.array(d, float))
            assert np.array_equal(Q[f, slot(*d)], expect), (d, f)


def mirror(blk, axis):
    """Reflect a [nf, z, y, x] block along `axis` (0 = x) and flip s_axis."""
    out = np.flip(blk, axis=3 - axis).copy()
    out[1 + axis] *= -1.0
    return out


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_mirror_symmetry_bitwise(axis):
    b = inputs.config1(seed=21)
    blk = np.array(b.block(0))
    Uo, amax, _ = run_step(b)
    bm = one(mirror(blk, axis), dt=b.dt)
    Um, amax_m, _ = run_step(bm)
    out = np.array(b.block(0, Uo))
    out_m = mirror(np.array(bm.block(0, Um)), axis)
    assert np.array_equal(out, out_m)
    assert amax[0] == amax_m[0]


@pytest.mark.parametrize("perm", [(1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0)])
def test_axis_permutation(perm):
    """Relabel the axes (and the momenta with them): the result matches to
    1e-14; only the order of sums over axes and tangential points changes."""
    b = inputs.config1(seed=22)
    blk = np.array(b.block(0))
    Uo, amax, _ = run_step(b)

    def permute(x):
        # x is [nf, z, y, x]; new axis a takes old axis perm[a]
        sp = x.transpose([0] + [3 - perm[2 - q] for q in range(3)]).copy()
        sp[1:4] = np.array(x[1:4])[list(perm)].transpose([0] + [3 - perm[2 - q] for q in range(3)])
        return sp

    bp = one(permute(blk), dt=b.dt)
    Up, amax_p, _ = run_step(bp)
    got = np.array(bp.interior(0, Up))
    ref = permute(np.array(b.block(0, Uo)))[:, 3:11, 3:11, 3:11]
    e = mixed_rel(got, ref, field_scales(permute(blk)))
    assert e.max() <= 1e-14
    assert abs(amax_p[0] - amax[0]) <= 1e-15 * amax[0]


def test_hydro_fields_independent_of_species():
    b11 = inputs.config1(seed=23)
    blk = np.array(b11.block(0))
    b6 = one(blk[:6].copy(), dt=b11.dt)
    U11, a11, _ = run_step(b11)
    U6, a6, _ = run_step(b6)
    assert np.array_equal(np.array(b11.block(0, U11))[:6], np.array(b6.block(0, U6)))
    assert a11[0] == a6[0]


def test_dt_zero_is_identity_and_reports_speed():
    b = inputs.config1(seed=24)
    Uo, amax, st = run_step(b, dt=0.0)
    assert np.array_equal(Uo, b.U)
    _, amax2, _ = run_step(b)
    assert amax[0] == amax2[0] > 0 and st[0] == 0


def test_status_flags_bad_subgrid_only():
    good = inputs.config1(seed=25)
    blk = np.array(good.block(0))
    bad = blk.copy()
    bad[0, 7, 7, 7] = -1.0        # negative density inside
    b = inputs.pack_blocks([blk, bad, blk], [0.125] * 3, dt=good.dt)
    Uo, amax, st = run_step(b)
    assert st[0] == 0 and st[2] == 0 and (st[1] & 1)
    assert np.array_equal(np.array(b.block(0, Uo)), np.array(b.block(2, Uo)))


def test_reconstruct_flux_divergence_compose_to_step():
    b = inputs.random_batch(3, seed=26, species=(0, 5))
    Q, qo = oracle.reconstruct(b.U, b.offset, b.h, b.n_species, b.fstride)
    F, fo, amax, st = oracle.flux(Q, qo, b.offset, b.h, b.n_species, b.fstride)
    Ud = oracle.divergence(F, fo, b.U, b.offset, b.h, b.n_species, b.fstride, b.dt)
    Us, amax_s, st_s = run_step(b)
    assert np.array_equal(Ud, Us) and np.array_equal(amax, amax_s)
    assert np.array_equal(st, st_s)


def test_periodic_conservation_config2():
    """Every face shared by two subgrids is computed from identical data on
    both sides, so the fluxes telescope: the totals change only by the
    rounding of the sums (bound 1e-13 relative)."""
    b = inputs.config2()
    Uo, amax, st = run_step(b)
    assert np.all(st == 0)
    # momenta start at zero: their scale is sum(sqrt(rho * E)), a momentum
    mom_scale = sum(np.sum(np.sqrt(b.interior(s)[0] * b.interior(s)[4])) for s in range(b.n_sub))
    for f in range(11):
        tin = sum(np.sum(b.interior(s)[f]) for s in range(b.n_sub))
        tout = sum(np.sum(b.interior(s, Uo)[f]) for s in range(b.n_sub))
        mag = sum(np.sum(np.abs(b.interior(s)[f])) for s in range(b.n_sub))
        if f in (1, 2, 3):
            mag = mom_scale
        assert abs(tout - tin) <= 1e-13 * mag, (f, tout - tin, mag)
    # and something did happen
    assert not np.array_equal(Uo, b.U)


def test_invalid_arguments_rejected():
    import ctypes
    b = inputs.config1()
    prm = oracle.params()
    bad_species = np.array([7], dtype=np.int32)
    ba = oracle._BatchArgs(b.offset, b.h, bad_species, b.fstride)
    out = np.zeros_like(b.U)
    am = np.zeros(1)
    st = np.zeros(1, dtype=np.int32)
    dp = ctypes.POINTER(ctypes.c_double)
    rc = oracle.raw_call("hydro_ref_step", ctypes.byref(prm), ctypes.byref(ba.struct),
                         b.U.ctypes.data_as(dp), out.ctypes.data_as(dp), am.ctypes.data_as(dp),
                         st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert rc == -1
    ba2 = oracle._BatchArgs(b.offset, b.h, b.n_species, 2000)
    rc = oracle.raw_call("hydro_ref_step", ctypes.byref(prm), ctypes.byref(ba2.struct),
                         b.U.ctypes.data_as(dp), out.ctypes.data_as(dp), am.ctypes.data_as(dp),
                         st.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    assert rc == -1
