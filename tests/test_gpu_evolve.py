"""Device-resident time integration on the GPU: ghost fill, the rate form of
the fused stage, the CFL reduction, the RK3 stage combination, captured RK3
steps against the oracle-driven RK3, and a GPU Sod tube converging to the
exact Riemann solution."""
import numpy as np
import pytest

import oracle
import riemann
from driver import density_profile, rk3_evolve, sod_refill
from gpu_util import device_batch, torch
from mesh_util import box_batch, refill
from metrics import max_err_step
from paper_2210_06439_amd import hydro, inputs

pytestmark = pytest.mark.gpu

GAMMA = 5.0 / 3.0


def _stale(b):
    """Copy of b.U with every ghost cell overwritten."""
    U = b.U.copy()
    for s in range(b.n_sub):
        blk = b.block(s, U)
        inner = blk[:, 3:11, 3:11, 3:11].copy()
        blk[...] = -7.5
        blk[:, 3:11, 3:11, 3:11] = inner
    return U


@pytest.mark.parametrize("nsub,periodic", [((4, 4, 4), (True, True, True)),
                                           ((4, 2, 3), (False, True, False))])
def test_fill_ghosts_bitwise(nsub, periodic):
    T = torch()
    rng = np.random.default_rng(11)
    nx, ny, nz = nsub
    G = rng.uniform(0.5, 2.0, size=(11, nz * 8, ny * 8, nx * 8))
    want = box_batch(G, nsub, 1.0 / 32, periodic)
    db = hydro.DeviceBatch(_stale(want), want.offset, want.h, want.n_species, want.fstride)
    gm = hydro.DeviceGhostMap(*hydro.box_ghost_map(*nsub, periodic=periodic))
    status = T.zeros(db.n_sub, dtype=T.int32, device="cuda")
    hydro.fill_ghosts(db.struct, gm, db.U, status)
    T.cuda.synchronize()
    assert np.array_equal(db.U.cpu().numpy(), want.U)
    assert not status.any().item()


def test_fill_ghosts_bad_entry_flags_only_that_subgrid():
    T = torch()
    rng = np.random.default_rng(12)
    G = rng.uniform(0.5, 2.0, size=(6, 8, 8, 16))
    want = box_batch(G, (2, 1, 1), 0.1, (True, True, True))
    src, mode = hydro.box_ghost_map(2, 1, 1)
    src = src.copy()
    src[27 + 4] = 99                        # subgrid 1, direction (0,-1,-1)
    db = hydro.DeviceBatch(_stale(want), want.offset, want.h, want.n_species, want.fstride)
    status = T.zeros(2, dtype=T.int32, device="cuda")
    hydro.fill_ghosts(db.struct, hydro.DeviceGhostMap(src, mode), db.U, status)
    T.cuda.synchronize()
    st = status.cpu().numpy()
    assert st[0] == 0 and st[1] == hydro.STATUS_BADMETA
    got = db.U.cpu().numpy()
    assert np.array_equal(want.block(0, got), want.block(0))


def test_rate_matches_oracle_step():
    """U + h R(U) against the oracle's step with dt = h (so dt/h = 1)."""
    T = torch()
    b = inputs.random_batch(6, seed=13, species=(0, 5))
    db = device_batch(b)
    R = T.zeros_like(db.U)
    amax = T.zeros(db.n_sub, dtype=T.float64, device="cuda")
    status = T.full((db.n_sub,), 16, dtype=T.int32, device="cuda")
    hydro.rate(hydro.params(), db.struct, db.U, R, amax, status)
    T.cuda.synchronize()
    Rh = R.cpu().numpy()
    worst = 0.0
    for s in range(b.n_sub):
        sub = b.subset([s])
        h = float(b.h[s])
        Ur, ar, _ = oracle.step(sub.U, sub.offset, sub.h, sub.n_species, sub.fstride, h)
        got = sub.U.copy()
        sub.block(0, got)[:, 3:11, 3:11, 3:11] += h * b.interior(s, Rh)
        worst = max(worst, max_err_step(sub, got, Ur))
        assert abs(amax[s].item() - ar[0]) <= 1e-13 * ar[0]
    assert worst <= 1e-12, worst
    assert np.all(status.cpu().numpy() == 16)       # bits are ORed in


def test_cfl_dt_and_clock():
    T = torch()
    b = inputs.random_batch(40, seed=14)
    db = device_batch(b)
    rng = np.random.default_rng(15)
    a = rng.uniform(0.5, 3.0, size=40)
    a[7] = 0.0                                       # a subgrid at rest is skipped
    amax = T.as_tensor(a).cuda()
    clock = T.zeros(3, dtype=T.float64, device="cuda")
    want = 0.4 * np.min(b.h[a > 0] / a[a > 0])
    hydro.cfl_dt(db.struct, amax, 0.4, 1.0, clock)
    T.cuda.synchronize()
    t, dt, n = clock.tolist()
    assert dt == want and t == want and n == 1.0
    t_end = 2.5 * want
    clock.zero_()
    for _ in range(4):
        hydro.cfl_dt(db.struct, amax, 0.4, t_end, clock)
    T.cuda.synchronize()
    t, dt, n = clock.tolist()
    assert t == t_end and dt == 0.0 and n == 3.0


def test_rk_update():
    T = torch()
    b = inputs.random_batch(3, seed=16, species=(0, 5))
    db = device_batch(b)
    rng = np.random.default_rng(17)
    Uk = T.as_tensor(rng.normal(size=b.U.shape)).cuda()
    R = T.as_tensor(rng.normal(size=b.U.shape)).cuda()
    out = T.full_like(db.U, 3.25)
    clock = T.as_tensor(np.array([0.0, 0.01, 0.0])).cuda()
    hydro.rk_update(db.struct, 0.75, db.U, 0.25, Uk, R, clock, out)
    T.cuda.synchronize()
    o, u0, uk, r = (x.cpu().numpy() for x in (out, db.U, Uk, R))
    for s in range(b.n_sub):
        a0, ak, ar = b.interior(s, u0), b.interior(s, uk), b.interior(s, r)
        want = 0.75 * a0 + 0.25 * (ak + 0.01 * ar)
        size = 0.75 * np.abs(a0) + 0.25 * (np.abs(ak) + 0.01 * np.abs(ar))
        # a few roundings (contracted or not) of terms of this size
        assert np.all(np.abs(b.interior(s, o) - want) <= 4 * 2.0 ** -52 * size)
        blk = b.block(s, o)
        assert np.all(blk[:, :3] == 3.25)            # ghosts untouched
    clock[1] = 0.0
    hydro.rk_update(db.struct, 0.75, db.U, 0.25, Uk, R, clock, out)
    T.cuda.synchronize()
    o = out.cpu().numpy()
    for s in range(b.n_sub):
        assert np.array_equal(b.interior(s, o), b.interior(s, u0))


def _oracle_step(b):
    def step(U, dt):
        Uo, amax, st = oracle.step(U, b.offset, b.h, b.n_species, b.fstride, dt)
        assert np.all(st == 0)
        return Uo, amax
    return step


def test_rk3_plan_matches_oracle_driver():
    """Three RK3 steps on a 32^3 periodic mesh (64 subgrids, config-2 data)."""
    T = torch()
    nsub = (4, 4, 4)
    rho, vx, vy, vz, p, spc, h = inputs.config2_fields(seed=1002, N=32)
    G = inputs.conserved_from_primitive(rho, vx, vy, vz, p, spc)
    b = box_batch(G, nsub, h, (True, True, True))
    dt0 = inputs.cfl_dt(rho, vx, vy, vz, p, h)
    t_end = 2.5 * dt0
    Uo, n_or = rk3_evolve(b, _oracle_step(b), t_end, refill(b, nsub, (True, True, True)))
    db = device_batch(b)
    gm = hydro.DeviceGhostMap(*hydro.box_ghost_map(*nsub))
    rk = hydro.RK3(hydro.params(), db, gm, db.U, cfl=0.4, t_end=t_end)
    n_gpu = rk.run_to_end(chunk=4)
    T.cuda.synchronize()
    assert n_gpu == n_or
    assert rk.clock[0].item() == t_end
    assert not rk.status.any().item()
    Ug = db.U.cpu().numpy()
    assert max_err_step(b, Ug, Uo) <= 1e-12 * 3 * n_or
    # conservation of the periodic mesh, every field, over the whole run
    for f in range(11):
        tot0 = sum(float(np.sum(b.interior(s)[f])) for s in range(b.n_sub))
        tot1 = sum(float(np.sum(b.interior(s, Ug)[f])) for s in range(b.n_sub))
        scale = sum(float(np.sum(np.abs(b.interior(s)[f]))) for s in range(b.n_sub))
        if f in (1, 2, 3):
            scale = sum(float(np.sum(np.sqrt(np.abs(b.interior(s)[0] * b.interior(s)[4]))))
                        for s in range(b.n_sub))
        assert abs(tot1 - tot0) <= 1e-13 * scale, f
    rk.close()


def _gpu_sod(N, axis=0):
    b = inputs.sod_chain(N, axis=axis)
    nsub = [1, 1, 1]
    nsub[axis] = N // 8
    periodic = [True, True, True]
    periodic[axis] = False
    db = device_batch(b)
    gm = hydro.DeviceGhostMap(*hydro.box_ghost_map(*nsub, periodic=tuple(periodic)))
    rk = hydro.RK3(hydro.params(), db, gm, db.U, cfl=0.4, t_end=0.2)
    n = rk.run_to_end(chunk=32)
    U = db.U.cpu().numpy()
    assert not rk.status.any().item()
    rk.close()
    return b, U, n


def test_gpu_sod_converges_and_matches_oracle():
    LEFT, RIGHT = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    errs = {}
    for N in (64, 128):
        b, U, n = _gpu_sod(N)
        rho = density_profile(b, U, 0)
        exact = riemann.cell_average_density(np.arange(N + 1) / N, 0.2, 0.5, LEFT, RIGHT, GAMMA)
        errs[N] = float(np.mean(np.abs(rho - exact)))
        if N == 64:
            Uo, n_or = rk3_evolve(b, _oracle_step(b), 0.2, sod_refill(b, 0))
            assert n == n_or
            rho_o = density_profile(b, Uo, 0)
            assert np.max(np.abs(rho - rho_o)) <= 1e-10
    # the oracle's bounds for the same problem
    assert errs[64] < 1.0e-2 and errs[128] < 4.85e-3, errs
    assert np.log2(errs[64] / errs[128]) >= 0.5, errs


def test_gpu_sod_along_z_matches_x():
    bx, Ux, nx = _gpu_sod(64, 0)
    bz, Uz, nz = _gpu_sod(64, 2)
    assert nx == nz
    # the fused kernel forms x/y and z faces in different summation orders, so
    # the two runs agree to rounding growth over ~65 steps, not bitwise
    assert np.max(np.abs(density_profile(bx, Ux, 0) - density_profile(bz, Uz, 2))) <= 1e-10


def test_fused_rk_stage_matches_rate_and_update():
    """U_out = a U0 + b (U + dt L(U)) in one launch, against the rate form and
    the stage combination; dt = 0 returns U0; U_out may be U0."""
    T = torch()
    b = inputs.random_batch(6, seed=18, species=(0, 5))
    db = device_batch(b)
    rng = np.random.default_rng(19)
    U0 = T.as_tensor(b.U * (1.0 + 0.01 * rng.standard_normal(b.U.shape))).cuda()
    amax = T.zeros(db.n_sub, dtype=T.float64, device="cuda")
    R = T.zeros_like(db.U)
    ref = T.zeros_like(db.U)
    out = T.zeros_like(db.U)
    clock = T.as_tensor(np.array([0.0, b.dt, 0.0])).cuda()
    hydro.rate(hydro.params(), db.struct, db.U, R, amax)
    hydro.rk_update(db.struct, 0.75, U0, 0.25, db.U, R, clock, ref)
    status = T.zeros(db.n_sub, dtype=T.int32, device="cuda")
    hydro.rk_stage(hydro.params(), db.struct, db.U, out, U0, 0.75, 0.25, clock, amax, status)
    T.cuda.synchronize()
    assert max_err_step(b, out.cpu().numpy(), ref.cpu().numpy()) <= 1e-12
    assert not status.any().item()
    # in place on U0
    U0c = U0.clone()
    hydro.rk_stage(hydro.params(), db.struct, db.U, U0c, U0c, 0.75, 0.25, clock, amax)
    T.cuda.synchronize()
    o, c = out.cpu().numpy(), U0c.cpu().numpy()
    for s in range(b.n_sub):
        assert np.array_equal(b.interior(s, o), b.interior(s, c))
    # dt = 0: the stage is the identity on U0
    clock[1] = 0.0
    hydro.rk_stage(hydro.params(), db.struct, db.U, out, U0, 0.75, 0.25, clock, amax)
    T.cuda.synchronize()
    o, u0 = out.cpu().numpy(), U0.cpu().numpy()
    for s in range(b.n_sub):
        assert np.array_equal(b.interior(s, o), b.interior(s, u0))
