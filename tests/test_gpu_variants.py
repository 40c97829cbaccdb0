"""Method variants on the GPU against the oracle: the symmetric-speed
(Kurganov-Tadmor 2000) flux and the velocity reconstruction in the fused and
the plain paths (and in the captured forms), Colella-Woodward steepening and
flattening in both paths and the device RK3, and the entropy-tracer
re-synchronisation."""
import numpy as np
import pytest

import oracle
from gpu_util import device_batch, gpu_plain, gpu_step, rel, torch
from metrics import max_err_step
from paper_2210_06439_amd import hydro, inputs

pytestmark = pytest.mark.gpu

SYM = hydro.KT_SYMMETRIC
VEL = hydro.VELOCITY
ST, FL = hydro.STEEPEN, hydro.FLATTEN


def _flow_batch():
    """Subgrids with flow (rotating binary star, 32^3), and random states."""
    c3 = inputs.config3(N=32).subset([0, 9, 21, 42, 63])
    rb = inputs.random_batch(4, seed=91, species=(0, 5))
    blocks = [np.array(c3.block(s)) for s in range(c3.n_sub)] + \
             [np.array(rb.block(s)) for s in range(rb.n_sub)]
    return inputs.pack_blocks(blocks, list(c3.h) + list(rb.h), dt=min(c3.dt, rb.dt))


def test_symmetric_fused_matches_oracle():
    b = _flow_batch()
    Ug, ag, sg = gpu_step(b, flags=SYM)
    Ur, ar, sr = oracle.step(b.U, b.offset, b.h, b.n_species, b.fstride, b.dt, flags=SYM)
    assert max_err_step(b, Ug, Ur) <= 1e-12
    assert rel(ag, ar) <= 1e-13 and np.array_equal(sg, sr)
    # the flag changes the result where there is flow
    U0, _, _ = gpu_step(b)
    assert max_err_step(b, U0, Ur) > 1e-9


def test_symmetric_plain_bitwise():
    """Bitwise where no cell takes the dual-energy branch (its pow comes from
    each side's libm), within 1e-12 on the rotating-star subgrids."""
    rb = inputs.random_batch(4, seed=91, species=(0, 5))
    Qg, Fg, Ug, ag, sg = gpu_plain(rb, flags=SYM)
    Q, qo = oracle.reconstruct(rb.U, rb.offset, rb.h, rb.n_species, rb.fstride)
    F, fo, a, st = oracle.flux(Q, qo, rb.offset, rb.h, rb.n_species, rb.fstride, flags=SYM)
    assert np.array_equal(Fg, F)
    assert np.array_equal(ag, a) and np.array_equal(sg, st)
    Ur, _, _ = oracle.step(rb.U, rb.offset, rb.h, rb.n_species, rb.fstride, rb.dt, flags=SYM)
    for s in range(rb.n_sub):
        assert np.array_equal(rb.interior(s, Ug), rb.interior(s, Ur))
    b = _flow_batch()
    _, _, Ug, ag, _ = gpu_plain(b, flags=SYM)
    Ur, ar, _ = oracle.step(b.U, b.offset, b.h, b.n_species, b.fstride, b.dt, flags=SYM)
    assert max_err_step(b, Ug, Ur) <= 1e-12 and rel(ag, ar) <= 1e-13


@pytest.mark.parametrize("flags", [VEL, VEL | SYM])
def test_velocity_fused_matches_oracle(flags):
    b = _flow_batch()
    Ug, ag, sg = gpu_step(b, flags=flags)
    Ur, ar, sr = oracle.step(b.U, b.offset, b.h, b.n_species, b.fstride, b.dt, flags=flags)
    assert max_err_step(b, Ug, Ur) <= 1e-12
    assert rel(ag, ar) <= 1e-13 and np.array_equal(sg, sr)
    U0, _, _ = gpu_step(b, flags=flags & SYM)
    assert max_err_step(b, U0, Ur) > 1e-9


def test_velocity_fused_launch_shapes_agree_bitwise():
    b = _flow_batch()
    ref = gpu_step(b, flags=VEL, variant=0)
    for v in range(1, hydro.variant_count()):
        got = gpu_step(b, flags=VEL, variant=v)
        assert all(np.array_equal(x, y) for x, y in zip(got, ref)), v


def test_velocity_plain_matches_oracle():
    """Q is bitwise (divisions and PPM in the oracle's order); the step is
    bitwise where no point takes the dual-energy pow, else within 1e-12."""
    b = _flow_batch()
    Qg, Fg, Ug, ag, sg = gpu_plain(b, flags=VEL)
    Q, qo = oracle.reconstruct(b.U, b.offset, b.h, b.n_species, b.fstride, flags=VEL)
    assert np.array_equal(Qg, Q)
    Ur, ar, sr = oracle.step(b.U, b.offset, b.h, b.n_species, b.fstride, b.dt, flags=VEL)
    assert max_err_step(b, Ug, Ur) <= 1e-12 and rel(ag, ar) <= 1e-13
    assert np.array_equal(sg, sr)
    rb = inputs.random_batch(4, seed=92, species=(0, 5))
    _, _, Ug, ag, _ = gpu_plain(rb, flags=VEL)
    Ur, ar, _ = oracle.step(rb.U, rb.offset, rb.h, rb.n_species, rb.fstride, rb.dt, flags=VEL)
    for s in range(rb.n_sub):
        assert np.array_equal(rb.interior(s, Ug), rb.interior(s, Ur))
    assert np.array_equal(ag, ar)


def test_velocity_graph_plan_matches_eager():
    T = torch()
    b = _flow_batch()
    db = device_batch(b)
    ref = gpu_step(b, flags=VEL)
    U_out = db.U.clone()
    amax = T.zeros(db.n_sub, dtype=T.float64, device="cuda")
    status = T.zeros(db.n_sub, dtype=T.int32, device="cuda")
    plan = hydro.Plan(hydro.params(dt=b.dt, flags=VEL), db.struct, db.U, U_out, amax, status)
    for _ in range(2):
        U_out.fill_(0.0)
        plan.launch()
        T.cuda.synchronize()
        Uo = U_out.cpu().numpy()
        for s in range(b.n_sub):
            assert np.array_equal(b.interior(s, Uo), b.interior(s, ref[0]))
        assert np.array_equal(amax.cpu().numpy(), ref[1])
    plan.close()


def test_velocity_rk3_matches_oracle_driver():
    """Device-resident RK3 steps with the option on a periodic rotating-star
    box, against the test-side RK3 driver around the oracle."""
    from driver import rk3_evolve
    from mesh_util import box_batch, interiors_to_global, refill
    T = torch()
    c3 = inputs.config3(N=16)
    G = interiors_to_global(c3, c3.U, (2, 2, 2))
    b = box_batch(G, (2, 2, 2), float(c3.h[0]), (True, True, True), dt=float(c3.dt))
    fill = refill(b, (2, 2, 2), (True, True, True))

    def step(U, dt):
        Uo, amax, st = oracle.step(U, b.offset, b.h, b.n_species, b.fstride, dt, flags=VEL)
        assert np.all(st == 0)
        return Uo, amax

    t_end = 1.0
    Uo, n_or = rk3_evolve(b, step, t_end, fill, max_steps=3)
    db = device_batch(b)
    gm = hydro.DeviceGhostMap(*hydro.box_ghost_map(2, 2, 2))
    rk = hydro.RK3(hydro.params(flags=VEL), db, gm, db.U, cfl=0.4, t_end=t_end)
    rk.launch(n_or)
    T.cuda.synchronize()
    assert int(rk.clock[2].item()) == n_or == 3
    assert not rk.status.any().item()
    assert max_err_step(b, db.U.cpu().numpy(), Uo) <= 1e-12 * 3 * n_or
    rk.close()


@pytest.mark.parametrize("flags", [ST, FL, ST | FL, ST | FL | VEL, ST | FL | SYM])
def test_cw_options_plain_matches_oracle(flags):
    """Random states (both detectors fire often, no dual-energy pow): Q, F and
    the step are bitwise the oracle's.  Rotating-star subgrids (the pow of
    the dual-energy cells comes from each side's libm): within 1e-12."""
    rb = inputs.random_batch(4, seed=93, species=(0, 5))
    Qg, Fg, Ug, ag, sg = gpu_plain(rb, flags=flags)
    Q, qo = oracle.reconstruct(rb.U, rb.offset, rb.h, rb.n_species, rb.fstride, flags=flags)
    assert np.array_equal(Qg, Q)
    Q0, _ = oracle.reconstruct(rb.U, rb.offset, rb.h, rb.n_species, rb.fstride,
                               flags=flags & (VEL | SYM))
    assert not np.array_equal(Q, Q0)
    Ur, ar, sr = oracle.step(rb.U, rb.offset, rb.h, rb.n_species, rb.fstride, rb.dt, flags=flags)
    for s in range(rb.n_sub):
        assert np.array_equal(rb.interior(s, Ug), rb.interior(s, Ur))
    assert np.array_equal(ag, ar) and np.array_equal(sg, sr)
    b = _flow_batch()
    Qg, _, Ug, ag, sg = gpu_plain(b, flags=flags)
    Q, _ = oracle.reconstruct(b.U, b.offset, b.h, b.n_species, b.fstride, flags=flags)
    assert np.max(np.abs(Qg - Q) / np.maximum(np.abs(Q), 1e-300)) <= 1e-12
    Ur, ar, sr = oracle.step(b.U, b.offset, b.h, b.n_species, b.fstride, b.dt, flags=flags)
    assert max_err_step(b, Ug, Ur) <= 1e-12 and rel(ag, ar) <= 1e-13
    assert np.array_equal(sg, sr)


@pytest.mark.parametrize("flags", [ST, FL, ST | FL, ST | FL | VEL, ST | FL | SYM])
def test_cw_options_fused_matches_oracle(flags):
    """The fused kernel forms each line's cell pressures from its window:
    within 1e-12 of the oracle on random states (both detectors fire often)
    and on a generic periodic flow, the same in every launch shape.  (The
    rotating star is left out: its flow is divergence-free, so the detectors'
    compression test is decided by rounding there.)"""
    from mesh_util import generic_periodic_box
    for b in (inputs.random_batch(4, seed=93, species=(0, 5)), generic_periodic_box()):
        Ug, ag, sg = gpu_step(b, flags=flags)
        Ur, ar, sr = oracle.step(b.U, b.offset, b.h, b.n_species, b.fstride, b.dt, flags=flags)
        assert max_err_step(b, Ug, Ur) <= 1e-12
        assert rel(ag, ar) <= 1e-13 and np.array_equal(sg, sr)
        U0, _, _ = gpu_step(b, flags=flags & (VEL | SYM))
        assert max_err_step(b, U0, Ur) > 1e-9
    ref = gpu_step(b, flags=flags, variant=0)
    for v in range(1, hydro.variant_count()):
        got = gpu_step(b, flags=flags, variant=v)
        assert all(np.array_equal(x, y) for x, y in zip(got, ref)), v


def test_cw_options_rk3_matches_oracle_driver():
    """Device-resident RK3 with steepening and flattening on a generic
    periodic flow, against the test-side RK3 driver around the oracle."""
    from driver import rk3_evolve
    from mesh_util import generic_periodic_box, refill
    T = torch()
    b = generic_periodic_box()
    fill = refill(b, (2, 2, 2), (True, True, True))
    flags = ST | FL

    def step(U, dt):
        Uo, amax, st = oracle.step(U, b.offset, b.h, b.n_species, b.fstride, dt, flags=flags)
        assert np.all(st == 0)
        return Uo, amax

    Uo, n_or = rk3_evolve(b, step, 1.0, fill, max_steps=3)
    db = device_batch(b)
    gm = hydro.DeviceGhostMap(*hydro.box_ghost_map(2, 2, 2))
    rk = hydro.RK3(hydro.params(flags=flags), db, gm, db.U, cfl=0.4, t_end=1.0)
    rk.launch(n_or)
    T.cuda.synchronize()
    assert int(rk.clock[2].item()) == n_or == 3
    assert not rk.status.any().item()
    assert max_err_step(b, db.U.cpu().numpy(), Uo) <= 1e-12 * 3 * n_or
    rk.close()


def test_unknown_flag_is_rejected():
    b = inputs.config1()
    with pytest.raises(hydro.HydroError):
        gpu_step(b, flags=16)


def test_tau_resync_matches_oracle():
    T = torch()
    b = inputs.config3(N=32).subset(list(range(0, 64, 3)))
    db = device_batch(b)
    hydro.tau_resync(hydro.params(), db.struct, db.U)
    T.cuda.synchronize()
    Ug = db.U.cpu().numpy()
    Ur = oracle.tau_resync(b.U, b.offset, b.h, b.n_species, b.fstride)
    changed = 0
    for s in range(b.n_sub):
        g, r, i0 = b.block(s, Ug), b.block(s, Ur), b.block(s)
        assert np.array_equal(np.delete(g, 5, axis=0), np.delete(r, 5, axis=0))
        # tau: one pow on each side (device and host libm), a few ulp apart
        assert np.all(np.abs(g[5] - r[5]) <= 4 * 2.0 ** -52 * np.abs(r[5]))
        changed += int(np.count_nonzero(r[5] != i0[5]))
    assert changed > 100
