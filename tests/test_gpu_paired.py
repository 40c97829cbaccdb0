"""The paired body: subgrids without species are swept two planes per step by
a second body in the same launch.  Its results are the 11-field body's bits
(that body still sweeps them in the split-8 shape, whose parts hold single
planes), in every launch shape and in the rate and Runge-Kutta stage forms;
in a mixed batch every subgrid's result is its result alone; steps of
different sizes on one stream leave each other's scratch alone; and plans,
which pick their instance from the species counts at creation, replay the
eager results, also after the counts change."""
import numpy as np
import pytest

import oracle
from gpu_util import device_batch, gpu_step, rel, torch
from metrics import max_err_step
from paper_2210_06439_amd import hydro, inputs

pytestmark = pytest.mark.gpu


def _variant(name):
    return next(v for v in range(hydro.variant_count()) if hydro.variant_name(v) == name)


def test_paired_equals_the_11_field_body_in_every_shape():
    b = inputs.random_batch(12, seed=77, species=(0, 0))
    ref = gpu_step(b, variant=_variant("split-8"))
    for v in range(hydro.variant_count()):
        got = gpu_step(b, variant=v)
        for x, y in zip(ref, got):
            assert np.array_equal(x, y), hydro.variant_name(v)
    Ur, ar, sr = oracle.step(b.U, b.offset, b.h, b.n_species, b.fstride, b.dt)
    assert max_err_step(b, ref[0], Ur) <= 1e-12
    assert rel(ref[1], ar) <= 1e-13 and np.array_equal(ref[2], sr)


def test_mixed_batch_hands_each_subgrid_over_once():
    b = inputs.random_batch(40, seed=78, species=(0, 5))
    assert (b.n_species == 0).sum() >= 4 and (b.n_species > 0).sum() >= 4
    U, a, st = gpu_step(b, variant=_variant("persistent-1x-dynamic"))
    for s in range(b.n_sub):
        one = b.subset([s])
        U1, a1, s1 = gpu_step(one, dt=b.dt, variant=_variant("persistent-2x"))
        assert np.array_equal(one.interior(0, U1), b.interior(s, U)), s
        assert a1[0] == a[s] and s1[0] == st[s], s


def test_scratch_is_left_clean_for_a_larger_batch():
    """A later step with more subgrids on the same stream reads the split
    shapes' per-subgrid counters at other words, so each step must leave all
    the words it used zero."""
    small = inputs.random_batch(6, seed=79, species=(0, 0))
    big = inputs.random_batch(9, seed=80, species=(0, 5))
    want = gpu_step(big, variant=_variant("persistent-1x"))
    for _ in range(2):
        gpu_step(small, variant=_variant("persistent-2x"))
        got = gpu_step(big, variant=_variant("split-2"))
        for x, y in zip(want, got):
            assert np.array_equal(x, y)


def test_rate_and_stage_forms_alone_and_in_a_batch():
    """40 subgrids take the split-4 shape (paired body), one alone the split-8
    shape (11-field body): the rate and the stage combination agree bitwise."""
    T = torch()
    b = inputs.random_batch(40, seed=81, species=(0, 0))
    rng = np.random.default_rng(82)
    U0h = b.U * (1.0 + 0.01 * rng.standard_normal(b.U.shape))

    def run(batch, U0_host):
        db = device_batch(batch)
        R = T.zeros_like(db.U)
        out = T.zeros_like(db.U)
        U0 = T.as_tensor(U0_host).cuda()
        amax = T.zeros(db.n_sub, dtype=T.float64, device="cuda")
        clock = T.as_tensor(np.array([0.0, batch.dt, 0.0])).cuda()
        hydro.rate(hydro.params(), db.struct, db.U, R, amax)
        hydro.rk_stage(hydro.params(), db.struct, db.U, out, U0, 0.75, 0.25, clock, amax)
        T.cuda.synchronize()
        return R.cpu().numpy(), out.cpu().numpy()

    Rb, Ob = run(b, U0h)
    for s in (0, 17, 39):
        one = b.subset([s])
        U0one = U0h[b.offset[s]:b.offset[s] + one.U.size].copy()
        R1, O1 = run(one, U0one)
        assert np.array_equal(one.interior(0, R1), b.interior(s, Rb)), s
        assert np.array_equal(one.interior(0, O1), b.interior(s, Ob)), s


def _plan_run(T, db, dt, replays=2):
    U_out = db.U.clone()
    amax = T.zeros(db.n_sub, dtype=T.float64, device="cuda")
    status = T.zeros(db.n_sub, dtype=T.int32, device="cuda")
    plan = hydro.Plan(hydro.params(dt=dt), db.struct, db.U, U_out, amax, status)
    outs = []
    for _ in range(replays):
        U_out.fill_(0.0)
        plan.launch()
        T.cuda.synchronize()
        outs.append((U_out.cpu().numpy(), amax.cpu().numpy(), status.cpu().numpy()))
    return plan, outs


def test_plan_with_the_paired_body_matches_eager():
    """140 subgrids, some without species: the plan takes the instance with
    the paired body (the one-sweep shape), its replays equal the eager step."""
    T = torch()
    b = inputs.random_batch(140, seed=83, species=(0, 5))
    assert (b.n_species == 0).any()
    want = gpu_step(b)
    plan, outs = _plan_run(T, device_batch(b), b.dt)
    plan.close()
    for got in outs:
        for s in range(b.n_sub):
            assert np.array_equal(b.interior(s, got[0]), b.interior(s, want[0])), s
        assert np.array_equal(got[1], want[1]) and np.array_equal(got[2], want[2])


def test_plan_without_the_paired_body_stays_correct_after_counts_change():
    """A plan made while every subgrid had species takes the instance without
    the paired body; species counts rewritten to 0 afterwards are swept by its
    11-field body, with the same bits as an eager step on the new counts
    (which pairs those subgrids)."""
    T = torch()
    b = inputs.random_batch(140, seed=84, species=(5,))
    db = device_batch(b)
    U_plan = db.U.clone()
    am_p = T.zeros(db.n_sub, dtype=T.float64, device="cuda")
    st_p = T.zeros(db.n_sub, dtype=T.int32, device="cuda")
    plan = hydro.Plan(hydro.params(dt=b.dt), db.struct, db.U, U_plan, am_p, st_p)
    ns = b.n_species.copy()
    ns[::3] = 0
    db.n_species.copy_(T.as_tensor(ns).cuda())
    plan.launch()
    T.cuda.synchronize()
    plan.close()
    U_e = db.U.clone()
    am_e = T.zeros(db.n_sub, dtype=T.float64, device="cuda")
    st_e = T.zeros(db.n_sub, dtype=T.int32, device="cuda")
    hydro.step(hydro.params(dt=b.dt), db.struct, db.U, U_e, am_e, st_e)
    T.cuda.synchronize()
    got, want = U_plan.cpu().numpy(), U_e.cpu().numpy()
    for s in range(b.n_sub):
        assert np.array_equal(b.interior(s, got), b.interior(s, want)), s
    assert np.array_equal(am_p.cpu().numpy(), am_e.cpu().numpy())
    assert np.array_equal(st_p.cpu().numpy(), st_e.cpu().numpy())
