"""The serving loop on the GPU: every request's result is the same bits alone
and in the mix, and matches the oracle; a small real-time Poisson stream
completes with latency percentiles."""
import numpy as np
import pytest

import oracle
from metrics import max_err_step
from paper_2210_06439_amd import hydro, inputs, serving

pytestmark = pytest.mark.gpu

SLOT = serving.NF_MAX * inputs.FSTRIDE


@pytest.fixture(scope="module")
def cat():
    oracle.build()
    b = inputs.random_batch(24, seed=71, species=(5,))
    return b, hydro.DeviceBatch.from_inputs(b)


def _requests(b):
    rng = np.random.default_rng(72)
    out = []
    for rid in range(10):
        n = int(rng.integers(1, 7))
        idx = np.sort(rng.choice(b.n_sub, size=n, replace=False))
        out.append(serving.Request(rid, idx, b.h[idx], b.n_species[idx],
                                   int(rng.choice([1, 2, 3, 4])), 0.0))
    return out


def _serve(db, reqs, n_slots, dt, flags=0, lanes=1):
    be = serving.GpuBackend(n_slots, catalogue=db, flags=flags)
    finals = {}

    def grab(req, slots, copy):
        finals[req.rid] = be.read(slots, copy)

    recs = serving.HydroServer(be, dt, lanes=lanes).run(reqs, realtime=False, on_complete=grab)
    return recs, finals


@pytest.mark.parametrize("lanes", [1, 2])
def test_alone_equals_in_the_mix_and_matches_oracle(cat, lanes):
    """In the mix -- with one lane, or with two whose ticks overlap on the
    device -- each request's result is the bits of the request served alone."""
    b, db = cat
    reqs = _requests(b)
    recs, mixed = _serve(db, reqs, 12, b.dt, lanes=lanes)   # 12 slots: admission has to wait
    if lanes == 2:
        assert {r.lane for r in recs} == {0, 1}
    assert all(not r.rejected and r.status == 0 for r in recs)
    starts = sorted(r.ticks[0] for r in recs)
    assert starts[-1] > 0                          # some requests joined later ticks
    for r in reqs:
        _, alone = _serve(db, [r], 12, b.dt)
        assert np.array_equal(alone[r.rid], mixed[r.rid]), r.rid
        sub = b.subset(r.source)
        U = sub.U
        for _ in range(r.steps):
            U, _, _ = oracle.step(U, sub.offset, sub.h, sub.n_species, sub.fstride, b.dt)
        got = sub.U.copy()
        for s in range(r.n):
            got[int(sub.offset[s]):int(sub.offset[s]) + SLOT] = mixed[r.rid][s].reshape(-1)
        assert max_err_step(sub, got, U) <= 1e-12 * r.steps


def test_served_with_method_options(cat):
    """Velocity reconstruction with Colella-Woodward steepening and
    flattening in every tick: each request matches the oracle with the same
    options (random states: no detector sits on its threshold)."""
    b, db = cat
    flags = hydro.VELOCITY | hydro.STEEPEN | hydro.FLATTEN
    reqs = _requests(b)[:5]
    recs, out = _serve(db, reqs, 12, b.dt, flags=flags)
    assert all(not r.rejected and r.status == 0 for r in recs)
    for r in reqs:
        sub = b.subset(r.source)
        U = sub.U
        for _ in range(r.steps):
            U, _, _ = oracle.step(U, sub.offset, sub.h, sub.n_species, sub.fstride, b.dt,
                                  flags=flags)
        got = sub.U.copy()
        for s in range(r.n):
            got[int(sub.offset[s]):int(sub.offset[s]) + SLOT] = out[r.rid][s].reshape(-1)
        assert max_err_step(sub, got, U) <= 1e-12 * r.steps
    # and the options made a difference
    _, plain = _serve(db, reqs[:1], 12, b.dt)
    assert not np.array_equal(plain[reqs[0].rid], out[reqs[0].rid])


def test_host_array_sources(cat):
    b, db = cat
    idx = np.array([3, 7, 11])
    host = np.stack([b.U[int(b.offset[i]):int(b.offset[i]) + SLOT] for i in idx])
    r_host = serving.Request(0, host, b.h[idx], b.n_species[idx], 2, 0.0)
    r_cat = serving.Request(1, idx, b.h[idx], b.n_species[idx], 2, 0.0)
    _, a = _serve(db, [r_host], 4, b.dt)
    _, c = _serve(db, [r_cat], 4, b.dt)
    assert np.array_equal(a[0], c[1])


def test_realtime_poisson_stream(cat):
    b, db = cat
    reqs = serving.poisson_requests(40, rate=2000.0, catalogue_n=b.n_sub, h=b.h,
                                    n_species=b.n_species, seed=73, median_n=4,
                                    max_n=12)
    be = serving.GpuBackend(16, catalogue=db)
    recs = serving.HydroServer(be, b.dt, lanes=2).run(reqs, realtime=True)
    assert all(not r.rejected for r in recs)
    for r in recs:
        assert r.completed > r.arrival and len(r.ticks) == r.steps
    s = serving.summarize(recs)
    assert s["requests"] == 40 and s["nonzero_status"] == 0
    assert 0 < s["latency_ms"]["p50"] <= s["latency_ms"]["p99"]
