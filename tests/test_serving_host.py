"""Host logic of the serving loop, driven by a CPU backend that runs the
oracle: admission against the slot budget, first-come-first-served order,
continuous batching (sessions at different stages share ticks), slot reuse,
rejection, and each result equal to the same request stepped alone."""
import numpy as np
import pytest

import oracle
from paper_2210_06439_amd import inputs, serving
from paper_2210_06439_amd.inputs import FSTRIDE

SLOT = serving.NF_MAX * FSTRIDE


class OracleBackend:
    """Serving backend on the CPU oracle: two host copies of the slot pool,
    ticks computed at launch, a tick counter as the clock."""

    def __init__(self, n_slots, catalogue):
        self.n_slots = n_slots
        self.cat = catalogue
        self.copies = [np.zeros(n_slots * SLOT), np.zeros(n_slots * SLOT)]
        self.ticks = []          # per tick: (group0 rids, group1 rids)
        self.lanes = []          # per tick: its lane
        self.loads = []          # per load call: rids

    def start(self):
        self.clock = 0.0
        return 0.0

    def now(self, t0):
        return self.clock

    def idle_until(self, t0, t):
        self.clock = max(self.clock, t)

    def load(self, sessions):
        self.loads.append([s.req.rid for s in sessions])
        for s in sessions:
            for slot, idx in zip(s.slots, s.req.source):
                blk = self.cat.U[int(self.cat.offset[idx]):int(self.cat.offset[idx]) + SLOT]
                for c in range(2):
                    self.copies[c][slot * SLOT:(slot + 1) * SLOT] = blk

    max_lanes = 2

    def launch_tick(self, groups, dt, tick_no, lane=0):
        self.ticks.append(tuple([s.req.rid for s in g] for g in groups))
        self.lanes.append(lane)
        status = {}
        for g in range(2):
            for s in groups[g]:
                off = s.slots * SLOT
                U_out, _, st = oracle.step(self.copies[g], off, s.req.h, s.req.n_species,
                                           FSTRIDE, dt)
                for o in off:
                    self.copies[1 - g][o:o + SLOT] = U_out[o:o + SLOT]
                status[id(s)] = int(np.bitwise_or.reduce(st))
        self.clock += 1.0
        return (self.clock, status)

    def wait_tick(self, handle, t0):
        return handle

    def finish(self):
        pass

    def read(self, slots, copy):
        return np.stack([self.copies[copy][s * SLOT:(s + 1) * SLOT] for s in slots])


@pytest.fixture(scope="module")
def catalogue():
    oracle.build()
    return inputs.random_batch(12, seed=61, species=(5,))


def _req(rid, idx, steps, arrival, cat):
    idx = np.asarray(idx)
    return serving.Request(rid, idx, cat.h[idx], cat.n_species[idx], steps, arrival)


def _alone(cat, idx, steps, dt):
    """The request's subgrids stepped alone with the oracle."""
    sub = cat.subset(np.asarray(idx))
    U = sub.U
    for _ in range(steps):
        U, _, _ = oracle.step(U, sub.offset, sub.h, sub.n_species, sub.fstride, dt)
    return sub, U


def test_fifo_admission_under_budget(catalogue):
    be = OracleBackend(8, catalogue)
    srv = serving.HydroServer(be, dt=catalogue.dt)
    reqs = [_req(0, [0, 1, 2, 3, 4], 2, 0.0, catalogue),
            _req(1, [5, 6, 7, 8], 1, 0.0, catalogue),      # does not fit next to 0
            _req(2, [9], 1, 0.0, catalogue)]               # fits, but waits behind 1
    recs = srv.run(reqs, realtime=False)
    assert be.loads[0] == [0]
    assert be.ticks[0] == ([0], []) and be.ticks[1] == ([], [0])
    # 1 and 2 are admitted together once 0 has finished and its slots are back
    assert be.loads[1] == [1, 2]
    assert be.ticks[2] == ([1, 2], [])
    assert [r.ticks for r in recs] == [[0, 1], [2], [2]]
    assert srv.pool.free == 8


def test_sessions_at_different_stages_share_ticks(catalogue):
    be = OracleBackend(12, catalogue)
    srv = serving.HydroServer(be, dt=catalogue.dt)
    reqs = [_req(0, [0, 1], 4, 0.0, catalogue),
            _req(1, [2, 3, 4], 2, 1.0, catalogue),
            _req(2, [5], 1, 1.5, catalogue)]
    finals = {}

    def grab(req, slots, copy):
        finals[req.rid] = be.read(slots, copy)

    recs = srv.run(reqs, realtime=True, on_complete=grab)
    # request 1 joins while request 0 is mid-session: some tick has both parities
    assert any(g0 and g1 for g0, g1 in be.ticks)
    assert all(not r.rejected for r in recs)
    for r in reqs:
        sub, U = _alone(catalogue, r.source, r.steps, catalogue.dt)
        got = finals[r.rid]
        for s in range(r.n):
            blk = U[int(sub.offset[s]):int(sub.offset[s]) + SLOT]
            assert np.array_equal(got[s], blk), (r.rid, s)


def test_two_lanes_keep_sessions_in_order_and_results_alone(catalogue):
    """Sessions dealt to two lanes: each runs its stages in one lane, in
    consecutive ticks of that lane, both lanes carry work, and every result
    is the request stepped alone."""
    be = OracleBackend(12, catalogue)
    srv = serving.HydroServer(be, dt=catalogue.dt, lanes=2)
    reqs = [_req(i, [(3 * i + k) % 12 for k in range(1 + i % 3)], 1 + i % 4, 0.3 * i, catalogue)
            for i in range(10)]
    finals = {}

    def grab(req, slots, copy):
        finals[req.rid] = be.read(slots, copy)

    recs = srv.run(reqs, realtime=True, on_complete=grab)
    assert all(not r.rejected for r in recs)
    assert set(be.lanes) == {0, 1}
    for r in recs:
        assert all(be.lanes[t] == r.lane for t in r.ticks)
        lane_ticks = [t for t, q in enumerate(be.lanes) if q == r.lane]
        first = lane_ticks.index(r.ticks[0])
        assert r.ticks == lane_ticks[first:first + r.steps]
    for r in reqs:
        sub, U = _alone(catalogue, r.source, r.steps, catalogue.dt)
        for s in range(r.n):
            assert np.array_equal(finals[r.rid][s], U[int(sub.offset[s]):int(sub.offset[s]) + SLOT])
    with pytest.raises(ValueError):
        serving.HydroServer(be, dt=catalogue.dt, lanes=3)


def test_oversize_and_empty_requests_are_rejected(catalogue):
    be = OracleBackend(3, catalogue)
    srv = serving.HydroServer(be, dt=catalogue.dt)
    reqs = [_req(0, [0, 1, 2, 3], 1, 0.0, catalogue),
            _req(1, [4], 0, 0.0, catalogue),
            _req(2, [5, 6], 1, 0.0, catalogue)]
    recs = srv.run(reqs, realtime=False)
    assert recs[0].rejected and recs[1].rejected and not recs[2].rejected
    assert recs[2].ticks == [0]


def test_slots_are_reused_and_latency_recorded(catalogue):
    be = OracleBackend(4, catalogue)
    srv = serving.HydroServer(be, dt=catalogue.dt)
    reqs = [_req(i, [i % 12, (i + 3) % 12], 1 + (i % 3), 0.25 * i, catalogue) for i in range(9)]
    recs = srv.run(reqs, realtime=True)
    assert all(not r.rejected for r in recs)
    assert srv.pool.free == 4
    for r in recs:
        assert len(r.ticks) == r.steps and r.ticks == list(range(r.ticks[0], r.ticks[0] + r.steps))
        assert r.latency >= r.steps - 1e-12
    # never more than 4 resident subgrids in one tick
    for g0, g1 in be.ticks:
        assert 2 * (len(g0) + len(g1)) <= 4
    summ = serving.summarize(recs)
    assert summ["requests"] == 9 and summ["subgrid_steps"] == sum(2 * r.steps for r in reqs)


def test_request_generator_statistics():
    reqs = serving.poisson_requests(400, rate=100.0, catalogue_n=4096,
                                    h=np.ones(4096), n_species=np.full(4096, 5), seed=7)
    arr = np.array([r.arrival for r in reqs])
    assert np.all(np.diff(arr) > 0)
    gaps = np.diff(np.concatenate([[0.0], arr]))
    assert abs(np.mean(gaps) - 0.01) < 0.002
    sizes = np.array([r.n for r in reqs])
    assert sizes.min() >= 1 and sizes.max() <= 4096
    assert 60 < np.median(sizes) < 260
    for r in reqs[:20]:
        assert len(np.unique(r.source)) == r.n and r.steps in (1, 2, 4)


def test_slots_for_budget():
    assert serving.slots_for_budget(64 * 10 ** 9) == 64 * 10 ** 9 // (2 * 11 * 2752 * 8)
    assert serving.slots_for_budget(2 * 11 * 2752 * 8 - 1) == 0
