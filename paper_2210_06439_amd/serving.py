"""Serving loop for hydro-step requests: continuous batching over resident state.

A request is a session: n subgrids (each a 14^3 block with frozen ghosts) that
must each be advanced S forward-Euler stages with the server's dt.  The
server keeps every admitted subgrid resident in device memory until its
session ends, and advances all admitted sessions together: one *tick* is one
fused step over every subgrid that still has a stage to do, whichever
session it belongs to.  Requests that arrive while ticks are running join at
the next tick (continuous batching), as soon as the memory budget has room
for them.

Memory.  The budget buys a fixed pool of slots.  A slot holds one subgrid
twice (two ping-pong copies of nf_max fields at fstride), so a resident
subgrid costs 2 * nf_max * fstride * 8 bytes.  Admission is first come,
first served: the oldest waiting request is admitted when the free slots
cover it (a request larger than the whole pool is rejected).  Slots are
returned when the tick that finishes a session has completed on the device.

Ticks.  A session's stage k reads copy k % 2 and writes copy (k + 1) % 2.
A tick is one launch of the fused step with per-subgrid input and output
offsets into one pool buffer, so sessions at even and odd stages advance
together; new sessions are copied in on a copy stream that the tick waits
for.  The host builds and launches tick t+1 while tick t runs, and retires
the oldest tick (completions, freed slots) before it launches a third.

Lanes.  With lanes > 1 the sessions are dealt to several lanes at
admission (each to the lane with the fewest resident subgrids); every lane
runs its own sequence of ticks on its own stream, so the ticks of different
lanes overlap on the device: the tail of one tick (its last, partly filled
round of workgroups) runs beside the start of another lane's tick, and one
lane's launch gaps are filled by the other.  A session stays in its lane,
so its stages still run one after another.

The arithmetic is the library's fused step; a session's result does not
depend on what else is in its ticks (the kernel computes each subgrid on its
own), so a request gives the same bits alone and in the mix.

The loop talks to the device through a backend object (``GpuBackend`` here;
the tests also drive it with a CPU backend of their own).
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Optional

import numpy as np

from . import inputs
from .inputs import FSTRIDE

NF_MAX = 11


@dataclasses.dataclass
class Request:
    """One hydro-step request.

    source: backend-specific reference to the n input blocks (for GpuBackend,
            indices into its catalogue, or a host array [n, nf_max, fstride]).
    h, n_species: per-subgrid cell size and species count (length n).
    steps: stages to apply.  arrival: seconds after the start of the run.
    """
    rid: int
    source: object
    h: np.ndarray
    n_species: np.ndarray
    steps: int
    arrival: float = 0.0

    @property
    def n(self) -> int:
        return int(len(self.h))


@dataclasses.dataclass
class Record:
    rid: int
    n: int
    steps: int
    arrival: float
    lane: int = 0
    admitted: float = float("nan")
    completed: float = float("nan")
    status: int = 0
    rejected: bool = False
    ticks: list = dataclasses.field(default_factory=list)

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


class SlotPool:
    """Free list of slot indices (a slot = one resident subgrid)."""

    def __init__(self, n_slots: int):
        self.n_slots = int(n_slots)
        self._free = collections.deque(range(self.n_slots))

    @property
    def free(self) -> int:
        return len(self._free)

    def alloc(self, n: int) -> Optional[np.ndarray]:
        if n > len(self._free):
            return None
        return np.array([self._free.popleft() for _ in range(n)], dtype=np.int64)

    def release(self, slots: np.ndarray) -> None:
        self._free.extend(int(s) for s in slots)


@dataclasses.dataclass
class _Session:
    req: Request
    rec: Record
    slots: np.ndarray
    launched: int = 0          # stages launched so far
    status: int = 0


def slots_for_budget(budget_bytes: int, nf_max: int = NF_MAX, fstride: int = FSTRIDE) -> int:
    return int(budget_bytes // (2 * nf_max * fstride * 8))


class HydroServer:
    """Continuous-batching loop over a backend (see module docstring)."""

    def __init__(self, backend, dt: float, lanes: int = 1):
        self.be = backend
        self.dt = float(dt)
        self.pool = SlotPool(backend.n_slots)
        self.lanes = int(lanes)
        if self.lanes < 1 or self.lanes > getattr(backend, "max_lanes", 1):
            raise ValueError(f"{self.lanes} lanes: the backend supports "
                             f"{getattr(backend, 'max_lanes', 1)}")

    def run(self, requests, realtime: bool = True,
            on_complete: Optional[Callable] = None) -> list:
        """Serve `requests` (sorted by arrival or not).  With realtime, a
        request becomes visible at its arrival time on the host clock; else
        all are visible at once.  on_complete(session_request, slots,
        final_copy) is called after the session's last tick has completed
        and before its slots are returned.  Returns one Record per request,
        in request order."""
        reqs = sorted(requests, key=lambda r: r.arrival)
        recs = {r.rid: Record(r.rid, r.n, r.steps, r.arrival) for r in reqs}
        pending = collections.deque(reqs)
        waiting = collections.deque()
        L = self.lanes
        active: list[list[_Session]] = [[] for _ in range(L)]
        resident = [0] * L                  # subgrids admitted to each lane and not yet done
        inflight = collections.deque()      # (tick handle, sessions finishing, all sessions, lane)
        lane_inflight = [0] * L
        next_lane = 0
        tick_no = 0
        t0 = self.be.start()

        def now():
            return self.be.now(t0)

        while pending or waiting or any(active) or inflight:
            t = now() if realtime else float("inf")
            while pending and pending[0].arrival <= t:
                waiting.append(pending.popleft())
            # first come, first served admission against the slot budget
            admitted = []
            while waiting:
                r = waiting[0]
                if r.n > self.pool.n_slots or r.steps <= 0 or r.n == 0:
                    rec = recs[r.rid]
                    rec.rejected = True
                    waiting.popleft()
                    continue
                slots = self.pool.alloc(r.n)
                if slots is None:
                    break
                waiting.popleft()
                rec = recs[r.rid]
                rec.admitted = now()
                s = _Session(r, rec, slots)
                lane = min(range(L), key=lambda q: (resident[q], q))
                rec.lane = lane
                resident[lane] += r.n
                admitted.append(s)
                active[lane].append(s)
            if admitted:
                self.be.load(admitted)
            # the next lane (in turn) with sessions and fewer than two ticks in flight
            lane = None
            for q in range(L):
                c = (next_lane + q) % L
                if active[c] and lane_inflight[c] < 2:
                    lane = c
                    break
            # retire the oldest tick when no lane can launch, or when every
            # lane that could is busy
            if inflight and (lane is None or len(inflight) >= 2 * L):
                item = inflight.popleft()
                lane_inflight[item[3]] -= 1
                for s in item[1]:
                    resident[item[3]] -= s.req.n
                self._retire(item, t0, on_complete)
                continue
            if lane is None:
                if pending and realtime:
                    self.be.idle_until(t0, pending[0].arrival)
                continue
            groups = ([], [])
            for s in active[lane]:
                groups[s.launched % 2].append(s)
            if L == 1:
                handle = self.be.launch_tick(groups, self.dt, tick_no)
            else:
                handle = self.be.launch_tick(groups, self.dt, tick_no, lane=lane)
            finishing = []
            for s in active[lane]:
                s.launched += 1
                s.rec.ticks.append(tick_no)
                if s.launched == s.req.steps:
                    finishing.append(s)
            inflight.append((handle, finishing, list(active[lane]), lane))
            lane_inflight[lane] += 1
            active[lane] = [s for s in active[lane] if s.launched < s.req.steps]
            next_lane = (lane + 1) % L
            tick_no += 1
        self.be.finish()
        return [recs[r.rid] for r in requests]

    def _retire(self, item, t0, on_complete):
        handle, finishing, members, _ = item
        t_end, status = self.be.wait_tick(handle, t0)
        for s in members:
            st = status.get(id(s), 0)
            s.status |= st
        for s in finishing:
            s.rec.completed = t_end
            s.rec.status = s.status
            if on_complete is not None:
                on_complete(s.req, s.slots, s.launched % 2)
            self.pool.release(s.slots)


def summarize(records, cells_per_subgrid: int = 512) -> dict:
    """Throughput and latency percentiles of a finished run."""
    done = [r for r in records if not r.rejected]
    if not done:
        return {"requests": 0}
    lat = np.array([r.latency for r in done])
    first = min(r.arrival for r in done)
    last = max(r.completed for r in done)
    work = sum(r.n * r.steps for r in done)
    span = max(last - first, 1e-12)
    return {
        "requests": len(done), "rejected": len(records) - len(done),
        "subgrid_steps": int(work),
        "cell_updates_per_s": work * cells_per_subgrid / span,
        "subgrid_steps_per_s": work / span,
        "makespan_s": span,
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                       "p99": float(np.percentile(lat, 99) * 1e3),
                       "mean": float(np.mean(lat) * 1e3)},
        "ticks": int(max(max(r.ticks) for r in done) + 1),
        "nonzero_status": int(sum(1 for r in done if r.status)),
    }


def poisson_requests(n_requests: int, rate: float, catalogue_n: int, h, n_species,
                     seed: int = 1005, max_n: int = 4096, median_n: float = 128.0,
                     sigma: float = 1.5, steps=(1, 2, 4)) -> list:
    """Requests over a catalogue of catalogue_n subgrids (the seeded stream of
    inputs.config5_requests) with their per-subgrid metadata."""
    out = []
    for i, (t, idx, S) in enumerate(inputs.config5_requests(
            n_requests, rate, seed=seed, pool=catalogue_n, max_sub=max_n,
            median_n=median_n, sigma=sigma, steps=steps)):
        out.append(Request(i, idx, np.asarray(h)[idx], np.asarray(n_species)[idx], S, t))
    return out


def mean_work(n_requests: int, catalogue_n: int, seed: int = 1005, **kw) -> float:
    """E[n * S] of the request distribution, estimated from one draw."""
    reqs = poisson_requests(n_requests, 1.0, catalogue_n, np.ones(catalogue_n),
                            np.zeros(catalogue_n, dtype=np.int32), seed=seed, **kw)
    return float(np.mean([r.n * r.steps for r in reqs]))


class GpuBackend:
    """Device side of the serving loop on the HIP library.

    The pool is one device buffer of 2 x n_slots slot-sized regions of
    nf_max * fstride doubles: copy c of slot q starts at element
    (c * n_slots + q) * slot.  A tick is a single launch of the fused step
    with per-subgrid input and output offsets, so sessions at even stages
    (copy 0 -> 1) and at odd stages (copy 1 -> 0) advance together.  New
    sessions are copied in on a second stream, which the tick waits for.  A
    catalogue (a DeviceBatch whose subgrids each fill one slot-sized region,
    offset[s] = s * nf_max * fstride) lets requests name their inputs by
    index; host arrays are accepted too.  `flags` are the method options of
    every tick (hydro_params.flags).
    """

    IDX_RING = 8

    def __init__(self, n_slots: int, catalogue=None, gamma=5.0 / 3.0, de_switch=1e-3,
                 nf_max: int = NF_MAX, fstride: int = FSTRIDE, flags: int = 0,
                 max_lanes: int = 2):
        import torch

        from . import hydro
        self.torch, self.hydro = torch, hydro
        hydro.lib()
        self.n_slots = int(n_slots)
        self.nf_max, self.fstride = nf_max, fstride
        self.slot_elems = nf_max * fstride
        dev = torch.device("cuda")
        self.pool = torch.zeros(2 * self.n_slots * self.slot_elems, dtype=torch.float64,
                                device=dev)
        self.catalogue = catalogue
        if catalogue is not None:
            off = catalogue.offset.cpu().numpy()
            if catalogue.fstride != fstride or np.any(off != np.arange(len(off)) * self.slot_elems):
                raise ValueError("catalogue subgrids must each fill one slot-sized region")
        self.gamma, self.de_switch, self.flags = gamma, de_switch, int(flags)
        self.max_lanes = int(max_lanes)
        self.lane_streams = [torch.cuda.Stream() for _ in range(self.max_lanes)]
        self.compute = self.lane_streams[0]
        self.copy = torch.cuda.Stream()
        self._load_ev = None
        self.tick_log = []      # per retired tick: (subgrids, GPU start s, GPU end s)
        # pinned staging for the gather indices of a load call (catalogue
        # rows, then the two copies' slot rows), a ring of them, and their
        # device twin.  A load call reuses the oldest pinned buffer once its
        # copy has run; the copy stream's gathers wait for CUs that a tick's
        # persistent kernel holds, so with a single buffer the host would
        # wait for a whole tick there, launching and retiring nothing.
        self._idx_h = [torch.empty(3 * self.n_slots, dtype=torch.int64, pin_memory=True)
                       for _ in range(self.IDX_RING)]
        self._idx_ev = [None] * self.IDX_RING
        self._idx_next = 0
        self._idx_d = torch.empty(3 * self.n_slots, dtype=torch.int64, device=dev)
        # ring of metadata buffers: two ticks in flight per lane, one being filled
        n = 2 * self.n_slots
        self.ring = []
        for _ in range(2 * self.max_lanes + 1):
            self.ring.append({
                "off_h": torch.empty(self.n_slots, dtype=torch.int64, pin_memory=True),
                "oo_h": torch.empty(self.n_slots, dtype=torch.int64, pin_memory=True),
                "h_h": torch.empty(self.n_slots, dtype=torch.float64, pin_memory=True),
                "ns_h": torch.empty(self.n_slots, dtype=torch.int32, pin_memory=True),
                "off": torch.empty(self.n_slots, dtype=torch.int64, device=dev),
                "oo": torch.empty(self.n_slots, dtype=torch.int64, device=dev),
                "h": torch.empty(self.n_slots, dtype=torch.float64, device=dev),
                "ns": torch.empty(self.n_slots, dtype=torch.int32, device=dev),
                "amax": torch.empty(self.n_slots, dtype=torch.float64, device=dev),
                "status": torch.empty(self.n_slots, dtype=torch.int32, device=dev),
                "status_h": torch.empty(self.n_slots, dtype=torch.int32, pin_memory=True),
            })
        del n

    def warmup(self, dt: float):
        """One tiny load, two ticks and a read, so that every kernel the loop
        uses is loaded before a timed run (a kernel's first launch loads its
        code)."""
        from types import SimpleNamespace
        n = min(2, self.n_slots)
        if n == 0:
            return
        src = np.zeros(n, dtype=np.int64) if self.catalogue is not None else np.zeros(
            (n, self.nf_max, self.fstride))
        req = Request(-1, src, np.full(n, 1.0), np.zeros(n, dtype=np.int32), 2)
        sess = [SimpleNamespace(req=req, slots=np.arange(n, dtype=np.int64))]
        self.start()
        self.load(sess)
        for lane in range(self.max_lanes):     # every lane's stream (and its scratch)
            self.wait_tick(self.launch_tick((sess, []), 0.0, 2 * lane, lane=lane), 0.0)
            self.wait_tick(self.launch_tick(([], sess), 0.0, 2 * lane + 1, lane=lane), 0.0)
        self.read(sess[0].slots, 0)
        self.torch.cuda.synchronize()

    # -- clock ---------------------------------------------------------------
    def start(self):
        torch = self.torch
        torch.cuda.synchronize()
        self.ev0 = torch.cuda.Event(enable_timing=True)
        self.ev0.record(self.compute)
        self.ev0.synchronize()
        self._load_ev = None
        return time.perf_counter()

    def now(self, t0):
        return time.perf_counter() - t0

    def idle_until(self, t0, t_arrival):
        while True:
            left = t_arrival - self.now(t0)
            if left <= 0:
                return
            time.sleep(min(left, 2e-4) if left > 1e-3 else 0)

    # -- data movement -------------------------------------------------------
    def _rows(self):
        return self.pool.view(2 * self.n_slots, self.slot_elems)

    def load(self, sessions):
        """Copy the new sessions' blocks into both copies of their slots, in one
        gather per call (copy stream; the next tick waits for it)."""
        torch = self.torch
        rows = self._rows()
        host = [s for s in sessions
                if isinstance(s.req.source, np.ndarray) and s.req.source.dtype.kind == "f"]
        cat = [s for s in sessions if not (isinstance(s.req.source, np.ndarray)
                                           and s.req.source.dtype.kind == "f")]
        with torch.cuda.stream(self.copy):
            if cat:
                q = self._idx_next
                self._idx_next = (q + 1) % self.IDX_RING
                if self._idx_ev[q] is not None:
                    self._idx_ev[q].synchronize()       # this pinned index buffer is free
                m = int(sum(s.req.n for s in cat))
                ih = self._idx_h[q].numpy()
                np.concatenate([np.asarray(s.req.source, dtype=np.int64) for s in cat],
                               out=ih[:m])
                slots = np.concatenate([s.slots for s in cat])
                ih[m:2 * m] = slots
                ih[2 * m:3 * m] = slots + self.n_slots
                idx = self._idx_d[:3 * m]
                # the device twin is rewritten by the next call's copy, behind
                # this call's gathers on the same stream
                idx.copy_(self._idx_h[q][:3 * m], non_blocking=True)
                self._idx_ev[q] = torch.cuda.Event()
                self._idx_ev[q].record(self.copy)
                # each catalogue block read once, written to both copies
                self.hydro.copy_blocks(self.catalogue.U, idx[:m], self.pool, idx[m:2 * m],
                                       idx[2 * m:3 * m], row_elems=self.slot_elems,
                                       stream=self.copy)
            for s in host:
                q = torch.as_tensor(np.concatenate([s.slots, s.slots + self.n_slots]),
                                    device="cuda")
                blk = torch.as_tensor(s.req.source.reshape(s.req.n, self.slot_elems)).to("cuda")
                rows.index_copy_(0, q, torch.cat([blk, blk]))
            ev = torch.cuda.Event()
            ev.record(self.copy)
        self._load_ev = ev

    def read(self, slots, copy):
        """Host copy [n, nf_max, fstride] of the given slots of one copy."""
        torch = self.torch
        torch.cuda.synchronize()
        idx = torch.as_tensor(np.asarray(slots) + copy * self.n_slots, device="cuda")
        v = self._rows().index_select(0, idx)
        return v.cpu().numpy().reshape(len(slots), self.nf_max, self.fstride)

    # -- ticks ---------------------------------------------------------------
    def launch_tick(self, groups, dt, tick_no, lane: int = 0):
        torch, hydro = self.torch, self.hydro
        b = self.ring[tick_no % len(self.ring)]
        sess = list(groups[0]) + list(groups[1])
        par = [0] * len(groups[0]) + [1] * len(groups[1])
        sizes = [s.req.n for s in sess]
        p = int(sum(sizes))
        rows = ([id(s) for s in sess], np.cumsum([0] + sizes[:-1]) if sess else np.zeros(0, int),
                sizes)
        if p:
            slots = np.concatenate([s.slots for s in sess])
            parity = np.repeat(np.asarray(par, dtype=np.int64), sizes)
            n, se = self.n_slots, self.slot_elems
            np.multiply(slots + parity * n, se, out=b["off_h"].numpy()[:p])
            np.multiply(slots + (1 - parity) * n, se, out=b["oo_h"].numpy()[:p])
            np.concatenate([s.req.h for s in sess], out=b["h_h"].numpy()[:p])
            np.concatenate([s.req.n_species for s in sess], out=b["ns_h"].numpy()[:p],
                           casting="unsafe")
        st = self.lane_streams[lane]
        with torch.cuda.stream(st):
            if self._load_ev is not None:
                # the latest load (every session of this tick was loaded by it
                # or by an earlier one, which the copy stream ran first)
                st.wait_event(self._load_ev)
            e0 = torch.cuda.Event(enable_timing=True)
            e0.record(st)
            if p:
                b["off"][:p].copy_(b["off_h"][:p], non_blocking=True)
                b["oo"][:p].copy_(b["oo_h"][:p], non_blocking=True)
                b["h"][:p].copy_(b["h_h"][:p], non_blocking=True)
                b["ns"][:p].copy_(b["ns_h"][:p], non_blocking=True)
                batch = hydro.Batch(p, self.fstride, b["off"].data_ptr(), b["h"].data_ptr(),
                                    b["ns"].data_ptr())
                hydro.step_io(hydro.params(self.gamma, self.de_switch, dt, self.flags), batch,
                              b["oo"],
                              self.pool, self.pool, b["amax"], b["status"], stream=st)
                b["status_h"][:p].copy_(b["status"][:p], non_blocking=True)
            e = torch.cuda.Event(enable_timing=True)
            e.record(st)
        return (e, rows, tick_no, e0, p)

    def wait_tick(self, handle, t0):
        e, rows, tick_no, e0, p = handle
        e.synchronize()
        t_end = self.ev0.elapsed_time(e) * 1e-3
        self.tick_log.append((p, self.ev0.elapsed_time(e0) * 1e-3, t_end))
        ids, starts, sizes = rows
        status = {}
        if ids:
            sh = self.ring[tick_no % len(self.ring)]["status_h"].numpy()[:p]
            red = np.bitwise_or.reduceat(sh, starts) if p else np.zeros(len(ids), np.int32)
            status = {sid: int(v) for sid, v, k in zip(ids, red, sizes) if k and v}
        return t_end, status

    def finish(self):
        self.torch.cuda.synchronize()
