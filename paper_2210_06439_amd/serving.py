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
The kernel takes one input and one output buffer, so a tick is two launches:
the sessions at an even stage (copy 0 -> 1) on one stream and those at an odd
stage (copy 1 -> 0) on a second stream.  The two run concurrently; each tick
waits for both launches of the previous tick.  The host builds and launches
tick t+1 while tick t runs, and retires tick t (completions, freed slots)
before it launches tick t+2.

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

    def __init__(self, backend, dt: float):
        self.be = backend
        self.dt = float(dt)
        self.pool = SlotPool(backend.n_slots)

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
        active: list[_Session] = []
        inflight = collections.deque()      # (tick handle, sessions finishing at it, all sessions in it)
        tick_no = 0
        t0 = self.be.start()

        def now():
            return self.be.now(t0)

        while pending or waiting or active or inflight:
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
                admitted.append(s)
                active.append(s)
            if admitted:
                self.be.load(admitted)
            # retire the oldest tick first when two are in flight
            if len(inflight) >= 2 or (inflight and not active):
                self._retire(inflight.popleft(), t0, on_complete)
                continue
            if not active:
                if pending and realtime:
                    self.be.idle_until(t0, pending[0].arrival)
                continue
            groups = ([], [])
            for s in active:
                groups[s.launched % 2].append(s)
            handle = self.be.launch_tick(groups, self.dt, tick_no)
            finishing = []
            for s in active:
                s.launched += 1
                s.rec.ticks.append(tick_no)
                if s.launched == s.req.steps:
                    finishing.append(s)
            inflight.append((handle, finishing, list(active)))
            active = [s for s in active if s.launched < s.req.steps]
            tick_no += 1
        self.be.finish()
        return [recs[r.rid] for r in requests]

    def _retire(self, item, t0, on_complete):
        handle, finishing, members = item
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

    The pool is two device buffers (copy 0 and copy 1) of n_slots slots of
    nf_max * fstride doubles.  A catalogue (a DeviceBatch whose subgrids each
    fill one slot-sized region, i.e. offset[s] = s * nf_max * fstride) lets
    requests name their inputs by index; host arrays are accepted too.
    """

    def __init__(self, n_slots: int, catalogue=None, gamma=5.0 / 3.0, de_switch=1e-3,
                 nf_max: int = NF_MAX, fstride: int = FSTRIDE):
        import torch

        from . import hydro
        self.torch, self.hydro = torch, hydro
        hydro.lib()
        self.n_slots = int(n_slots)
        self.nf_max, self.fstride = nf_max, fstride
        self.slot_elems = nf_max * fstride
        dev = torch.device("cuda")
        self.copies = [torch.zeros(self.n_slots * self.slot_elems, dtype=torch.float64, device=dev)
                       for _ in range(2)]
        self.catalogue = catalogue
        if catalogue is not None:
            off = catalogue.offset.cpu().numpy()
            if catalogue.fstride != fstride or np.any(off != np.arange(len(off)) * self.slot_elems):
                raise ValueError("catalogue subgrids must each fill one slot-sized region")
        self.gamma, self.de_switch = gamma, de_switch
        self.streams = [torch.cuda.Stream(), torch.cuda.Stream()]
        # ring of metadata buffers: three ticks (two in flight, one being filled)
        self.ring = []
        for _ in range(3):
            sets = []
            for _g in range(2):
                sets.append({
                    "off_h": torch.empty(self.n_slots, dtype=torch.int64, pin_memory=True),
                    "h_h": torch.empty(self.n_slots, dtype=torch.float64, pin_memory=True),
                    "ns_h": torch.empty(self.n_slots, dtype=torch.int32, pin_memory=True),
                    "off": torch.empty(self.n_slots, dtype=torch.int64, device=dev),
                    "h": torch.empty(self.n_slots, dtype=torch.float64, device=dev),
                    "ns": torch.empty(self.n_slots, dtype=torch.int32, device=dev),
                    "amax": torch.empty(self.n_slots, dtype=torch.float64, device=dev),
                    "status": torch.empty(self.n_slots, dtype=torch.int32, device=dev),
                    "status_h": torch.empty(self.n_slots, dtype=torch.int32, pin_memory=True),
                })
            self.ring.append(sets)
        self._prev = None

    # -- clock ---------------------------------------------------------------
    def start(self):
        torch = self.torch
        torch.cuda.synchronize()
        self.ev0 = torch.cuda.Event(enable_timing=True)
        self.ev0.record(self.streams[0])
        self.ev0.synchronize()
        self._prev = None
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
    def _slot_view(self, c):
        return self.copies[c].view(self.n_slots, self.slot_elems)

    def load(self, sessions):
        torch = self.torch
        s0 = self.streams[0]
        with torch.cuda.stream(s0):
            for s in sessions:
                slots = torch.as_tensor(s.slots, device="cuda")
                src = s.req.source
                if isinstance(src, np.ndarray) and src.dtype.kind == "f":
                    blk = torch.as_tensor(src.reshape(s.req.n, self.slot_elems)).to(
                        "cuda", non_blocking=False)
                else:
                    cat = self.catalogue.U.view(-1, self.slot_elems)
                    blk = cat.index_select(0, torch.as_tensor(np.asarray(src), device="cuda"))
                for c in range(2):
                    self._slot_view(c).index_copy_(0, slots, blk)

    def read(self, slots, copy):
        """Host copy [n, nf_max, fstride] of the given slots of one copy."""
        torch = self.torch
        torch.cuda.synchronize()
        v = self._slot_view(copy).index_select(0, torch.as_tensor(slots, device="cuda"))
        return v.cpu().numpy().reshape(len(slots), self.nf_max, self.fstride)

    # -- ticks ---------------------------------------------------------------
    def launch_tick(self, groups, dt, tick_no):
        torch, hydro = self.torch, self.hydro
        bufs = self.ring[tick_no % 3]
        prm = hydro.params(self.gamma, self.de_switch, dt)
        evs, members = [], []
        for g in range(2):
            st = self.streams[g]
            if self._prev is not None:
                for e in self._prev:
                    st.wait_event(e)
            sess = groups[g]
            b = bufs[g]
            n = sum(s.req.n for s in sess)
            rows = []
            if n:
                off = b["off_h"].numpy()
                hh = b["h_h"].numpy()
                ns = b["ns_h"].numpy()
                p = 0
                for s in sess:
                    k = s.req.n
                    off[p:p + k] = s.slots * self.slot_elems
                    hh[p:p + k] = s.req.h
                    ns[p:p + k] = s.req.n_species
                    rows.append((id(s), p, k))
                    p += k
                with torch.cuda.stream(st):
                    b["off"][:n].copy_(b["off_h"][:n], non_blocking=True)
                    b["h"][:n].copy_(b["h_h"][:n], non_blocking=True)
                    b["ns"][:n].copy_(b["ns_h"][:n], non_blocking=True)
                    batch = hydro.Batch(n, self.fstride, b["off"].data_ptr(), b["h"].data_ptr(),
                                        b["ns"].data_ptr())
                    hydro.step(prm, batch, self.copies[g], self.copies[1 - g], b["amax"],
                               b["status"], stream=st)
                    b["status_h"][:n].copy_(b["status"][:n], non_blocking=True)
            e = torch.cuda.Event(enable_timing=True)
            e.record(st)
            evs.append(e)
            members.append(rows)
        self._prev = evs
        return (evs, members, tick_no)

    def wait_tick(self, handle, t0):
        evs, members, tick_no = handle
        for e in evs:
            e.synchronize()
        t_end = max(self.ev0.elapsed_time(e) for e in evs) * 1e-3
        bufs = self.ring[tick_no % 3]
        status = {}
        for g in range(2):
            sh = bufs[g]["status_h"].numpy()
            for sid, p, k in members[g]:
                v = int(np.bitwise_or.reduce(sh[p:p + k])) if k else 0
                status[sid] = v
        return t_end, status

    def finish(self):
        self.torch.cuda.synchronize()
