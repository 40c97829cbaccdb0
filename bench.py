#!/usr/bin/env python3
"""Benchmark of the fused FP64 hydro stage on one MI355X.

Workload (timed): the 128^3 binary-star mesh, 4096 subgrids of 8^3 cells
with 3 ghost layers and 5 passive species (11 fields), all in one fused
persistent launch replayed from a hipGraph; inputs are resident in HBM
before the timed region.  A step is one stage over the whole batch.

Also reported: the 64^3 Sod-like mesh (512 subgrids) launched one subgrid at
a time (unfused three-kernel form and fused form) against one batched
launch, the step latency percentiles, the roofline of the fused kernel, and
the CPU oracle's rate on a bounded sample of the same workload.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6     # MI355X vector FP64 (published)
HBM_PEAK_GBPS = 8000.0      # MI355X HBM3E (published)

# HBM traffic of the fused kernel, from two counter passes over
# `bench.py --traffic-probe` (one fused step on the 128^3 batch, then a copy of
# COPY_BYTES).  The counter file also holds the hash of the kernel sources the
# counts were taken with; traffic is reported only while those are unchanged.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fused_binary_star_4096_traffic.md")
KERNEL_SOURCES = ("paper_2210_06439_amd/csrc/fused.hip", "paper_2210_06439_amd/csrc/hydro_internal.hpp")
COPY_BYTES = 512 * 1024 * 1024


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_per_launch():
    """HBM bytes per fused launch from the committed counter summary, scaled by
    the copy calibration, or None if the kernel changed since it was taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            lines = f.read().splitlines()
    except OSError:
        return None, "no counter summary"
    vals = {}
    for ln in lines:
        parts = ln.split()
        if len(parts) == 3 and parts[0] == "counter:":
            vals[parts[1]] = parts[2]
    try:
        if vals["sources_sha256"] != kernel_source_hash():
            return None, "kernel changed since the counters were taken"
        copy_kib = float(vals["copy_bytes"]) / 1024.0
        f_scale = copy_kib / float(vals["copy_FETCH_SIZE_KiB"])
        w_scale = copy_kib / float(vals["copy_WRITE_SIZE_KiB"])
        fetch = float(vals["k_fused_FETCH_SIZE_KiB"]) * f_scale * 1024.0
        write = float(vals["k_fused_WRITE_SIZE_KiB"]) * w_scale * 1024.0
    except (KeyError, ValueError, ZeroDivisionError):
        return None, "counter summary incomplete"
    return {"bytes": fetch + write, "read_bytes": fetch, "write_bytes": write,
            "fetch_scale": f_scale, "write_scale": w_scale}, None


def traffic_probe():
    """One fused step on the 128^3 batch, then a device copy of COPY_BYTES
    (the calibration for FETCH_SIZE / WRITE_SIZE); run under rocprofv3 --pmc."""
    import torch

    from paper_2210_06439_amd import hydro, inputs
    torch.cuda.set_device(0)
    b = inputs.config3()
    db = hydro.DeviceBatch.from_inputs(b)
    U_out = db.U.clone()
    amax = torch.zeros(db.n_sub, dtype=torch.float64, device="cuda")
    plan = hydro.Plan(hydro.params(dt=b.dt), db.struct, db.U, U_out, amax)
    plan.launch()
    torch.cuda.synchronize()
    plan.close()
    src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"traffic_probe": True, "copy_bytes": COPY_BYTES,
                      "sources_sha256": kernel_source_hash()}), flush=True)


def timed_plan(plan, steps, warmup, torch):
    for _ in range(warmup):
        plan.launch()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(stream)
        plan.launch()
        b.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([a.elapsed_time(b) for a, b in evs])
    return wall, per


def plain_batched_stages(torch, hydro, db, prm, reps=5):
    """The unfused form with one launch per stage over the whole batch: each
    stage's time and its algorithmic HBM rate (Q and F round-trip HBM)."""
    n = db.n_sub
    nf = 6 + db.n_species_host.astype(np.int64)
    qo, qn = db.q_layout()
    fo, fn = db.f_layout()
    Q = torch.zeros(qn, dtype=torch.float64, device="cuda")
    F = torch.zeros(fn, dtype=torch.float64, device="cuda")
    amax = torch.zeros(n, dtype=torch.float64, device="cuda")
    U_out = db.U.clone()
    u_bytes = int(np.sum(nf * 2744 * 8))
    q_bytes, f_bytes = qn * 8, fn * 8
    i_bytes = int(np.sum(nf * 512 * 8))
    prm_cw = hydro.params(gamma=prm.gamma, de_switch=prm.de_switch, dt=prm.dt,
                          flags=prm.flags | hydro.STEEPEN | hydro.FLATTEN)
    stages = {
        "reconstruct": (lambda: hydro.reconstruct(prm, db.struct, db.U, Q, qo), u_bytes + q_bytes),
        "flux": (lambda: hydro.flux(prm, db.struct, Q, qo, F, fo, amax), q_bytes + f_bytes),
        "divergence": (lambda: hydro.divergence(prm, db.struct, F, fo, db.U, U_out),
                       f_bytes + 2 * i_bytes),
        # the Colella-Woodward options run in this form only
        "reconstruct_steepen_flatten": (lambda: hydro.reconstruct(prm_cw, db.struct, db.U, Q, qo),
                                        u_bytes + q_bytes),
    }
    out = {}
    stream = torch.cuda.current_stream()
    for name, (fn_, nbytes) in stages.items():
        fn_()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn_()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": ms, "algorithmic_bytes": nbytes,
                     "GB_per_s": nbytes / (ms * 1e-3) / 1e9,
                     "hbm_frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS}
        log(f"plain batched {name}: {ms:.3f} ms, {out[name]['GB_per_s']:.0f} GB/s")
    return out


def subgrid16_plain(torch, hydro, inputs, reps=5):
    """The plain stages of the library built for 16^3 subgrids on the same
    128^3 binary-star mesh (512 subgrids): time per stage and the mesh's
    cell-update rate, beside the 8^3 build's plain stages."""
    U, off, h, ns, fs, dt = inputs.config3_subgrid16()
    db = hydro.DeviceBatch(U, off, h, ns, fs, n=16)
    del U
    prm = hydro.params(dt=dt)
    qo, qn = db.q_layout()
    fo, fn = db.f_layout()
    Q = torch.zeros(qn, dtype=torch.float64, device="cuda")
    F = torch.zeros(fn, dtype=torch.float64, device="cuda")
    amax = torch.zeros(db.n_sub, dtype=torch.float64, device="cuda")
    U_out = db.U.clone()
    stages = {
        "reconstruct": lambda: hydro.reconstruct(prm, db.struct, db.U, Q, qo, n=16),
        "flux": lambda: hydro.flux(prm, db.struct, Q, qo, F, fo, amax, n=16),
        "divergence": lambda: hydro.divergence(prm, db.struct, F, fo, db.U, U_out, n=16),
    }
    out = {"workload": "128^3 binary-star mesh: 512 subgrids of 16^3 (+3 ghosts), 11 fields"}
    stream = torch.cuda.current_stream()
    total = 0.0
    for name, fn_ in stages.items():
        fn_()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn_()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name + "_ms"] = ms
        total += ms
    out["ms_per_stage"] = total
    out["cell_updates_per_s"] = db.n_sub * 16 ** 3 / (total * 1e-3)
    log(f"plain stages at 16^3: {total:.3f} ms per stage "
        f"({out['cell_updates_per_s']:.3e} cell-updates/s)")
    # the fused step of the 16^3 build: each subgrid's eight 8^3 tiles
    # stepped in place by the 8^3 fused kernel (compiled there for the 22^3
    # blocks' row pitch)
    L = hydro.lib(16)
    status = torch.zeros(db.n_sub, dtype=torch.int32, device="cuda")
    fused = lambda: L.hydro_step(ctypes.byref(prm), ctypes.byref(db.struct), hydro._ptr(db.U),
                                 hydro._ptr(U_out), hydro._ptr(amax), hydro._ptr(status), None)
    for _ in range(3):
        assert fused() == 0
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(2 * reps):
        fused()
    e1.record(stream)
    torch.cuda.synchronize()
    fms = e0.elapsed_time(e1) / (2 * reps)
    out["fused_ms"] = fms
    out["fused_cell_updates_per_s"] = db.n_sub * 16 ** 3 / (fms * 1e-3)
    out["fused_nonzero_status"] = int(status.any().item())
    log(f"fused step at 16^3 (8^3 tiles): {fms:.3f} ms ({out['fused_cell_updates_per_s']:.3e} "
        f"cell-updates/s)")
    del Q, F, U_out, db, status
    torch.cuda.empty_cache()
    return out


def per_subgrid_vs_batched(torch, hydro, b, db, label, reps):
    """One subgrid per launch (unfused three-kernel form and fused form)
    against one batched launch, on the same batch."""
    prm = hydro.params(dt=b.dt)
    n = db.n_sub
    U_out = db.U.clone()
    amax = torch.zeros(n, dtype=torch.float64, device="cuda")
    status = torch.zeros(n, dtype=torch.int32, device="cuda")
    Q = torch.zeros(hydro.q_elems(5), dtype=torch.float64, device="cuda")
    F = torch.zeros(hydro.f_elems(5), dtype=torch.float64, device="cuda")
    zero = torch.zeros(1, dtype=torch.int64, device="cuda")
    views = [db.view(s, 1) for s in range(n)]

    def unfused():
        for s in range(n):
            hydro.reconstruct(prm, views[s], db.U, Q, zero)
            hydro.flux(prm, views[s], Q, zero, F, zero, amax[s:s + 1], status[s:s + 1])
            hydro.divergence(prm, views[s], F, zero, db.U, U_out)

    def fused_each():
        for s in range(n):
            hydro.step(prm, views[s], db.U, U_out, amax[s:s + 1], status[s:s + 1])

    def batched():
        hydro.step(prm, db.struct, db.U, U_out, amax, status)

    out = {}
    for name, fn in (("per_subgrid_unfused", unfused), ("per_subgrid_fused", fused_each),
                     ("batched_fused", batched)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[name] = {"ms": dt * 1e3, "cell_updates_per_s": b.cell_updates / dt}
        log(f"{label} {name}: {dt * 1e3:.2f} ms")
    out["speedup_batched_vs_per_subgrid_unfused"] = (
        out["per_subgrid_unfused"]["ms"] / out["batched_fused"]["ms"])
    out["speedup_batched_vs_per_subgrid_fused"] = (
        out["per_subgrid_fused"]["ms"] / out["batched_fused"]["ms"])
    del U_out, Q, F
    return out


def plain_vs_batched(torch, hydro, inputs, reps=3):
    """Config 2 (64^3, 512 subgrids): one subgrid per launch vs one batched
    launch, and the batched unfused stages."""
    b = inputs.config2()
    db = hydro.DeviceBatch.from_inputs(b)
    out = per_subgrid_vs_batched(torch, hydro, b, db, "config2", reps)
    out["plain_batched_stages"] = plain_batched_stages(torch, hydro, db, hydro.params(dt=b.dt))
    return out


def serving_run(torch, hydro, serving, b, db, peak_subgrids_per_s, n_requests, budget_gb,
                lanes=2):
    """Continuous-batching serving of Poisson request streams drawn from the
    128^3 batch.  The loop's capacity is measured first: the same kind of
    stream with every request visible at once (the queue never empties),
    with one lane and with `lanes` lanes.  The offered loads 0.3/0.6/0.9 are
    fractions of that capacity (with `lanes` lanes), so a load below 1 is
    one the loop can sustain; each is also given against the kernel's batched
    peak."""
    n_slots = serving.slots_for_budget(int(budget_gb * 1e9))
    be = serving.GpuBackend(n_slots, catalogue=db, max_lanes=lanes)
    be.warmup(b.dt)
    work = serving.mean_work(4000, b.n_sub)
    out = {"budget_GB": budget_gb, "slots": n_slots, "requests_per_load": n_requests,
           "kernel_peak_subgrid_steps_per_s": peak_subgrids_per_s,
           "mean_subgrid_steps_per_request": work, "lanes": lanes, "loads": {}}
    cap = {}
    for nl in sorted({1, lanes}):
        reqs = serving.poisson_requests(n_requests, 1.0, b.n_sub, b.h, b.n_species, seed=1006)
        for r in reqs:
            r.arrival = 0.0                  # all queued at the start
        summ = serving.summarize(serving.HydroServer(be, b.dt, lanes=nl).run(reqs, realtime=False))
        cap[nl] = summ["subgrid_steps_per_s"]
        log(f"serving capacity, {nl} lane(s): {cap[nl]:.3e} subgrid-steps/s "
            f"({cap[nl] / peak_subgrids_per_s:.3f} of the kernel's batched peak)")
    capacity = cap[lanes]
    out["capacity_subgrid_steps_per_s"] = {str(k): v for k, v in cap.items()}
    out["capacity_over_kernel_peak"] = capacity / peak_subgrids_per_s
    for load in (0.3, 0.6, 0.9):
        rate = load * capacity / work
        reqs = serving.poisson_requests(n_requests, rate, b.n_sub, b.h, b.n_species)
        recs = serving.HydroServer(be, b.dt, lanes=lanes).run(reqs, realtime=True)
        summ = serving.summarize(recs)
        summ["offered_requests_per_s"] = rate
        summ["offered_subgrid_steps_per_s"] = rate * work
        summ["offered_over_kernel_peak"] = rate * work / peak_subgrids_per_s
        summ["delivered_over_offered"] = summ["subgrid_steps_per_s"] / (rate * work)
        out["loads"][str(load)] = summ
        log(f"serving load {load} of capacity: {summ['cell_updates_per_s']:.3e} cell-updates/s "
            f"({summ['delivered_over_offered']:.3f} of offered), "
            f"p50 {summ['latency_ms']['p50']:.2f} ms, p99 {summ['latency_ms']['p99']:.2f} ms, "
            f"{summ['ticks']} ticks")
    del be
    torch.cuda.empty_cache()
    return out


def rk3_timing(torch, hydro, db, n_per_dim, periodic, steps):
    """Device-resident SSP-RK3 time steps: three fused stages that read their
    ghost cells through the neighbour map, the on-device CFL step size and
    the stage combinations, replayed as one hipGraph per time step.  Also
    times the standalone ghost fill (hydro_fill_ghosts) of the same batch."""
    gm = hydro.DeviceGhostMap(*hydro.box_ghost_map(*n_per_dim, periodic=periodic))
    hydro.fill_ghosts(db.struct, gm, db.U)
    torch.cuda.synchronize()
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record(torch.cuda.current_stream())
    for _ in range(5):
        hydro.fill_ghosts(db.struct, gm, db.U)
    f1.record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    fill_ms = f0.elapsed_time(f1) / 5
    rk = hydro.RK3(hydro.params(), db, gm, db.U, cfl=0.4)
    rk.launch(2)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    rk.launch(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    st = int(rk.status.any().item())
    t_sim = float(rk.clock[0].item())
    rk.close()
    cells = db.n_sub * 512
    return {"ms_per_time_step": ms, "stages_per_step": 3,
            "stage_cell_updates_per_s": 3 * cells / (ms * 1e-3),
            "time_steps_per_s": 1e3 / ms, "simulated_time": t_sim,
            "nonzero_status": st, "ghost_fill_ms": fill_ms}


def _launch_set(torch, hydro, cat_db, picks):
    """Batch descriptors of a set of launches that each take the subgrids
    picks[l] of a resident catalogue: all launches' metadata in one device
    buffer, outputs (U_out at the catalogue's offsets, amax and status) in
    buffers of their own."""
    cat_off = cat_db.offset.cpu().numpy()
    cat_h = cat_db.h.cpu().numpy()
    cat_ns = cat_db.n_species_host
    idx = np.concatenate(picks)
    off = torch.as_tensor(cat_off[idx]).cuda()
    h = torch.as_tensor(cat_h[idx]).cuda()
    ns = torch.as_tensor(cat_ns[idx].astype(np.int32)).cuda()
    amax = torch.zeros(len(idx), dtype=torch.float64, device="cuda")
    status = torch.zeros(len(idx), dtype=torch.int32, device="cuda")
    launches, start = [], 0
    for p in picks:
        n = len(p)
        b = hydro.Batch(n, cat_db.fstride, off.data_ptr() + 8 * start, h.data_ptr() + 8 * start,
                        ns.data_ptr() + 4 * start)
        launches.append((b, amax[start:start + n], status[start:start + n], cat_ns[p]))
        start += n
    return {"launches": launches, "keep": (off, h, ns), "amax": amax, "status": status}


def _time_launches(torch, hydro, prm, cat_db, U_out, ls, variant=None):
    """Every launch of the set once (warm-up), then once more timed: HIP
    events around each launch and around the whole set."""
    def go(timed):
        evs = []
        for b, am, st, _ in ls["launches"]:
            if timed:
                e = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                e[0].record(torch.cuda.current_stream())
            hydro.step(prm, b, cat_db.U, U_out, am, st, variant=variant)
            if timed:
                e[1].record(torch.cuda.current_stream())
                evs.append(e)
        return evs
    go(False)
    torch.cuda.synchronize()
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(torch.cuda.current_stream())
    evs = go(True)
    z.record(torch.cuda.current_stream())
    torch.cuda.synchronize()
    per = np.array([x.elapsed_time(y) for x, y in evs])
    return a.elapsed_time(z), per


def config4_run(torch, hydro, inputs, costmodel, n_launches):
    """Config 4: uneven AMR batches.  A catalogue of 8192 subgrids of the
    binary-star field at levels 0-4 (0 or 5 species each) stays resident;
    each launch takes n = clip(round(lognormal(ln 256, 1.5)), 1, 8192) of
    them (seeded, without repetition).  The launches run back to back with
    the default launch shape for their size, again after autotuning every
    size bucket that occurs, and with the one-sweep shape (persistent-2x)
    for all of them."""
    cat = inputs.config4(launch=9, n_override=8192)
    db = hydro.DeviceBatch.from_inputs(cat)
    rng = np.random.default_rng([1004, 200])
    sizes = np.clip(np.round(np.exp(rng.normal(np.log(256), 1.5, n_launches))), 1,
                    cat.n_sub).astype(int)
    picks = [np.sort(rng.choice(cat.n_sub, n, replace=False)) for n in sizes]
    ls = _launch_set(torch, hydro, db, picks)
    prm = hydro.params(dt=cat.dt)
    U_out = db.U.clone()
    flops = sum(costmodel.cost(nsp)[0] for *_, nsp in ls["launches"])
    cells = int(sizes.sum()) * 512
    out = {"workload": f"{n_launches} launches of lognormal(ln 256, 1.5) sizes in [1, 8192] "
                       "drawn from 8192 resident binary-star subgrids at levels 0-4, 0 or 5 "
                       "species mixed",
           "launches": n_launches, "subgrid_steps": int(sizes.sum()),
           "size_p50": float(np.median(sizes)), "size_max": int(sizes.max()),
           "flops": flops}

    def record(name, total_ms, per):
        kern = float(per.sum())
        out[name] = {"ms_total": total_ms, "cell_updates_per_s": cells / (total_ms * 1e-3),
                     "kernel_ms_sum": kern,
                     "fp64_tflops": flops / (kern * 1e-3) / 1e12,
                     "alu_frac": flops / (kern * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                     "launch_ms": {"p50": float(np.percentile(per, 50)),
                                   "p99": float(np.percentile(per, 99)),
                                   "max": float(per.max())}}
        log(f"config4 {name}: {total_ms:.2f} ms for {n_launches} launches, "
            f"{out[name]['cell_updates_per_s']:.3e} cell-updates/s, launch p50 "
            f"{out[name]['launch_ms']['p50']:.3f} p99 {out[name]['launch_ms']['p99']:.3f} ms")

    record("one_sweep", *_time_launches(torch, hydro, prm, db, U_out, ls, variant=1))
    record("default_shapes", *_time_launches(torch, hydro, prm, db, U_out, ls))
    # autotune one launch of every power-of-two size bucket that occurs
    tuned = {}
    for (b, am, st, _), n in zip(ls["launches"], sizes):
        key = int(np.ceil(np.log2(max(n, 1))))
        if key not in tuned:
            best, _ = hydro.autotune(prm, b, db.U, U_out, am, st, reps=3)
            tuned[key] = hydro.variant_name(best)
    out["tuned_shapes"] = {str(2 ** k): v for k, v in sorted(tuned.items())}
    record("tuned", *_time_launches(torch, hydro, prm, db, U_out, ls))
    st = ls["status"].cpu().numpy()
    out["nonzero_status"] = int(np.count_nonzero(st))
    del U_out, ls, db
    torch.cuda.empty_cache()
    return out


def six_field_run(torch, hydro, inputs, costmodel, b, kern11_ms, steps, warmup):
    """Subgrids without species (6 fields): the 128^3 binary-star batch with
    its species removed and the 64^3 blast, each captured in a plan and timed
    as config 3; per-subgrid kernel time against config 3's (11 fields)."""
    out = {}
    t0 = time.perf_counter()
    bs = inputs.pack_blocks([np.array(b.block(s))[:6] for s in range(b.n_sub)], b.h, dt=b.dt,
                            name="binary-star-6")
    log(f"6-field binary star packed in {time.perf_counter() - t0:.1f} s")
    sedov = inputs.sedov(64)
    per11 = kern11_ms * 1e3 / b.n_sub
    for name, bb in (("binary_star_6_fields", bs), ("sedov64", sedov)):
        dt = bb.dt if bb.dt > 0.0 else 1e-4
        d = hydro.DeviceBatch.from_inputs(bb)
        U_out = d.U.clone()
        am = torch.zeros(d.n_sub, dtype=torch.float64, device="cuda")
        st = torch.zeros(d.n_sub, dtype=torch.int32, device="cuda")
        plan = hydro.Plan(hydro.params(dt=dt), d.struct, d.U, U_out, am, st)
        _, per = timed_plan(plan, steps, warmup, torch)
        plan.close()
        ms = float(np.mean(per))
        flops = costmodel.cost(bb.n_species)[0]
        out[name] = {"subgrids": bb.n_sub, "kernel_ms": ms,
                     "per_subgrid_us": ms * 1e3 / bb.n_sub,
                     "per_subgrid_vs_11_fields": ms * 1e3 / bb.n_sub / per11,
                     "cell_updates_per_s": bb.cell_updates / (ms * 1e-3),
                     "alu_frac": flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
                     "variant": hydro.variant_name(hydro.selected_variant(bb.n_sub)),
                     "nonzero_status": int(st.any().item())}
        log(f"{name}: kernel {ms:.3f} ms, {out[name]['per_subgrid_us']:.3f} us per subgrid "
            f"({out[name]['per_subgrid_vs_11_fields']:.3f} of config 3's)")
        del d, U_out
    out["config3_per_subgrid_us"] = per11
    torch.cuda.empty_cache()
    return out


def single_subgrid_latency(torch, hydro, inputs, reps=200):
    """Config 1: one subgrid per launch, eager and replayed from a plan; HIP
    events around each launch."""
    b = inputs.config1()
    db = hydro.DeviceBatch.from_inputs(b)
    prm = hydro.params(dt=b.dt)
    U_out = db.U.clone()
    amax = torch.zeros(1, dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = {"workload": "one 8^3 subgrid (+3 ghosts), 11 fields",
           "shape": hydro.variant_name(hydro.selected_variant(1))}
    for name, fn in (("eager", lambda: hydro.step(prm, db.struct, db.U, U_out, amax, status)),
                     ("one_sweep", lambda: hydro.step(prm, db.struct, db.U, U_out, amax, status,
                                                      variant=1))):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        evs = []
        for _ in range(reps):
            e = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            e[0].record(torch.cuda.current_stream())
            fn()
            e[1].record(torch.cuda.current_stream())
            evs.append(e)
        torch.cuda.synchronize()
        per = np.array([x.elapsed_time(y) for x, y in evs])
        out[name] = {"p50_ms": float(np.percentile(per, 50)), "p99_ms": float(np.percentile(per, 99))}
    plan = hydro.Plan(prm, db.struct, db.U, U_out, amax, status)
    _, per = timed_plan(plan, reps, 5, torch)
    plan.close()
    out["graph"] = {"p50_ms": float(np.percentile(per, 50)), "p99_ms": float(np.percentile(per, 99))}
    log(f"config1 one subgrid ({out['shape']}): eager p50 {out['eager']['p50_ms'] * 1e3:.1f} us, "
        f"graph p50 {out['graph']['p50_ms'] * 1e3:.1f} us, one sweep p50 "
        f"{out['one_sweep']['p50_ms'] * 1e3:.1f} us")
    return out


def _oracle_slice(args):
    """Oracle steps over subgrids of one slice until the time is up (one process)."""
    b, idx, seconds = args
    import oracle
    done = 0
    t0 = time.perf_counter()
    elapsed = 0.0
    while elapsed < seconds:                   # cycles through the slice if it runs out
        start = done % len(idx)
        part = np.sort(idx[start:start + 16])
        sub = b.subset(part)
        oracle.step(sub.U, sub.offset, sub.h, sub.n_species, sub.fstride, b.dt)
        done += len(part)
        elapsed = time.perf_counter() - t0
    return done, elapsed


def cpu_baseline(b, seconds, procs):
    """The oracle, single-threaded, on a random subset of the workload; then
    the same in `procs` processes on disjoint slices (forked before the GPU
    is touched).  Each leg runs for about `seconds`."""
    import multiprocessing

    import oracle
    oracle.build()
    order = np.random.default_rng(0).permutation(b.n_sub)
    done, elapsed = _oracle_slice((b, order, seconds))
    out = {"value": done * 512 / elapsed, "unit": "cell-updates/s", "cores": 1,
           "kind": "oracle",
           "sample": f"{done} subgrid steps over the 4096 subgrids of the 128^3 binary-star "
                     f"batch (random order, seed 0), single thread, {elapsed:.1f} s",
           "cpu": _cpu_model(), "host": _host_cpus()}
    if procs > 1:
        slices = [(b, order[p::procs], seconds) for p in range(procs)]
        with multiprocessing.get_context("fork").Pool(procs) as pool:
            t0 = time.perf_counter()
            res = pool.map(_oracle_slice, slices)
            wall = time.perf_counter() - t0
        n = sum(d for d, _ in res)
        out["all_cores"] = {"value": n * 512 / wall, "unit": "cell-updates/s", "cores": procs,
                            "sample": f"{n} subgrid steps in {procs} processes, {wall:.1f} s",
                            "note": "one process per core of the CPU share a one-GPU job gets "
                                    "(16 on the MI355X box), whatever the host shows in all"}
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_cpus():
    """What the timing host shows of its CPUs: logical CPUs of the machine,
    the ones this process may run on, and lscpu's sockets and cores."""
    out = {"logical_cpus": os.cpu_count(), "model": _cpu_model()}
    try:
        out["usable_cpus"] = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        pass
    try:
        import subprocess
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in txt.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() in ("Socket(s)", "Core(s) per socket", "Thread(s) per core",
                             "Model name", "CPU max MHz"):
                out[k.strip()] = v.strip()
    except (OSError, ValueError, subprocess.SubprocessError):
        pass
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--cpu-procs", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-rk3", action="store_true")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-config4", action="store_true")
    ap.add_argument("--config4-launches", type=int, default=200)
    ap.add_argument("--rk3-steps", type=int, default=10)
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-budget-gb", type=float, default=64.0)
    ap.add_argument("--traffic-probe", action="store_true",
                    help="one fused step and a calibration copy, for counter runs")
    ap.add_argument("--only-config4", action="store_true",
                    help="the config-4 launches alone (for a kernel trace of them)")
    ap.add_argument("--only-subgrid16", action="store_true",
                    help="the 16^3 build's plain stages and fused step alone (for a kernel trace)")
    ap.add_argument("--no-six-field", action="store_true")
    ap.add_argument("--only-six-field", action="store_true",
                    help="config 3, then its 6-field form and the 64^3 blast, timed alone "
                         "(for a kernel trace of them)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the hydro stage is measured on a single "
              "MI355X (multi-GPU sharding is a design note, not built).", file=sys.stderr)
        sys.exit(2)
    if args.traffic_probe:
        traffic_probe()
        return
    if args.only_subgrid16:
        import torch

        from paper_2210_06439_amd import hydro, inputs
        torch.cuda.set_device(0)
        print(json.dumps({"subgrid16_plain": subgrid16_plain(torch, hydro, inputs)}), flush=True)
        return
    if args.only_config4:
        import torch

        from paper_2210_06439_amd import costmodel, hydro, inputs
        torch.cuda.set_device(0)
        print(json.dumps({"config4": config4_run(torch, hydro, inputs, costmodel,
                                                 args.config4_launches)}), flush=True)
        return

    from paper_2210_06439_amd import inputs
    t0 = time.perf_counter()
    b = inputs.config3()
    log(f"config3 generated in {time.perf_counter() - t0:.1f} s ({b.n_sub} subgrids)")
    cpu = None
    if not args.no_cpu_baseline:
        # on the CPU, before the GPU is initialised (the worker processes are forked)
        cpu = cpu_baseline(b, args.cpu_seconds, args.cpu_procs)
        log(f"oracle: {cpu['value']:.3e} cell-updates/s on 1 core"
            + (f", {cpu['all_cores']['value']:.3e} on {cpu['all_cores']['cores']}"
               if "all_cores" in cpu else ""))

    import torch

    from paper_2210_06439_amd import costmodel, hydro, serving

    torch.cuda.set_device(0)
    db = hydro.DeviceBatch.from_inputs(b)
    prm = hydro.params(dt=b.dt)
    U_out = db.U.clone()
    amax = torch.zeros(db.n_sub, dtype=torch.float64, device="cuda")
    status = torch.zeros(db.n_sub, dtype=torch.int32, device="cuda")
    best, times = hydro.autotune(prm, db.struct, db.U, U_out, amax, status, reps=3)
    log("autotune: " + ", ".join(f"{hydro.variant_name(v)}={t:.3f}ms" for v, t in enumerate(times))
        + f" -> {hydro.variant_name(best)}")
    plan = hydro.Plan(prm, db.struct, db.U, U_out, amax, status)
    wall, per = timed_plan(plan, args.steps, args.warmup, torch)
    if args.only_six_field:
        plan.close()
        print(json.dumps({"six_field": six_field_run(torch, hydro, inputs, costmodel, b,
                                                     float(np.mean(per)), args.steps,
                                                     args.warmup)}), flush=True)
        return
    st = status.cpu().numpy()
    if np.any(st != 0):
        log(f"WARNING: nonzero status words: {np.unique(st)}")
    ms_per_step = wall * 1e3 / args.steps
    value = b.cell_updates / (wall / args.steps)
    kern_ms = float(np.mean(per))
    flops, nbytes = costmodel.cost(b.n_species)
    achieved_tf = flops / (kern_ms * 1e-3) / 1e12
    achieved_gbps = nbytes / (kern_ms * 1e-3) / 1e9
    log(f"config3 fused: {ms_per_step:.3f} ms/step wall, kernel {kern_ms:.3f} ms, "
        f"{value:.3e} cell-updates/s, {achieved_tf:.1f} TFLOP/s, {achieved_gbps:.0f} GB/s")
    plan.close()
    variants = None
    if not args.no_variants:
        # the method variants on the same batch, each captured the same way
        variants = {}
        cw = hydro.STEEPEN | hydro.FLATTEN
        for name, fl in (("kt_symmetric", hydro.KT_SYMMETRIC), ("velocity", hydro.VELOCITY),
                         ("velocity+kt_symmetric", hydro.VELOCITY | hydro.KT_SYMMETRIC),
                         ("steepen+flatten", cw), ("velocity+steepen+flatten", hydro.VELOCITY | cw)):
            vplan = hydro.Plan(hydro.params(dt=b.dt, flags=fl), db.struct, db.U, U_out, amax,
                               status)
            vwall, vper = timed_plan(vplan, max(5, args.steps // 2), args.warmup, torch)
            vplan.close()
            vms = float(np.mean(vper))
            variants[name] = {"flags": fl, "kernel_ms": vms,
                              "cell_updates_per_s": b.cell_updates / (vms * 1e-3),
                              "relative_to_default": kern_ms / vms,
                              "nonzero_status": int(status.any().item())}
            log(f"variant {name}: kernel {vms:.3f} ms ({kern_ms / vms:.3f} of the default rate)")
    traffic, why = traffic_per_launch()
    if traffic is None:
        log(f"traffic: null ({why})")
    else:
        log(f"traffic: {traffic['bytes'] / 1e9:.3f} GB per launch "
            f"({traffic['bytes'] / nbytes:.3f} x algorithmic)")

    result = {
        "metric": "FP64 hydro cell-updates/s, batched vs per-subgrid launch; p50/p99 step latency",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "128^3 binary-star mesh: 4096 subgrids of 8^3 (+3 ghosts), "
                               "11 fields, one fused persistent launch in a hipGraph",
                   "subgrids": b.n_sub, "cells_per_step": b.cell_updates,
                   "variant": hydro.variant_name(best)},
        "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99))},
        "roofline": {"bound": "alu", "achieved": achieved_tf, "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved_tf / FP64_PEAK_TFLOPS,
                     "traffic": None if traffic is None else traffic["bytes"],
                     "kernel": "k_fused<false, false, false, false>", "flops_per_launch": flops,
                     "kernel_ms": kern_ms},
        "hbm": {"achieved": achieved_gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved_gbps / HBM_PEAK_GBPS, "bytes_per_launch": nbytes,
                "traffic_bytes_per_launch": None if traffic is None else traffic["bytes"],
                "traffic_over_algorithmic": None if traffic is None else traffic["bytes"] / nbytes},
    }
    if variants is not None:
        result["variants"] = variants
    if not args.no_six_field:
        result["six_field"] = six_field_run(torch, hydro, inputs, costmodel, b, kern_ms,
                                            max(20, args.steps // 4), args.warmup)
    if not args.no_plain:
        # the same comparison on the 128^3 batch (4096 subgrids), one timed pass
        result["per_subgrid_vs_batched_config3"] = per_subgrid_vs_batched(torch, hydro, b, db,
                                                                          "config3", 1)
    del U_out
    torch.cuda.empty_cache()
    if not args.no_config4:
        result["config4"] = config4_run(torch, hydro, inputs, costmodel, args.config4_launches)
        result["config1_latency"] = single_subgrid_latency(torch, hydro, inputs)
    if not args.no_serving:
        result["serving"] = serving_run(torch, hydro, serving, b, db, b.n_sub / (kern_ms * 1e-3),
                                        args.serving_requests, args.serving_budget_gb)
    if not args.no_rk3:
        # config 3's mesh with outflow boundaries (evolves db.U in place)
        result["rk3_binary_star"] = rk3_timing(torch, hydro, db, (16, 16, 16),
                                               (False, False, False), args.rk3_steps)
        log(f"rk3 128^3 binary star: {result['rk3_binary_star']['ms_per_time_step']:.3f} ms "
            f"per time step")
        sb = inputs.sedov(64)
        sdb = hydro.DeviceBatch.from_inputs(sb)
        result["rk3_sedov"] = rk3_timing(torch, hydro, sdb, (8, 8, 8), (True, True, True),
                                         args.rk3_steps)
        result["rk3_sedov"]["workload"] = "64^3 Sedov blast, 512 subgrids, 6 fields, periodic"
        log(f"rk3 64^3 sedov: {result['rk3_sedov']['ms_per_time_step']:.3f} ms per time step")
        del sdb
    del db
    torch.cuda.empty_cache()
    if not args.no_plain:
        result["plain_vs_batched"] = plain_vs_batched(torch, hydro, inputs)
        result["subgrid16_plain"] = subgrid16_plain(torch, hydro, inputs)
    if cpu is not None:
        result["cpu_baseline"] = cpu
        result["cpu_baseline"]["gpu_over_cpu"] = value / cpu["value"]
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
