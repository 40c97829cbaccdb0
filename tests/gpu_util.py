"""Helpers for the GPU tests: run the library's paths on a SubgridBatch."""
from __future__ import annotations

import numpy as np

from paper_2210_06439_amd import hydro


def torch():
    import torch as t
    return t


def device_batch(b):
    return hydro.DeviceBatch.from_inputs(b)


def gpu_step(b, dt=None, variant=None, db=None, flags=0):
    """Fused step; returns (U_out host array, amax, status)."""
    T = torch()
    db = db or device_batch(b)
    dt = b.dt if dt is None else dt
    U_out = db.U.clone()
    amax = T.zeros(db.n_sub, dtype=T.float64, device="cuda")
    status = T.zeros(db.n_sub, dtype=T.int32, device="cuda")
    hydro.step(hydro.params(dt=dt, flags=flags), db.struct, db.U, U_out, amax, status,
               variant=variant)
    T.cuda.synchronize()
    return U_out.cpu().numpy(), amax.cpu().numpy(), status.cpu().numpy()


def gpu_plain(b, dt=None, db=None, flags=0):
    """Unfused reconstruct -> flux -> divergence; returns (Q, F, U_out, amax, status)."""
    T = torch()
    db = db or device_batch(b)
    dt = b.dt if dt is None else dt
    prm = hydro.params(dt=dt, flags=flags)
    qo, qn = db.q_layout()
    fo, fn = db.f_layout()
    Q = T.zeros(qn, dtype=T.float64, device="cuda")
    F = T.zeros(fn, dtype=T.float64, device="cuda")
    amax = T.zeros(db.n_sub, dtype=T.float64, device="cuda")
    status = T.zeros(db.n_sub, dtype=T.int32, device="cuda")
    U_out = db.U.clone()
    hydro.reconstruct(prm, db.struct, db.U, Q, qo)
    hydro.flux(prm, db.struct, Q, qo, F, fo, amax, status)
    hydro.divergence(prm, db.struct, F, fo, db.U, U_out)
    T.cuda.synchronize()
    return (Q.cpu().numpy(), F.cpu().numpy(), U_out.cpu().numpy(), amax.cpu().numpy(),
            status.cpu().numpy())


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))
