"""Status words on the GPU against the oracle's, on a batch where one subgrid
holds a NaN, one a zero-pressure cold flow (p <= 0 at every point), one an
infinite energy, and the rest clean data: in every path (fused step in each
launch shape, the stage-wise plain path, the step with output offsets, the
Runge-Kutta stage form, the step that reads ghosts through a map) each
subgrid's status equals the oracle's, and every clean subgrid's output is
bitwise what it is in a batch of clean subgrids alone.  Also: block cells
that no stencil reads may hold NaN without reaching any output."""
import numpy as np
import pytest

import oracle
from gpu_util import device_batch, gpu_plain, gpu_step, torch
from metrics import max_err_step
from paper_2210_06439_amd import hydro, inputs

pytestmark = pytest.mark.gpu
NB, NG, NI = 14, 3, 8


def _cold_block():
    one = np.ones((NB, NB, NB))
    return np.stack([one, one, 0.5 * one, 0.25 * one, 0.65625 * one, 0 * one])


def _bad_batch():
    """Subgrids: 0 clean, 1 NaN density, 2 clean, 3 cold flow with tau = 0,
    4 +inf energy, 5 clean (6 fields)."""
    clean = inputs.random_batch(3, seed=451, species=(0, 5))
    blocks = [np.array(clean.block(s)) for s in range(3)]
    nan_b = np.array(inputs.config1(seed=452).block(0))
    nan_b[0, 5, 6, 4] = np.nan
    inf_b = np.array(inputs.config1(seed=453).block(0))
    inf_b[4, 7, 4, 6] = np.inf
    order = [blocks[0], nan_b, blocks[1], _cold_block(), inf_b, blocks[2]]
    h = [clean.h[0], 0.125, clean.h[1], 0.125, 0.125, clean.h[2]]
    b = inputs.pack_blocks(order, h, dt=min(clean.dt, 0.01))
    return b, [0, 2, 5]


def _ref(b, U=None):
    U = b.U if U is None else U
    return oracle.step(U, b.offset, b.h, b.n_species, b.fstride, b.dt)


def _clean_alone(b, clean):
    sub = b.subset(clean)
    Ug, ag, sg = gpu_step(sub, dt=b.dt)
    return sub, Ug, ag, sg


def _check(b, clean, Ug, ag, sg, sr, label):
    print(f"{label}: status {list(sg)} oracle {list(sr)}", flush=True)
    assert np.array_equal(sg, sr), label
    sub, Uc, ac, _ = _clean_alone(b, clean)
    for n, s in enumerate(clean):
        assert np.array_equal(b.interior(s, Ug), sub.interior(n, Uc)), (label, s)
        assert ag[s] == ac[n], (label, s)


def test_oracle_status_of_the_bad_batch():
    b, clean = _bad_batch()
    _, _, sr = _ref(b)
    assert list(sr) == [0, 4, 0, 2, 4, 0]


@pytest.mark.parametrize("variant", list(range(4)))
def test_fused_step_status_matches_oracle(variant):
    b, clean = _bad_batch()
    Ug, ag, sg = gpu_step(b, variant=variant)
    Ur, ar, sr = _ref(b)
    _check(b, clean, Ug, ag, sg, sr, f"fused variant {variant}")
    assert max_err_step(b, Ug, Ur, idx=clean, ref_batch=None) <= 1e-12
    # the cold flow stays uniform and finite
    assert np.all(np.isfinite(b.interior(3, Ug)))


def test_plain_path_status_matches_oracle():
    b, clean = _bad_batch()
    Q, qo = oracle.reconstruct(b.U, b.offset, b.h, b.n_species, b.fstride)
    _, _, ar, sr = oracle.flux(Q, qo, b.offset, b.h, b.n_species, b.fstride)
    Qg, Fg, Ug, ag, sg = gpu_plain(b)
    print(f"plain: status {list(sg)} oracle {list(sr)}", flush=True)
    assert np.array_equal(sg, sr)
    Ur, _, _ = _ref(b)
    for s in clean:
        assert np.array_equal(b.interior(s, Ug), b.interior(s, Ur))
        assert ag[s] == ar[s]


def test_step_io_status_matches_oracle():
    T = torch()
    b, clean = _bad_batch()
    db = device_batch(b)
    out = T.zeros_like(db.U)
    out_off = T.as_tensor(b.offset).cuda()
    amax = T.zeros(b.n_sub, dtype=T.float64, device="cuda")
    status = T.full((b.n_sub,), 99, dtype=T.int32, device="cuda")
    hydro.step_io(hydro.params(dt=b.dt), db.struct, out_off, db.U, out, amax, status)
    T.cuda.synchronize()
    Ug = out.cpu().numpy()
    _, _, sr = _ref(b)
    _check(b, clean, Ug, amax.cpu().numpy(), status.cpu().numpy(), sr, "step_io")


def test_rk_stage_status_matches_oracle():
    """The stage form U_out = a U0 + b (U + dt L(U)) with U0 = U: status ORs
    into the incoming words, which start at zero here."""
    T = torch()
    b, clean = _bad_batch()
    db = device_batch(b)
    out = db.U.clone()
    clock = T.tensor([0.0, b.dt], dtype=T.float64, device="cuda")
    amax = T.zeros(b.n_sub, dtype=T.float64, device="cuda")
    status = T.zeros(b.n_sub, dtype=T.int32, device="cuda")
    hydro.rk_stage(hydro.params(), db.struct, db.U, out, db.U, 0.0, 1.0, clock, amax, status)
    T.cuda.synchronize()
    _, _, sr = _ref(b)
    sg = status.cpu().numpy()
    print(f"rk_stage: status {list(sg)} oracle {list(sr)}", flush=True)
    assert np.array_equal(sg, sr)


def _self_map(n):
    """Every subgrid its own periodic neighbour in all 26 directions."""
    src = np.repeat(np.arange(n, dtype=np.int32), 27)
    return src, np.zeros_like(src)


def _self_wrapped(b):
    out = b.U.copy()
    for s in range(b.n_sub):
        blk = b.block(s, out)
        inner = np.array(blk[:, NG:NG + NI, NG:NG + NI, NG:NG + NI])
        blk[...] = np.pad(inner, ((0, 0), (NG, NG), (NG, NG), (NG, NG)), mode="wrap")
    return out


def test_gathered_step_status_matches_oracle():
    """Ghosts read through a map in which each subgrid is its own periodic
    neighbour; the block's own ghost layers hold NaN and are never read."""
    T = torch()
    b, clean = _bad_batch()
    Uw = _self_wrapped(b)
    Ur, ar, sr = _ref(b, Uw)
    spoiled = Uw.copy()
    for s in range(b.n_sub):
        blk = b.block(s, spoiled)
        inner = np.array(blk[:, NG:NG + NI, NG:NG + NI, NG:NG + NI])
        blk[...] = np.nan
        blk[:, NG:NG + NI, NG:NG + NI, NG:NG + NI] = inner
    db = device_batch(b)
    db.U.copy_(T.as_tensor(spoiled))
    gm = hydro.DeviceGhostMap(*_self_map(b.n_sub))
    out = db.U.clone()
    amax = T.zeros(b.n_sub, dtype=T.float64, device="cuda")
    status = T.zeros(b.n_sub, dtype=T.int32, device="cuda")
    hydro.step_gather(hydro.params(dt=b.dt), db.struct, gm, db.U, out, amax, status)
    T.cuda.synchronize()
    sg = status.cpu().numpy()
    Ug = out.cpu().numpy()
    print(f"gather: status {list(sg)} oracle {list(sr)}", flush=True)
    assert np.array_equal(sg, sr)
    assert max_err_step(b, Ug, Ur, idx=clean) <= 1e-12
    for s in clean:
        assert np.all(np.isfinite(b.interior(s, Ug)))


def test_unread_block_cells_never_reach_the_outputs():
    """NaN in every block cell with two or more coordinates in the outermost
    ghost layers (no face's stencils reach them): every output bitwise as
    with the original values, status clear, in every launch shape."""
    b = inputs.random_batch(5, seed=454, species=(0, 5))
    ref = [gpu_step(b, variant=v) for v in range(4)]
    outer = [np.isin(np.arange(NB), (0, NB - 1))] * 3
    kk, jj, ii = np.meshgrid(*outer, indexing="ij")
    unread = (kk.astype(int) + jj + ii) >= 2
    U = b.U.copy()
    for s in range(b.n_sub):
        b.block(s, U)[:, unread] = np.nan
    bn = inputs.SubgridBatch(U=U, offset=b.offset, h=b.h, n_species=b.n_species,
                             fstride=b.fstride, dt=b.dt)
    for v in range(4):
        Ug, ag, sg = gpu_step(bn, variant=v)
        assert np.all(sg == 0)
        assert np.array_equal(ag, ref[v][1])
        for s in range(b.n_sub):
            assert np.array_equal(b.interior(s, Ug), b.interior(s, ref[v][0])), (v, s)
