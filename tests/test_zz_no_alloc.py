"""hydro_step_noalloc (the step for callers that cannot allocate) against
hydro_step, through the C ABI: bit for bit on two calls in a row, the second
with a smaller batch, in launch shapes that use the fixed scratch and in
ones that do not; no library workspace is allocated on a stream that only
runs it; batches beyond its scratch are refused."""
import ctypes

import numpy as np
import pytest

from gpu_util import device_batch, torch
from paper_2210_06439_amd import hydro, inputs

pytestmark = pytest.mark.gpu


def _run(fn, b, stream=None):
    T = torch()
    db = device_batch(b)
    out = db.U.clone()
    amax = T.zeros(db.n_sub, dtype=T.float64, device="cuda")
    status = T.full((db.n_sub,), 7, dtype=T.int32, device="cuda")
    fn(hydro.params(dt=b.dt), db.struct, db.U, out, amax, status, stream=stream)
    T.cuda.synchronize()
    return out.cpu().numpy(), amax.cpu().numpy(), status.cpu().numpy()


def _same(x, y):
    return all(np.array_equal(p, q) for p, q in zip(x, y))


@pytest.mark.parametrize("sizes", [(20, 7), (300, 100), (64, 3)])
def test_noalloc_equals_step_on_two_calls(sizes):
    T = torch()
    c3 = inputs.config3(N=64)                         # 512 subgrids of the binary star
    rng = np.random.default_rng(sum(sizes))
    batches = [c3.subset(np.sort(rng.choice(c3.n_sub, n, replace=False))) for n in sizes]
    want = [_run(hydro.step, b) for b in batches]     # the reference (default stream)
    stream = T.cuda.Stream()                           # a stream no eager call has used
    before = int(hydro.lib().hydro_workspace_bytes())
    for b, ref in zip(batches, want):
        shape = hydro.variant_name(hydro.selected_variant(b.n_sub))
        with T.cuda.stream(stream):
            got = _run(hydro.step_noalloc, b, stream=stream)
        print(f"n={b.n_sub} shape {shape}: bitwise {_same(got, ref)}", flush=True)
        assert _same(got, ref), (b.n_sub, shape)
        assert np.all(got[2] == 0)
    # the library allocated no workspace for the calls on the new stream
    assert int(hydro.lib().hydro_workspace_bytes()) == before


def test_noalloc_refuses_batches_beyond_its_scratch():
    T = torch()
    n = hydro.NOALLOC_MAX_SUB + 1
    off = T.zeros(1, dtype=T.int64, device="cuda")
    h = T.ones(1, dtype=T.float64, device="cuda")
    ns = T.zeros(1, dtype=T.int32, device="cuda")
    U = T.zeros(16, dtype=T.float64, device="cuda")
    batch = hydro.Batch(n, inputs.FSTRIDE, off.data_ptr(), h.data_ptr(), ns.data_ptr())
    rc = hydro.lib().hydro_step_noalloc(ctypes.byref(hydro.params(dt=0.0)), ctypes.byref(batch),
                                        ctypes.c_void_p(U.data_ptr()),
                                        ctypes.c_void_p(U.data_ptr() + 64), ctypes.c_void_p(h.data_ptr()),
                                        None, None)
    assert rc == hydro.ESCRATCH
    assert b"scratch" in hydro.lib().hydro_strerror(rc)
