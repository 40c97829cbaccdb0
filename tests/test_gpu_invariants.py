"""The oracle's invariants, run directly on the GPU: linear data reconstructed
exactly, mirror symmetry (also with the Colella-Woodward options) and
axis-permutation symmetry of the step, in the plain form (which evaluates in
the oracle's order: bitwise) and in the fused form (which sums in another
order: to rounding)."""
import numpy as np
import pytest

from gpu_util import gpu_plain, gpu_step
from metrics import field_scales, mixed_rel
from paper_2210_06439_amd import hydro, inputs
from test_oracle_invariants import DIRS, NB, mirror, slot

pytestmark = pytest.mark.gpu


def one(block, h=0.125, dt=0.0):
    return inputs.pack_blocks([block], [h], dt=dt)


def test_linear_data_reconstructed_exactly_plain():
    """U_f = a_f + beta_f . (i, j, k) with dyadic coefficients: Q_f(c, d) =
    U_f(c) + (beta_f . d)/2 bitwise, at every one of the 26 points."""
    rng = np.random.default_rng(0)
    nf = 11
    a = rng.integers(-8, 9, nf) / 4.0
    beta = rng.integers(-8, 9, (nf, 3)) / 8.0
    k, j, i = np.meshgrid(np.arange(NB), np.arange(NB), np.arange(NB), indexing="ij")
    blk = np.stack([a[f] + beta[f, 0] * i + beta[f, 1] * j + beta[f, 2] * k for f in range(nf)])
    # a positive density and energy so the point states are physical
    blk[0] = 4.0 + np.abs(blk[0])
    blk[4] = 40.0 + np.abs(blk[4])
    b = one(blk)
    Q = gpu_plain(b, dt=0.0)[0].reshape(nf, 26, 10, 10, 10)
    for d in DIRS:
        for f in range(nf):
            if f in (0, 4):
                continue
            expect = blk[f, 2:12, 2:12, 2:12] + 0.5 * (beta[f] @ np.array(d, float))
            assert np.array_equal(Q[f, slot(*d)], expect), (d, f)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("flags", [0, hydro.VELOCITY, hydro.STEEPEN | hydro.FLATTEN])
def test_mirror_symmetry(axis, flags):
    b = inputs.config1(seed=21)
    blk = np.array(b.block(0))
    bm = one(mirror(blk, axis), dt=b.dt)
    S = field_scales(blk)
    # fused: to rounding
    Uo, ao, _ = gpu_step(b, flags=flags)
    Um, am, _ = gpu_step(bm, flags=flags)
    out = np.array(b.block(0, Uo))[:, 3:11, 3:11, 3:11]
    out_m = mirror(np.array(bm.block(0, Um)), axis)[:, 3:11, 3:11, 3:11]
    assert float(mixed_rel(out, out_m, S).max()) <= 1e-13
    assert abs(ao[0] - am[0]) <= 1e-15 * ao[0]
    # plain: bitwise
    _, _, Up, ap, _ = gpu_plain(b, flags=flags)
    _, _, Upm, apm, _ = gpu_plain(bm, flags=flags)
    assert np.array_equal(np.array(b.block(0, Up)), mirror(np.array(bm.block(0, Upm)), axis))
    assert ap[0] == apm[0]


@pytest.mark.parametrize("perm", [(1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0)])
def test_axis_permutation(perm):
    b = inputs.config1(seed=22)
    blk = np.array(b.block(0))

    def permute(x):
        sp = x.transpose([0] + [3 - perm[2 - q] for q in range(3)]).copy()
        sp[1:4] = np.array(x[1:4])[list(perm)].transpose([0] + [3 - perm[2 - q] for q in range(3)])
        return sp

    bp = one(permute(blk), dt=b.dt)
    S = field_scales(permute(blk))
    for runner in (gpu_step, lambda bb: gpu_plain(bb)[2:]):
        res, resp = runner(b), runner(bp)
        Uo, ao, Up, ap = res[0], res[1], resp[0], resp[1]
        got = np.array(bp.interior(0, Up))
        ref = permute(np.array(b.block(0, Uo)))[:, 3:11, 3:11, 3:11]
        assert float(mixed_rel(got, ref, S).max()) <= 1e-13
        assert abs(ap[0] - ao[0]) <= 1e-15 * ao[0]
