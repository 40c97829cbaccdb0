"""The host-side ghost map of a box of subgrids means what the padded global
field means: wrap along periodic axes, zero-gradient copy along the others."""
import numpy as np
import pytest

from mesh_util import apply_map, box_batch
from paper_2210_06439_amd import hydro


@pytest.mark.parametrize("nsub,periodic", [((2, 2, 2), (True, True, True)),
                                           ((3, 2, 1), (False, True, True)),
                                           ((2, 1, 2), (False, False, False))])
def test_box_map_reproduces_padding(nsub, periodic):
    rng = np.random.default_rng(5)
    nx, ny, nz = nsub
    G = rng.normal(size=(6, nz * 8, ny * 8, nx * 8))
    want = box_batch(G, nsub, 0.1, periodic)
    stale = want.U.copy()
    for s in range(want.n_sub):
        blk = want.block(s, stale)
        inner = blk[:, 3:11, 3:11, 3:11].copy()
        blk[...] = np.nan
        blk[:, 3:11, 3:11, 3:11] = inner
    src, mode = hydro.box_ghost_map(*nsub, periodic=periodic)
    got = apply_map(want, stale, src, mode)
    assert np.array_equal(got, want.U)


def test_box_map_entries():
    src, mode = hydro.box_ghost_map(3, 1, 1, periodic=(False, True, True))
    src, mode = src.reshape(3, 27), mode.reshape(3, 27)
    left, right = 9 * 1 + 3 * 1 + 0, 9 * 1 + 3 * 1 + 2
    assert src[0, left] == 0 and mode[0, left] == 1        # outflow at the low end
    assert src[0, right] == 1 and mode[0, right] == 0
    assert src[2, right] == 2 and mode[2, right] == 1      # outflow at the high end
    up = 9 * 1 + 3 * 2 + 1
    assert src[1, up] == 1 and mode[1, up] == 0            # y wraps onto itself
