"""The self-similar point-blast solution used to check the blast-wave runs:
its energy constant matches the textbook values, and it has the known
behaviour at the shock and at the centre."""
import numpy as np

import sedov
from paper_2210_06439_amd import inputs


def test_energy_constant_textbook_values():
    # xi0 = 1.033 for gamma = 1.4 and 1.152 for gamma = 5/3 (3-D point blast)
    assert abs(sedov.xi0(1.4) - 1.033) < 1e-3
    assert abs(sedov.xi0(5.0 / 3.0) - 1.152) < 1e-3


def test_profile_limits():
    g53 = 5.0 / 3.0
    eta, f, g, h, _ = sedov.profile(g53)
    assert abs(g[-1] - 4.0) < 1e-12 and abs(f[-1] - 0.75) < 1e-12
    # near the centre the gas is at rest relative to homologous expansion:
    # u / (R' eta) -> 1/gamma, and the density vanishes
    assert abs(f[0] / eta[0] - 1.0 / g53) < 1e-3
    assert g[0] < 1e-10
    # the pressure stays finite at the centre (about 0.3 of its shock value)
    assert 0.2 < h[0] / h[-1] < 0.5


def test_mass_inside_the_shock_is_the_swept_mass():
    """4 pi R^3 rho0 int g eta^2 = (4/3) pi R^3 rho0."""
    eta, f, g, h, _ = sedov.profile(5.0 / 3.0)
    assert abs(np.trapezoid(g * eta * eta, eta) - 1.0 / 3.0) < 2e-5


def test_sedov_input_energy_and_symmetry():
    b = inputs.sedov(N=32)
    E = inputs.sedov_energy(b)
    amb = 1e-5 / (2.0 / 3.0)
    assert abs(E - (1.0 + amb)) < 1e-12
    blk0 = b.interior(0)            # corner subgrid of the octant below the centre
    far = b.interior(b.n_sub - 1)   # the opposite corner subgrid
    assert np.array_equal(blk0[4], far[4][::-1, ::-1, ::-1])
