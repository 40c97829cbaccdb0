"""Pins for the oracle's point state (ideal gas with dual-energy switch) and
its central-upwind face flux with tensor Simpson quadrature (Sec. II: the
`flux` kernel integrates the flux with Newton-Cotes quadrature)."""
import math

import numpy as np
import pytest

import oracle

G = 5.0 / 3.0


def ulp_close(a, b, n=4):
    a, b = np.asarray(a, float), np.asarray(b, float)
    tol = n * np.spacing(np.maximum(np.abs(a), np.abs(b)))
    assert np.all(np.abs(a - b) <= tol), (a, b)


def test_gas_at_rest():
    # rho = 1, s = 0, E = 3/2: p = (gamma-1) E = 1, c = sqrt(5/3); flux along
    # x carries only the pressure in the x-momentum slot.
    V = [1.0, 0.0, 0.0, 0.0, 1.5, 1.0]
    F, un, cs, p, st = oracle.state_flux(V, 0)
    assert p == 1.0 and un == 0.0 and st == 0
    assert cs == math.sqrt(5.0 / 3.0)
    assert list(F) == [0.0, 1.0, 0.0, 0.0, 0.0, 0.0]


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_moving_gas_closed_form(axis):
    # rho = 2, s_axis = 2 (v = 1), E = 4: e_k = 1, e_i = 3, p = 2,
    # c = sqrt(gamma p / rho) = sqrt(5/3).  Fluxes: F_rho = 2,
    # F_s_axis = s v + p = 4, F_E = (E + p) v = 6, F_tau = tau v.
    V = np.array([2.0, 0.0, 0.0, 0.0, 4.0, 0.75, 0.5, 1.5])
    V[1 + axis] = 2.0
    F, un, cs, p, st = oracle.state_flux(V, axis)
    assert (un, p, st) == (1.0, 2.0, 0)
    ulp_close(cs, math.sqrt(5.0 / 3.0), 2)
    expect = np.zeros(8)
    expect[0] = 2.0
    expect[1 + axis] = 4.0
    expect[4] = 6.0
    expect[5] = 0.75
    expect[6], expect[7] = 0.5, 1.5
    assert np.array_equal(F, expect)


def test_moving_gas_other_axis_momentum():
    # Flux along y of a gas moving along x: F_sx = s_x v_y = 0, pressure in sy.
    V = [2.0, 2.0, 0.0, 0.0, 4.0, 0.75]
    F, un, cs, p, st = oracle.state_flux(V, 1)
    assert un == 0.0 and p == 2.0
    assert list(F) == [0.0, 0.0, 2.0, 0.0, 0.0, 0.0]


def test_dual_energy_switch_fires():
    # Cold fast gas: rho = 1, v = 10, E = 50 + 1e-4, so e_i = 1e-4 < 1e-3 E and
    # the pressure comes from the entropy tracer: p = (gamma-1) tau^gamma.
    tau = 2.0
    V = [1.0, 10.0, 0.0, 0.0, 50.0 + 1e-4, tau]
    F, un, cs, p, st = oracle.state_flux(V, 0)
    ulp_close(p, (2.0 / 3.0) * tau ** G, 2)
    assert st == 0
    # ... and does not fire when e_i is large enough.
    V2 = [1.0, 10.0, 0.0, 0.0, 50.0 + 1.0, tau]
    _, _, _, p2, _ = oracle.state_flux(V2, 0)
    ulp_close(p2, (2.0 / 3.0) * 1.0, 8)


def test_status_bits():
    assert oracle.state_flux([-1.0, 0, 0, 0, 1.0, 1.0], 0)[4] & 1
    # p = 0 exactly (E = 0 at rest, switch does not fire since 0 < 0 is false)
    assert oracle.state_flux([1.0, 0, 0, 0, 0.0, 1.0], 0)[4] & 2
    assert oracle.state_flux([1.0, 0, 0, 0, 1.5, 1.0], 0)[4] == 0


def _states(rng, nf=11, n=9):
    rho = rng.uniform(0.5, 2.0, n)
    s = rng.normal(0, 0.3, (3, n))
    p = rng.uniform(0.5, 2.0, n)
    E = p / (G - 1) + 0.5 * (s ** 2).sum(0) / rho
    tau = (p / (G - 1)) ** (1 / G)
    spc = [rho * w for w in rng.uniform(0, 0.2, (nf - 6, n))]
    return np.stack([rho, *s, E, tau, *spc]).T.copy()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_equal_sides_give_physical_flux(axis):
    """V_L = V_R = V at every point: the dissipation term vanishes and the
    central-upwind flux is F(V) for any a+, a- (uniform V over the face)."""
    rng = np.random.default_rng(axis)
    V = _states(rng, n=1)[0]
    VL = np.tile(V, (9, 1))
    Fbar, a, st = oracle.face(VL, VL.copy(), axis)
    F, un, cs, p, _ = oracle.state_flux(V, axis)
    ulp_close(Fbar, F, 8)
    assert a == max(un + cs, -(un - cs))
    assert st == 0


def test_supersonic_gives_upwind_flux():
    """All waves move right (u - c > 0 on both sides): a- = 0, so the flux is
    F(V_L) point by point, averaged with Simpson weights."""
    rng = np.random.default_rng(7)
    VL = _states(rng)
    VR = _states(rng)
    for V in (VL, VR):
        V[:, 1] = V[:, 0] * 5.0           # v_x = 5 > c (c < 2.3 here)
        V[:, 4] = (V[:, 4] - 0.0) + 0.5 * 25.0 * V[:, 0]
    Fbar, a, _ = oracle.face(VL, VR, 0)
    Fs = np.array([oracle.state_flux(v, 0)[0] for v in VL])
    w = np.outer([1, 4, 1], [1, 4, 1]).reshape(-1) / 36.0
    expect = (w[:, None] * Fs).sum(0)
    np.testing.assert_allclose(Fbar, expect, rtol=1e-14, atol=1e-14)


def test_simpson_exact_for_bicubic():
    """With the same state on both sides and a constant hydro state, the
    species flux is spc(t) * u_n; the 9-point tensor Simpson average of a
    bicubic spc(t_b, t_b2) over [-1,1]^2 is its exact mean."""
    rng = np.random.default_rng(3)
    base = _states(rng, n=1)[0]
    c = rng.integers(-4, 5, size=(4, 4)) / 8.0
    c[0, 0] = 4.0
    V = np.tile(base, (9, 1))
    for t2 in (-1, 0, 1):
        for t1 in (-1, 0, 1):
            val = sum(c[i, j] * t1 ** i * t2 ** j for i in range(4) for j in range(4))
            V[(t2 + 1) * 3 + (t1 + 1), 6] = val
    Fbar, _, _ = oracle.face(V, V.copy(), 2)
    un = oracle.state_flux(base, 2)[1]
    mom = [1.0, 0.0, 1.0 / 3.0, 0.0]          # mean of t^i over [-1, 1]
    exact = sum(c[i, j] * mom[i] * mom[j] for i in range(4) for j in range(4))
    assert abs(Fbar[6] - exact * un) <= 1e-14 * max(1.0, abs(exact * un))


def test_face_speed_uses_both_sides_and_all_points():
    """a+ is the max of u+c over all 18 point-sides, a- the min of u-c."""
    rng = np.random.default_rng(11)
    VL, VR = _states(rng), _states(rng)
    _, a, _ = oracle.face(VL, VR, 1)
    speeds = []
    for V in np.concatenate([VL, VR]):
        _, un, cs, _, _ = oracle.state_flux(V, 1)
        speeds += [un + cs, -(un - cs)]
    assert a == max(speeds)


def test_face_mirror_negates_odd_fields():
    """Swap the sides and reflect the normal momentum: the flux of every field
    except the normal momentum changes sign, the normal momentum's does not."""
    rng = np.random.default_rng(5)
    VL, VR = _states(rng), _states(rng)
    F1, a1, _ = oracle.face(VL, VR, 0)
    ML, MR = VR.copy(), VL.copy()
    ML[:, 1] *= -1
    MR[:, 1] *= -1
    F2, a2, _ = oracle.face(ML, MR, 0)
    sign = -np.ones(11)
    sign[1] = 1.0
    assert np.array_equal(F2, sign * F1) and a1 == a2
