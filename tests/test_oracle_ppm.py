"""Pins for the oracle's one-dimensional PPM (Colella-Woodward 1984 with
monotonised-central slopes), the reconstruction named in Sec. II.

Each hand-computed case below exercises one branch; the expected values were
worked out by hand in exact rational arithmetic (derivations in comments).
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

import oracle


def close(x, fr, rel=4e-16):
    v = float(fr)
    assert abs(x - v) <= rel * max(abs(v), 1.0), (x, v)


def test_uniform_is_exact():
    assert oracle.ppm1d([3.25] * 5) == (3.25, 3.25)


def test_linear_is_exact():
    # u_m = 2 + m: every slope is 1, interfaces are u0 +- 1/2, nothing limited.
    assert oracle.ppm1d([0.0, 1.0, 2.0, 3.0, 4.0]) == (2.5, 1.5)
    assert oracle.ppm1d([4.0, 3.0, 2.0, 1.0, 0.0]) == (1.5, 2.5)


def test_extremum_is_flattened():
    # u = 0,1,2,1,0: slopes 1, 0 (Delta+ Delta- < 0), -1; q+ = q- = 3/2 + 1/6
    # = 5/3, so (q+ - u0)(u0 - q-) = (-1/3)(1/3) < 0 -> both set to u0 = 2.
    assert oracle.ppm1d([0.0, 1.0, 2.0, 1.0, 0.0]) == (2.0, 2.0)


def test_smooth_unchanged():
    # u = 0,1,3,6,10: slopes 3/2, 5/2, 7/2 (none limited);
    # q+ = 9/2 - 1/6 = 13/3, q- = 2 - 1/6 = 11/6; a = q+ - u0 = 4/3,
    # b = u0 - q- = 7/6: neither b > 2a nor a > 2b -> unchanged.
    qp, qm = oracle.ppm1d([0.0, 1.0, 3.0, 6.0, 10.0])
    close(qp, Fr(13, 3))
    close(qm, Fr(11, 6))


def test_overshoot_minus_side():
    # u = 0,1,4,5,6: slopes 2 (limited by 2|Delta-| = 2), 2 (limited), 1;
    # q+ = 9/2 + 1/6 = 14/3, q- = 5/2; dq = 13/6, m6 = 5/2,
    # dq m6 = 65/12 > dq^2 = 169/36 -> q- = 3 u0 - 2 q+ = 8/3.
    qp, qm = oracle.ppm1d([0.0, 1.0, 4.0, 5.0, 6.0])
    close(qp, Fr(14, 3))
    close(qm, Fr(8, 3))


def test_overshoot_plus_side():
    # u = 0,1,2,5,6: slopes 1, 2 (limited), 2 (limited);
    # q+ = 7/2, q- = 3/2 - 1/6 = 4/3; dq = 13/6, m6 = -5/2,
    # -dq^2 = -169/36 > dq m6 = -65/12 -> q+ = 3 u0 - 2 q- = 10/3.
    qp, qm = oracle.ppm1d([0.0, 1.0, 2.0, 5.0, 6.0])
    close(qp, Fr(10, 3))
    close(qm, Fr(4, 3))


def test_slope_limiter_active():
    # u = 0,0,1,10,10: slopes 0, min(5, 2*1) = 2, 0;
    # q+ = 11/2 + 1/3 = 35/6, q- = 1/2 - 1/3 = 1/6;
    # a = 29/6 > 2b = 10/6 -> q+ = 3 - 2/6 = 8/3.
    qp, qm = oracle.ppm1d([0.0, 0.0, 1.0, 10.0, 10.0])
    close(qp, Fr(8, 3))
    close(qm, Fr(1, 6))


def test_step_profile_flat_branch():
    # u = 0,0,0,1,1: every slope is 0 (a zero one-sided difference each);
    # q+ = 1/2, q- = 0 -> (q+ - u0)(u0 - q-) = 0 -> flattened to u0 = 0.
    assert oracle.ppm1d([0.0, 0.0, 0.0, 1.0, 1.0]) == (0.0, 0.0)


@pytest.mark.parametrize("seed", range(5))
def test_reversal_swaps_faces_bitwise(seed):
    rng = np.random.default_rng(seed)
    for _ in range(2000):
        u = rng.normal(size=5) * 10.0 ** rng.integers(-3, 4)
        qp, qm = oracle.ppm1d(u)
        rp, rm = oracle.ppm1d(u[::-1].copy())
        assert (rp, rm) == (qm, qp)


def _clamp_rule(u):
    """Exact rational PPM written in the equivalent clamp form of the CW84
    monotonicity step: with a = q+ - u0, b = u0 - q-, flatten if a b <= 0,
    else limit |b| to 2|a| and |a| to 2|b| (signs kept)."""
    u = [Fr(x) for x in u]

    def slope(l, c, r):
        dm, dp = c - l, r - c
        if dm * dp <= 0:
            return Fr(0)
        d = (dm + dp) / 2
        m = min(abs(d), 2 * abs(dm), 2 * abs(dp))
        return m if d > 0 else -m

    s = [slope(u[0], u[1], u[2]), slope(u[1], u[2], u[3]), slope(u[2], u[3], u[4])]
    qp = (u[2] + u[3]) / 2 - (s[2] - s[1]) / 6
    qm = (u[1] + u[2]) / 2 - (s[1] - s[0]) / 6
    a, b = qp - u[2], u[2] - qm
    if a * b <= 0:
        return u[2], u[2]
    sg = 1 if a > 0 else -1
    A, B = abs(a), abs(b)
    a2 = sg * min(A, 2 * B)
    b2 = sg * min(B, 2 * A)
    return u[2] + a2, u[2] - b2


@pytest.mark.parametrize("seed", range(3))
def test_matches_clamp_characterisation(seed):
    """The oracle's (dq, m6) branch tests agree with the clamp form on small
    dyadic inputs, where the oracle's own arithmetic is exact."""
    rng = np.random.default_rng(100 + seed)
    for _ in range(3000):
        u = rng.integers(-16, 17, size=5) / 4.0
        qp, qm = oracle.ppm1d(u)
        ep, em = _clamp_rule(u)
        assert abs(qp - float(ep)) <= 1e-14 * max(1.0, abs(float(ep)))
        assert abs(qm - float(em)) <= 1e-14 * max(1.0, abs(float(em)))


@pytest.mark.parametrize("seed", range(3))
def test_no_new_extrema(seed):
    """After limiting, the parabola has no interior extremum and the face
    values lie between the neighbouring cell values (monotonicity)."""
    rng = np.random.default_rng(200 + seed)
    for _ in range(3000):
        u = rng.normal(size=5)
        qp, qm = oracle.ppm1d(u)
        u0 = u[2]
        if qp == u0 and qm == u0:
            continue
        dq = qp - qm
        m6 = 6.0 * (u0 - 0.5 * (qp + qm))
        assert abs(m6) <= abs(dq) * (1 + 1e-12) + 1e-15
        lo, hi = min(u[2], u[3]), max(u[2], u[3])
        assert lo - 1e-14 <= qp <= hi + 1e-14
        lo, hi = min(u[1], u[2]), max(u[1], u[2])
        assert lo - 1e-14 <= qm <= hi + 1e-14
