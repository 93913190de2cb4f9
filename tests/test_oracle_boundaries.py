"""Pins of the oracle's interface schemes (Sec. 2.3, Eqs. (9)-(12)) by
interpolation identities and exact special cases."""
import math

import numpy as np
import pytest

import oracle
from tests.textbook import EX, EY, OPP, W9, feq9

QS_LOW = [0.0, 0.05, 0.2, 0.37, 0.5]
QS_HIGH = [0.5000001, 0.6, 0.75, 0.93, 1.0]


def _phi(s, a=0.41, b=-0.07, c=0.013):
    return a + b * s + c * s * s


@pytest.mark.parametrize("q", QS_LOW)
@pytest.mark.parametrize("i", [1, 2, 5, 8])
def test_bouzidi_low_q_is_quadratic_interpolation(q, i):
    """q <= 1/2: the population leaving x_f towards the wall comes back to x_f
    from the point x_f - (1 - 2q) e_i; Eq. (9) is the Lagrange interpolant of
    f_i^+ through x_f, x_f - e_i, x_f - 2 e_i evaluated there."""
    got = oracle.bouzidi(q, i, _phi(0), _phi(-1), _phi(-2), 9.9, 9.9, 1, 1, 1.0, 0.0, 0.0)
    assert abs(got - _phi(-(1 - 2 * q))) < 1e-15
    lin = oracle.bouzidi(q, i, _phi(0, c=0), _phi(-1, c=0), 7.7, 9.9, 9.9, 1, 0, 1.0, 0.0, 0.0)
    assert abs(lin - _phi(-(1 - 2 * q), c=0)) < 1e-15


@pytest.mark.parametrize("q", QS_HIGH)
@pytest.mark.parametrize("i", [3, 4, 6, 7])
def test_bouzidi_high_q_is_quadratic_interpolation(q, i):
    """q > 1/2: f_i^+(x_f), reflected, sits at x_f + (2q - 1) e_i at t + dt;
    f_ibar^+(x_f) and f_ibar^+(x_f - e_i) sit at x_f - e_i and x_f - 2 e_i.
    Eq. (10) is their Lagrange interpolant at x_f."""
    got = oracle.bouzidi(q, i, _phi(2 * q - 1), 7.7, 7.7, _phi(-1), _phi(-2), 1, 1, 1.0, 0.0, 0.0)
    assert abs(got - _phi(0)) < 1e-14
    lin = oracle.bouzidi(q, i, _phi(2 * q - 1, c=0), 7.7, 7.7, _phi(-1, c=0), 6.6, 0, 0, 1.0, 0, 0)
    assert abs(lin - _phi(0, c=0)) < 1e-14


@pytest.mark.parametrize("i", range(1, 9))
def test_bouzidi_half_q_is_halfway_bounce_back(i):
    for have1, have2 in [(1, 1), (1, 0), (0, 0)]:
        lo = oracle.bouzidi(0.5, i, 0.3, 0.7, 1.1, 0.2, 0.9, have1, have2, 1.0, 0.0, 0.0)
        hi = oracle.bouzidi(0.5 + 1e-12, i, 0.3, 0.7, 1.1, 0.2, 0.9, have1, have2, 1.0, 0.0, 0.0)
        assert abs(lo - 0.3) < 1e-15
        assert abs(hi - 0.3) < 1e-11


@pytest.mark.parametrize("q", QS_LOW + QS_HIGH)
@pytest.mark.parametrize("i", range(1, 9))
def test_bouzidi_moving_wall_keeps_uniform_equilibrium(q, i):
    """A wall moving with the fluid's uniform velocity U returns exactly the
    equilibrium population f_ibar^eq(U): pins the wall term and its sign."""
    U = (0.031, -0.017)
    fe = feq9(1.0, *U)
    ib = OPP[i]
    for have1, have2 in [(1, 1), (1, 0), (0, 0)]:
        got = oracle.bouzidi(q, i, fe[i], fe[i], fe[i], fe[ib], fe[ib], have1, have2, 1.0, *U)
        assert abs(got - fe[ib]) < 2e-16 * 8


def _linear_steady_g(T_w, G, q, tau, w):
    """Steady D2Q5 BGK populations for T(s) = T_w + G (s - q) along e_i (s from
    x_f): g_i = w (T - tau e_i . grad T) before collision."""
    def T(s):
        return T_w + G * (s - q)
    gi_post = lambda s: w * (T(s) - (tau - 1) * G)   # post-collision, direction i
    gib_post = lambda s: w * (T(s) + (tau - 1) * G)  # post-collision, direction ibar
    exact_gib = w * (T(0) + tau * G)                  # after streaming at x_f
    return gi_post(0), gi_post(-1), gib_post(0), exact_gib


@pytest.mark.parametrize("q", [0.05, 0.3, 0.5, 0.71, 1.0])
@pytest.mark.parametrize("tau", [0.55, 1.0, 1.7])
def test_thermal_wall_exact_for_linear_profiles(q, tau):
    """Eqs. (11)-(12) reproduce the steady linear-conduction populations with
    the wall temperature T_w at x_f + q e_i, for any q and relaxation time."""
    w, Tw, G = 0.1, 0.8, -0.03
    gi0, gi1, gib0, exact = _linear_steady_g(Tw, G, q, tau, w)
    got = oracle.thermal_link(q, 1, gi0, gi1, gib0, 1, w, Tw)
    assert abs(got - exact) < 1e-15


@pytest.mark.parametrize("q", [0.01, 0.5, 0.8, 1.0])
def test_thermal_wall_special_cases(q):
    w, Tw = 0.1, 0.65
    assert abs(oracle.thermal_link(q, 2, w * Tw, w * Tw, w * Tw, 1, w, Tw) - w * Tw) < 1e-16
    assert abs(oracle.thermal_link(0.5, 2, 0.3, 0.9, 0.4, 1, w, Tw) - (-0.3 + 2 * w * Tw)) < 1e-16
    assert abs(oracle.thermal_link(q, 2, 0.3, 0.9, 0.4, 0, w, Tw) - (-0.3 + 2 * w * Tw)) < 1e-16


def test_link_fraction_hand_values():
    """Circle of radius 1.5 centred on the origin, seen from fluid nodes."""
    r = 1.5
    assert oracle.link_q(-2.0, 0.0, r, 1) == 0.5
    assert abs(oracle.link_q(-2.0, -1.0, r, 1) - (2 - math.sqrt(1.25))) < 1e-15
    assert abs(oracle.link_q(-2.0, -2.0, r, 5) - (2 - 1.5 / math.sqrt(2))) < 1e-15
    assert abs(oracle.link_q(-2.0, -1.0, r, 5) - (3 - math.sqrt(3.5)) / 2) < 1e-15
    assert abs(oracle.link_q(1.0, 2.0, r, 4) - (2 - math.sqrt(1.25))) < 1e-15
    # a node on the circle is solid: the wall sits at the far end of the link
    assert oracle.link_q(-2.5, 0.0, 1.5, 1) == 1.0
