"""Pins of the oracle's collision (Sec. 2.1, Eqs. (5)-(6)) against textbook
special cases and exact invariants, independent of its own formulas."""
import numpy as np
import pytest

import lbm_inputs
from oracle import Oracle
from tests.textbook import EX, EY, bgk_guo_collide, feq9, geq5


def _random_node(seed):
    r = lbm_inputs.random_state(18, seed)
    rho, ux, uy, T = 1 + 0.1 * (r[0] - 0.5), 0.1 * (r[1] - 0.5), 0.1 * (r[2] - 0.5), r[3]
    f = feq9(rho, ux, uy) * (1 + 0.2 * (r[4:13] - 0.5))
    g = geq5(T, ux, uy) + 0.05 * (r[13:18] - 0.5)
    return f, g


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_mrt_with_equal_rates_is_bgk_with_guo_forcing(seed):
    """All D2Q9 rates equal to s turns the MRT operator into BGK with Guo's
    forcing; all D2Q5 rates equal to s_a turns it into BGK.  This pins M, M^-1,
    m^eq, the forcing moments and the half-force velocity together."""
    nu, alpha = 0.07, 0.03
    s = 1.0 / (3 * nu + 0.5)
    sa = 1.0 / (5 * alpha + 0.5)
    g_grav, beta, Tref, body = 2e-3, 0.3, 0.25, 1.5e-4
    o = Oracle(nx=8, ny=8, nu=nu, alpha=alpha, s_e=s, s_eps=s, s_q=s, sT_e=sa, sT_p=sa,
               gravity=g_grav, beta=beta, T_ref=Tref, body_fx=body)
    f, g = _random_node(seed)
    fo, go, m = o.collide_node(f, g)
    T = g.sum()
    rho = f.sum()
    Fx, Fy = body, rho * g_grav * beta * (T - Tref)
    ref, (rr, ux, uy) = bgk_guo_collide(f, s, Fx, Fy)
    np.testing.assert_allclose(fo, ref, rtol=0, atol=2e-15)
    np.testing.assert_allclose(go, g - sa * (g - geq5(T, ux, uy)), rtol=0, atol=2e-15)
    np.testing.assert_allclose(m, [rr, ux, uy, T], rtol=0, atol=1e-15)


@pytest.mark.parametrize("seed", [4, 5])
def test_collision_invariants_default_rates(seed):
    """rho and T are collision invariants; the momentum gains exactly F."""
    o = Oracle(nx=8, ny=8, nu=0.02, alpha=0.01, gravity=1e-3, beta=0.5, body_fx=3e-5)
    f, g = _random_node(seed)
    fo, go, m = o.collide_node(f, g)
    rho, T = f.sum(), g.sum()
    Fx, Fy = 3e-5, rho * 1e-3 * 0.5 * T
    assert abs(fo.sum() - rho) < 4e-16
    assert abs(go.sum() - T) < 4e-16
    assert abs((EX * fo).sum() - (EX * f).sum() - Fx) < 1e-16
    assert abs((EY * fo).sum() - (EY * f).sum() - Fy) < 1e-16


def test_equilibrium_is_a_fixed_point_without_force():
    o = Oracle(nx=8, ny=8, nu=0.013, alpha=0.2, s_e=1.1, s_eps=1.3, s_q=1.7, sT_e=0.9, sT_p=1.6)
    f = feq9(1.03, 0.04, -0.07)
    g = geq5(0.6, 0.04, -0.07)
    fo, go, _ = o.collide_node(f, g)
    np.testing.assert_allclose(fo, f, rtol=4 * 2.2e-16, atol=0)
    np.testing.assert_allclose(go, g, rtol=4 * 2.2e-16, atol=0)


def test_default_rates_follow_the_transport_coefficients():
    """s_nu from nu = (1/s - 1/2)/3, s_a from alpha = (4 + a)/10 (1/s - 1/2),
    and the default free rates of the stated magic combinations."""
    nu, alpha = 0.0391046, 0.0558638
    o = Oracle(nx=8, ny=8, nu=nu, alpha=alpha)
    s9, s5, w5 = o.rates()
    snu = s9[7]
    assert abs((1 / snu - 0.5) / 3 - nu) < 1e-15
    assert s9[8] == snu and s9[1] == snu and s9[2] == snu
    assert abs((1 / snu - 0.5) * (1 / s9[4] - 0.5) - 3 / 16) < 1e-15
    assert s9[4] == s9[6]
    assert abs((1 / s5[1] - 0.5) * 0.2 - alpha) < 1e-15
    assert abs((1 / s5[1] - 0.5) * (1 / s5[3] - 0.5) - 0.25) < 1e-15
    np.testing.assert_allclose(w5, [0.6, 0.1, 0.1, 0.1, 0.1], rtol=0, atol=1e-16)
