"""Closed-form flows that pin the oracle's lattice update, walls and buoyancy.

Poiseuille and Couette channels, steady conduction between isothermal walls,
Taylor-Green and thermal-wave decay, Rayleigh-Benard onset, and conservation.
"""
import numpy as np
import pytest

import lbm_inputs
from oracle import Oracle


@pytest.mark.parametrize("nu", [0.02, 1 / 6, 0.3])
def test_poiseuille_exact(nu):
    """Body-force driven channel with halfway walls: u(y) = F (y+1/2)(H-1/2-y)/(2 rho0 nu).
    With the default free rates (magic combination 3/16) the discrete steady
    state is the parabola itself."""
    ny, F = 12, 1e-5
    o = Oracle(nx=8, ny=ny, nu=nu, alpha=0.1, body_fx=F)
    o.step(int(40 * ny * ny / nu / 9.87))
    f = o.fields()
    y = np.arange(ny)
    exact = F * (y + 0.5) * (ny - 0.5 - y) / (2 * nu)
    err = np.abs(f["ux"] - exact[:, None]).max() / exact.max()
    assert err < 1e-11, err
    assert np.abs(f["uy"]).max() < 1e-15


def test_couette_exact():
    """Top wall moving at U: u(y) = U (y + 1/2) / H."""
    ny, U = 12, 0.01
    o = Oracle(nx=8, ny=ny, nu=1 / 6, alpha=0.1, wall_ux=(0.0, U))
    o.step(3000)
    f = o.fields()
    y = np.arange(ny)
    exact = U * (y + 0.5) / ny
    assert np.abs(f["ux"] - exact[:, None]).max() / U < 1e-12


@pytest.mark.parametrize("rates", [(0.0, 0.0), (1.3, 0.7), (0.4, 1.9)])
def test_linear_conduction_exact(rates):
    """Hot bottom wall T=1, cold top T=0: T(y) = 1 - (y+1/2)/H for any rates."""
    ny = 16
    o = Oracle(nx=8, ny=ny, nu=0.1, alpha=0.15, wall_T=(1.0, 0.0), sT_e=rates[0], sT_p=rates[1])
    o.step(6000)
    f = o.fields()
    y = np.arange(ny)
    assert np.abs(f["T"] - (1 - (y + 0.5) / ny)[:, None]).max() < 1e-12


def _taylor_green_rate_error(N, nu=0.02, U0=0.01, s_e=0.0, s_q=0.0):
    k = 2 * np.pi / N
    x = np.arange(N)[None, :] + 0.0
    y = np.arange(N)[:, None] + 0.0
    ux = -U0 * np.cos(k * x) * np.sin(k * y)
    uy = U0 * np.sin(k * x) * np.cos(k * y)
    rho = 1 - 0.75 * U0 ** 2 * (np.cos(2 * k * x) + np.cos(2 * k * y))
    o = Oracle(nx=N, ny=N, periodic_y=1, nu=nu, alpha=0.1, s_e=s_e, s_eps=s_e, s_q=s_q)
    o.set_equilibrium(rho, ux, uy, np.zeros((N, N)))
    steps = int(round(0.5 / (2 * nu * k * k)))
    o.step(steps)
    amp = np.sum(o.fields()["ux"] * ux) / np.sum(ux * ux)
    return abs(-np.log(amp) / steps / (2 * nu * k * k) - 1)


@pytest.mark.parametrize("free", [(0.0, 0.0), (1.4, 1.1)])
def test_taylor_green_viscosity_second_order(free):
    """Shear-wave decay rate 2 nu k^2 with nu = (1/s_nu - 1/2)/3, approached
    at second order in the resolution, whatever the free rates."""
    e16, e32, e64 = (_taylor_green_rate_error(N, s_e=free[0], s_q=free[1]) for N in (16, 32, 64))
    assert e64 < 5e-3
    assert 3.2 < e32 / e64 < 4.8 and 3.2 < e16 / e32 < 4.8


def _thermal_wave_rate_error(N, alpha=0.02):
    k = 2 * np.pi / N
    T = 0.5 * np.sin(k * np.arange(N))[None, :] * np.ones((8, 1))
    o = Oracle(nx=N, ny=8, periodic_y=1, nu=0.1, alpha=alpha)
    one, zero = np.ones((8, N)), np.zeros((8, N))
    o.set_equilibrium(one, zero, zero, T)
    steps = int(round(0.5 / (alpha * k * k)))
    o.step(steps)
    amp = np.sum(o.fields()["T"] * T) / np.sum(T * T)
    return abs(-np.log(amp) / steps / (alpha * k * k) - 1)


def test_thermal_wave_diffusivity_second_order():
    """Temperature wave decay rate alpha k^2 with alpha = (4+a)/10 (1/s_a - 1/2)."""
    e16, e32, e64 = (_thermal_wave_rate_error(N) for N in (16, 32, 64))
    assert e64 < 5e-4
    assert 3.2 < e32 / e64 < 4.8 and 3.2 < e16 / e32 < 4.8


def _rb_mode_amplitudes(ratio, H=16, steps=9000):
    """Rayleigh-Benard cell of the critical wavelength 2 pi / 3.117 H between a
    hot bottom and a cold top wall; returns |mode-1 amplitude of u_y| over time."""
    W = int(round(2 * np.pi / 3.117 * H))
    nu = alpha = 0.05
    gbeta = ratio * 1707.76 * nu * alpha / H ** 3
    o = Oracle(nx=W, ny=H, nu=nu, alpha=alpha, gravity=1.0, beta=gbeta, wall_T=(1.0, 0.0),
               T_ref=0.5, T_fluid0=0.5)
    y = np.arange(H)[:, None] + 0.0
    x = np.arange(W)[None, :] + 0.0
    T = 1 - (y + 0.5) / H + 0.01 * np.sin(np.pi * (y + 0.5) / H) * np.cos(2 * np.pi * x / W)
    o.set_equilibrium(np.ones((H, W)), np.zeros((H, W)), np.zeros((H, W)), T)
    amps = []
    for _ in range(3):
        o.step(steps // 3)
        amps.append(np.abs(np.fft.fft(o.fields()["uy"], axis=1)[:, 1]).sum())
    return amps


def test_rayleigh_benard_onset_sign():
    """Classical linear stability (rigid walls): Ra_c = 1707.76.  Below it the
    convective mode decays, above it the mode grows: pins the sign and size of
    the Boussinesq coupling (hot fluid rises against gravity)."""
    below = _rb_mode_amplitudes(0.8)
    above = _rb_mode_amplitudes(1.2)
    assert below[2] < 0.2 * below[0]
    assert above[2] > 5 * above[0]


def test_mass_and_heat_conserved_without_particles():
    """Periodic box: sum f and sum g are invariants of collision and streaming."""
    N = 24
    rho, ux, uy, T = lbm_inputs.smooth_fields(N, N, seed=11)
    o = Oracle(nx=N, ny=N, periodic_y=1, nu=0.05, alpha=0.03, gravity=1e-3, beta=0.1)
    o.set_equilibrium(rho, ux, uy, T)
    f0, g0 = o.populations()
    o.step(1000)
    f1, g1 = o.populations()
    assert abs(f1.sum() - f0.sum()) / f0.sum() < 1e-13
    assert abs(g1.sum() - g0.sum()) / np.abs(g0).sum() < 1e-13


def test_mass_conserved_with_moving_wall():
    """Halfway bounce-back with a tangentially moving wall loses no mass."""
    rho, ux, uy, T = lbm_inputs.smooth_fields(16, 16, seed=12)
    o = Oracle(nx=16, ny=16, nu=0.05, alpha=0.03, wall_ux=(0.02, -0.01), wall_T=(0.3, 0.0))
    o.set_equilibrium(rho, ux, uy, T)
    f0, _ = o.populations()
    o.step(500)
    f1, _ = o.populations()
    assert abs(f1.sum() - f0.sum()) / f0.sum() < 1e-13


# ----------------------------------------------------------- closed cavity
# Side walls at x = -1/2 and nx - 1/2 (periodic_x = 0): the same halfway
# bounce-back and anti-bounce-back as the flat y walls, pinned the same way.

@pytest.mark.parametrize("rates", [(0.0, 0.0), (1.3, 0.7), (0.4, 1.9)])
def test_side_wall_conduction_exact(rates):
    """Hot left wall T=1, cold right wall T=0, periodic y:
    T(x) = 1 - (x+1/2)/W for any rates."""
    nx = 16
    o = Oracle(nx=nx, ny=8, periodic_x=0, periodic_y=1, nu=0.1, alpha=0.15, side_T=(1.0, 0.0),
               sT_e=rates[0], sT_p=rates[1])
    o.step(6000)
    f = o.fields()
    x = np.arange(nx)
    assert np.abs(f["T"] - (1 - (x + 0.5) / nx)[None, :]).max() < 1e-12


@pytest.mark.parametrize("nu", [0.02, 1 / 6])
def test_side_wall_poiseuille_exact(nu):
    """Uniform buoyancy force F = rho g beta (T - T_ref) along +y between the
    side walls (T = 1 everywhere, walls included, periodic y):
    u_y(x) = F (x+1/2)(W-1/2-x) / (2 rho0 nu), u_x = 0."""
    nx, G = 12, 1e-5
    o = Oracle(nx=nx, ny=8, periodic_x=0, periodic_y=1, nu=nu, alpha=0.1, gravity=1.0, beta=G,
               T_ref=0.0, T_fluid0=1.0, side_T=(1.0, 1.0))
    o.set_equilibrium(np.ones((8, nx)), np.zeros((8, nx)), np.zeros((8, nx)), np.ones((8, nx)))
    o.step(int(40 * nx * nx / nu / 9.87))
    f = o.fields()
    x = np.arange(nx)
    exact = G * (x + 0.5) * (nx - 0.5 - x) / (2 * nu)
    err = np.abs(f["uy"] - exact[None, :]).max() / exact.max()
    assert err < 1e-11, err
    assert np.abs(f["ux"]).max() < 1e-15


def test_closed_cavity_conserves_mass():
    """Four walls (moving lid and bottom, resting sides, corners included):
    sum f is invariant."""
    rho, ux, uy, T = lbm_inputs.smooth_fields(20, 16, seed=13)
    o = Oracle(nx=20, ny=16, periodic_x=0, nu=0.05, alpha=0.03, wall_ux=(0.02, -0.01),
               wall_T=(0.3, 0.0), side_T=(0.7, 0.1), gravity=1e-3, beta=0.1)
    o.set_equilibrium(rho, ux, uy, T)
    f0, _ = o.populations()
    o.step(500)
    f1, _ = o.populations()
    assert abs(f1.sum() - f0.sum()) / f0.sum() < 1e-13
