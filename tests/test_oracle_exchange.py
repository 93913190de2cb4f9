"""Pins of the oracle's momentum exchange (Sec. 2.4, Eqs. (13)-(14)) and of
its wall Nusselt number by conservation laws the lattice obeys exactly.

Bookkeeping of one step, for a fluid with no body force (gravity 0):
* collision keeps the mass and momentum of every node;
* pull streaming carries each post-collision population f_i^+(y) to y + e_i
  and keeps its momentum e_i f_i^+ and its angular momentum
  (y + e_i - X) x e_i f_i^+ = (y - X) x e_i f_i^+ about any point X;
* a static flat wall returns f_i^+ as f_ibar at the same node; with the fluid
  at rest near both walls the two walls' exchanges cancel;
* at a link (x_f, i) of a particle the fluid loses f_i^+(x_f), which would
  have entered the solid, and gains the reflected f_ibar(x_f) from it: mass
  f_i^+ - f_ibar, momentum e_i (f_i^+ + f_ibar), angular momentum
  (x_f - X) x e_i (f_i^+ + f_ibar).
Eq. (13) gives the link dF = f_i^+ (e_i - u_w) - f_ibar (e_ibar - u_w)
= e_i (f_i^+ + f_ibar) - u_w (f_i^+ - f_ibar), and Eq. (14) its torque
(x_w - X) x dF with the wall point x_w = x_f + q e_i.  Summed over a
particle's links, with dM, dJ, dL the changes of the fluid's mass, momentum
and angular momentum over the step (no node changes its owner):
* translation (u_w = U):  F = -dJ + U dM;
* rotation about a fixed centre (u_w = Omega z x (x_w - X)) of a circle:
  (x_w - X) x u_w = Omega R^2 at every wall point (x_w on the circle), and
  e_i x e_i = 0, so  T = -dL + Omega R^2 dM.
A wrong factor or sign in Eq. (13), a dropped u_w term, the lever x_f - X
in place of x_w - X, or u_w taken at x_f instead of x_w breaks one of these.
The sums use exactly rounded summation (math.fsum).
"""
import math

import numpy as np
import pytest

from oracle import Oracle
from tests.gpu_util import nusselt_from_fields
from tests.textbook import EX, EY

# no body force; a particle so heavy that it keeps its velocity over the step
HEAVY = dict(gravity=0.0, beta=0.0, repulsion=0, particle_T=1.0, T_fluid0=0.0, rho_ratio=1e12,
             nu=0.05, alpha=0.05)
NX = NY = 64


def _offsets(nx, X, ii, jj):
    dx = ii - X[0]
    dx = np.where(dx > nx / 2, dx - nx, np.where(dx < -nx / 2, dx + nx, dx))
    return dx, jj - X[1]


def _fluid_totals(o, X):
    """Mass, momentum and angular momentum about X of the fluid (pre-collision
    populations of the fluid nodes), exactly rounded sums; the owner map."""
    f, _ = o.populations()
    owner = o.fields()["owner"]
    fl = owner < 0
    jj, ii = np.nonzero(fl)
    dx, dy = _offsets(owner.shape[1], X, ii, jj)
    ff = f[:, fl]
    M = math.fsum(ff.ravel())
    Jx = math.fsum(np.concatenate([EX[i] * ff[i] for i in range(9)]))
    Jy = math.fsum(np.concatenate([EY[i] * ff[i] for i in range(9)]))
    L = math.fsum(np.concatenate([(dx * EY[i] - dy * EX[i]) * ff[i] for i in range(9)]))
    return M, Jx, Jy, L, owner


def _bump(X, seed, amp=0.03, rc=20.0):
    """Smooth fields that differ from rest only within rc of X (zero at the
    walls and the periodic seam, also after one step)."""
    rng = np.random.default_rng(seed)
    y, x = np.mgrid[0:NY, 0:NX].astype(float)
    dx, dy = _offsets(NX, X, x, y)
    r2 = (dx * dx + dy * dy) / (rc * rc)
    w = np.where(r2 < 1.0, (1.0 - r2) ** 2, 0.0)
    a, b, c = rng.uniform(-1.0, 1.0, 3)
    return 1.0 + 0.02 * a * w, amp * b * w, amp * c * w, 0.3 * w


def _one_step(rows, X, flow_seed, ellipse=False):
    o = Oracle(nx=NX, ny=NY, **HEAVY)
    (o.set_particles_ellipse if ellipse else o.set_particles)(rows)
    if flow_seed is not None:
        o.set_equilibrium(*_bump(X, flow_seed))
    M0, Jx0, Jy0, L0, ow0 = _fluid_totals(o, X)
    o.step(1)
    M1, Jx1, Jy1, L1, ow1 = _fluid_totals(o, X)
    # the balances hold link by link only while no node changes its owner
    assert (ow0 == ow1).all()
    return o.particles()[0], M1 - M0, Jx1 - Jx0, Jy1 - Jy0, L1 - L0


@pytest.mark.parametrize("flow_seed", [None, 1, 2])
@pytest.mark.parametrize("X,U", [((31.37, 32.21), (0.013, 0.021)),
                                 ((30.83, 31.62), (0.02, -0.013)),
                                 ((32.41, 30.77), (-0.017, 0.011))])
def test_force_is_the_fluid_momentum_lost_through_the_links(X, U, flow_seed):
    """Translating disk: Eqs. (13) summed over the links equal -dJ + U dM of
    the fluid over one step (magnitude, sign and the u_w term of Eq. (13))."""
    R = 8.3
    P, dM, dJx, dJy, _ = _one_step([[X[0], X[1], R, U[0], U[1], 0.0, 0.0]], X, flow_seed)
    Fx, Fy = -dJx + U[0] * dM, -dJy + U[1] * dM
    scale = math.hypot(Fx, Fy)
    assert scale > 0.05
    assert abs(P[7] - Fx) <= 1e-13 * scale and abs(P[8] - Fy) <= 1e-13 * scale, (P[7:9], Fx, Fy)
    # the u_w term of Eq. (13) is resolved: it exceeds the tolerance by far
    assert abs(U[0] * dM) + abs(U[1] * dM) > 1e-8 * scale


@pytest.mark.parametrize("flow_seed", [None, 3])
def test_force_balance_translating_ellipse(flow_seed):
    """The same balance for an ellipse (Sec. 2.6.2), whose wall points lie on
    the ellipse."""
    X, U = (31.37, 32.21), (0.013, 0.021)
    rows = [[X[0], X[1], 10.5, 6.2, U[0], U[1], 0.4, 0.0]]
    P, dM, dJx, dJy, _ = _one_step(rows, X, flow_seed, ellipse=True)
    Fx, Fy = -dJx + U[0] * dM, -dJy + U[1] * dM
    scale = math.hypot(Fx, Fy)
    assert scale > 0.05
    assert abs(P[7] - Fx) <= 1e-13 * scale and abs(P[8] - Fy) <= 1e-13 * scale


@pytest.mark.parametrize("flow_seed", [None, 4, 5])
@pytest.mark.parametrize("X,R,Om", [((31.37, 32.21), 8.3, 0.005), ((32.08, 31.55), 6.7, -0.007)])
def test_torque_is_the_fluid_angular_momentum_lost_with_the_wall_point_lever(X, R, Om, flow_seed):
    """Spinning disk with a fixed centre: Eq. (14) summed over the links
    equals -dL + Omega R^2 dM (lever x_w - X, wall velocity at x_w)."""
    P, dM, _, _, dL = _one_step([[X[0], X[1], R, 0.0, 0.0, 0.0, Om]], X, flow_seed)
    Tz = -dL + Om * R * R * dM
    assert abs(Tz) > 1.0
    assert abs(P[9] - Tz) <= 1e-13 * abs(Tz), (P[9], Tz)
    assert abs(Om * R * R * dM) > 1e-8 * abs(Tz)


def test_nusselt_of_linear_conduction_is_one():
    """Steady conduction between a hot bottom wall (T = 1) and a cold top wall
    (T = 0): T(y) = 1 - (y + 1/2)/H for any rates, so the wall-normal heat
    flux is 1/H everywhere and the Nusselt number H/dT times the flux is 1
    at both walls, with the sign of the gradient: -1 at the bottom wall
    (temperature falls away from it), +1 at the top.  dT = particle_T -
    T_fluid0 = 1.  Both the oracle's Nusselt number and the helper applied
    to read-back fields are held to it."""
    nx, ny = 24, 20
    o = Oracle(nx=nx, ny=ny, nu=0.07, alpha=0.11, gravity=0.0, beta=0.0, wall_T=(1.0, 0.0),
               particle_T=1.0, T_fluid0=0.0)
    y = np.arange(ny, dtype=float)[:, None] * np.ones((1, nx))
    T = 1.0 - (y + 0.5) / ny
    o.set_equilibrium(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)), T)
    o.step(200)
    fo = o.fields()
    assert np.abs(fo["T"] - T).max() < 1e-12
    nb, nt = o.nusselt()
    assert abs(nb + 1.0) < 1e-11 and abs(nt - 1.0) < 1e-11, (nb, nt)
    hb, ht = nusselt_from_fields(fo["T"], fo["owner"], (1.0, 0.0))
    assert abs(hb + 1.0) < 1e-11 and abs(ht - 1.0) < 1e-11, (hb, ht)


def test_nusselt_scales_with_the_temperature_difference_and_skips_solids():
    """Doubling the wall temperature difference doubles the flux and the
    reference dT = particle_T - T_fluid0 (held at 1) turns that into Nu = 2;
    a particle touching a wall row removes its nodes from the average
    without changing the value of a linear profile."""
    nx, ny = 40, 24
    o = Oracle(nx=nx, ny=ny, nu=0.07, alpha=0.11, gravity=0.0, beta=0.0, wall_T=(2.0, 0.0),
               particle_T=1.0, T_fluid0=0.0, repulsion=0)
    y = np.arange(ny, dtype=float)[:, None] * np.ones((1, nx))
    T = 2.0 * (1.0 - (y + 0.5) / ny)
    o.set_particles([[20.3, 3.1, 3.4, 0.0, 0.0, 0.0, 0.0]])
    o.set_equilibrium(np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)), T)
    fo = o.fields()
    assert (fo["owner"][0] >= 0).any()
    nb, nt = o.nusselt()
    assert abs(nb + 2.0) < 1e-12 and abs(nt - 2.0) < 1e-12, (nb, nt)
    hb, ht = nusselt_from_fields(fo["T"], fo["owner"], (2.0, 0.0))
    assert abs(hb + 2.0) < 1e-12 and abs(ht - 2.0) < 1e-12
