"""Pins of the oracle's elliptical particles (Sec. 2.6.2, App. A): semi-axes
a along the body axis at angle theta and b across it.

Each pin uses a formulation of the ellipse other than the oracle's implicit
b^2 u^2 + a^2 v^2 <= a^2 b^2: the focal definition (distances to the foci
sum to at most 2a), the parametric boundary, numerical quadrature over the
area, the reflection property of the normal, mirror symmetry of a whole
step, and physics of settling ellipses."""
import math

import numpy as np
import pytest

import oracle
from oracle import Oracle, OracleError
from tests.textbook import EX, EY, feq9

QUIET = dict(gravity=0.0, beta=0.0, repulsion=0, particle_T=0.0, T_fluid0=0.0)


def _foci(X, Y, a, b, th):
    c = math.sqrt(a * a - b * b)
    return (X + c * math.cos(th), Y + c * math.sin(th)), (X - c * math.cos(th), Y - c * math.sin(th))


def _focal_excess(x, y, X, Y, a, b, th):
    """|x - F1| + |x - F2| - 2a: negative inside, positive outside."""
    (f1x, f1y), (f2x, f2y) = _foci(X, Y, a, b, th)
    return math.hypot(x - f1x, y - f1y) + math.hypot(x - f2x, y - f2y) - 2.0 * a


def _boundary(X, Y, a, b, th, phi):
    c, s = math.cos(th), math.sin(th)
    u, v = a * np.cos(phi), b * np.sin(phi)
    return X + u * c - v * s, Y + u * s + v * c


SHAPES = [(7.3, 3.1, 0.0), (7.3, 3.1, math.pi / 3), (9.0, 4.5, 2.2), (6.2, 5.9, -0.7),
          (12.5, 6.25, math.pi / 2)]


@pytest.mark.parametrize("a,b,th", SHAPES)
def test_solid_test_matches_the_focal_definition(a, b, th):
    """Every offset on a grid around the centre is inside exactly when the
    distances to the two foci sum to at most 2a (offsets within 1e-9 of the
    boundary are skipped)."""
    X, Y = 0.37, -0.21
    checked = 0
    for j in range(-14, 15):
        for i in range(-14, 15):
            e = _focal_excess(i, j, X, Y, a, b, th)
            if abs(e) < 1e-9:
                continue
            assert oracle.inside_shape(i - X, j - Y, a, b, th) == (e < 0), (i, j)
            checked += 1
    assert checked > 800


def test_solid_count_approaches_the_area():
    """Semi-axes, not full axes: the number of nodes inside tends to pi a b."""
    a, b = 40.3, 17.1
    for th in (0.0, 0.4, 1.3):
        n = sum(oracle.inside_shape(i - 0.3, j + 0.2, a, b, th)
                for j in range(-42, 43) for i in range(-42, 43))
        assert abs(n / (math.pi * a * b) - 1.0) < 0.01


def test_circle_reduces_to_the_disk_test():
    for dx, dy in [(3.0, 4.0), (3.0, 4.0000001), (-2.5, 1.1)]:
        assert oracle.inside_shape(dx, dy, 5.0, 5.0, 1.234) == (dx * dx + dy * dy <= 25.0)
        for i in range(1, 9):
            assert oracle.link_q_ellipse(dx, dy, 5.0, 5.0, 0.8, i) == oracle.link_q(dx, dy, 5.0, i)


def test_link_fraction_hand_values():
    """Axis-aligned ellipse a = 4, b = 2 centred at the origin."""
    assert abs(oracle.link_q_ellipse(4.5, 0.0, 4.0, 2.0, 0.0, 3) - 0.5) < 1e-15
    assert abs(oracle.link_q_ellipse(0.0, 2.75, 4.0, 2.0, 0.0, 4) - 0.75) < 1e-15
    # (3 - t)^2/16 + (2 - t)^2/4 = 1  ->  5 t^2 - 22 t + 9 = 0
    t = (22.0 - math.sqrt(304.0)) / 10.0
    assert abs(oracle.link_q_ellipse(3.0, 2.0, 4.0, 2.0, 0.0, 7) - t) < 1e-15


@pytest.mark.parametrize("a,b,th", SHAPES)
def test_link_fraction_hits_the_nearer_boundary_point(a, b, th):
    """For every link of a grid of nodes: x_w = x_f + q e_i satisfies the
    focal equation, and the points before it on the link are outside."""
    X, Y = 0.37, -0.21
    n = 0
    for j in range(-14, 15):
        for i in range(-14, 15):
            if _focal_excess(i, j, X, Y, a, b, th) <= 1e-9:
                continue
            for d in range(1, 9):
                if _focal_excess(i + EX[d], j + EY[d], X, Y, a, b, th) > -1e-9:
                    continue
                q = oracle.link_q_ellipse(i - X, j - Y, a, b, th, d)
                assert 0.0 < q <= 1.0
                assert abs(_focal_excess(i + q * EX[d], j + q * EY[d], X, Y, a, b, th)) < 1e-9
                for t in np.linspace(0.0, q, 7)[:-1]:
                    assert _focal_excess(i + t * EX[d], j + t * EY[d], X, Y, a, b, th) > -1e-9
                n += 1
    assert n > 100


@pytest.mark.parametrize("th", [0.0, 0.35, math.pi / 3, 2.0])
def test_link_set_and_owner_map_brute_force(th):
    """Links and owner map of two ellipses in a closed cavity against an
    enumeration with the focal test."""
    nx, ny = 48, 40
    P = [(14.3, 20.2, 9.0, 4.0, th), (35.6, 17.9, 7.5, 3.5, -th + 0.3)]
    o = Oracle(nx=nx, ny=ny, periodic_x=0, **QUIET)
    o.set_particles_ellipse([[x, y, a, b, 0, 0, t, 0] for x, y, a, b, t in P])

    def owner_of(i, j):
        if not (0 <= i < nx and 0 <= j < ny):
            return -2
        for k, (x, y, a, b, t) in enumerate(P):
            e = _focal_excess(i, j, x, y, a, b, t)
            assert abs(e) > 1e-9
            if e < 0:
                return k
        return -1

    own = np.array([[owner_of(i, j) for i in range(nx)] for j in range(ny)])
    np.testing.assert_array_equal(o.fields()["owner"], own)
    expect = set()
    for j in range(ny):
        for i in range(nx):
            if own[j, i] != -1:
                continue
            for d in range(1, 9):
                k = owner_of(i + EX[d], j + EY[d])
                if k >= 0:
                    expect.add((j * nx + i, d, k))
    L = o.links()
    got = set(zip(L["node"].tolist(), L["dir"].tolist(), L["particle"].tolist()))
    assert got == expect and len(got) > 50


@pytest.mark.parametrize("a,b,th", SHAPES)
def test_refill_direction_follows_the_reflection_normal(a, b, th):
    """On the boundary the outward normal bisects the angle between the
    focal radii; the refill direction maximises it over the eight lattice
    vectors (points near a tie skipped)."""
    if a == b:
        return
    (f1x, f1y), (f2x, f2y) = _foci(0.0, 0.0, a, b, th)
    n = 0
    for phi in np.linspace(0.0, 2 * math.pi, 97)[:-1]:
        x, y = _boundary(0.0, 0.0, a, b, th, phi)
        r1, r2 = math.hypot(x - f1x, y - f1y), math.hypot(x - f2x, y - f2y)
        nx_ = (x - f1x) / r1 + (x - f2x) / r2
        ny_ = (y - f1y) / r1 + (y - f2y) / r2
        scores = [nx_ * EX[d] + ny_ * EY[d] for d in range(1, 9)]
        top = sorted(scores)[-2:]
        if top[1] - top[0] < 1e-6 * max(1.0, abs(top[1])):
            continue
        assert oracle.refill_direction(x, y, a, b, th) == 1 + int(np.argmax(scores))
        n += 1
    assert n > 80


def test_mass_and_inertia_match_quadrature():
    """Constant force and torque over one step: du = F/M, dOmega = T/I with
    M and I of the ellipse, compared with midpoint quadrature of rho dA and
    rho |x|^2 dA over the area."""
    a, b, rho_ratio = 6.0, 2.5, 1.7
    p = oracle.make_params(rho_ratio=rho_ratio)
    h = 0.01
    g = np.arange(-a + h / 2, a, h)
    X, Y = np.meshgrid(g, np.arange(-b + h / 2, b, h))
    inside = (X / a) ** 2 + (Y / b) ** 2 <= 1.0
    M_q = rho_ratio * inside.sum() * h * h
    I_q = rho_ratio * ((X ** 2 + Y ** 2) * inside).sum() * h * h
    out = oracle.newton_euler_ellipse(p, [10.0, 10.0, a, 0.0, 0.0, 0.3, 0.0], b, 1e-3, 0.0, 1e-2)
    assert abs((1e-3 / out[3]) / M_q - 1.0) < 2e-3
    assert abs((1e-2 / out[6]) / I_q - 1.0) < 2e-3
    # trapezoidal angle: theta advances by half the new rotation rate
    assert abs(out[5] - (0.3 + 0.5 * out[6])) < 1e-16
    disk = oracle.newton_euler(p, [10.0, 10.0, a, 0.0, 0.0, 0.3, 0.0], 1e-3, 0.0, 1e-2)
    np.testing.assert_array_equal(oracle.newton_euler_ellipse(p, [10.0, 10.0, a, 0, 0, 0.3, 0], a,
                                                              1e-3, 0.0, 1e-2), disk)


@pytest.mark.parametrize("th", [0.0, 0.6, math.pi / 2, 2.5])
def test_wall_repulsion_uses_the_supporting_line(th):
    """The gap to each flat wall is the centre's distance minus the largest
    extent of the boundary normal to the wall (parametric sampling); the
    force scale is the particle's immersed weight pi a b (rho_p - rho_f) g."""
    a, b = 8.0, 3.0
    nx, ny = 60, 50
    p = oracle.make_params(nx=nx, ny=ny, periodic_x=0, rho_ratio=1.5, gravity=1e-4, rep_eps=1e-3,
                           rep_range=3.0)
    xs, ys = _boundary(0.0, 0.0, a, b, th, np.linspace(0, 2 * math.pi, 200001))
    hx, hy = xs.max(), ys.max()
    C = math.pi * a * b * 0.5 * 1e-4
    x, y = -0.5 + hx + 1.2, ny - 0.5 - hy - 2.1
    fx, fy = oracle.repulsion_walls_ellipse(p, x, y, a, b, th)
    assert abs(fx - C / 1e-3 * ((1.2 - 3.0) / 3.0) ** 2) < 1e-9 * abs(fx)
    assert abs(fy + C / 1e-3 * ((2.1 - 3.0) / 3.0) ** 2) < 1e-8 * abs(fy)
    fx, fy = oracle.repulsion_walls_ellipse(p, 30.0, 25.0, a, b, th)
    assert fx == 0.0 and fy == 0.0


def test_pair_repulsion_along_the_centre_line():
    """The gap is the centre distance minus each shape's extent along the
    centre line (found by bisection on the focal test); equal and opposite
    forces; equal to the disk formula for two circles."""
    p = oracle.make_params(nx=200, ny=200, periodic_x=1, rho_ratio=1.5, gravity=1e-4)
    P = (50.0, 60.0, 9.0, 4.0, 0.4)
    Q = (50.0 + 7.2, 60.0 + 8.8, 7.0, 3.0, 2.1)

    def extent(S, ux, uy):
        lo, hi = 0.0, S[2]
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if _focal_excess(S[0] + mid * ux, S[1] + mid * uy, *S) < 0:
                lo = mid
            else:
                hi = mid
        return lo

    d = math.hypot(Q[0] - P[0], Q[1] - P[1])
    ux, uy = (Q[0] - P[0]) / d, (Q[1] - P[1]) / d
    gap = d - extent(P, ux, uy) - extent(Q, -ux, -uy)
    assert 0 < gap < 3.0
    C = math.pi * math.sqrt(P[2] * P[3] * Q[2] * Q[3]) * 0.5 * 1e-4
    mag = C / 1e-3 * ((gap - 3.0) / 3.0) ** 2
    fp = oracle.repulsion_pair_ellipse(p, P, Q)
    fq = oracle.repulsion_pair_ellipse(p, Q, P)
    np.testing.assert_allclose(fp, [-mag * ux, -mag * uy], rtol=1e-9)
    np.testing.assert_allclose(fp, -fq, rtol=1e-14)
    np.testing.assert_array_equal(oracle.repulsion_pair_ellipse(p, (1, 2, 5, 5, 0.3), (12, 2.5, 4, 4, 1)),
                                  oracle.repulsion_pair(p, 1, 2, 5, 12, 2.5, 4))


def _comoving(U, th, y=20.2):
    nx, ny = 56, 44
    o = Oracle(nx=nx, ny=ny, nu=0.05, alpha=0.05, **QUIET)
    o.set_particles_ellipse([[15.3, y, 8.0, 3.5, U[0], U[1], th, 0.0],
                             [40.1, 23.6, 6.5, 4.0, U[0], U[1], th + 1.7, 0.0]])
    shape = (ny, nx)
    o.set_equilibrium(np.ones(shape), np.full(shape, U[0]), np.full(shape, U[1]), np.zeros(shape))
    o.step(1)
    return o


def test_uniform_flow_with_comoving_ellipses_has_no_force():
    """Galilean invariance (Eq. (13)) with inclined ellipses translating with
    the fluid: no force, and the populations stay the uniform equilibrium.
    Each lattice line through a convex body holds one link at each end, and
    their isotropic parts cancel in force and torque (the two wall points
    lie on the line); what remains of the torque is the u_w term of the
    modified momentum exchange, which is exactly quadratic in U and
    vanishes at rest and for mirror-symmetric layouts."""
    U = (0.02, -0.01)
    o = _comoving(U, 0.7)
    out = o.particles()
    assert np.abs(out[:, 7:9]).max() < 1e-14
    f, _ = o.populations()
    fe = feq9(1.0, *U)
    keep = o.fields()["owner"] < 0
    keep[:2] = keep[-2:] = False
    for i in range(9):
        assert np.abs(f[i][keep] - fe[i]).max() < 1e-15
    T1 = out[:, 9]
    T2 = _comoving((2 * U[0], 2 * U[1]), 0.7).particles()[:, 9]
    np.testing.assert_allclose(T2, 4.0 * T1, rtol=1e-9)
    assert np.abs(_comoving((0.0, 0.0), 0.7).particles()[:, 7:10]).max() < 1e-14
    # axis-aligned ellipse on a lattice row, flow along its axis: no torque
    assert abs(_comoving((0.02, 0.0), 0.0, y=20.0).particles()[0, 9]) < 1e-14


def test_mirror_image_step():
    """Mirroring the cavity about its vertical centre line maps an ellipse
    at angle theta to pi - theta: every field and particle of the mirrored
    run is the mirror image of the original (u_x, Omega and the torque
    change sign)."""
    nx, ny = 48, 64
    kw = dict(nx=nx, ny=ny, periodic_x=0, nu=0.05, alpha=0.04, gravity=2e-4, beta=0.3,
              rho_ratio=1.5, particle_T=1.0)
    row = [17.3, 40.2, 8.0, 3.5, 0.01, -0.004, 1.0, 0.002]
    mir = [nx - 1 - row[0], row[1], row[2], row[3], -row[4], row[5], math.pi - row[6], -row[7]]
    o1, o2 = Oracle(**kw), Oracle(**kw)
    o1.set_particles_ellipse([row])
    o2.set_particles_ellipse([mir])
    np.testing.assert_array_equal(o1.fields()["owner"], o2.fields()["owner"][:, ::-1])
    o1.step(60)
    o2.step(60)
    f1, f2 = o1.fields(), o2.fields()
    np.testing.assert_array_equal(f1["owner"], f2["owner"][:, ::-1])
    fluid = f1["owner"] < 0
    for k, sgn in (("rho", 1), ("ux", -1), ("uy", 1), ("T", 1)):
        assert np.abs(f1[k][fluid] - sgn * f2[k][:, ::-1][fluid]).max() < 1e-12
    p1, p2 = o1.particles()[0], o2.particles()[0]
    assert abs(p1[0] - (nx - 1 - p2[0])) < 1e-12 and abs(p1[1] - p2[1]) < 1e-12
    assert abs(p1[3] + p2[3]) < 1e-12 and abs(p1[4] - p2[4]) < 1e-12
    assert abs(p1[5] - (math.pi - p2[5])) < 1e-12 and abs(p1[6] + p2[6]) < 1e-12


def test_inclined_ellipse_glides_and_turns_broadside():
    """A heavy ellipse released at 60 degrees drifts sideways towards its
    lower end (it glides along its long axis: u_x < 0 with u_y < 0, the
    velocity between the vertical and the axis) and turns towards the
    broadside orientation (Omega < 0), as settling ellipses do at finite
    Reynolds number."""
    o = Oracle(nx=64, ny=160, periodic_x=0, nu=0.05, alpha=0.05, gravity=1e-4, rho_ratio=1.5)
    o.set_particles_ellipse([[31.8, 120.0, 8.0, 4.0, 0.0, 0.0, math.pi / 3, 0.0]])
    o.step(500)
    x, y, _, ux, uy, th, om = o.particles()[0, :7]
    assert uy < 0 and ux < 0
    assert 0 < ux / uy < 1 / math.tan(math.pi / 3)
    assert om < 0 and th < math.pi / 3


def test_invalid_ellipses_are_rejected():
    o = Oracle(nx=40, ny=40, **QUIET)
    for row in ([20, 20, 5.0, 6.0, 0, 0, 0, 0], [20, 20, 5.0, 1.0, 0, 0, 0, 0],
                [20, 20, 5.0, float("nan"), 0, 0, 0, 0]):
        with pytest.raises(OracleError):
            o.set_particles_ellipse([row])
