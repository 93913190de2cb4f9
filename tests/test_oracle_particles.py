"""Pins of the oracle's particle side: the link set (Sec. 3), the owner map,
repulsion (Sec. 2.4, Eq. (15)), Newton-Euler motion (Sec. 2.2), the momentum
exchange (Sec. 2.4, Eqs. (13)-(14)) and refilling (Sec. 2.5)."""
import math

import numpy as np
import pytest

import lbm_inputs
import oracle
from oracle import Oracle, OracleError
from tests.textbook import EX, EY, feq9, geq5

QUIET = dict(gravity=0.0, beta=0.0, repulsion=0, particle_T=0.0, T_fluid0=0.0)


def _links_set(o):
    L = o.links()
    return set(zip(L["node"].tolist(), L["dir"].tolist(), L["particle"].tolist())), L


def _row(x, y, r, ux=0.0, uy=0.0, th=0.0, om=0.0):
    return [x, y, r, ux, uy, th, om]


@pytest.mark.parametrize("cx", [10.0, 0.0, 31.0])
def test_links_of_a_three_by_three_disk(cx):
    """r = 1.5 centred on a node: the 3 x 3 block of nodes is solid.  Counting
    by hand: 3 links per axis direction and 5 per diagonal direction, 32 in
    all; also across the periodic seam."""
    nx = 32
    o = Oracle(nx=nx, ny=24, **QUIET)
    o.set_particles([_row(cx, 10.0, 1.5)])
    owner = o.fields()["owner"]
    solid = {(int(i), int(j)) for j, i in zip(*np.nonzero(owner >= 0))}
    c = int(cx)
    assert solid == {((c + a) % nx, 10 + b) for a in (-1, 0, 1) for b in (-1, 0, 1)}
    links, L = _links_set(o)
    assert len(links) == 32
    for d in range(1, 9):
        assert sum(1 for (_, dd, _) in links if dd == d) == (3 if d <= 4 else 5)
    expect = {((c - 2) % nx, 10, 1): 0.5, ((c - 2) % nx, 9, 1): 2 - math.sqrt(1.25),
              ((c - 2) % nx, 8, 5): 2 - 1.5 / math.sqrt(2), ((c + 2) % nx, 12, 7): 2 - 1.5 / math.sqrt(2)}
    got = {(int(n) % nx, int(n) // nx, int(d)): q for n, d, q in zip(L["node"], L["dir"], L["q"])}
    for key, q in expect.items():
        assert abs(got[key] - q) < 1e-15


def _line_id(node, d, nx):
    i, j = node % nx, node // nx
    if EY[d] == 0:
        return j
    if EX[d] == 0:
        return i
    return ((i - j) if EX[d] == EY[d] else (i + j)) % nx


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_link_set_invariants_random_layouts(seed):
    """Per particle and direction at most one link per lattice line; at most
    12N - 12 links per particle with N = INT(x_c + d/2) - INT(x_c - d/2) + 3
    (Sec. 3); for an isolated particle every lattice line through its solid
    nodes holds exactly one link in each of its two directions."""
    nx, ny = 48, 40
    P = lbm_inputs.rsa_particles(nx, ny, 4, 9.0 + seed % 3, min_gap=4.0, seed=seed)
    o = Oracle(nx=nx, ny=ny, **QUIET)
    o.set_particles(P)
    links, L = _links_set(o)
    owner = o.fields()["owner"].ravel()
    for p in range(len(P)):
        mine = [(n, d) for (n, d, pp) in links if pp == p]
        N = math.floor(P[p, 0] + P[p, 2]) - math.floor(P[p, 0] - P[p, 2]) + 3
        assert len(mine) <= 12 * N - 12
        solid = np.nonzero(owner == p)[0]
        for d in range(1, 9):
            lines = [_line_id(n, d, nx) for (n, dd) in mine if dd == d]
            assert len(lines) == len(set(lines))
            through = {_line_id(int(k), d, nx) for k in solid}
            assert set(lines) == through
    for n, d, p in links:
        i, j = n % nx, n // nx
        assert owner[n] == -1
        assert owner[((j + EY[d]) * nx + (i + EX[d]) % nx)] == p


@pytest.mark.parametrize("seed", [6, 7])
def test_owner_counts_match_row_chords(seed):
    """Solid nodes per row equal the integers inside the chord
    [x_c - sqrt(r^2 - dy^2), x_c + sqrt(r^2 - dy^2)] (generic centres)."""
    nx, ny = 40, 40
    P = lbm_inputs.rsa_particles(nx, ny, 3, 11.3, min_gap=2.0, seed=seed)
    o = Oracle(nx=nx, ny=ny, **QUIET)
    o.set_particles(P)
    owner = o.fields()["owner"]
    for p, (x, y, r) in enumerate(P[:, :3]):
        for j in range(ny):
            h2 = r * r - (j - y) ** 2
            n = 0 if h2 < 0 else math.floor(x + math.sqrt(h2)) - math.ceil(x - math.sqrt(h2)) + 1
            assert (owner[j] == p).sum() == n


def test_repulsion_hand_values():
    p = oracle.make_params(nx=100, ny=100, gravity=2e-4, rho_ratio=1.5, rep_eps=1e-3, rep_range=3.0)
    C = math.pi * 25 * 0.5 * 2e-4
    f = oracle.repulsion_pair(p, 10.0, 50.0, 5.0, 22.0, 50.0, 5.0)  # gap 2
    assert abs(f[0] - (-C / 1e-3 * (1 / 3) ** 2)) < 1e-15 and f[1] == 0.0
    g = oracle.repulsion_pair(p, 22.0, 50.0, 5.0, 10.0, 50.0, 5.0)
    np.testing.assert_array_equal(g, -f)
    assert (oracle.repulsion_pair(p, 10.0, 50.0, 5.0, 23.5, 50.0, 5.0) == 0).all()
    # across the periodic seam: centres 1 and 89 are 12 apart
    s = oracle.repulsion_pair(p, 1.0, 50.0, 5.0, 89.0, 50.0, 5.0)
    assert abs(s[0] - C / 1e-3 / 9) < 1e-15
    w = oracle.repulsion_walls(p, 1.0, 5.5, 5.0)  # gap to the bottom wall plane y=-1/2 is 1
    assert abs(w[1] - C / 1e-3 * (2 / 3) ** 2) < 1e-15 and w[0] == 0.0   # periodic x: no side walls
    w = oracle.repulsion_walls(p, 1.0, 99.5 - 5.0 - 2.0, 5.0)  # gap 2 to the top wall plane y=99.5
    assert abs(w[1] + C / 1e-3 / 9) < 1e-15
    # a closed cavity also pushes off its side walls at x = -1/2 and nx - 1/2
    pc = oracle.make_params(nx=90, ny=100, periodic_x=0, gravity=2e-4, rho_ratio=1.5, rep_eps=1e-3,
                            rep_range=3.0)
    w = oracle.repulsion_walls(pc, 5.5, 50.0, 5.0)   # gap 1 to the left wall
    assert abs(w[0] - C / 1e-3 * (2 / 3) ** 2) < 1e-15 and w[1] == 0.0
    w = oracle.repulsion_walls(pc, 89.5 - 5.0 - 2.0, 50.0, 5.0)   # gap 2 to the right wall
    assert abs(w[0] + C / 1e-3 / 9) < 1e-15
    c = oracle.repulsion_walls(pc, 5.5, 5.5, 5.0)   # a corner: both walls at gap 1
    assert abs(c[0] - C / 1e-3 * (2 / 3) ** 2) < 1e-15 and abs(c[1] - C / 1e-3 * (2 / 3) ** 2) < 1e-15
    # and no minimum image across a side wall: centres 1 and 89 are 88 apart
    assert (oracle.repulsion_pair(pc, 1.0, 50.0, 5.0, 89.0, 50.0, 5.0) == 0).all()


def test_newton_euler_constant_force_is_exact_quadratic():
    p = oracle.make_params(nx=1000, ny=100, rho_ratio=2.0)
    st = np.array([500.0, 40.0, 4.0, 0.01, -0.02, 0.3, 0.001])
    M = 2.0 * math.pi * 16
    I = 0.5 * M * 16
    Fx, Fy, Tz = 3e-3, -1e-2, 2e-3
    s = st.copy()
    for n in range(1, 41):
        s = oracle.newton_euler(p, s, Fx, Fy, Tz)
        assert abs(s[0] - (500 + 0.01 * n + 0.5 * Fx / M * n * n)) < 1e-12
        assert abs(s[1] - (40 - 0.02 * n + 0.5 * Fy / M * n * n)) < 1e-12
        assert abs(s[5] - (0.3 + 0.001 * n + 0.5 * Tz / I * n * n)) < 1e-13
        assert abs(s[3] - (0.01 + Fx / M * n)) < 1e-15
    assert s[2] == 4.0


def test_uniform_flow_with_comoving_particle_has_no_force():
    """Galilean invariance of the modified momentum exchange (Eq. (13)): a
    particle translating with the fluid's uniform velocity feels no force,
    and interpolated bounce-back leaves the uniform equilibrium unchanged."""
    nx, ny, U = 48, 40, (0.02, -0.01)
    o = Oracle(nx=nx, ny=ny, periodic_y=0, nu=0.05, alpha=0.05, **QUIET)
    P = lbm_inputs.rsa_particles(nx, ny, 3, 10.4, min_gap=4.0, seed=9)
    P[:, 3], P[:, 4] = U
    o.set_particles(P)
    shape = (ny, nx)
    o.set_equilibrium(np.ones(shape), np.full(shape, U[0]), np.full(shape, U[1]), np.zeros(shape))
    owner0 = o.fields()["owner"]
    o.step(1)
    out = o.particles()
    assert np.abs(out[:, 7:9]).max() < 1e-14
    f, _ = o.populations()
    fe = feq9(1.0, *U)
    owner1 = o.fields()["owner"]
    # away from the flat walls (which are at rest) and the refilled nodes
    keep = (owner0 < 0) & (owner1 < 0)
    keep[:2] = keep[-2:] = False
    for i in range(9):
        assert np.abs(f[i][keep] - fe[i]).max() < 1e-15


def test_momentum_exchange_signs():
    """A particle held in a uniform stream is dragged downstream; a particle
    spinning in fluid at rest feels a torque against its rotation."""
    nx, ny = 48, 40
    shape = (ny, nx)
    o = Oracle(nx=nx, ny=ny, nu=0.05, alpha=0.05, **QUIET)
    o.set_particles([_row(24.3, 20.2, 6.0)])
    o.set_equilibrium(np.ones(shape), np.full(shape, 0.02), np.zeros(shape), np.zeros(shape))
    o.step(1)
    fx, fy = o.particles()[0, 7:9]
    assert fx > 0 and abs(fy) < 0.05 * fx
    o = Oracle(nx=nx, ny=ny, nu=0.05, alpha=0.05, **QUIET)
    o.set_particles([_row(24.3, 20.2, 6.0, om=0.01)])
    o.step(1)
    assert o.particles()[0, 9] < 0


def test_refill_node_quadratic_extrapolation_and_constraint():
    """Eq. (16) is exact for populations quadratic along e_c; afterwards the
    macroscopic velocity (with the half force at T = T_w) equals u_w and the
    temperature populations are g^eq(T_w, u_w) (Eq. (17))."""
    g_grav, beta, Tw = 1e-3, 0.2, 0.9
    o = Oracle(nx=8, ny=8, gravity=g_grav, beta=beta, particle_T=Tw, body_fx=1e-5)
    base = feq9(1.02, 0.01, 0.03)
    slope = 0.01 * np.arange(1, 10)
    curv = 0.002 * np.arange(9)
    fk = [base + slope * k + curv * k * k for k in (1, 2, 3)]
    uw = (0.015, -0.004)
    fo, go = o.refill_node(3, *fk, *uw)
    rho = base.sum()
    assert abs(fo.sum() - rho) < 1e-15
    Fx, Fy = 1e-5, rho * g_grav * beta * Tw
    ux = ((EX * fo).sum() + Fx / 2) / rho
    uy = ((EY * fo).sum() + Fy / 2) / rho
    assert abs(ux - uw[0]) < 1e-16 and abs(uy - uw[1]) < 1e-16
    # only the momentum changed: the other moments of the extrapolation stay
    d = fo - base
    assert abs((EX * EX * d).sum()) < 1e-15 and abs((EX * EY * d).sum()) < 1e-15
    np.testing.assert_allclose(go, geq5(Tw, *uw), rtol=0, atol=1e-16)
    lin = o.refill_node(2, base + slope, base + 2 * slope, base * 0, *uw)[0]
    assert abs(lin.sum() - rho) < 1e-15
    eq = o.refill_node(0, base, base, base, *uw)[0]
    assert abs(eq.sum() - 1.0) < 1e-15


def test_newborn_nodes_move_with_the_particle():
    """After a step that uncovers nodes, each newborn node carries the rigid
    velocity U + Omega x (x - X) of its former particle and T = T_w."""
    nx, ny = 40, 32
    o = Oracle(nx=nx, ny=ny, nu=0.1, alpha=0.1, gravity=0.0, beta=0.0, repulsion=0, particle_T=0.7)
    o.set_particles([_row(20.0, 15.5, 5.3, ux=0.3, uy=-0.2, om=0.02)])
    own0 = o.fields()["owner"]
    o.step(1)
    f = o.fields()
    P = o.particles()[0]
    newborn = (own0 >= 0) & (f["owner"] < 0)
    assert newborn.sum() >= 3
    j, i = np.nonzero(newborn)
    ux = P[3] - P[6] * (j - P[1])
    uy = P[4] + P[6] * (i - P[0])
    assert np.abs(f["ux"][newborn] - ux).max() < 1e-15
    assert np.abs(f["uy"][newborn] - uy).max() < 1e-15
    assert np.abs(f["T"][newborn] - 0.7).max() < 1e-15


def test_overspeed_is_reported():
    o = Oracle(nx=40, ny=32, **QUIET)
    o.set_particles([_row(20.0, 15.5, 5.3, ux=0.6)])
    with pytest.raises(OracleError) as e:
        o.step(1)
    assert e.value.rc == -5


def test_invalid_parameters_are_rejected():
    with pytest.raises(OracleError):
        Oracle(nx=4, ny=32)
    with pytest.raises(OracleError):
        Oracle(nx=32, ny=32, periodic_x=2)
    cav = Oracle(nx=32, ny=32, periodic_x=0)
    with pytest.raises(OracleError):   # no wrapping into a closed cavity
        cav.set_particles([_row(33.0, 10, 3)])
    o = Oracle(nx=32, ny=32, periodic_y=1)
    with pytest.raises(OracleError):
        o.set_particles([_row(10, 10, 3)])


@pytest.mark.parametrize("cx,cy", [(2.3, 20.0), (29.6, 2.4), (1.9, 37.2)])
def test_links_next_to_cavity_walls_brute_force(cx, cy):
    """In a closed cavity nothing wraps: the link set of a disk touching a
    side wall (and, in the corners, a y wall) is the brute-force set over the
    nodes of the lattice alone, and the disk owns no node beyond the walls."""
    nx, ny, r = 32, 40, 4.7
    o = Oracle(nx=nx, ny=ny, periodic_x=0, **QUIET)
    o.set_particles([_row(cx, cy, r)])
    links, _ = _links_set(o)

    def solid(i, j):
        return 0 <= i < nx and 0 <= j < ny and (i - cx) ** 2 + (j - cy) ** 2 <= r * r

    expect = set()
    for j in range(ny):
        for i in range(nx):
            if solid(i, j):
                continue
            for d in range(1, 9):
                if solid(i + EX[d], j + EY[d]):
                    expect.add((j * nx + i, d, 0))
    assert links == expect and len(links) > 0
    owner = o.fields()["owner"]
    assert (owner == 0).sum() == sum(solid(i, j) for j in range(ny) for i in range(nx))
