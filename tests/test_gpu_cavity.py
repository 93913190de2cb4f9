"""GPU (gfx950) parity with the CPU oracle in the closed cavity: static side
walls at x = -1/2 and x = nx - 1/2 (no-slip, Dirichlet side temperature)
besides the flat y walls, through the C ABI.

Same bar as the periodic channel: fields within 1e-12 of the oracle, owner
maps and link sets bit-identical, particle states within 1e-12.
"""
import numpy as np
import pytest

import lbm_inputs
from paper_2308_16597_amd import params as P
from tests.gpu_util import U_FF, compare_fields, compare_links, compare_particles, make_pair

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("nx,ny", [(300, 70), (65, 64), (8, 9)])
def test_cavity_lattice_parity(nx, ny):
    """No particles: all four walls, the y walls moving and at their own
    temperatures, the side walls at two others; buoyancy; ragged tiles and
    the smallest lattice (every node next to a wall)."""
    _say("cavity lattice parity", nx, ny)
    kw = dict(nx=nx, ny=ny, periodic_x=0, nu=0.03, alpha=0.02, gravity=1e-3, beta=0.2, T_ref=0.1,
              wall_T=(0.8, 0.1), wall_ux=(0.01, -0.02), side_T=(0.6, 0.3))
    sim, orc = make_pair(**kw)
    rho, ux, uy, T = lbm_inputs.smooth_fields(nx, ny, seed=nx * ny)
    sim.set_equilibrium(rho, ux, uy, T)
    orc.set_equilibrium(rho, ux, uy, T)
    for steps in (1, 99):
        sim.step(steps)
        orc.step(steps)
        errs = compare_fields(sim.fields(), orc.fields())
        _say("  after", orc.steps_done, errs)


@pytest.mark.parametrize("case", ["sides", "corners"])
def test_cavity_owner_and_links_bit_exact(case):
    """Disks touching the side walls and sitting in the corners: the owner
    map and the link set stop at the walls (nothing wraps)."""
    nx, ny = 200, 120
    if case == "sides":
        rows = np.array([[5.6, 60.2, 6.0, 0, 0, 0, 0], [194.3, 40.7, 6.5, 0, 0, 0, 0],
                         [-0.2, 90.1, 5.0, 0, 0, 0, 0], [199.4, 100.3, 5.5, 0, 0, 0, 0]])
    else:
        rows = np.array([[5.2, 5.9, 6.0, 0, 0, 0, 0], [194.1, 6.3, 6.0, 0, 0, 0, 0],
                         [4.8, 113.6, 6.0, 0, 0, 0, 0], [193.7, 114.2, 6.0, 0, 0, 0, 0]])
    _say("cavity links", case)
    kw = dict(nx=nx, ny=ny, periodic_x=0, max_particles=len(rows), max_diameter=14.0,
              gravity=1e-4, beta=0.5, rho_ratio=2.0)
    sim, orc = make_pair(**kw)
    sim.set_particles(rows)
    orc.set_particles(rows)
    np.testing.assert_array_equal(sim.fields()["owner"], orc.fields()["owner"])
    n, dq = compare_links(sim.links(), orc.links())
    _say("  links", n, "max dq", dq)
    assert n > 0


def test_cavity_particles_parity():
    """Particles moving into the side walls and a corner, inside the wall
    repulsion range (they bounce off): side-wall repulsion, refilling next to
    the walls, link collection and the link pass without wrap, 60 steps in
    three pieces.  Every disk starts with a layer of fluid nodes between it
    and the walls."""
    rows = np.array([[6.0, 40.2, 5.0, -0.05, 0.01, 0.0, 0.002],
                     [120.0, 50.1, 6.0, 0.04, -0.02, 0.0, -0.003],
                     [5.8, 6.1, 5.0, -0.03, -0.03, 0.0, 0.004],
                     [64.2, 70.7, 5.5, 0.0, 0.02, 0.0, 0.0]])
    kw = dict(nx=128, ny=96, periodic_x=0, nu=0.08, alpha=0.06, gravity=1e-4, beta=0.5,
              particle_T=1.0, rho_ratio=2.0, side_T=(0.2, 0.0), wall_T=(0.0, 0.1),
              rep_eps=3e-3, max_particles=4, max_diameter=14.0)
    sim, orc = make_pair(torch_memory=False, **kw)
    sim.set_particles(rows)
    orc.set_particles(rows)
    for _ in range(3):
        sim.step(20)
        orc.step(20)
        ef = compare_fields(sim.fields(), orc.fields(), u_floor=U_FF)
        ep = compare_particles(sim.particles(), orc.particles(), u_floor=U_FF)
        compare_links(sim.links(), orc.links(), q_abs=1e-12)
        _say("cavity particles at", orc.steps_done, ef, ep)
    po = orc.particles()
    assert (po[:, 0] - po[:, 2] > -0.5).all() and (po[:, 0] + po[:, 2] < 127.5).all()


def test_cavity_graph_replay_equals_eager_steps():
    """Whole 6-step cycles replayed from a captured graph give the bits of
    single steps in the cavity too."""
    from paper_2308_16597_amd import lbm
    rows = np.array([[8.3, 30.2, 6.0, -0.03, -0.02, 0.0, 0.004],
                     [118.6, 50.5, 7.0, 0.03, 0.03, 0.0, -0.005]])
    kw = dict(nx=128, ny=96, periodic_x=0, nu=0.05, alpha=0.04, gravity=1e-4, beta=0.5,
              side_T=(0.3, 0.0), rho_ratio=2.0, max_particles=2, max_diameter=14.0)
    eager = lbm.Sim(lbm.lbm_params_default(**kw))
    graph = lbm.Sim(lbm.lbm_params_default(**kw))
    eager.set_particles(rows)
    graph.set_particles(rows)
    for _ in range(36):
        eager.step(1)
    graph.step(36)
    fe, fg = eager.fields(), graph.fields()
    for k in ("rho", "ux", "uy", "T", "owner"):
        np.testing.assert_array_equal(fg[k], fe[k], err_msg=k)
    np.testing.assert_array_equal(graph.particles(), eager.particles())
    eager.close()
    graph.close()


def test_cavity_rejects_particles_outside_and_seeding():
    from paper_2308_16597_amd import lbm
    kw = dict(nx=64, ny=64, periodic_x=0, max_particles=2, max_diameter=12.0)
    sim = lbm.Sim(lbm.lbm_params_default(**kw))
    for rows in ([[-0.6, 30.0, 5.0, 0, 0, 0, 0]], [[63.6, 30.0, 5.0, 0, 0, 0, 0]]):
        with pytest.raises(lbm.LbmError) as e:
            sim.set_particles(rows)
        assert e.value.rc == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError) as e:
        sim.seed_particles(2, 10.0, 1.0, 1)
    assert e.value.rc == lbm.LBM_EINVAL
    sim.close()


def test_e4_cavity_parity_full_lattice():
    """The paper's benchmark case itself (closed 4000^2 cavity, 60 x 80 hot
    particles of diameter 40, Pr 5, Gr_p 60, rho_p/rho_f = 1.1) in the launch
    configuration the benchmark times: link set at t_0 bit-exact, then every
    field and particle after two steps within 1e-12 of the oracle."""
    kw = P.workload_params("e4_cavity")
    rows = lbm_inputs.workload_particles(P.WORKLOADS["e4_cavity"])
    sim, orc = make_pair(**kw)
    sim.set_particles(rows)
    orc.set_particles(rows)
    n, dq = compare_links(sim.links(), orc.links())
    _say("e4 cavity links", n, "max dq", dq)
    sim.step(2)
    orc.step(2)
    ef = compare_fields(sim.fields(), orc.fields(), u_floor=U_FF)
    ep = compare_particles(sim.particles(), orc.particles(), u_floor=U_FF)
    _say("e4 cavity after 2 steps", ef, ep)
    compare_links(sim.links(), orc.links(), q_abs=1e-12)
