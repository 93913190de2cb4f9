"""GPU (gfx950) parity with the CPU oracle, through the C ABI.

FP64 bar: fields within 1e-12 of the oracle (max abs difference over fluid
nodes / max abs oracle value), owner maps and link sets bit-identical, link
fractions within 2 ulp, particle states within 1e-12.
"""
import numpy as np
import pytest

import lbm_inputs
from paper_2308_16597_amd import params as P
from tests.gpu_util import U_FF, compare_fields, compare_links, compare_particles, make_pair

pytestmark = pytest.mark.gpu

C1 = P.workload_params("small")
C1_PHYS = {k: v for k, v in C1.items() if k not in ("nx", "ny", "max_particles", "max_diameter")}


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("nx,ny,periodic_y", [(300, 70, 0), (257, 33, 1), (64, 64, 0)])
def test_lattice_parity_smooth_fields(nx, ny, periodic_y):
    """No particles: walls (moving, isothermal), buoyancy, body force, ragged tiles."""
    _say("lattice parity", nx, ny, periodic_y)
    kw = dict(nx=nx, ny=ny, periodic_y=periodic_y, nu=0.03, alpha=0.02, gravity=1e-3, beta=0.2,
              T_ref=0.1, body_fx=1e-6, wall_T=(0.8, 0.1), wall_ux=(0.01, -0.02))
    sim, orc = make_pair(**kw)
    rho, ux, uy, T = lbm_inputs.smooth_fields(nx, ny, seed=nx + ny)
    sim.set_equilibrium(rho, ux, uy, T)
    orc.set_equilibrium(rho, ux, uy, T)
    for steps in (1, 99):
        sim.step(steps)
        orc.step(steps)
        errs = compare_fields(sim.fields(), orc.fields())
        _say("  after", orc.steps_done, errs)


def test_free_rates_and_a_T_parity():
    kw = dict(nx=96, ny=40, nu=0.05, alpha=0.04, s_e=1.2, s_eps=1.4, s_q=1.1, sT_e=0.9, sT_p=1.3,
              a_T=-1.0, gravity=2e-3, beta=0.3, wall_T=(1.0, 0.0))
    sim, orc = make_pair(**kw)
    rho, ux, uy, T = lbm_inputs.smooth_fields(96, 40, seed=5)
    sim.set_equilibrium(rho, ux, uy, T)
    orc.set_equilibrium(rho, ux, uy, T)
    sim.step(50)
    orc.step(50)
    compare_fields(sim.fields(), orc.fields())


@pytest.mark.parametrize("case", ["small", "seam", "walls", "touching", "tiny"])
def test_owner_and_links_bit_exact(case):
    """Given bit-identical particle input, owner maps and link sets are equal
    and link fractions agree within 2 ulp."""
    nx, ny = 256, 256
    if case == "small":
        rows = lbm_inputs.rsa_particles(nx, ny, 20, 12, 1.0, 1)
    elif case == "seam":
        rows = np.array([[0.3, 100.2, 6.0, 0, 0, 0, 0], [255.7, 40.9, 7.5, 0, 0, 0, 0],
                         [128.0, 128.0, 6.0, 0, 0, 0, 0]])
    elif case == "walls":
        rows = np.array([[40.25, 6.1, 6.0, 0, 0, 0, 0], [90.5, 249.4, 6.0, 0, 0, 0, 0],
                         [150.0, 5.5, 5.0, 0, 0, 0, 0]])
    elif case == "touching":
        rows = np.array([[50.0, 50.0, 6.0, 0, 0, 0, 0], [62.0, 50.0, 6.0, 0, 0, 0, 0],
                         [56.0, 60.4, 6.0, 0, 0, 0, 0], [80.1, 80.3, 6.0, 0, 0, 0, 0],
                         [91.9, 80.3, 6.0, 0, 0, 0, 0]])
    else:
        rows = np.array([[20.5, 20.5, 1.2, 0, 0, 0, 0], [30.0, 30.0, 1.5, 0, 0, 0, 0],
                         [40.3, 41.7, 1.01, 0, 0, 0, 0]])
    _say("links", case, len(rows))
    sim, orc = make_pair(nx=nx, ny=ny, max_particles=len(rows), max_diameter=16.0, **C1_PHYS)
    sim.set_particles(rows)
    orc.set_particles(rows)
    np.testing.assert_array_equal(sim.fields()["owner"], orc.fields()["owner"])
    n, dq = compare_links(sim.links(), orc.links())
    _say("  links", n, "max dq", dq)
    assert n > 0


def test_small_workload_parity_100_and_200_steps():
    """256^2, 20 hot particles of diameter 12, Pr 0.7, Ra 1e5 (seed 1)."""
    rows = lbm_inputs.rsa_particles(256, 256, 20, 12.0, 1.0, 1)
    sim, orc = make_pair(**C1)
    sim.set_particles(rows)
    orc.set_particles(rows)
    for target in (100, 200):
        n = target - orc.steps_done
        sim.step(n)
        orc.step(n)
        ef = compare_fields(sim.fields(), orc.fields(), u_floor=U_FF)
        ep = compare_particles(sim.particles(), orc.particles(), u_floor=U_FF)
        _say("small workload step", target, ef, ep)
        compare_links(sim.links(), orc.links(), q_abs=1e-12)


def test_fast_particles_refill_parity():
    """Particles moving and spinning fast enough to uncover nodes every step:
    exercises refilling, the owner map update and the flags."""
    rows = np.array([[40.3, 30.2, 6.0, 0.15, -0.05, 0.0, 0.01],
                     [100.6, 50.5, 7.0, -0.2, 0.1, 0.0, -0.02],
                     [1.2, 25.0, 5.0, -0.12, 0.0, 0.0, 0.0],
                     [70.0, 8.5, 4.5, 0.0, -0.1, 0.0, 0.03]])
    kw = dict(nx=128, ny=64, nu=0.08, alpha=0.06, gravity=1e-4, beta=0.5, particle_T=1.0,
              rho_ratio=3.0, max_particles=4, max_diameter=14.0)
    sim, orc = make_pair(torch_memory=False, **kw)
    sim.set_particles(rows)
    orc.set_particles(rows)
    for _ in range(3):
        sim.step(10)
        orc.step(10)
        compare_fields(sim.fields(), orc.fields(), u_floor=U_FF)
        compare_particles(sim.particles(), orc.particles(), u_floor=U_FF)
    _say("fast particles ok at", orc.steps_done)


def test_deterministic_replay_is_bitwise():
    rows = lbm_inputs.rsa_particles(256, 256, 20, 12.0, 1.0, 1)
    from paper_2308_16597_amd import lbm
    out = []
    for _ in range(2):
        sim = lbm.Sim(lbm.lbm_params_default(**C1))
        sim.set_particles(rows)
        sim.step(60)
        f = sim.fields()
        out.append((f, sim.particles()))
        sim.close()
    for k in ("rho", "ux", "uy", "T"):
        np.testing.assert_array_equal(out[0][0][k], out[1][0][k])
    np.testing.assert_array_equal(out[0][1], out[1][1])


def test_seed_particles_matches_input_generator():
    from paper_2308_16597_amd import lbm
    sim = lbm.Sim(lbm.lbm_params_default(**C1))
    sim.seed_particles(20, 12.0, 1.0, 1)
    got = sim.particles()[:, :7]
    np.testing.assert_array_equal(got, lbm_inputs.rsa_particles(256, 256, 20, 12.0, 1.0, 1))


def test_overspeed_reported_as_unstable():
    from paper_2308_16597_amd import lbm
    sim = lbm.Sim(lbm.lbm_params_default(nx=64, ny=64, max_particles=1, max_diameter=12.0))
    sim.set_particles([[32.0, 32.0, 5.0, 0.7, 0.0, 0.0, 0.0]])
    sim.step(1)
    with pytest.raises(lbm.LbmError) as e:
        sim.sync()
    assert e.value.rc == lbm.LBM_EUNSTABLE
    # a fresh particle set clears the error
    sim.set_particles([[32.0, 32.0, 5.0, 0.0, 0.0, 0.0, 0.0]])
    sim.step(2)
    sim.sync()


def test_invalid_particles_rejected():
    from paper_2308_16597_amd import lbm
    sim = lbm.Sim(lbm.lbm_params_default(nx=64, ny=64, max_particles=2, max_diameter=12.0))
    for rows in ([[10, 10, 7.0, 0, 0, 0, 0]], [[10, 10, 0.5, 0, 0, 0, 0]],
                 [[np.nan, 10, 5.0, 0, 0, 0, 0]], [[10, 80, 5.0, 0, 0, 0, 0]],
                 [[10, 10, 5.0, 0, 0, 0, 0]] * 3):
        with pytest.raises(lbm.LbmError) as e:
            sim.set_particles(rows)
        assert e.value.rc == lbm.LBM_EINVAL


def test_paper_scale_parity_full_lattice():
    """The benchmark workload itself (4000^2, 4800 particles of diameter 20,
    Ra 1e8, seeded with gaps >= 3), in the launch configuration the benchmark
    times: link set at t_0 bit-exact, then every field and particle after two
    steps within 1e-12 of the oracle."""
    kw = P.workload_params("paper_scale")
    w = P.WORKLOADS["paper_scale"]
    rows = lbm_inputs.rsa_particles(w["nx"], w["ny"], w["n"], w["d"], w["gap"], w["seed"])
    sim, orc = make_pair(**kw)
    sim.set_particles(rows)
    orc.set_particles(rows)
    n, dq = compare_links(sim.links(), orc.links())
    _say("paper scale links", n, "max dq", dq)
    sim.step(2)
    orc.step(2)
    ef = compare_fields(sim.fields(), orc.fields(), u_floor=U_FF)
    ep = compare_particles(sim.particles(), orc.particles(), u_floor=U_FF)
    _say("paper scale after 2 steps", ef, ep)
    compare_links(sim.links(), orc.links(), q_abs=1e-12)


def test_dense_workload_parity_full_lattice():
    """The dense workload (4096^2, 64000 particles of diameter 10, 30 % solid,
    Ra 1e8, gaps >= 3) in the launch configuration the benchmark times, FP64
    storage: link set at t_0 bit-exact (about 6.2 M links), then every field
    and particle after one step within 1e-12 of the oracle."""
    kw = P.workload_params("dense")
    w = P.WORKLOADS["dense"]
    rows = lbm_inputs.rsa_particles(w["nx"], w["ny"], w["n"], w["d"], w["gap"], w["seed"])
    sim, orc = make_pair(**kw)
    sim.set_particles(rows)
    orc.set_particles(rows)
    n, dq = compare_links(sim.links(), orc.links())
    _say("dense links", n, "max dq", dq)
    sim.step(1)
    orc.step(1)
    ef = compare_fields(sim.fields(), orc.fields(), u_floor=U_FF)
    ep = compare_particles(sim.particles(), orc.particles(), u_floor=U_FF)
    _say("dense after 1 step", ef, ep)


def test_graph_replays_equal_eager_steps():
    """lbm_step replays a captured graph of six overlapped steps for whole
    cycles; stepping one step per call never does.  Three calls of 36 steps
    (the graph is captured by the first and replayed six times per call),
    with field reads between them, must give the bits of 108 single steps."""
    from paper_2308_16597_amd import lbm
    rows = np.array([[40.3, 30.2, 6.0, 0.05, -0.02, 0.0, 0.004],
                     [100.6, 50.5, 7.0, -0.06, 0.03, 0.0, -0.005],
                     [70.0, 70.5, 4.5, 0.0, -0.03, 0.0, 0.006]])
    kw = dict(nx=128, ny=96, nu=0.05, alpha=0.04, gravity=1e-4, beta=0.5, particle_T=1.0,
              rho_ratio=2.0, max_particles=3, max_diameter=14.0)
    eager = lbm.Sim(lbm.lbm_params_default(**kw))
    graph = lbm.Sim(lbm.lbm_params_default(**kw))
    eager.set_particles(rows)
    graph.set_particles(rows)
    for call in range(3):
        for _ in range(36):
            eager.step(1)
        graph.step(36)
        fe, fg = eager.fields(), graph.fields()
        for k in ("rho", "ux", "uy", "T", "owner"):
            np.testing.assert_array_equal(fg[k], fe[k], err_msg=f"call {call}: {k}")
        np.testing.assert_array_equal(graph.particles(), eager.particles())
        _say("graph replay call", call, "bitwise equal to single steps")
    eager.close()
    graph.close()


def test_direct_addressing_parity_and_switching():
    """The direct-addressing link pass (a thread per node, no collection,
    FP64 atomic force sums) on the small workload: 60 steps direct, 60
    indirect, 60 direct again, then every field and particle within 1e-12 of
    the oracle (forces within 1e-9: their summation order differs)."""
    from paper_2308_16597_amd import lbm
    rows = lbm_inputs.rsa_particles(256, 256, 20, 12.0, 1.0, 1)
    sim, orc = make_pair(**C1)
    sim.set_particles(rows)
    orc.set_particles(rows)
    with pytest.raises(lbm.LbmError) as e:
        sim.set_addressing(7)
    assert e.value.rc == lbm.LBM_EINVAL
    for mode in ("direct", "indirect", "direct"):
        sim.set_addressing(mode)
        sim.step(60)
        orc.step(60)
        ef = compare_fields(sim.fields(), orc.fields(), u_floor=U_FF)
        ep = compare_particles(sim.particles(), orc.particles(), u_floor=U_FF)
        _say("addressing", mode, "at step", orc.steps_done, ef, ep)
    n, dq = compare_links(sim.links(), orc.links(), q_abs=1e-12)   # collected on demand
    assert n > 0
    other = lbm.Sim(lbm.lbm_params_default(**C1))
    other.set_particles(rows)
    other.set_addressing("direct")
    with pytest.raises(lbm.LbmError) as e:
        lbm.step_many([sim, other], [1, 1])
    assert e.value.rc == lbm.LBM_EINVAL
    other.close()


def test_large_window_particles_parity():
    """Particles of diameter 30 (windows 34 wide): the per-particle kernels
    give each particle a whole block of 256 lanes instead of a wavefront.
    Moving, spinning, refilling every step, close to each other and to the
    walls: 60 steps against the oracle, links bit-exact at the start."""
    rows = np.array([[40.3, 40.2, 15.0, 0.06, -0.02, 0.0, 0.004],
                     [80.6, 45.5, 14.0, -0.05, 0.03, 0.0, -0.006],
                     [60.2, 85.4, 13.5, 0.02, -0.06, 0.0, 0.005],
                     [140.0, 20.7, 15.0, -0.04, 0.0, 0.0, 0.0]])
    kw = dict(nx=180, ny=120, nu=0.06, alpha=0.05, gravity=1e-4, beta=0.5, particle_T=1.0,
              rho_ratio=1.8, max_particles=4, max_diameter=30.0)
    sim, orc = make_pair(torch_memory=False, **kw)
    sim.set_particles(rows)
    orc.set_particles(rows)
    compare_links(sim.links(), orc.links())
    for _ in range(3):
        sim.step(20)
        orc.step(20)
        ef = compare_fields(sim.fields(), orc.fields(), u_floor=U_FF)
        ep = compare_particles(sim.particles(), orc.particles(), u_floor=U_FF)
        compare_links(sim.links(), orc.links(), q_abs=1e-12)
        _say("large windows at", orc.steps_done, ef, ep)
