"""In-place (AA) streaming on the GPU (gfx950), through the C ABI.

The in-place layout keeps one population set and alternates two kernels;
the collision, the wall rules, the link pass and the refill compute the same
values as in the two-set layout, so a run gives the same bits in both
layouts.  Each case steps a two-set run and an in-place run through odd and
even step counts (single steps and replays of captured six-step graphs),
reading fields in both parities, and compares every field and particle bit
for bit; one case also holds the in-place run to the oracle.
"""
import numpy as np
import pytest

import lbm_inputs
from paper_2308_16597_amd import lbm
from paper_2308_16597_amd import params as P
from tests.gpu_util import U_FF, compare_fields, compare_links, compare_particles, make_pair

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _pair(**kw):
    a = lbm.Sim(lbm.lbm_params_default(streaming="two_sets", **kw))
    b = lbm.Sim(lbm.lbm_params_default(streaming="in_place", **kw))
    return a, b


def _same(a, b, what):
    fa, fb = a.fields(), b.fields()
    for k in ("rho", "ux", "uy", "T", "owner"):
        np.testing.assert_array_equal(fb[k], fa[k], err_msg=f"{what}: {k}")
    if a.params.max_particles > 0:
        np.testing.assert_array_equal(b.particles(), a.particles(), err_msg=what)


def _walk(a, b, chunks=(1, 1, 5, 12, 36, 7)):
    """Step both runs through odd and even counts, comparing after each."""
    done = 0
    for n in chunks:
        a.step(n)
        b.step(n)
        done += n
        _same(a, b, f"after {done} steps")
    return done


@pytest.mark.parametrize("nx,ny,periodic_x,periodic_y", [(300, 70, 1, 0), (257, 33, 1, 1), (65, 64, 0, 0)])
def test_lattice_in_place_equals_two_sets(nx, ny, periodic_x, periodic_y):
    """No particles: moving and isothermal walls, side walls, buoyancy, body
    force, periodic y, ragged tiles; started from smooth fields at both
    parities."""
    kw = dict(nx=nx, ny=ny, periodic_x=periodic_x, periodic_y=periodic_y, nu=0.03, alpha=0.02,
              gravity=1e-3, beta=0.2, T_ref=0.1, body_fx=1e-6, wall_T=(0.8, 0.1),
              wall_ux=(0.01, -0.02), side_T=(0.6, 0.3))
    a, b = _pair(**kw)
    rho, ux, uy, T = lbm_inputs.smooth_fields(nx, ny, seed=nx + ny)
    a.set_equilibrium(rho, ux, uy, T)
    b.set_equilibrium(rho, ux, uy, T)
    _walk(a, b)
    # re-initialise at the odd parity (the state is then written pushed)
    a.step(1)
    b.step(1)
    a.set_equilibrium(rho, ux, uy, T)
    b.set_equilibrium(rho, ux, uy, T)
    _walk(a, b, (1, 6, 13))
    a.close()
    b.close()


@pytest.mark.parametrize("storage", ["f64", "f32", "shift_f16", "shift_bf16"])
def test_small_workload_in_place_equals_two_sets(storage):
    """The small workload (256^2, 20 hot particles) in every storage mode."""
    kw = P.workload_params("small", lbm.STORE[storage])
    kw.pop("storage")
    rows = lbm_inputs.workload_particles(P.WORKLOADS["small"])
    a, b = _pair(storage=storage, **kw)
    a.set_particles(rows)
    b.set_particles(rows)
    n = _walk(a, b, (1, 1, 7, 36, 55))
    compare_links(b.links(), a.links(), q_ulps=0)
    _say("small workload", storage, "bitwise equal over", n, "steps")
    a.close()
    b.close()


def test_fast_particles_cavity_and_ellipses_in_place_equals_two_sets():
    """Particles fast enough to refill every step, in a closed cavity, circles
    and ellipses spinning, bouncing off the side walls."""
    kw = dict(nx=128, ny=96, periodic_x=0, nu=0.08, alpha=0.06, gravity=1e-4, beta=0.5,
              particle_T=1.0, rho_ratio=2.0, side_T=(0.2, 0.0), wall_T=(0.0, 0.1), wall_ux=(0.01, 0.0),
              rep_eps=3e-3, max_particles=4, max_diameter=20.0)
    rows = np.array([[40.3, 30.2, 6.0, 6.0, 0.15, -0.05, 0.0, 0.01],
                     [100.6, 50.5, 9.0, 4.0, -0.2, 0.1, 0.7, -0.02],
                     [7.2, 25.0, 5.0, 5.0, -0.05, 0.0, 0.0, 0.0],
                     [70.0, 8.5, 8.0, 3.0, 0.0, -0.1, 2.0, 0.03]])
    a, b = _pair(**kw)
    a.set_particles_ellipse(rows)
    b.set_particles_ellipse(rows)
    _walk(a, b, (1, 2, 3, 12, 24, 1))
    a.close()
    b.close()


def test_in_place_small_workload_oracle_parity():
    """The in-place layout held to the oracle: the small workload over 100
    steps at the FP64 bar."""
    kw = P.workload_params("small")
    rows = lbm_inputs.workload_particles(P.WORKLOADS["small"])
    sim, orc = make_pair(streaming="in_place", **kw)
    sim.set_particles(rows)
    orc.set_particles(rows)
    for n in (37, 63):
        sim.step(n)
        orc.step(n)
        ef = compare_fields(sim.fields(), orc.fields(), u_floor=U_FF)
        ep = compare_particles(sim.particles(), orc.particles(), u_floor=U_FF)
        _say("in place vs oracle at", orc.steps_done, ef, ep)
    compare_links(sim.links(), orc.links(), q_abs=1e-12)


def test_in_place_direct_addressing_oracle_parity():
    kw = P.workload_params("small")
    rows = lbm_inputs.workload_particles(P.WORKLOADS["small"])
    sim, orc = make_pair(streaming="in_place", **kw)
    sim.set_particles(rows)
    orc.set_particles(rows)
    sim.set_addressing("direct")
    sim.step(41)
    orc.step(41)
    compare_fields(sim.fields(), orc.fields(), u_floor=U_FF)
    compare_particles(sim.particles(), orc.particles(), u_floor=U_FF)


def test_in_place_batched_runs_equal_runs_alone():
    """lbm_step_many over in-place runs of unequal sizes and step counts (their
    parities differ within a batch) gives the bits of each run stepped alone;
    a batch may not mix layouts."""
    specs = [dict(nx=128, ny=96, n=6, d=12.0, seed=3), dict(nx=200, ny=64, n=4, d=10.0, seed=8),
             dict(nx=96, ny=160, n=9, d=14.0, seed=5)]
    base = dict(nu=0.05, alpha=0.04, gravity=1e-4, beta=0.5, rho_ratio=1.5, storage="shift_bf16")

    def make(spec, streaming):
        s = lbm.Sim(lbm.lbm_params_default(nx=spec["nx"], ny=spec["ny"], max_particles=spec["n"],
                                           max_diameter=spec["d"], streaming=streaming, **base))
        s.set_particles(lbm_inputs.rsa_particles(spec["nx"], spec["ny"], spec["n"], spec["d"], 3.0,
                                                 spec["seed"]))
        return s

    alone = [make(s, "in_place") for s in specs]
    mixed = [make(s, "in_place") for s in specs]
    mixed[1].step(1)   # a run one step ahead: the batch holds both parities
    alone[1].step(1)
    for counts in ([13, 12, 25], [36, 7, 12], [6, 6, 6]):
        lbm.step_many(mixed, counts)
        for s, n in zip(alone, counts):
            s.step(n)
        for s, t in zip(alone, mixed):
            _same(s, t, f"batched {counts}")
    other = make(specs[0], "two_sets")
    with pytest.raises(lbm.LbmError) as e:
        lbm.step_many([mixed[0], other], [1, 1])
    assert e.value.rc == lbm.LBM_EINVAL
    for s in alone + mixed + [other]:
        s.close()


def test_in_place_paper_scale_equals_two_sets():
    """The benchmark workload (4000^2, 4800 particles) in the launch
    configuration the benchmark times: 13 steps (two graph cycles and a
    single step on each side) bit for bit."""
    kw = P.workload_params("paper_scale")
    rows = lbm_inputs.workload_particles(P.WORKLOADS["paper_scale"])
    a = lbm.Sim(lbm.lbm_params_default(streaming="two_sets", **kw))
    a.set_particles(rows)
    a.step(13)
    fa, pa = a.fields(), a.particles()
    a.close()
    del a
    b = lbm.Sim(lbm.lbm_params_default(streaming="in_place", **kw))
    b.set_particles(rows)
    b.step(13)
    fb, pb = b.fields(), b.particles()
    for k in ("rho", "ux", "uy", "T", "owner"):
        np.testing.assert_array_equal(fb[k], fa[k], err_msg=k)
    np.testing.assert_array_equal(pb, pa)
    b.close()
