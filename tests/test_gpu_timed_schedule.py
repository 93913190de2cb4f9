"""The launch configurations the benchmark and the server time, held to the
oracle directly (not only through bit-equality with other GPU paths):

* the paper-scale workload (4000^2, 4800 particles of diameter 20) stepped
  13 times by one lbm_step call, as lbm_step schedules it: a 6-step cycle
  captured as a HIP graph and replayed twice (particle kernels on the
  second stream, concurrent with the lattice kernel), then one eager step;
* calls of step counts that are not multiples of 6, which replay the
  graphs kept for each step state;
* FP64 runs advanced together by lbm_step_many (batched kernels over a run
  table, graph replays, unequal step counts), each against its own oracle
  run.

Bar (FP64): owner maps and link sets bit-identical, fields within 1e-12 of
the oracle (velocities on the flow's scale U_ff), particles within 1e-12,
force and torque within 1e-9.  After 13 steps at 4000^2 the two sides'
positions differ by an ulp or two of |X| ~ 4000 (9e-13 each), which moves
a link fraction q by up to r |dX| / |(x_w - X) . e_i|; there q is held to
2 ulp of its definition evaluated at the GPU's own particle state."""
import numpy as np
import pytest

import lbm_inputs
from gpu_util import U_FF, check_q_of_own_particles, compare_fields, compare_links, compare_particles, make_pair
from oracle import Oracle
from paper_2308_16597_amd import lbm
from paper_2308_16597_amd import params as P

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.mark.timeout(900)
def test_paper_scale_graph_schedule_matches_oracle():
    kw = P.workload_params("paper_scale")
    w = P.WORKLOADS["paper_scale"]
    rows = lbm_inputs.rsa_particles(w["nx"], w["ny"], w["n"], w["d"], w["gap"], w["seed"])
    sim, orc = make_pair(**kw)
    sim.set_particles(rows)
    orc.set_particles(rows)
    _say("paper scale: 13 steps in one lbm_step call (2 graph replays + 1 eager step)")
    sim.step(13)
    orc.step(13)
    ef = compare_fields(sim.fields(), orc.fields(), u_floor=U_FF)
    pg = sim.particles()
    ep = compare_particles(pg, orc.particles(), u_floor=U_FF)
    lg = sim.links()
    n, dq = compare_links(lg, orc.links(), check_q=False)
    qu = check_q_of_own_particles(lg, pg, w["nx"])
    assert sim.stats()["steps"] == 13
    _say("paper scale after 13 scheduled steps", ef, ep, "links", n, "max |dq| vs oracle", dq,
         "q vs its definition at the GPU's positions (ulp)", qu)
    sim.close()
    orc.close()


def _small_run(nx, ny, rows, d):
    kw = dict(nx=nx, ny=ny, nu=0.05, alpha=0.04, gravity=1e-4, beta=0.5, particle_T=1.0,
              rho_ratio=2.0, max_particles=len(rows), max_diameter=d)
    return kw, np.asarray(rows, dtype=float)


FAST = [[40.3, 30.2, 6.0, 0.05, -0.02, 0.0, 0.004],
        [100.6, 50.5, 7.0, -0.06, 0.03, 0.0, -0.005],
        [1.2, 25.0, 5.0, -0.04, 0.0, 0.0, 0.0],
        [70.0, 70.5, 4.5, 0.0, -0.03, 0.0, 0.006]]


def test_uneven_step_calls_replay_per_state_graphs_against_oracle():
    """Calls of 20, 10 and 7 steps start from changing step states; each
    state's graph is captured once and replayed later.  Held to the oracle
    after every call, and to single eager steps bit for bit."""
    kw, rows = _small_run(128, 96, FAST, 14.0)
    sim, orc = make_pair(**kw)
    eager = lbm.Sim(lbm.lbm_params_default(**kw))
    for r in (sim, orc, eager):
        r.set_particles(rows)
    done = 0
    for call, n in enumerate([20, 20, 10, 20, 7, 20, 20]):
        sim.step(n)
        orc.step(n)
        for _ in range(n):
            eager.step(1)
        done += n
        fg, fe = sim.fields(), eager.fields()
        for k in ("rho", "ux", "uy", "T", "owner"):
            np.testing.assert_array_equal(fg[k], fe[k], err_msg=f"call {call}: {k}")
        np.testing.assert_array_equal(sim.particles(), eager.particles())
        ef = compare_fields(fg, orc.fields(), u_floor=U_FF)
        compare_particles(sim.particles(), orc.particles(), u_floor=U_FF)
        _say("call", call, "of", n, "steps (", done, "in all ):", ef)
    assert sim.stats()["steps"] == done
    for r in (sim, orc, eager):
        r.close()


def test_batched_fp64_runs_match_oracle():
    """Three FP64 runs of different shapes advanced by lbm_step_many with
    unequal step counts per call, each compared with its own oracle run."""
    specs = [_small_run(128, 96, FAST, 14.0),
             _small_run(160, 80, lbm_inputs.rsa_particles(160, 80, 6, 8.0, 3.0, 11), 8.0),
             _small_run(96, 128, lbm_inputs.rsa_particles(96, 128, 5, 12.0, 3.0, 7), 12.0)]
    sims, orcs = [], []
    for kw, rows in specs:
        s, o = make_pair(**kw)
        s.set_particles(rows)
        o.set_particles(rows)
        sims.append(s)
        orcs.append(o)
    calls = [[7, 12, 18], [30, 30, 0], [23, 5, 40], [36, 36, 36], [0, 13, 2]]
    for c, counts in enumerate(calls):
        lbm.step_many(sims, counts)
        for s, o, n in zip(sims, orcs, counts):
            o.step(n)
        for r, (s, o) in enumerate(zip(sims, orcs)):
            ef = compare_fields(s.fields(), o.fields(), u_floor=U_FF)
            ep = compare_particles(s.particles(), o.particles(), u_floor=U_FF)
            compare_links(s.links(), o.links(), q_abs=1e-12)
            _say("batched call", c, "run", r, ef, ep)
    for r in sims + orcs:
        r.close()
