"""The serving form on the GPU: several runs advanced together by
lbm_step_many (batched step kernels over a run table, graph replay of
6-step cycles) give bit-for-bit the results of each run advanced alone by
lbm_step; the request loop completes a small mix under a binding memory
budget with the same results as the runs alone."""
import ctypes

import numpy as np
import pytest

import lbm_inputs
from paper_2308_16597_amd import lbm, params, serve

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _runs(storage):
    """Three runs of different shapes: moving particles (window 18),
    a particle-free lattice with smooth initial fields, small particles
    (window 12)."""
    fast = np.array([[40.3, 30.2, 6.0, 0.05, -0.02, 0.0, 0.004],
                     [100.6, 50.5, 7.0, -0.06, 0.03, 0.0, -0.005],
                     [1.2, 25.0, 5.0, -0.04, 0.0, 0.0, 0.0],
                     [70.0, 70.5, 4.5, 0.0, -0.03, 0.0, 0.006]])
    base = dict(storage=lbm.STORE[storage], T_shift=0.0, nu=0.05, alpha=0.04, gravity=1e-4,
                beta=0.5, particle_T=1.0, rho_ratio=2.0)
    a = (dict(base, nx=128, ny=96, max_particles=4, max_diameter=14.0), fast, None)
    b = (dict(base, nx=96, ny=64, wall_T=(0.7, 0.1), wall_ux=(0.01, 0.0)), None,
         lbm_inputs.smooth_fields(96, 64, seed=3))
    c = (dict(base, nx=160, ny=80, max_particles=6, max_diameter=8.0),
         lbm_inputs.rsa_particles(160, 80, 6, 8.0, 3.0, 11), None)
    return [a, b, c]


def _make(run):
    kw, rows, fields = run
    sim = lbm.Sim(lbm.lbm_params_default(**kw))
    if rows is not None:
        sim.set_particles(rows)
    if fields is not None:
        sim.set_equilibrium(*fields)
    return sim


def _state(sim):
    f = sim.fields()
    p = sim.particles()
    return f, p


def _same(a, b, what):
    fa, pa = a
    fb, pb = b
    for k in ("rho", "ux", "uy", "T", "owner"):
        np.testing.assert_array_equal(fa[k], fb[k], err_msg=f"{what}: {k}")
    np.testing.assert_array_equal(pa, pb, err_msg=f"{what}: particles")


# step counts per call: unequal counts split a call into segments of
# different run sets; calls of 36 steps replay the captured 6-step cycle
CALLS = [[7, 12, 18], [30, 30, 0], [23, 5, 40], [36, 36, 36], [36, 36, 36], [0, 13, 2], [36, 36, 36]]


@pytest.mark.parametrize("storage", ["f64", "shift_bf16"])
def test_same_alone_and_in_mix(storage):
    runs = _runs(storage)
    alone = []
    for r, run in enumerate(runs):
        sim = _make(run)
        snaps = []
        for call in CALLS:
            sim.step(call[r])
            snaps.append(_state(sim))
        sim.sync()
        sim.close()
        alone.append(snaps)
    mix = [_make(run) for run in runs]
    for c, call in enumerate(CALLS):
        lbm.step_many(mix, call)
        for r in range(len(runs)):
            _same(_state(mix[r]), alone[r][c], f"{storage} call {c} run {r}")
        _say(storage, "call", c, call, "bitwise equal")
    for s in mix:
        s.sync()
        s.close()


def test_link_pass_block_sizes_give_the_same_bits():
    """A run alone takes a link-pass block of 128, 256 or 512 threads by its
    particle size (windows 12, 18 and 34 here: d = 8, 14, 30), a batch 256
    for every run; the force and torque sums keep one order whatever the
    block size, so every field and particle matches bit for bit."""
    base = dict(nu=0.05, alpha=0.04, gravity=1e-4, beta=0.5, particle_T=1.0, rho_ratio=2.0)
    runs = [(dict(base, nx=160, ny=80, max_particles=6, max_diameter=8.0),
             lbm_inputs.rsa_particles(160, 80, 6, 8.0, 3.0, 11), None),
            (dict(base, nx=128, ny=96, max_particles=4, max_diameter=14.0),
             lbm_inputs.rsa_particles(128, 96, 4, 14.0, 3.0, 5), None),
            (dict(base, nx=192, ny=128, max_particles=3, max_diameter=30.0),
             np.array([[50.3, 60.2, 14.0, 0.02, -0.01, 0.0, 0.001],
                       [130.6, 70.5, 12.5, -0.03, 0.02, 0.0, -0.002],
                       [96.0, 25.3, 10.0, 0.0, 0.03, 0.0, 0.0]]), None)]
    alone = [_make(r) for r in runs]
    mix = [_make(r) for r in runs]
    for n in (1, 5, 36):
        for sim in alone:
            sim.step(n)
        lbm.step_many(mix, [n] * len(mix))
        for r, (a, b) in enumerate(zip(alone, mix)):
            _same(_state(a), _state(b), f"run {r} after +{n} steps")
    for sim in alone + mix:
        sim.close()


def test_edge_runs_alone_and_in_mix():
    """A batch of a run created for particles that holds none, a run with a
    single particle and an 8 x 9 lattice (the smallest accepted) with
    moving walls: every run matches itself alone bit for bit (the empty run
    adds no blocks to the per-particle grids)."""
    base = dict(nu=0.05, alpha=0.04, gravity=1e-4, beta=0.5, particle_T=1.0, rho_ratio=2.0)
    runs = [(dict(base, nx=96, ny=64, max_particles=3, max_diameter=12.0), None,
             lbm_inputs.smooth_fields(96, 64, seed=8)),
            (dict(base, nx=80, ny=72, max_particles=1, max_diameter=12.0),
             np.array([[39.6, 35.2, 6.0, 0.03, -0.02, 0.0, 0.002]]), None),
            (dict(base, nx=8, ny=9, wall_T=(0.9, 0.1), wall_ux=(0.02, -0.01)), None,
             lbm_inputs.smooth_fields(8, 9, seed=9))]
    alone = [_make(r) for r in runs]
    mix = [_make(r) for r in runs]
    for call in ([13, 7, 20], [36, 36, 36], [0, 12, 5], [36, 36, 36]):
        for sim, n in zip(alone, call):
            sim.step(n)
        lbm.step_many(mix, call)
        for r, (a, b) in enumerate(zip(alone, mix)):
            _same(_state(a), _state(b), f"run {r} after call {call}")
        _say("edge runs", call, "bitwise equal")
    for sim in alone + mix:
        sim.close()


def test_step_many_argument_errors():
    runs = _runs("f64")
    a, b = _make(runs[0]), _make(runs[1])
    with pytest.raises(lbm.LbmError) as e:
        lbm.step_many([a, a], [1, 1])
    assert e.value.rc == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError) as e:
        lbm.step_many([a, b], [1, -1])
    assert e.value.rc == lbm.LBM_EINVAL
    c = _make(_runs("shift_bf16")[2])
    with pytest.raises(lbm.LbmError) as e:
        lbm.step_many([a, c], [1, 1])
    assert e.value.rc == lbm.LBM_EINVAL
    for s in (a, b, c):
        s.close()


def test_request_loop_matches_runs_alone():
    """Six small requests, all arriving at t = 0, under a budget that holds
    about two of them: every request completes, and the final particle
    states equal those of the same request run alone with lbm_step."""
    reqs = lbm_inputs.serving_requests(6, seed=7, L_range=(96, 160), np_range=(3, 12),
                                       d_range=(8, 12), Ra_range=(1e4, 1e5), steps_range=(60, 200))
    sizes = [lbm.lbm_bytes_required(serve.request_params(r)[0]) for r in reqs]
    budget = int(2.2 * max(sizes))
    srv = serve.Server(budget, chunk=48)
    recs = srv.run(reqs, np.zeros(len(reqs)))
    _say("request loop:", [(r["rid"], r["status"], round(r["latency"], 3)) for r in recs])
    assert all(r["status"] == "ok" for r in recs)
    first_done = min(r["done"] for r in recs)
    assert any(r["admit"] >= first_done for r in recs)   # the budget made some wait
    for r, rec in zip(reqs, recs):
        p, _ = serve.request_params(r)
        sim = lbm.Sim(p)
        sim.seed_particles(r["n"], r["d"], srv.gap, r["seed"])
        sim.step(r["steps"])
        np.testing.assert_array_equal(sim.particles(), rec["particles"], err_msg=f"request {r['rid']}")
        sim.close()
    s = serve.summarize(recs, max(r["done"] for r in recs))
    _say("summary", s)
    assert s["completed"] == len(reqs) and s["p99_s"] >= s["p50_s"] > 0
