"""Edge cases of the particle path on the GPU against the oracle: a run with
a single particle, a run filled to its particle capacity, particles removed
from a run that had them (the step then runs with no particle at all over
buffers that still hold the earlier set) and set again, and particles whose
windows all lie in one row band (the link pass's particle order is then the
order along x alone), and particles near the far end of lattices 65 535
nodes long; the last two also with in-place streaming.  Same bar as the other FP64 parity tests: fields within
1e-12 (velocities on the flow's scale), particles within 1e-12, owner maps
and link sets bit-identical, link fractions within 1e-12 after steps."""
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


def _check(sim, orc, what):
    ef = compare_fields(sim.fields(), orc.fields(), u_floor=U_FF)
    ep = compare_particles(sim.particles(), orc.particles(), u_floor=U_FF)
    nl, dq = compare_links(sim.links(), orc.links(), q_abs=1e-12)
    _say(" ", what, "after", orc.steps_done, "steps:", ef, ep, "links", nl, "max |dq|", dq)
    return nl


def test_one_particle():
    """A single moving, spinning particle (steps 7 and 30: an eager start and
    replays of the captured 6-step cycles)."""
    _say("one particle, 96 x 80")
    kw = dict(C1_PHYS, nx=96, ny=80, max_particles=1, max_diameter=12.0)
    rows = np.array([[47.3, 40.6, 6.0, 0.01, -0.02, 0.0, 0.001]])
    sim, orc = make_pair(**kw)
    sim.set_particles(rows)
    orc.set_particles(rows)
    for n in (7, 23):
        sim.step(n)
        orc.step(n)
        assert _check(sim, orc, "one particle") > 0


def test_particles_at_capacity():
    """As many particles as the run was created for."""
    _say("particles at capacity, 128 x 128")
    n = 9
    kw = dict(C1_PHYS, nx=128, ny=128, max_particles=n, max_diameter=12.0)
    rows = lbm_inputs.rsa_particles(128, 128, n, 12.0, 1.0, 21)
    assert len(rows) == n
    sim, orc = make_pair(**kw)
    sim.set_particles(rows)
    orc.set_particles(rows)
    for steps in (12, 24):
        sim.step(steps)
        orc.step(steps)
        _check(sim, orc, "at capacity")
    with pytest.raises(Exception):
        sim.set_particles(lbm_inputs.rsa_particles(128, 128, n + 1, 10.0, 1.0, 22))


@pytest.mark.parametrize("streaming", ["two_sets", "in_place"])
def test_particles_removed_then_set_again(streaming):
    """Three particles for 10 steps; then none (the particle kernels have no
    work and the buffers still hold the earlier set) for 13 steps; then two
    others.  Each set restarts the fluid at rest on both sides."""
    _say("particles removed and set again, 112 x 72,", streaming)
    kw = dict(C1_PHYS, nx=112, ny=72, max_particles=4, max_diameter=14.0, streaming=streaming)
    sim, orc = make_pair(**kw)
    first = np.array([[20.4, 30.2, 6.0, 0.02, 0.0, 0.0, 0.0],
                      [60.7, 40.9, 7.0, -0.01, 0.01, 0.0, 0.002],
                      [100.1, 20.3, 5.5, 0.0, -0.02, 0.0, 0.0]])
    sim.set_particles(first)
    orc.set_particles(first)
    sim.step(10)
    orc.step(10)
    _check(sim, orc, "three particles")
    none = np.zeros((0, 7))
    sim.set_particles(none)
    orc.set_particles(none)
    sim.step(13)
    orc.step(13)
    assert _check(sim, orc, "no particles") == 0
    fg = sim.fields()
    assert (fg["owner"] == -1).all()
    assert len(sim.particles()) == 0
    second = np.array([[30.2, 50.5, 6.5, 0.0, 0.01, 0.0, -0.001], [85.6, 35.1, 6.0, 0.015, 0.0, 0.0, 0.0]])
    sim.set_particles(second)
    orc.set_particles(second)
    sim.step(9)
    orc.step(9)
    assert _check(sim, orc, "two particles") > 0


def test_particles_in_one_row_band():
    """Eight particles side by side in one row band of a wide channel."""
    _say("one row band, 256 x 64")
    kw = dict(C1_PHYS, nx=256, ny=64, max_particles=8, max_diameter=12.0)
    xs = 16.0 + 31.0 * np.arange(8) + 0.37
    rows = np.stack([xs, np.full(8, 30.6), np.full(8, 5.5), np.zeros(8), np.full(8, -0.01), np.zeros(8),
                     np.zeros(8)], axis=1)
    sim, orc = make_pair(**kw)
    sim.set_particles(rows)
    orc.set_particles(rows)
    sim.step(15)
    orc.step(15)
    _check(sim, orc, "one row band")


@pytest.mark.parametrize("streaming", ["two_sets", "in_place"])
@pytest.mark.parametrize("shape", ["wide", "tall"])
def test_extreme_coordinates(shape, streaming):
    """Lattices at the largest accepted edge (65 535 nodes): link records
    and newborn candidates pack a node as x | y << 16, so particles near
    the far end (and across the periodic seam at x = 65 535) use the top
    bits of both halves."""
    _say("extreme coordinates", shape, streaming)
    if shape == "wide":
        nx, ny = 65535, 48
        rows = np.array([[10.3, 20.6, 6.0, 0.02, 0.0, 0.0, 0.001],
                         [40000.7, 24.2, 6.0, -0.02, 0.01, 0.0, 0.0],
                         [65532.2, 22.9, 6.0, 0.03, 0.0, 0.0, -0.002]])
    else:
        nx, ny = 48, 65535
        rows = np.array([[20.6, 20.2, 6.0, 0.0, -0.02, 0.0, 0.001],
                         [24.2, 40000.6, 6.0, 0.01, 0.02, 0.0, 0.0],
                         [22.9, 65510.3, 6.0, 0.0, 0.03, 0.0, -0.002]])
    kw = dict(C1_PHYS, nx=nx, ny=ny, max_particles=3, max_diameter=12.0, streaming=streaming)
    sim, orc = make_pair(**kw)
    sim.set_particles(rows)
    orc.set_particles(rows)
    lg, lo = sim.links(), orc.links()
    compare_links(lg, lo)
    far = lg["node"] % nx if shape == "wide" else lg["node"] // nx
    assert far.max() >= 65500
    for n in (1, 2):
        sim.step(n)
        orc.step(n)
        _check(sim, orc, shape)
