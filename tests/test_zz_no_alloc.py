"""lbm_step_many_noalloc, the batched step for callers that cannot allocate
device memory: through the C ABI it gives bit for bit what lbm_step_many
gives on the same runs, on two calls in a row (the second over fewer,
smaller runs, so the fixed array keeps the first call's larger tables), and
it rejects calls whose tables exceed its fixed array before enqueuing work."""
import numpy as np
import pytest

import lbm_inputs
from paper_2308_16597_amd import lbm

pytestmark = pytest.mark.gpu

FAST = np.array([[40.3, 30.2, 6.0, 0.05, -0.02, 0.0, 0.004],
                 [100.6, 50.5, 7.0, -0.06, 0.03, 0.0, -0.005],
                 [1.2, 25.0, 5.0, -0.04, 0.0, 0.0, 0.0],
                 [70.0, 70.5, 4.5, 0.0, -0.03, 0.0, 0.006]])


def _say(*a):
    print(*a, flush=True)


def _specs(storage):
    base = dict(storage=lbm.STORE[storage], T_shift=0.0, nu=0.05, alpha=0.04, gravity=1e-4,
                beta=0.5, particle_T=1.0, rho_ratio=2.0)
    return [
        (dict(base, nx=128, ny=96, max_particles=4, max_diameter=14.0), FAST, None),
        (dict(base, nx=96, ny=64, wall_T=(0.7, 0.1), wall_ux=(0.01, 0.0)), None,
         lbm_inputs.smooth_fields(96, 64, seed=3)),
        (dict(base, nx=160, ny=80, max_particles=6, max_diameter=8.0),
         lbm_inputs.rsa_particles(160, 80, 6, 8.0, 3.0, 11), None),
        (dict(base, nx=256, ny=192, max_particles=12, max_diameter=16.0),
         lbm_inputs.rsa_particles(256, 192, 12, 16.0, 3.0, 5), None),
    ]


def _make(spec):
    kw, rows, fields = spec
    sim = lbm.Sim(lbm.lbm_params_default(**kw))
    if rows is not None:
        sim.set_particles(rows)
    if fields is not None:
        sim.set_equilibrium(*fields)
    return sim


def _same(a, b, what):
    fa, fb = a.fields(), b.fields()
    for k in ("rho", "ux", "uy", "T", "owner"):
        np.testing.assert_array_equal(fa[k], fb[k], err_msg=f"{what}: {k}")
    np.testing.assert_array_equal(a.particles(), b.particles(), err_msg=f"{what}: particles")
    assert a.stats()["steps"] == b.stats()["steps"]


@pytest.mark.parametrize("storage", ["f64", "shift_bf16"])
def test_noalloc_equals_step_many_on_two_calls(storage):
    specs = _specs(storage)
    ref = [_make(s) for s in specs]
    new = [_make(s) for s in specs]
    # call 1: four runs, unequal counts (several segments, one of a single run)
    c1 = [17, 9, 30, 12]
    _say(storage, "call 1: four runs", c1)
    lbm.lbm_step_many([s.handle for s in ref], c1)
    lbm.lbm_step_many_noalloc([s.handle for s in new], c1)
    for r, (a, b) in enumerate(zip(ref, new)):
        _same(a, b, f"call 1 run {r}")
    # call 2: a smaller input, the two smallest runs only
    c2 = [11, 6]
    _say(storage, "call 2: two runs", c2)
    lbm.lbm_step_many([ref[1].handle, ref[2].handle], c2)
    lbm.lbm_step_many_noalloc([new[1].handle, new[2].handle], c2)
    for r in (1, 2):
        _same(ref[r], new[r], f"call 2 run {r}")
    # the runs left out keep their state
    for r in (0, 3):
        _same(ref[r], new[r], f"untouched run {r}")
    for s in ref + new:
        s.close()


def test_noalloc_rejects_tables_beyond_its_array():
    # 17 runs of 4096^2 (FP16 in place: 65 536 lattice blocks each) need
    # 17 x 512 KiB of block map: more than the 8 MiB array
    kw = dict(nx=4096, ny=4096, storage=lbm.STORE["shift_f16"], streaming="in_place")
    sims = [lbm.Sim(lbm.lbm_params_default(**kw)) for _ in range(17)]
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_step_many_noalloc([s.handle for s in sims], [1] * 17)
    assert e.value.rc == lbm.LBM_EINVAL and "fixed array" in str(e.value)
    for s in sims:
        assert s.stats()["steps"] == 0
        s.close()
    # more than 64 runs in one call
    small = [lbm.Sim(lbm.lbm_params_default(nx=8, ny=8)) for _ in range(65)]
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_step_many_noalloc([s.handle for s in small], [1] * 65)
    assert e.value.rc == lbm.LBM_EINVAL
    for s in small:
        s.close()
