"""The mixed-precision storage forms against the FP64 oracle.

Small workload (256^2, 20 hot particles d = 12, Pr 0.7, Ra 1e5), 2000 steps:
populations stored as FP32, or as shifted deviations (f_i - w_i rho0,
g_k - w_k T_shift with T_shift = 0, the initial fluid temperature) in
FP32, FP16 or BF16, collided in FP32; momentum exchange, its reduction and the particle update stay FP64.
The test prints the error report (velocity and temperature L2 errors over
nodes fluid in both runs, largest particle displacement, wall Nusselt
numbers at the end and averaged over the run) and asserts the stated bounds.
"""
import numpy as np
import pytest

import lbm_inputs
from oracle import Oracle
from paper_2308_16597_amd import params as P
from tests.gpu_util import form_errors, nusselt_from_fields

pytestmark = pytest.mark.gpu

STEPS, EVERY = 2000, 250
C1 = P.workload_params("small")
ROWS = lbm_inputs.rsa_particles(256, 256, 20, 12.0, 1.0, 1)
# stated bounds: L2 velocity error, L2 temperature error, largest particle
# displacement (lattice units), relative Nusselt error (time-averaged).
# FP32 and FP16: accuracy statements (about twice the errors measured on
# gfx950).  BF16 keeps 8 significand bits, so small temperature increments
# of the cold fluid are largely rounded away (eps_T 0.39 measured): it is a
# throughput form, and its bounds (1.5 x the measured errors: eps_u 0.058,
# eps_T 0.39, dX 0.33, dNu 0.031) only guard that result against change.
BOUNDS = {
    "f32": (1e-4, 1e-5, 1e-3, 1e-4),
    "shift_f32": (1e-4, 1e-5, 1e-3, 1e-4),
    "shift_f16": (2e-3, 1.5e-2, 0.02, 2e-3),
    "shift_bf16": (0.09, 0.6, 0.5, 0.05),
}


@pytest.fixture(scope="module")
def oracle_snapshots():
    okw = {k: v for k, v in C1.items() if k not in ("storage", "max_particles", "max_diameter")}
    o = Oracle(**okw)
    o.set_particles(ROWS)
    snaps = []
    for _ in range(STEPS // EVERY):
        o.step(EVERY)
        f = o.fields()
        snaps.append((f, o.particles(), nusselt_from_fields(f["T"], f["owner"], (0.0, 0.0))))
    return snaps


@pytest.mark.parametrize("form", ["f32", "shift_f32", "shift_f16", "shift_bf16"])
def test_precision_form_error_report(oracle_snapshots, form):
    from paper_2308_16597_amd import lbm
    kw = dict(C1, storage=form, T_shift=0.0)
    sim = lbm.Sim(lbm.lbm_params_default(**kw))
    sim.set_particles(ROWS)
    nu_g, nu_o = [], []
    for fo, po, nuo in oracle_snapshots:
        sim.step(EVERY)
        fg, pg = sim.fields(), sim.particles()
        nu_g.append(nusselt_from_fields(fg["T"], fg["owner"], (0.0, 0.0)))
        nu_o.append(nuo)
    err = form_errors(fg, fo, pg, po)
    nug, nuo = np.array(nu_g), np.array(nu_o)
    err["Nu_final_rel"] = float(np.abs(nug[-1] - nuo[-1]).max() / np.abs(nuo[-1]).max())
    err["Nu_mean_rel"] = float(np.abs(nug.mean(0) - nuo.mean(0)).max() / np.abs(nuo.mean(0)).max())
    print(f"form {form} after {STEPS} steps: {err}", flush=True)
    bu, bT, bX, bN = BOUNDS[form]
    assert err["eps_u"] <= bu and err["eps_T"] <= bT and err["max_dX"] <= bX, err
    assert err["Nu_mean_rel"] <= bN, err
