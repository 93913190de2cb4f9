"""Host-side parameter mapping (no GPU work).

* Physical <-> lattice units through the conversion factors l*, t*, T* the
  paper tabulates for each case (Sec. 2.6): x = x_lat l*, nu = nu_lat l*^2/t*,
  g = g_lat l*/t*^2, beta = beta_lat / T*.
* Dimensionless groups (Sec. 2.6): U_ref = sqrt(g pi d (rho_p/rho_f - 1)/2),
  Re_p = U_ref d / nu, Ar = sqrt(g d^3 (rho_p/rho_f - 1)) / nu,
  Gr_p = g beta dT d^3 / nu^2, and Ra = Pr Gr on a length L0 (Sec. 2.1).
* `from_dimensionless` maps (H, Ra, Pr, d, rho_ratio) to lattice parameters
  at a free-fall Mach number: U_ff = Ma c_s, nu = U_ff H sqrt(Pr/Ra),
  alpha = nu/Pr, g beta dT = U_ff^2 / H (dT = 1), and g from U_ref = U_ff.
  Ra is taken on the channel height H.
"""
import math

CS = 1.0 / math.sqrt(3.0)


def physical_to_lattice(l_star, t_star, T_star=None, nu=None, alpha=None, g=None, beta=None,
                        length=None):
    out = {}
    if nu is not None:
        out["nu"] = nu * t_star / l_star ** 2
    if alpha is not None:
        out["alpha"] = alpha * t_star / l_star ** 2
    if g is not None:
        out["g"] = g * t_star ** 2 / l_star
    if beta is not None:
        out["beta"] = beta * T_star
    if length is not None:
        out["length"] = length / l_star
    return out


def groups(g, d, nu, rho_ratio, beta_dT=None):
    u_ref = math.sqrt(g * math.pi * d * (rho_ratio - 1.0) / 2.0)
    out = dict(U_ref=u_ref, Re_p=u_ref * d / nu,
               Ar=math.sqrt(g * d ** 3 * (rho_ratio - 1.0) / nu ** 2))
    if beta_dT is not None:
        out["Gr_p"] = g * beta_dT * d ** 3 / nu ** 2
    return out


def from_dimensionless(H, Ra, Pr, d, rho_ratio, Ma=0.1):
    u_ff = Ma * CS
    nu = u_ff * H * math.sqrt(Pr / Ra)
    alpha = nu / Pr
    gbeta = u_ff ** 2 / H
    g = 2.0 * u_ff ** 2 / (math.pi * d * (rho_ratio - 1.0))
    return dict(nu=nu, alpha=alpha, gravity=g, beta=gbeta / g)


# Workloads: sizes and physics of the cases the library is exercised on.
WORKLOADS = {
    # 256^2 channel, 20 hot particles of diameter 12, Pr 0.7, Ra 1e5, 200 steps
    "small": dict(nx=256, ny=256, n=20, d=12.0, seed=1, gap=1.0, Ra=1e5, Pr=0.7, rho_ratio=1.5,
                  steps=200),
    # 4000^2 channel, 4800 hot particles of diameter 20, Pr 0.7, Ra 1e8, 2000 steps;
    # seeded outside the repulsion range s = 3 of each other and of the walls
    "paper_scale": dict(nx=4000, ny=4000, n=4800, d=20.0, seed=2, gap=3.0, Ra=1e8, Pr=0.7,
                        rho_ratio=1.5, steps=2000),
    # 4096^2, 64000 particles of diameter 10 (30 % solid), Ra 1e8; seeded
    # outside the repulsion range like the paper-scale workload (at gaps of 1
    # the contact spring accelerates particles past 0.5 lattice units per
    # step within 20 steps)
    "dense": dict(nx=4096, ny=4096, n=64000, d=10.0, seed=5, gap=3.0, Ra=1e8, Pr=0.7,
                  rho_ratio=1.5, steps=1000),
    # The paper's benchmark case (Sec. 2.6.3, the 4,800-particle sedimentation
    # and its parameter table): closed 4000^2 cavity with cold walls, 60 lines
    # of 80 hot particles of diameter 40 at 50 apart in the upper part
    # (37.7 % solid), rho_p/rho_f = 1.1, Pr 5, Gr_p 60, lattice parameters
    # as tabulated; 6000 steps in the paper's timing.
    "e4_cavity": dict(nx=4000, ny=4000, n=4800, d=40.0, layout="grid", rows=60, cols=80,
                      spacing=50.0, rho_ratio=1.1, closed=True, steps=6000,
                      lattice=dict(nu=0.01, alpha=0.002, gravity=7.84e-6, beta=1.20e-2)),
    # The paper's elliptical-particle case (Sec. 2.6.2 and its parameter
    # table): closed 1000 x 2000 cavity with cold walls, 129 hot ellipses of
    # axes 50 x 25 (6.3 % solid) in a circular cluster centred at
    # (0.5 W, 0.75 H): one in the centre and rings of 6, 12, 18, 24, 31, 37
    # at 60 apart, major axes horizontal; rho_p/rho_f = 1.5, Pr 5, Gr_p 10.
    "e3_ellipses": dict(nx=1000, ny=2000, n=129, d=50.0, d_minor=25.0, layout="rings",
                        centre=(499.5, 1499.5), rings=(6, 12, 18, 24, 31, 37), ring_spacing=60.0,
                        rho_ratio=1.5, closed=True, steps=2000,
                        lattice=dict(nu=0.01, alpha=0.002, gravity=9.8e-7, beta=8.16e-3)),
}


def workload_params(name, storage=0):
    """Parameter dict (lbm_params field names) of a named workload: hot
    particles (T = 1) in cold fluid (T = 0) between cold walls, gravity -y,
    repulsion on; periodic x, or a closed cavity with cold side walls.  The
    lattice parameters are the tabulated ones where the workload gives them,
    else mapped from (Ra, Pr) on the height."""
    w = WORKLOADS[name]
    phys = w.get("lattice") or from_dimensionless(w["ny"], w["Ra"], w["Pr"], w["d"], w["rho_ratio"])
    closed = bool(w.get("closed"))
    out = dict(nx=w["nx"], ny=w["ny"], storage=storage, rho0=1.0, nu=phys["nu"],
               alpha=phys["alpha"], gravity=phys["gravity"], beta=phys["beta"], T_ref=0.0,
               wall_T=(0.0, 0.0), wall_ux=(0.0, 0.0), T_fluid0=0.0, particle_T=1.0,
               rho_ratio=w["rho_ratio"], repulsion=1, rep_eps=1e-3, rep_range=3.0,
               max_particles=w["n"], max_diameter=w["d"], periodic_x=0 if closed else 1)
    if closed:
        out["side_T"] = (0.0, 0.0)
    return out


def mlups(mesh_size, steps, seconds):
    """Million lattice updates per second over the whole mesh, solid nodes
    included (Sec. 3): mesh size x iteration steps / (running time x 10^6)."""
    return mesh_size * steps / (seconds * 1e6)
