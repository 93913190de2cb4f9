/*
 * ptlbm_oracle.h -- plain, slow, single-threaded FP64 CPU oracle of the
 * particle-resolved thermal lattice Boltzmann method of Xu & Li,
 * "Particle-resolved thermal lattice Boltzmann simulation using OpenACC on
 * multi-GPUs" (arXiv 2308.16597).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.  Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load it.  It shares no source, header or table with the GPU library.
 *
 * Conventions (Sec. 2 of the paper; readings of silent points are listed in
 * the design notes of the repository):
 *   node (i, j) sits at (x, y) = (i, j); flat walls are halfway, at y = -1/2
 *   and y = ny - 1/2; x is periodic.  Node index k = j * nx + i.
 *   D2Q9 velocities e0..e8 = (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1) (-1,1)
 *   (-1,-1) (1,-1); D2Q5 uses e0..e4.
 *   Particles: input rows of 7 doubles (x, y, r, ux, uy, theta, omega);
 *   output rows of 10 doubles (the same 7, then Fx, Fy, Tz of the last step's
 *   momentum exchange, Sec. 2.4, Eqs. (13)-(14)).
 * All arithmetic is IEEE binary64; the library is built with
 * -ffp-contract=off so that no multiply-add is fused.
 */
#ifndef PTLBM_ORACLE_H
#define PTLBM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EUNSTABLE = -5 };

typedef struct {
    int32_t nx, ny;
    int32_t periodic_x;   /* 1: periodic; 0: side walls at x = -1/2 and nx - 1/2 (static,
                             no-slip, Dirichlet side_T) -- the closed cavity */
    int32_t periodic_y;   /* 0: flat walls at y (required with particles); 1: periodic */
    double rho0;          /* reference density */
    double nu;            /* kinematic viscosity (lattice units) */
    double alpha;         /* thermal diffusivity (lattice units) */
    double gravity;       /* magnitude of g; gravity points along -y */
    double beta;          /* thermal expansion coefficient */
    double T_ref;         /* T0 of the Boussinesq force */
    double body_fx;       /* uniform extra force density along +x */
    double s_e, s_eps, s_q;   /* D2Q9 free rates; <= 0 selects the default */
    double a_T;           /* D2Q5 equilibrium constant a of n_e^eq = a T */
    double sT_e, sT_p;    /* D2Q5 free rates; <= 0 selects the default */
    double wall_T[2];     /* Dirichlet temperature of the [bottom, top] wall */
    double wall_ux[2];    /* tangential velocity of the [bottom, top] wall */
    double T_fluid0;      /* initial fluid temperature */
    double particle_T;    /* particle surface temperature T_w */
    double rho_ratio;     /* particle / fluid density ratio */
    int32_t repulsion;    /* 1: spring repulsion on (Sec. 2.4, Eq. (15)) */
    double rep_eps;       /* stiffness epsilon_w */
    double rep_range;     /* threshold distance s */
    double side_T[2];     /* Dirichlet temperature of the [left, right] side wall */
} orc_params;

typedef struct orc_sim orc_sim;

/* Whole-lattice simulation. */
int  orc_create(const orc_params* p, orc_sim** out);
void orc_destroy(orc_sim* s);
const char* orc_last_error(const orc_sim* s);
/* Replace the particles and re-initialise the run: fluid at rest at rho0 and
 * T_fluid0 (equilibrium), step counter 0.  n may be 0. */
int  orc_set_particles(orc_sim* s, int32_t n, const double* rows7);
/* The same for ellipses (Sec. 2.6.2): rows of (x, y, a, b, ux, uy, theta,
 * omega), a the semi-axis along the body axis at angle theta from +x, b the
 * semi-axis across it, 1 < b <= a (b == a is a circle). */
int  orc_set_particles_ellipse(orc_sim* s, int32_t n, const double* rows8);
/* Re-initialise fluid nodes to f^eq(rho, u), g^eq(T, u) from the given fields
 * (nx*ny each, row-major); particles are kept; step counter 0. */
int  orc_set_equilibrium(orc_sim* s, const double* rho, const double* ux,
                         const double* uy, const double* T);
int  orc_step(orc_sim* s, int32_t nsteps);
int64_t orc_steps_done(const orc_sim* s);
/* Pre-collision macroscopics at t_n (Sec. 2.1): rho, u with the half force,
 * T; NaN inside solids.  owner: -1 fluid, else the particle index.  Any
 * pointer may be NULL. */
int  orc_read_fields(const orc_sim* s, double* rho, double* ux, double* uy,
                     double* T, int32_t* owner);
/* Pre-collision populations at t_n (9*nx*ny, 5*nx*ny, direction-major). */
int  orc_read_populations(const orc_sim* s, double* f, double* g);
int  orc_read_particles(const orc_sim* s, double* rows10, int32_t* n);
/* The fluid-particle links of the current state (Sec. 3): every fluid node
 * x_f and direction i with x_f + e_i inside particle p, in ascending (node,
 * direction) order, with the link fraction q. */
int  orc_read_links(const orc_sim* s, int32_t* node, int32_t* dir, int32_t* particle,
                    double* q, int64_t cap, int64_t* n_out);
/* Nusselt number at the two flat walls from the current temperature field. */
int  orc_nusselt(const orc_sim* s, double* nu_bottom, double* nu_top);

/* Single-node pieces of the method, exported for unit tests. */
void orc_collide_node(const orc_sim* s, const double f[9], const double g[5],
                      double fo[9], double go[5], double macro[4]);
double orc_link_q(double dx, double dy, double r, int32_t i);
double orc_link_q_ellipse(double dx, double dy, double a, double b, double theta, int32_t i);
int32_t orc_inside_shape(double dx, double dy, double a, double b, double theta);
int32_t orc_refill_direction(double dx, double dy, double a, double b, double theta);
double orc_bouzidi(double q, int32_t i, double fi_xf, double fi_xf1, double fi_xf2,
                   double fib_xf, double fib_xf1, int32_t have1, int32_t have2,
                   double rho0, double uwx, double uwy);
double orc_thermal_link(double q, int32_t i, double gi_xf, double gi_xf1, double gib_xf,
                        int32_t have1, double w5_i, double Tw);
void orc_repulsion_pair(const orc_params* p, double xp, double yp, double rp,
                        double xq, double yq, double rq, double out[2]);
void orc_repulsion_walls(const orc_params* p, double xp, double yp, double rp, double out[2]);
void orc_repulsion_pair_ellipse(const orc_params* p, double xp, double yp, double ap, double bp,
                                double thp, double xq, double yq, double aq, double bq,
                                double thq, double out[2]);
void orc_repulsion_walls_ellipse(const orc_params* p, double xp, double yp, double a, double b,
                                 double theta, double out[2]);
void orc_newton_euler(const orc_params* p, const double state7[7], double Fx, double Fy,
                      double Tz, double out7[7]);
void orc_newton_euler_ellipse(const orc_params* p, const double state7[7], double b, double Fx,
                              double Fy, double Tz, double out7[7]);
void orc_refill_node(const orc_sim* s, int32_t K, const double* f1, const double* f2,
                     const double* f3, double uwx, double uwy, double fo[9], double go[5]);
void orc_rates(const orc_sim* s, double s9[9], double s5[5], double w5[5]);

#ifdef __cplusplus
}
#endif
#endif
