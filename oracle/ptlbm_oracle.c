/*
 * ptlbm_oracle.c -- plain single-threaded FP64 CPU oracle of the
 * particle-resolved thermal LBM of Xu & Li (arXiv 2308.16597).
 *
 * TEST INFRASTRUCTURE ONLY: it checks the GPU path and is never part of it.
 *
 * Every function follows the paper's definitions in the paper's order:
 *   Sec. 2.1  Eqs. (5)-(6): D2Q9 MRT for f with a forcing term, D2Q5 MRT for g,
 *             macroscopic rho, u (with the half force), T and the buoyancy
 *             force F = rho g beta (T - T0) y^.
 *   Sec. 2.2  Eqs. (7)-(8): Newton-Euler motion of the rigid particles, same
 *             time step as the fluid.
 *   Sec. 2.3  Eqs. (9)-(10): quadratic interpolated bounce-back (Bouzidi) with
 *             a moving wall; Eqs. (11)-(12): the thermal curved-wall condition.
 *   Sec. 2.4  Eqs. (13)-(14): Galilean-invariant momentum exchange force and
 *             torque; Eq. (15): spring repulsion.
 *   Sec. 2.5  Eq. (16): normal extrapolation refilling with a velocity
 *             constraint; Eq. (17): equilibrium refilling of g.
 *   Sec. 3    links between fluid nodes and particles, collected anew every
 *             step.
 *   Sec. 2.6.2 and App. A: particles may be ellipses; the solid test, the link
 *             fraction, the refill normal, the repulsion gaps, mass and
 *             inertia then follow the ellipse (readings at the point of use).
 * Where the paper is silent (the MRT matrices, equilibria and forcing moments,
 * fallbacks when an interpolation stencil leaves the fluid, wall handling,
 * the integrator) the reading used is stated at the point of use.
 *
 * There is no blocking, fusion or reordering: each step runs the phases one
 * after the other over whole arrays.  The only shortcut is that the solid
 * test of a particle is evaluated over a bounding box that contains its shape,
 * which cannot change the result.
 */
#include "ptlbm_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static const double ORC_PI = 3.14159265358979323846;
#define PSTRIDE 11

/* ---------------------------------------------------------------- lattice */

/* D2Q9 velocities and weights; D2Q5 takes the first five velocities. */
static const int EX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double W9[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const double CS2 = 1.0 / 3.0;

/* Moment matrix of the D2Q9 MRT model (the paper defers M to earlier work;
 * reading: the orthogonal basis of Lallemand & Luo 2000, rows rho, e, eps,
 * j_x, q_x, j_y, q_y, p_xx, p_xy). */
static const double M9[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1},
};

/* Moment matrix of the D2Q5 MRT model (reading: rows T, j_x, j_y, e, p_xx). */
static const double N5[5][5] = {
    {1, 1, 1, 1, 1},
    {0, 1, 0, -1, 0},
    {0, 0, 1, 0, -1},
    {-4, 1, 1, 1, 1},
    {0, 1, -1, 1, -1},
};

/* ------------------------------------------------------------------ state */

struct orc_sim {
    orc_params p;
    int nx, ny;
    long n;                 /* nx * ny */
    double s9[9], s5[5];    /* diagonal relaxation matrices S and Q */
    double w5[5];           /* D2Q5 weights implied by a_T */
    double M9inv[9][9], N5inv[5][5];
    double *f, *g;          /* pre-collision populations at t_n, [dir][node] */
    double *fp, *gp;        /* post-collision populations */
    int32_t *owner, *owner_new;
    int np;
    double *P;              /* particles, np rows of PSTRIDE: x, y, a, u_x, u_y,
                               theta, Omega, F_x, F_y, T_z, b */
    int64_t steps;
    char err[256];
};

static void set_err(orc_sim* s, const char* msg) {
    if (s) snprintf(s->err, sizeof s->err, "%s", msg);
}

/* Inverse of a matrix with mutually orthogonal rows: M^-1 = M^T diag(1/|row|^2). */
static void orthogonal_inverse(int n, const double* M, double* Minv) {
    for (int a = 0; a < n; ++a) {
        double nrm = 0.0;
        for (int i = 0; i < n; ++i) nrm += M[a * n + i] * M[a * n + i];
        for (int i = 0; i < n; ++i) Minv[i * n + a] = M[a * n + i] / nrm;
    }
}

/* Relaxation rates.  s_nu follows from nu = cs^2 (1/s_nu - 1/2); the defaults
 * of the free rates are readings: s_e = s_eps = s_nu and s_q such that
 * (1/s_nu - 1/2)(1/s_q - 1/2) = 3/16; for D2Q5, alpha = cs_T^2 (1/s_a - 1/2)
 * with cs_T^2 = (4 + a)/10 and the free rates such that
 * (1/s_a - 1/2)(1/s_T - 1/2) = 1/4. */
static void derive_rates(orc_sim* s) {
    const orc_params* p = &s->p;
    double s_nu = 1.0 / (p->nu / CS2 + 0.5);
    double s_e = p->s_e > 0 ? p->s_e : s_nu;
    double s_eps = p->s_eps > 0 ? p->s_eps : s_nu;
    double lam_nu = 1.0 / s_nu - 0.5;
    double s_q = p->s_q > 0 ? p->s_q : 1.0 / (0.5 + (3.0 / 16.0) / lam_nu);
    double rates9[9] = {0.0, s_e, s_eps, 1.0, s_q, 1.0, s_q, s_nu, s_nu};
    memcpy(s->s9, rates9, sizeof rates9);

    double a = p->a_T;
    double w0 = (1.0 - a) / 5.0, wk = (4.0 + a) / 20.0;
    double w5[5] = {w0, wk, wk, wk, wk};
    memcpy(s->w5, w5, sizeof w5);
    double cs2T = (4.0 + a) / 10.0;
    double s_a = 1.0 / (p->alpha / cs2T + 0.5);
    double lam_a = 1.0 / s_a - 0.5;
    double s_T = 1.0 / (0.5 + 0.25 / lam_a);
    double sTe = p->sT_e > 0 ? p->sT_e : s_T;
    double sTp = p->sT_p > 0 ? p->sT_p : s_T;
    double rates5[5] = {0.0, s_a, s_a, sTe, sTp};
    memcpy(s->s5, rates5, sizeof rates5);
}

void orc_rates(const orc_sim* s, double s9[9], double s5[5], double w5[5]) {
    if (s9) memcpy(s9, s->s9, sizeof s->s9);
    if (s5) memcpy(s5, s->s5, sizeof s->s5);
    if (w5) memcpy(w5, s->w5, sizeof s->w5);
}

/* ------------------------------------------------------------ equilibria */

/* Second-order D2Q9 equilibrium (its moments are the m^eq of the MRT model). */
static void feq9(double rho, double ux, double uy, double out[9]) {
    double usq = ux * ux + uy * uy;
    for (int i = 0; i < 9; ++i) {
        double eu = EX[i] * ux + EY[i] * uy;
        out[i] = W9[i] * rho * (1.0 + eu / CS2 + (eu * eu) / (2.0 * CS2 * CS2) - usq / (2.0 * CS2));
    }
}

/* D2Q5 equilibrium with moments (T, u_x T, u_y T, a T, 0). */
static void geq5(const orc_sim* s, double T, double ux, double uy, double out[5]) {
    out[0] = s->w5[0] * T;
    for (int k = 1; k < 5; ++k) out[k] = s->w5[k] * T + 0.5 * T * (EX[k] * ux + EY[k] * uy);
}

/* --------------------------------------------------------------- collide */

/* One node of Eqs. (5)-(6), Sec. 2.1.  macro = (rho, ux, uy, T) with u
 * including the half force.  F = rho g beta (T - T0) y^ + (body_fx, 0); the
 * buoyancy is taken along +y so that hot fluid rises against gravity along -y.
 * The forcing term of Eq. (5) is read as the moment-space form
 * M^-1 (I - S/2) Fbar (Guo-type forcing). */
void orc_collide_node(const orc_sim* s, const double f[9], const double g[5],
                      double fo[9], double go[5], double macro[4]) {
    const orc_params* p = &s->p;
    double rho = 0.0, jx = 0.0, jy = 0.0, T = 0.0;
    for (int i = 0; i < 9; ++i) {
        rho += f[i];
        jx += EX[i] * f[i];
        jy += EY[i] * f[i];
    }
    for (int k = 0; k < 5; ++k) T += g[k];
    double Fx = p->body_fx;
    double Fy = rho * p->gravity * p->beta * (T - p->T_ref);
    double ux = (jx + 0.5 * Fx) / rho;
    double uy = (jy + 0.5 * Fy) / rho;
    if (macro) {
        macro[0] = rho;
        macro[1] = ux;
        macro[2] = uy;
        macro[3] = T;
    }

    /* flow: m = M f; f+ = f - M^-1 [ S (m - m^eq) - (I - S/2) Fbar ] */
    double m[9];
    for (int a = 0; a < 9; ++a) {
        m[a] = 0.0;
        for (int i = 0; i < 9; ++i) m[a] += M9[a][i] * f[i];
    }
    double usq = ux * ux + uy * uy;
    double meq[9] = {rho,
                     -2.0 * rho + 3.0 * rho * usq,
                     rho - 3.0 * rho * usq,
                     rho * ux,
                     -rho * ux,
                     rho * uy,
                     -rho * uy,
                     rho * (ux * ux - uy * uy),
                     rho * ux * uy};
    double uF = ux * Fx + uy * Fy;
    double Fb[9] = {0.0,
                    6.0 * uF,
                    -6.0 * uF,
                    Fx,
                    -Fx,
                    Fy,
                    -Fy,
                    2.0 * (ux * Fx - uy * Fy),
                    ux * Fy + uy * Fx};
    double dm[9];
    for (int a = 0; a < 9; ++a)
        dm[a] = s->s9[a] * (m[a] - meq[a]) - (1.0 - 0.5 * s->s9[a]) * Fb[a];
    for (int i = 0; i < 9; ++i) {
        double acc = 0.0;
        for (int a = 0; a < 9; ++a) acc += s->M9inv[i][a] * dm[a];
        fo[i] = f[i] - acc;
    }

    /* heat: n = N g; g+ = g - N^-1 Q (n - n^eq) */
    double nm[5];
    for (int a = 0; a < 5; ++a) {
        nm[a] = 0.0;
        for (int k = 0; k < 5; ++k) nm[a] += N5[a][k] * g[k];
    }
    double neq[5] = {T, ux * T, uy * T, p->a_T * T, 0.0};
    double dn[5];
    for (int a = 0; a < 5; ++a) dn[a] = s->s5[a] * (nm[a] - neq[a]);
    for (int k = 0; k < 5; ++k) {
        double acc = 0.0;
        for (int a = 0; a < 5; ++a) acc += s->N5inv[k][a] * dn[a];
        go[k] = g[k] - acc;
    }
}

/* ------------------------------------------------------------- geometry */

static int wrapi(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

/* Node-minus-centre offset along x with the minimum image on a periodic
 * axis: the plain difference, shifted by one period when it exceeds half. */
static double min_image(double d, int n, int periodic) {
    if (!periodic) return d;
    double h = 0.5 * n;
    if (d > h) return d - n;
    if (d < -h) return d + n;
    return d;
}

/* Particle shapes (Sec. 2.6.2 uses ellipses, the other cases circles): a
 * record holds the semi-axis a along the body axis at angle theta from +x
 * and the semi-axis b across it; b == a is a circle, evaluated with the
 * plain circle formulas.  (u, v) are the body-frame coordinates of an offset
 * (dx, dy): u along the body axis. */
static void to_body(double dx, double dy, double c, double s, double* u, double* v) {
    *u = dx * c + dy * s;
    *v = dy * c - dx * s;
}

/* Offset (dx, dy) from the centre inside the shape: dx^2 + dy^2 <= r^2 for a
 * circle; (u/a)^2 + (v/b)^2 <= 1 for an ellipse, evaluated as
 * b^2 u^2 + a^2 v^2 <= a^2 b^2.  On the boundary counts as inside. */
int32_t orc_inside_shape(double dx, double dy, double a, double b, double theta) {
    if (a == b) return dx * dx + dy * dy <= a * a;
    double u, v;
    to_body(dx, dy, cos(theta), sin(theta), &u, &v);
    return (u * u) * (b * b) + (v * v) * (a * a) <= (a * a) * (b * b);
}

/* A node is inside particle p when its offset from X_p (minimum image on a
 * periodic axis) is inside the shape (a node exactly on the boundary counts
 * as solid, so the link fraction q lies in (0, 1]). */
static int inside(const orc_sim* s, int i, int j, const double* P) {
    double dx = min_image((double)i - P[0], s->nx, s->p.periodic_x);
    double dy = min_image((double)j - P[1], s->ny, s->p.periodic_y);
    return orc_inside_shape(dx, dy, P[2], P[10], P[5]);
}

/* owner = lowest particle index whose disk holds the node, else -1. */
static void compute_owner(const orc_sim* s, int32_t* owner) {
    for (long k = 0; k < s->n; ++k) owner[k] = -1;
    for (int q = 0; q < s->np; ++q) {
        const double* P = s->P + PSTRIDE * q;   /* the box of half-width a holds the shape */
        int i0 = (int)floor(P[0] - P[2]), i1 = (int)floor(P[0] + P[2]) + 1;
        int j0 = (int)floor(P[1] - P[2]), j1 = (int)floor(P[1] + P[2]) + 1;
        for (int jj = j0; jj <= j1; ++jj) {
            int j = jj;
            if (s->p.periodic_y) j = wrapi(jj, s->ny);
            else if (jj < 0 || jj >= s->ny) continue;
            for (int ii = i0; ii <= i1; ++ii) {
                int i = ii;
                if (s->p.periodic_x) i = wrapi(ii, s->nx);
                else if (ii < 0 || ii >= s->nx) continue;
                long k = (long)j * s->nx + i;
                if (owner[k] >= 0) continue;
                if (inside(s, i, j, P)) owner[k] = q;
            }
        }
    }
}

/* Link fraction q = |x_f - x_w| / |x_f - x_b| (Sec. 2.3) for the circle of
 * radius r: (dx, dy) = x_f - X_c, x_w = x_f + q e_i is the nearer crossing of
 * the segment x_f -> x_f + e_i with the circle, the smaller root of
 * |d + t e_i|^2 = r^2.  Rounding is clamped so that q stays in [0, 1]. */
double orc_link_q(double dx, double dy, double r, int32_t i) {
    double a = (double)(EX[i] * EX[i] + EY[i] * EY[i]);
    double b = dx * EX[i] + dy * EY[i];
    double c = (dx * dx + dy * dy) - r * r;
    double disc = b * b - a * c;
    if (disc < 0.0) disc = 0.0;
    double q = (-b - sqrt(disc)) / a;
    if (q < 0.0) q = 0.0;
    if (q > 1.0) q = 1.0;
    return q;
}

/* The same for the ellipse of semi-axes a, b at angle theta (a circle when
 * b == a): in body coordinates the smaller root of
 * b^2 (u + t e_u)^2 + a^2 (v + t e_v)^2 = a^2 b^2. */
double orc_link_q_ellipse(double dx, double dy, double a, double b, double theta, int32_t i) {
    if (a == b) return orc_link_q(dx, dy, a, i);
    double c = cos(theta), s = sin(theta), u, v, eu, ev;
    to_body(dx, dy, c, s, &u, &v);
    to_body((double)EX[i], (double)EY[i], c, s, &eu, &ev);
    double a2 = a * a, b2 = b * b;
    double A = b2 * (eu * eu) + a2 * (ev * ev);
    double B = b2 * (u * eu) + a2 * (v * ev);
    double C = (b2 * (u * u) + a2 * (v * v)) - a2 * b2;
    double disc = B * B - A * C;
    if (disc < 0.0) disc = 0.0;
    double q = (-B - sqrt(disc)) / A;
    if (q < 0.0) q = 0.0;
    if (q > 1.0) q = 1.0;
    return q;
}

/* ---------------------------------------------------- boundary schemes */

/* Interpolated bounce-back, Sec. 2.3 Eqs. (9)-(10): the unknown f_ibar(x_f,
 * t + dt) for the link (x_f, i) crossing a wall moving at u_w.
 *   fi_xf  = f_i^+(x_f),  fi_xf1 = f_i^+(x_f - e_i),  fi_xf2 = f_i^+(x_f - 2e_i)
 *   fib_xf = f_ibar^+(x_f), fib_xf1 = f_ibar^+(x_f - e_i)
 *   have1, have2: whether x_f - e_i, x_f - 2e_i are fluid nodes.
 * The wall term 2 w_i rho0 (e_ibar . u_w) / cs^2 uses the D2Q9 weight and
 * rho0.  When a stencil node is not fluid (the paper is silent) the scheme
 * drops to Bouzidi's linear interpolation, then to halfway bounce-back. */
double orc_bouzidi(double q, int32_t i, double fi_xf, double fi_xf1, double fi_xf2,
                   double fib_xf, double fib_xf1, int32_t have1, int32_t have2,
                   double rho0, double uwx, double uwy) {
    int ib = OPP[i];
    double wall = 2.0 * W9[i] * rho0 * (EX[ib] * uwx + EY[ib] * uwy) / CS2;
    if (q <= 0.5) {
        if (have1 && have2)
            return q * (2.0 * q + 1.0) * fi_xf + (1.0 - 4.0 * q * q) * fi_xf1 -
                   q * (1.0 - 2.0 * q) * fi_xf2 + wall;
        if (have1) return 2.0 * q * fi_xf + (1.0 - 2.0 * q) * fi_xf1 + wall;
        return fi_xf + wall;
    }
    if (have1)
        return 1.0 / (q * (2.0 * q + 1.0)) * fi_xf + (2.0 * q - 1.0) / q * fib_xf -
               (2.0 * q - 1.0) / (2.0 * q + 1.0) * fib_xf1 +
               1.0 / (q * (2.0 * q + 1.0)) * wall;
    return 1.0 / (2.0 * q) * fi_xf + (2.0 * q - 1.0) / (2.0 * q) * fib_xf + wall / (2.0 * q);
}

/* Thermal curved-wall condition, Sec. 2.3 Eqs. (11)-(12):
 *   g_ibar(x_f) = c1 g_i^+(x_f) + c2 g_i^+(x_f - e_i) + c3 g_ibar^+(x_f)
 *                 + c4 (2 w_i T_w),
 * c1 = -1, c2 = c3 = (2q - 1)/(2q + 1), c4 = 2/(2q + 1); w_i is read as the
 * D2Q5 weight.  Without the node x_f - e_i it falls back to the
 * anti-bounce-back value of q = 1/2. */
double orc_thermal_link(double q, int32_t i, double gi_xf, double gi_xf1, double gib_xf,
                        int32_t have1, double w5_i, double Tw) {
    (void)i;
    if (!have1) return -gi_xf + 2.0 * w5_i * Tw;
    double c1 = -1.0;
    double c2 = (2.0 * q - 1.0) / (2.0 * q + 1.0);
    double c3 = (2.0 * q - 1.0) / (2.0 * q + 1.0);
    double c4 = 2.0 / (2.0 * q + 1.0);
    return (c1 * gi_xf + c2 * gi_xf1 + c3 * gib_xf) + c4 * (2.0 * w5_i * Tw);
}

/* ------------------------------------------------------ particle motion */

/* Distance from the centre to the boundary of a shape along the unit
 * direction (nx_, ny_): r for a circle; for an ellipse
 * a b / sqrt(b^2 n_u^2 + a^2 n_v^2) with (n_u, n_v) the direction in body
 * coordinates. */
static double radial_extent(double a, double b, double theta, double nx_, double ny_) {
    if (a == b) return a;
    double nu, nv;
    to_body(nx_, ny_, cos(theta), sin(theta), &nu, &nv);
    return (a * b) / sqrt((b * b) * (nu * nu) + (a * a) * (nv * nv));
}

/* Half-extents of a shape along x and along y (the distance from the centre
 * to its supporting lines): r for a circle; sqrt(a^2 c^2 + b^2 s^2) along x
 * and sqrt(a^2 s^2 + b^2 c^2) along y for an ellipse at angle theta. */
static void half_extents(double a, double b, double theta, double* hx, double* hy) {
    if (a == b) {
        *hx = a;
        *hy = a;
        return;
    }
    double c = cos(theta), s = sin(theta);
    *hx = sqrt((a * a) * (c * c) + (b * b) * (s * s));
    *hy = sqrt((a * a) * (s * s) + (b * b) * (c * c));
}

/* Radius of the disk of equal area: r for a circle, sqrt(a b) for an
 * ellipse (the force scale C of Eq. (15) is the particle's immersed weight
 * pi r^2 (rho_p - rho_f) g). */
static double area_radius(double a, double b) { return a == b ? a : sqrt(a * b); }

/* Spring repulsion, Sec. 2.4 Eq. (15), on particle p from particle q:
 * |x_s| is the surface gap along the centre line, |X_p - X_q| minus the two
 * shapes' extents along it (r_p + r_q for circles), the direction is the
 * centre line from q to p, s = rep_range, eps = rep_eps, and the force scale
 * C = pi r^2 (rho_p - rho_f) g is taken with r^2 = r_p r_q (equal-area radii)
 * so that the pair forces are equal and opposite. */
void orc_repulsion_pair_ellipse(const orc_params* p, double xp, double yp, double ap, double bp,
                                double thp, double xq, double yq, double aq, double bq,
                                double thq, double out[2]) {
    out[0] = 0.0;
    out[1] = 0.0;
    double dx = min_image(xp - xq, p->nx, p->periodic_x);
    double dy = yp - yq;
    double dist = sqrt(dx * dx + dy * dy);
    double ep = radial_extent(ap, bp, thp, dx / dist, dy / dist);
    double eq = radial_extent(aq, bq, thq, dx / dist, dy / dist);
    double gap = dist - ep - eq;
    if (gap > p->rep_range) return;
    double C = ORC_PI * (area_radius(ap, bp) * area_radius(aq, bq)) * (p->rho_ratio - 1.0) * p->rho0 *
               p->gravity;
    double t = (gap - p->rep_range) / p->rep_range;
    double mag = C / p->rep_eps * (t * t);
    out[0] = mag * (dx / dist);
    out[1] = mag * (dy / dist);
}

void orc_repulsion_pair(const orc_params* p, double xp, double yp, double rp,
                        double xq, double yq, double rq, double out[2]) {
    orc_repulsion_pair_ellipse(p, xp, yp, rp, rp, 0.0, xq, yq, rq, rq, 0.0, out);
}

/* Repulsion from the flat walls (the y walls, and the side walls of a
 * closed cavity): |x_s| is the distance from the wall plane to the particle
 * surface (the centre's distance minus the shape's half-extent normal to
 * the wall), the force points away from the wall; C with the particle's
 * own equal-area radius. */
void orc_repulsion_walls_ellipse(const orc_params* p, double xp, double yp, double a, double b,
                                 double theta, double out[2]) {
    out[0] = 0.0;
    out[1] = 0.0;
    double R = area_radius(a, b);
    double C = ORC_PI * (R * R) * (p->rho_ratio - 1.0) * p->rho0 * p->gravity;
    double hx, hy;
    half_extents(a, b, theta, &hx, &hy);
    if (!p->periodic_x) {
        double gap_l = (xp + 0.5) - hx;
        if (gap_l <= p->rep_range) {
            double t = (gap_l - p->rep_range) / p->rep_range;
            out[0] += C / p->rep_eps * (t * t);
        }
        double gap_r = ((p->nx - 0.5) - xp) - hx;
        if (gap_r <= p->rep_range) {
            double t = (gap_r - p->rep_range) / p->rep_range;
            out[0] -= C / p->rep_eps * (t * t);
        }
    }
    if (p->periodic_y) return;
    double gap_b = (yp + 0.5) - hy;
    if (gap_b <= p->rep_range) {
        double t = (gap_b - p->rep_range) / p->rep_range;
        out[1] += C / p->rep_eps * (t * t);
    }
    double gap_t = ((p->ny - 0.5) - yp) - hy;
    if (gap_t <= p->rep_range) {
        double t = (gap_t - p->rep_range) / p->rep_range;
        out[1] -= C / p->rep_eps * (t * t);
    }
}

void orc_repulsion_walls(const orc_params* p, double xp, double yp, double rp, double out[2]) {
    orc_repulsion_walls_ellipse(p, xp, yp, rp, rp, 0.0, out);
}

/* Newton-Euler update over one time step (Sec. 2.2 Eqs. (7)-(8); the
 * gyroscopic term vanishes in 2D).  Reading of the integrator: explicit
 * velocity update, trapezoidal position and angle update.  Mass and inertia:
 * M = rho_p pi a b with rho_p = rho_ratio rho0; I = M r^2 / 2 for a disk
 * (b == a = r), I = M (a^2 + b^2) / 4 for an ellipse.
 * state7 = (x, y, a, ux, uy, theta, omega); b the semi-axis across. */
void orc_newton_euler_ellipse(const orc_params* p, const double state7[7], double b, double Fx,
                              double Fy, double Tz, double out7[7]) {
    double r = state7[2];
    double mass = p->rho_ratio * p->rho0 * ORC_PI * r * b;
    double inertia = r == b ? 0.5 * mass * r * r : 0.25 * mass * (r * r + b * b);
    double ux = state7[3] + Fx / mass;
    double uy = state7[4] + Fy / mass;
    double om = state7[6] + Tz / inertia;
    double x = state7[0] + 0.5 * (state7[3] + ux);
    double y = state7[1] + 0.5 * (state7[4] + uy);
    double th = state7[5] + 0.5 * (state7[6] + om);
    if (p->periodic_x) {
        if (x < 0.0) x += p->nx;
        else if (x >= p->nx) x -= p->nx;
    }
    out7[0] = x;
    out7[1] = y;
    out7[2] = r;
    out7[3] = ux;
    out7[4] = uy;
    out7[5] = th;
    out7[6] = om;
}

void orc_newton_euler(const orc_params* p, const double state7[7], double Fx, double Fy,
                      double Tz, double out7[7]) {
    orc_newton_euler_ellipse(p, state7, state7[2], Fx, Fy, Tz, out7);
}

/* ------------------------------------------------------------- refilling */

/* Refill direction (Sec. 2.5): e_c maximises n . e_c over the moving
 * directions, n the outward normal at the newborn node, read as the
 * gradient of the shape's implicit function there: parallel to (dx, dy) for
 * a disk, to (b^2 u, a^2 v) in body coordinates for an ellipse.  The
 * unnormalised vector ranks the same; ties go to the lowest index. */
int32_t orc_refill_direction(double dx, double dy, double a, double b, double theta) {
    double gx = dx, gy = dy;
    if (a != b) {
        double cth = cos(theta), sth = sin(theta), u, v;
        to_body(dx, dy, cth, sth, &u, &v);
        double gu = (b * b) * u, gv = (a * a) * v;
        gx = gu * cth - gv * sth;
        gy = gu * sth + gv * cth;
    }
    int c = 1;
    double best = gx * EX[1] + gy * EY[1];
    for (int d = 2; d < 9; ++d) {
        double v = gx * EX[d] + gy * EY[d];
        if (v > best) {
            best = v;
            c = d;
        }
    }
    return c;
}

/* Refilling of one newborn node, Sec. 2.5.  K is the number of usable
 * extrapolation points x_new + k e_c, k = 1..K (the paper uses three; with
 * fewer the order drops, with none f takes the equilibrium at rho0 and the
 * local wall velocity).  f1..f3 are the pre-collision f at t + dt there.
 * Eq. (16): f = 3 f1 - 3 f2 + f3.  Velocity constraint (reading): rho stays
 * the sum of the extrapolated f and the momentum moments are replaced so that
 * the macroscopic velocity (with the half force, evaluated at T = T_w) equals
 * u_w; only the j-rows of M^-1 change f.  Eq. (17): g = g^eq(T_w, u_w). */
void orc_refill_node(const orc_sim* s, int32_t K, const double* f1, const double* f2,
                     const double* f3, double uwx, double uwy, double fo[9], double go[5]) {
    const orc_params* p = &s->p;
    if (K >= 3) {
        for (int a = 0; a < 9; ++a) fo[a] = 3.0 * f1[a] - 3.0 * f2[a] + f3[a];
    } else if (K == 2) {
        for (int a = 0; a < 9; ++a) fo[a] = 2.0 * f1[a] - f2[a];
    } else if (K == 1) {
        for (int a = 0; a < 9; ++a) fo[a] = f1[a];
    } else {
        feq9(p->rho0, uwx, uwy, fo);
    }
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int a = 0; a < 9; ++a) {
        rho += fo[a];
        jx += EX[a] * fo[a];
        jy += EY[a] * fo[a];
    }
    double Tw = p->particle_T;
    double Fx = p->body_fx;
    double Fy = rho * p->gravity * p->beta * (Tw - p->T_ref);
    double djx = (rho * uwx - 0.5 * Fx) - jx;
    double djy = (rho * uwy - 0.5 * Fy) - jy;
    /* delta f = M^-1 (0, 0, 0, djx, 0, djy, 0, 0, 0) */
    for (int a = 0; a < 9; ++a) fo[a] += s->M9inv[a][3] * djx + s->M9inv[a][5] * djy;
    geq5(s, Tw, uwx, uwy, go);
}

/* -------------------------------------------------------------- lifecycle */

static int validate(const orc_params* p, char* err, size_t n) {
    if (p->nx < 8 || p->ny < 8) return snprintf(err, n, "nx and ny must be >= 8"), 0;
    if (p->periodic_x != 0 && p->periodic_x != 1) return snprintf(err, n, "periodic_x must be 0 or 1"), 0;
    if (!(p->nu > 0) || !(p->alpha > 0)) return snprintf(err, n, "nu and alpha must be > 0"), 0;
    if (!(p->rho0 > 0)) return snprintf(err, n, "rho0 must be > 0"), 0;
    if (!(p->a_T > -4.0 && p->a_T <= 1.0)) return snprintf(err, n, "a_T out of (-4, 1]"), 0;
    if (p->s_e >= 2 || p->s_eps >= 2 || p->s_q >= 2 || p->sT_e >= 2 || p->sT_p >= 2)
        return snprintf(err, n, "relaxation rates must be < 2"), 0;
    return 1;
}

int orc_create(const orc_params* p, orc_sim** out) {
    *out = NULL;
    orc_sim* s = (orc_sim*)calloc(1, sizeof *s);
    if (!s) return ORC_ENOMEM;
    if (!validate(p, s->err, sizeof s->err)) {
        *out = s; /* keeps the message readable through orc_last_error */
        return ORC_EINVAL;
    }
    s->p = *p;
    s->nx = p->nx;
    s->ny = p->ny;
    s->n = (long)p->nx * p->ny;
    orthogonal_inverse(9, &M9[0][0], &s->M9inv[0][0]);
    orthogonal_inverse(5, &N5[0][0], &s->N5inv[0][0]);
    derive_rates(s);
    s->f = (double*)malloc(sizeof(double) * 9 * s->n);
    s->fp = (double*)malloc(sizeof(double) * 9 * s->n);
    s->g = (double*)malloc(sizeof(double) * 5 * s->n);
    s->gp = (double*)malloc(sizeof(double) * 5 * s->n);
    s->owner = (int32_t*)malloc(sizeof(int32_t) * s->n);
    s->owner_new = (int32_t*)malloc(sizeof(int32_t) * s->n);
    if (!s->f || !s->fp || !s->g || !s->gp || !s->owner || !s->owner_new) {
        orc_destroy(s);
        return ORC_ENOMEM;
    }
    *out = s;
    return orc_set_particles(s, 0, NULL);
}

void orc_destroy(orc_sim* s) {
    if (!s) return;
    free(s->f);
    free(s->fp);
    free(s->g);
    free(s->gp);
    free(s->owner);
    free(s->owner_new);
    free(s->P);
    free(s);
}

const char* orc_last_error(const orc_sim* s) { return s ? s->err : "null handle"; }

static void init_rest(orc_sim* s) {
    double fe[9], ge[5];
    feq9(s->p.rho0, 0.0, 0.0, fe);
    geq5(s, s->p.T_fluid0, 0.0, 0.0, ge);
    for (long k = 0; k < s->n; ++k) {
        int fluid = s->owner[k] < 0;
        for (int i = 0; i < 9; ++i) s->f[i * s->n + k] = fluid ? fe[i] : NAN;
        for (int i = 0; i < 5; ++i) s->g[i * s->n + k] = fluid ? ge[i] : NAN;
    }
}

/* rows: n rows of `cols` values; cols 7 = (x, y, r, ux, uy, theta, omega)
 * (circles), cols 8 = (x, y, a, b, ux, uy, theta, omega) (ellipses). */
static int set_particles_rows(orc_sim* s, int32_t n, const double* rows, int cols) {
    if (n < 0) return set_err(s, "negative particle count"), ORC_EINVAL;
    if (n > 0 && s->p.periodic_y) return set_err(s, "particles need walls in y"), ORC_EINVAL;
    free(s->P);
    s->P = NULL;
    s->np = n;
    if (n > 0) {
        s->P = (double*)calloc((size_t)n * PSTRIDE, sizeof(double));
        if (!s->P) return ORC_ENOMEM;
    }
    for (int q = 0; q < n; ++q) {
        const double* row = rows + (size_t)cols * q;
        double in[7], b;
        if (cols == 7) {
            for (int c = 0; c < 7; ++c) in[c] = row[c];
            b = row[2];
        } else {
            in[0] = row[0];
            in[1] = row[1];
            in[2] = row[2];
            b = row[3];
            for (int c = 3; c < 7; ++c) in[c] = row[c + 1];
        }
        double* P = s->P + PSTRIDE * q;
        if (!(in[2] > 1.0) || !isfinite(in[0]) || !isfinite(in[1]))
            return set_err(s, "particle radius must be > 1 and centre finite"), ORC_EINVAL;
        if (!(b > 1.0) || b > in[2])
            return set_err(s, "semi-axis b must lie in (1, a]"), ORC_EINVAL;
        if (2.0 * in[2] + 4.0 > s->nx) return set_err(s, "particle wider than the lattice"), ORC_EINVAL;
        double x = in[0];
        if (s->p.periodic_x) {
            x = fmod(in[0], (double)s->nx);
            if (x < 0) x += s->nx;
        } else if (x < -0.5 || x > s->nx - 0.5) {
            return set_err(s, "particle centre outside the cavity"), ORC_EINVAL;
        }
        P[0] = x;
        for (int c = 1; c < 7; ++c) P[c] = in[c];
        P[10] = b;
    }
    compute_owner(s, s->owner);
    init_rest(s);
    s->steps = 0;
    return ORC_OK;
}

int orc_set_particles(orc_sim* s, int32_t n, const double* rows7) {
    return set_particles_rows(s, n, rows7, 7);
}

int orc_set_particles_ellipse(orc_sim* s, int32_t n, const double* rows8) {
    return set_particles_rows(s, n, rows8, 8);
}

int orc_set_equilibrium(orc_sim* s, const double* rho, const double* ux, const double* uy,
                        const double* T) {
    for (long k = 0; k < s->n; ++k) {
        double fe[9], ge[5];
        int fluid = s->owner[k] < 0;
        feq9(rho[k], ux[k], uy[k], fe);
        geq5(s, T[k], ux[k], uy[k], ge);
        for (int i = 0; i < 9; ++i) s->f[i * s->n + k] = fluid ? fe[i] : NAN;
        for (int i = 0; i < 5; ++i) s->g[i * s->n + k] = fluid ? ge[i] : NAN;
    }
    s->steps = 0;
    return ORC_OK;
}

int64_t orc_steps_done(const orc_sim* s) { return s->steps; }

/* ------------------------------------------------------------------ step */

typedef struct {
    long node;
    int dir, part;
} link_t;

/* Fluid at the current time level and inside the lattice (rows beyond a
 * flat wall are not nodes). */
static int fluid_at(const orc_sim* s, const int32_t* owner, int i, int j) {
    if (!s->p.periodic_y && (j < 0 || j >= s->ny)) return 0;
    if (!s->p.periodic_x && (i < 0 || i >= s->nx)) return 0;
    i = wrapi(i, s->nx);
    j = wrapi(j, s->ny);
    return owner[(long)j * s->nx + i] < 0;
}

static long node_of(const orc_sim* s, int i, int j) {
    return (long)wrapi(j, s->ny) * s->nx + wrapi(i, s->nx);
}

/* Every (x_f, i, p): x_f fluid, x_f + e_i a node of particle p (Sec. 3), in
 * ascending node, then direction order. */
static long collect_links(const orc_sim* s, link_t* out) {
    long n = 0;
    for (long k = 0; k < s->n; ++k) {
        if (s->owner[k] >= 0) continue;
        int i = (int)(k % s->nx), j = (int)(k / s->nx);
        for (int d = 1; d < 9; ++d) {
            int tj = j + EY[d], ti = i + EX[d];
            if (!s->p.periodic_y && (tj < 0 || tj >= s->ny)) continue;
            if (!s->p.periodic_x && (ti < 0 || ti >= s->nx)) continue;
            int32_t o = s->owner[node_of(s, i + EX[d], tj)];
            if (o >= 0) {
                if (out) {
                    out[n].node = k;
                    out[n].dir = d;
                    out[n].part = o;
                }
                ++n;
            }
        }
    }
    return n;
}

static double link_q_of(const orc_sim* s, long k, int d, int part) {
    const double* P = s->P + PSTRIDE * part;
    int i = (int)(k % s->nx), j = (int)(k / s->nx);
    double dx = min_image((double)i - P[0], s->nx, s->p.periodic_x);
    double dy = min_image((double)j - P[1], s->ny, s->p.periodic_y);
    return orc_link_q_ellipse(dx, dy, P[2], P[10], P[5], d);
}

static int step_once(orc_sim* s) {
    const long N = s->n;
    const int nx = s->nx, ny = s->ny;
    const orc_params* p = &s->p;

    /* 1-3. macroscopics and collision at every fluid node (Sec. 2.1). */
    for (long k = 0; k < N; ++k) {
        double f[9], g[5], fo[9], go[5];
        if (s->owner[k] >= 0) {
            for (int i = 0; i < 9; ++i) s->fp[i * N + k] = NAN;
            for (int i = 0; i < 5; ++i) s->gp[i * N + k] = NAN;
            continue;
        }
        for (int i = 0; i < 9; ++i) f[i] = s->f[i * N + k];
        for (int i = 0; i < 5; ++i) g[i] = s->g[i * N + k];
        orc_collide_node(s, f, g, fo, go, NULL);
        for (int i = 0; i < 9; ++i) s->fp[i * N + k] = fo[i];
        for (int i = 0; i < 5; ++i) s->gp[i * N + k] = go[i];
    }

    /* 4. links at the particle positions of t_n (Sec. 3). */
    long nl = collect_links(s, NULL);
    link_t* links = (link_t*)malloc(sizeof(link_t) * (nl > 0 ? nl : 1));
    if (!links) return ORC_ENOMEM;
    collect_links(s, links);

    /* 5. streaming into s->f / s->g (reused as the t_n+1 arrays): pull from
     * the upstream node; flat walls use halfway bounce-back for f (with the
     * y wall's tangential velocity; side walls are at rest) and
     * anti-bounce-back for g (Dirichlet T_wall).  A diagonal population whose
     * upstream node lies beyond both a y wall and a side wall (a cavity
     * corner) is bounced back with the y wall's velocity and, being a
     * diagonal, has no g.  Populations coming from a particle are set in
     * step 6. */
    for (long k = 0; k < N; ++k) {
        for (int i = 0; i < 9; ++i) s->f[i * N + k] = NAN;
        for (int i = 0; i < 5; ++i) s->g[i * N + k] = NAN;
        if (s->owner[k] >= 0) continue;
        int x = (int)(k % nx), y = (int)(k / nx);
        for (int i = 0; i < 9; ++i) {
            int sy = y - EY[i], sx = x - EX[i];
            int outy = !p->periodic_y && (sy < 0 || sy >= ny);
            int outx = !p->periodic_x && (sx < 0 || sx >= nx);
            if (outy || outx) {
                int ib = OPP[i];
                double uw = outy ? p->wall_ux[sy < 0 ? 0 : 1] : 0.0;
                double Tw = outy ? p->wall_T[sy < 0 ? 0 : 1] : p->side_T[sx < 0 ? 0 : 1];
                s->f[i * N + k] = s->fp[ib * N + k] - 2.0 * W9[ib] * p->rho0 * (EX[ib] * uw) / CS2;
                if (i < 5) s->g[i * N + k] = -s->gp[ib * N + k] + 2.0 * s->w5[i] * Tw;
                continue;
            }
            long src = node_of(s, x - EX[i], sy);
            if (s->owner[src] >= 0) continue;
            s->f[i * N + k] = s->fp[i * N + src];
            if (i < 5) s->g[i * N + k] = s->gp[i * N + src];
        }
    }

    /* 6-7. each link: q, wall velocity, Bouzidi f (and the thermal g for the
     * axis directions), then the momentum exchange of Eqs. (13)-(14),
     * summed per particle in link order. */
    double* Fsum = (double*)calloc((size_t)(s->np > 0 ? s->np : 1) * 3, sizeof(double));
    if (!Fsum) {
        free(links);
        return ORC_ENOMEM;
    }
    for (long l = 0; l < nl; ++l) {
        long k = links[l].node;
        int i = links[l].dir, ib = OPP[i], part = links[l].part;
        const double* P = s->P + PSTRIDE * part;
        int x = (int)(k % nx), y = (int)(k / nx);
        double dx = min_image((double)x - P[0], nx, p->periodic_x);
        double dy = min_image((double)y - P[1], ny, p->periodic_y);
        double q = orc_link_q_ellipse(dx, dy, P[2], P[10], P[5], i);
        double rx = dx + q * EX[i], ry = dy + q * EY[i]; /* x_w - X_c */
        double uwx = P[3] - P[6] * ry, uwy = P[4] + P[6] * rx;
        int have1 = fluid_at(s, s->owner, x - EX[i], y - EY[i]);
        int have2 = have1 && fluid_at(s, s->owner, x - 2 * EX[i], y - 2 * EY[i]);
        long k1 = have1 ? node_of(s, x - EX[i], y - EY[i]) : k;
        long k2 = have2 ? node_of(s, x - 2 * EX[i], y - 2 * EY[i]) : k;
        double fi = s->fp[i * N + k];
        double fib = s->fp[ib * N + k];
        double fnew = orc_bouzidi(q, i, fi, s->fp[i * N + k1], s->fp[i * N + k2], fib,
                                  s->fp[ib * N + k1], have1, have2, p->rho0, uwx, uwy);
        s->f[ib * N + k] = fnew;
        if (i < 5) {
            s->g[ib * N + k] = orc_thermal_link(q, i, s->gp[i * N + k], s->gp[i * N + k1],
                                                s->gp[ib * N + k], have1, s->w5[i], p->particle_T);
        }
        /* Eq. (13): f_i^+(x_f)(e_i - u_w) - f_ibar(x_f, t+dt)(e_ibar - u_w) */
        double dFx = fi * (EX[i] - uwx) - fnew * (EX[ib] - uwx);
        double dFy = fi * (EY[i] - uwy) - fnew * (EY[ib] - uwy);
        Fsum[3 * part + 0] += dFx;
        Fsum[3 * part + 1] += dFy;
        Fsum[3 * part + 2] += rx * dFy - ry * dFx; /* Eq. (14), z component */
    }
    free(links);

    /* Every population of a fluid node must now be known (a NaN here can
     * only come from a population that no rule above produced, or from an
     * already unstable state). */
    for (long k = 0; k < N; ++k) {
        if (s->owner[k] >= 0) continue;
        for (int i = 0; i < 9; ++i) {
            if (isnan(s->f[i * N + k]) || (i < 5 && isnan(s->g[i * N + k]))) {
                free(Fsum);
                set_err(s, "NaN population after streaming");
                return ORC_EUNSTABLE;
            }
        }
    }

    /* 8. particle motion: hydrodynamic force, repulsion (evaluated at t_n for
     * all particles), net weight -(rho_p - rho_f) pi a b g y^ (pi r^2 for a
     * disk). */
    double* Pn = (double*)malloc(sizeof(double) * PSTRIDE * (s->np > 0 ? s->np : 1));
    if (!Pn) {
        free(Fsum);
        return ORC_ENOMEM;
    }
    int unstable = 0;
    for (int a = 0; a < s->np; ++a) {
        const double* P = s->P + PSTRIDE * a;
        double Rx = 0.0, Ry = 0.0;
        if (p->repulsion) {
            for (int b = 0; b < s->np; ++b) {
                if (b == a) continue;
                const double* Q = s->P + PSTRIDE * b;
                double fr[2];
                orc_repulsion_pair_ellipse(p, P[0], P[1], P[2], P[10], P[5], Q[0], Q[1], Q[2], Q[10],
                                           Q[5], fr);
                Rx += fr[0];
                Ry += fr[1];
            }
            double fw[2];
            orc_repulsion_walls_ellipse(p, P[0], P[1], P[2], P[10], P[5], fw);
            Rx += fw[0];
            Ry += fw[1];
        }
        double Fg = -(p->rho_ratio - 1.0) * p->rho0 * ORC_PI * P[2] * P[10] * p->gravity;
        double Fx = Fsum[3 * a + 0] + Rx;
        double Fy = (Fsum[3 * a + 1] + Ry) + Fg;
        double st[7], out[7];
        for (int c = 0; c < 7; ++c) st[c] = P[c];
        orc_newton_euler_ellipse(p, st, P[10], Fx, Fy, Fsum[3 * a + 2], out);
        double ddx = min_image(out[0] - P[0], nx, p->periodic_x), ddy = out[1] - P[1];
        if (!(ddx * ddx + ddy * ddy <= 0.25)) unstable = 1;
        double* O = Pn + PSTRIDE * a;
        for (int c = 0; c < 7; ++c) O[c] = out[c];
        O[7] = Fsum[3 * a + 0];
        O[8] = Fsum[3 * a + 1];
        O[9] = Fsum[3 * a + 2];
        O[10] = P[10];
    }
    free(Fsum);
    if (s->np > 0) memcpy(s->P, Pn, sizeof(double) * PSTRIDE * s->np);
    free(Pn);

    /* 9. owner at t_n+1; newborn = solid at t_n, fluid at t_n+1. */
    compute_owner(s, s->owner_new);

    /* 10. refilling of newborn nodes (Sec. 2.5).  The extrapolation reads only
     * nodes fluid at both t_n and t_n+1, whose streamed values are final. */
    for (long k = 0; k < N; ++k) {
        int32_t o = s->owner[k];
        if (o < 0 || s->owner_new[k] >= 0) continue;
        const double* P = s->P + PSTRIDE * o;
        int x = (int)(k % nx), y = (int)(k / nx);
        double dx = min_image((double)x - P[0], nx, p->periodic_x);
        double dy = min_image((double)y - P[1], ny, p->periodic_y);
        int c = orc_refill_direction(dx, dy, P[2], P[10], P[5]);
        int K = 0;
        double fs[3][9];
        for (int m = 1; m <= 3; ++m) {
            int xi = x + m * EX[c], yi = y + m * EY[c];
            if (!fluid_at(s, s->owner, xi, yi) || !fluid_at(s, s->owner_new, xi, yi)) break;
            long km = node_of(s, xi, yi);
            for (int a = 0; a < 9; ++a) fs[m - 1][a] = s->f[a * N + km];
            K = m;
        }
        double uwx = P[3] - P[6] * dy, uwy = P[4] + P[6] * dx;
        double fo[9], go[5];
        orc_refill_node(s, K, fs[0], fs[1], fs[2], uwx, uwy, fo, go);
        for (int a = 0; a < 9; ++a) s->f[a * N + k] = fo[a];
        for (int a = 0; a < 5; ++a) s->g[a * N + k] = go[a];
    }

    /* Covered nodes drop their populations; the new owner map takes over. */
    for (long k = 0; k < N; ++k) {
        if (s->owner_new[k] >= 0) {
            for (int i = 0; i < 9; ++i) s->f[i * N + k] = NAN;
            for (int i = 0; i < 5; ++i) s->g[i * N + k] = NAN;
        }
    }
    int32_t* t = s->owner;
    s->owner = s->owner_new;
    s->owner_new = t;
    s->steps += 1;
    if (unstable) return set_err(s, "particle moved more than 0.5 per step"), ORC_EUNSTABLE;
    return ORC_OK;
}

int orc_step(orc_sim* s, int32_t nsteps) {
    for (int32_t t = 0; t < nsteps; ++t) {
        int rc = step_once(s);
        if (rc != ORC_OK) return rc;
    }
    return ORC_OK;
}

/* ----------------------------------------------------------------- reads */

int orc_read_fields(const orc_sim* s, double* rho, double* ux, double* uy, double* T,
                    int32_t* owner) {
    const long N = s->n;
    for (long k = 0; k < N; ++k) {
        double m[4] = {NAN, NAN, NAN, NAN};
        if (s->owner[k] < 0) {
            double f[9], g[5], fo[9], go[5];
            for (int i = 0; i < 9; ++i) f[i] = s->f[i * N + k];
            for (int i = 0; i < 5; ++i) g[i] = s->g[i * N + k];
            orc_collide_node(s, f, g, fo, go, m);
        }
        if (rho) rho[k] = m[0];
        if (ux) ux[k] = m[1];
        if (uy) uy[k] = m[2];
        if (T) T[k] = m[3];
        if (owner) owner[k] = s->owner[k];
    }
    return ORC_OK;
}

int orc_read_populations(const orc_sim* s, double* f, double* g) {
    if (f) memcpy(f, s->f, sizeof(double) * 9 * s->n);
    if (g) memcpy(g, s->g, sizeof(double) * 5 * s->n);
    return ORC_OK;
}

int orc_read_particles(const orc_sim* s, double* rows10, int32_t* n) {
    if (n) *n = s->np;
    if (rows10)
        for (int q = 0; q < s->np; ++q) memcpy(rows10 + 10 * q, s->P + PSTRIDE * q, sizeof(double) * 10);
    return ORC_OK;
}

int orc_read_links(const orc_sim* s, int32_t* node, int32_t* dir, int32_t* particle, double* q,
                   int64_t cap, int64_t* n_out) {
    long nl = collect_links(s, NULL);
    if (n_out) *n_out = nl;
    if (!node && !dir && !particle && !q) return ORC_OK; /* count only */
    if (nl > cap) return ORC_EINVAL;
    link_t* links = (link_t*)malloc(sizeof(link_t) * (nl > 0 ? nl : 1));
    if (!links) return ORC_ENOMEM;
    collect_links(s, links);
    for (long l = 0; l < nl; ++l) {
        if (node) node[l] = (int32_t)links[l].node;
        if (dir) dir[l] = links[l].dir;
        if (particle) particle[l] = links[l].part;
        if (q) q[l] = link_q_of(s, links[l].node, links[l].dir, links[l].part);
    }
    free(links);
    return ORC_OK;
}

/* Nusselt number at each flat wall (the paper reports none; reading): the
 * one-sided wall-normal gradient between the wall (at half a spacing) and
 * the adjacent row, averaged over the fluid nodes of that row, scaled by
 * H / dT with H = ny and dT = particle_T - T_fluid0. */
int orc_nusselt(const orc_sim* s, double* nu_bottom, double* nu_top) {
    double dT = s->p.particle_T - s->p.T_fluid0;
    if (s->p.periodic_y || dT == 0.0) return ORC_EINVAL;
    double H = s->ny;
    for (int w = 0; w < 2; ++w) {
        int j = w == 0 ? 0 : s->ny - 1;
        double acc = 0.0;
        long cnt = 0;
        for (int i = 0; i < s->nx; ++i) {
            long k = (long)j * s->nx + i;
            if (s->owner[k] >= 0) continue;
            double T = 0.0;
            for (int a = 0; a < 5; ++a) T += s->g[a * s->n + k];
            acc += (T - s->p.wall_T[w]) / 0.5;
            ++cnt;
        }
        double v = cnt ? (acc / cnt) * H / dT : NAN;
        if (w == 0 && nu_bottom) *nu_bottom = v;
        if (w == 1 && nu_top) *nu_top = v;
    }
    return ORC_OK;
}
