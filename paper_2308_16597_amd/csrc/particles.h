// particles.h -- device-side building blocks of the particle side of a
// step: particle records, windows, the solid test, link fractions and the
// interpolated moving-wall and thermal-wall schemes (Sec. 2.3).
//
// Method: Xu & Li, arXiv 2308.16597 (equations cited at each piece).
#pragma once

#include "lattice.h"

namespace ptlbm {

// Particles per cell of the neighbour-search grid (cells are at least
// 2 r_max + s wide, so a cell of non-overlapping disks holds at most 4).
constexpr int BINCAP = 7;

// ------------------------------------------------------------- geometry ----
// The exact solid test shared by every kernel that builds or reads the
// solid map: dx = (i - X) with the minimum image along a periodic x axis
// (the plain difference in the closed cavity), dy = j - Y, inside when
// dx*dx + dy*dy <= r*r (no fused multiply-add: the translation unit is
// compiled with -ffp-contract=off).
__device__ __forceinline__ double min_image_x(double d, const LP& lp) {
    if (!lp.periodic_x) return d;
    const double h = 0.5 * lp.nx;
    if (d > h) return d - lp.nx;
    if (d < -h) return d + lp.nx;
    return d;
}

struct PState {   // one particle, FP64
    double x, y, r, ux, uy, th, om, b;   // r: semi-axis a along the body axis at th; b across it
};

// Whole-record global-memory accesses of the small structs kept in device
// arrays (their copy operations do not bind to address-space-qualified
// objects, so they go field by field; adjacent fields merge into wide
// accesses).
__device__ __forceinline__ PState ld_state(const PState* p) {
    const PT_GLOBAL double* q = (const PT_GLOBAL double*)p;
    return PState{q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7]};
}
__device__ __forceinline__ void st_state(PState* p, const PState& v) {
    PT_GLOBAL double* q = (PT_GLOBAL double*)p;
    q[0] = v.x; q[1] = v.y; q[2] = v.r; q[3] = v.ux; q[4] = v.uy; q[5] = v.th; q[6] = v.om; q[7] = v.b;
}
__device__ __forceinline__ uint2 ld_u2(const uint2* p) {
    const PT_GLOBAL unsigned* q = (const PT_GLOBAL unsigned*)p;
    return make_uint2(q[0], q[1]);
}
__device__ __forceinline__ void st_u2(uint2* p, uint2 v) {
    PT_GLOBAL unsigned* q = (PT_GLOBAL unsigned*)p;
    q[0] = v.x;
    q[1] = v.y;
}
__device__ __forceinline__ int2 ld_i2(const int2* p) {
    const PT_GLOBAL int* q = (const PT_GLOBAL int*)p;
    return make_int2(q[0], q[1]);
}
__device__ __forceinline__ void st_i2(int2* p, int2 v) {
    PT_GLOBAL int* q = (PT_GLOBAL int*)p;
    q[0] = v.x;
    q[1] = v.y;
}
__device__ __forceinline__ double4 ld_d4(const double4* p) {
    const PT_GLOBAL double* q = (const PT_GLOBAL double*)p;
    return make_double4(q[0], q[1], q[2], q[3]);
}
__device__ __forceinline__ void st_d4(double4* p, double4 v) {
    PT_GLOBAL double* q = (PT_GLOBAL double*)p;
    q[0] = v.x;
    q[1] = v.y;
    q[2] = v.z;
    q[3] = v.w;
}

// Window of a particle (Sec. 3): x from INT(x_c - r) - 1 to INT(x_c + r) + 1
// and likewise in y, INT read as floor.
struct Win {
    int x0, y0, nxw, nyw;
};
__device__ __forceinline__ Win window_of(const PState& P) {
    Win w;
    const int xa = (int)floor(P.x - P.r), xb = (int)floor(P.x + P.r);
    const int ya = (int)floor(P.y - P.r), yb = (int)floor(P.y + P.r);
    w.x0 = xa - 1;
    w.y0 = ya - 1;
    w.nxw = xb - xa + 3;
    w.nyw = yb - ya + 3;
    return w;
}
// A particle whose state is not finite or far outside the lattice is not
// processed (its kernels would address outside the buffers); the step
// reports it through the status word.
__device__ __forceinline__ bool particle_ok(const PState& P, const LP& lp) {
    return isfinite(P.x) && isfinite(P.y) && isfinite(P.r) && P.x >= -lp.nx && P.x <= 2.0 * lp.nx &&
           P.y >= -(double)lp.ny && P.y <= 2.0 * lp.ny;
}
__device__ __forceinline__ int wrap_x(int x, int nx) {
    x %= nx;
    return x < 0 ? x + nx : x;
}
// Column of lattice coordinate x: wrapped on a periodic axis; -1 beyond the
// side walls of the closed cavity (not a node).
__device__ __forceinline__ int col_of(int x, const LP& lp) {
    if (lp.periodic_x) return wrap_x(x, lp.nx);
    return (x >= 0 && x < lp.nx) ? x : -1;
}

// ---------------------------------------------------------------- shapes ----
// Particles are circles or ellipses (Sec. 2.6.2): semi-axis a = r along the
// body axis at angle th from +x, b across it; b == a is a circle and takes
// the plain circle formulas.  An ellipse is handled in body coordinates
// (u, v) = (dx c + dy s, dy c - dx s), c = cos th, s = sin th.
struct Shape {
    double a, b, c, s;
    bool circle;
};
__device__ __forceinline__ Shape shape_of(const PState& P) {
    Shape sh;
    sh.a = P.r;
    sh.b = P.b;
    sh.circle = P.b == P.r;
    sh.c = 1.0;
    sh.s = 0.0;
    if (!sh.circle) {
        sh.c = cos(P.th);
        sh.s = sin(P.th);
    }
    return sh;
}
// Solid test: dx^2 + dy^2 <= r^2, or b^2 u^2 + a^2 v^2 <= a^2 b^2.
__device__ __forceinline__ bool inside_shape(const Shape& sh, double dx, double dy) {
    if (sh.circle) return dx * dx + dy * dy <= sh.a * sh.a;
    const double u = dx * sh.c + dy * sh.s, v = dy * sh.c - dx * sh.s;
    return (u * u) * (sh.b * sh.b) + (v * v) * (sh.a * sh.a) <= (sh.a * sh.a) * (sh.b * sh.b);
}
// Distance from the centre to the boundary along the unit direction (nx, ny).
__device__ __forceinline__ double radial_extent(const Shape& sh, double nx, double ny) {
    if (sh.circle) return sh.a;
    const double nu = nx * sh.c + ny * sh.s, nv = ny * sh.c - nx * sh.s;
    return (sh.a * sh.b) / sqrt((sh.b * sh.b) * (nu * nu) + (sh.a * sh.a) * (nv * nv));
}
// Half-extents along x and y (distance from the centre to the supporting
// lines normal to the axes).
__device__ __forceinline__ void half_extents(const Shape& sh, double& hx, double& hy) {
    if (sh.circle) {
        hx = sh.a;
        hy = sh.a;
        return;
    }
    hx = sqrt((sh.a * sh.a) * (sh.c * sh.c) + (sh.b * sh.b) * (sh.s * sh.s));
    hy = sqrt((sh.a * sh.a) * (sh.s * sh.s) + (sh.b * sh.b) * (sh.c * sh.c));
}
// Radius of the disk of equal area (the repulsion force scale).
__device__ __forceinline__ double area_radius(const Shape& sh) { return sh.circle ? sh.a : sqrt(sh.a * sh.b); }

// Link fraction q of Sec. 2.3 for the circle: the nearer root of
// |d + t e_i|^2 = r^2, clamped to [0, 1].
__device__ __forceinline__ double link_q(double dx, double dy, double r, int i) {
    const double ex = EXd(i), ey = EYd(i);
    const double a = ex * ex + ey * ey;
    const double b = dx * ex + dy * ey;
    const double c = (dx * dx + dy * dy) - r * r;
    double disc = b * b - a * c;
    if (disc < 0.0) disc = 0.0;
    double q = (-b - sqrt(disc)) / a;
    if (q < 0.0) q = 0.0;
    if (q > 1.0) q = 1.0;
    return q;
}

// The same for either shape: for an ellipse the smaller root of
// b^2 (u + t e_u)^2 + a^2 (v + t e_v)^2 = a^2 b^2 in body coordinates.
__device__ __forceinline__ double link_q_shape(const Shape& sh, double dx, double dy, int i) {
    if (sh.circle) return link_q(dx, dy, sh.a, i);
    const double ex = EXd(i), ey = EYd(i);
    const double u = dx * sh.c + dy * sh.s, v = dy * sh.c - dx * sh.s;
    const double eu = ex * sh.c + ey * sh.s, ev = ey * sh.c - ex * sh.s;
    const double a2 = sh.a * sh.a, b2 = sh.b * sh.b;
    const double A = b2 * (eu * eu) + a2 * (ev * ev);
    const double B = b2 * (u * eu) + a2 * (v * ev);
    const double C = (b2 * (u * u) + a2 * (v * v)) - a2 * b2;
    double disc = B * B - A * C;
    if (disc < 0.0) disc = 0.0;
    double q = (-B - sqrt(disc)) / A;
    if (q < 0.0) q = 0.0;
    if (q > 1.0) q = 1.0;
    return q;
}

// Interpolated bounce-back, Sec. 2.3 Eqs. (9)-(10), with the linear and
// halfway fallbacks when stencil nodes are not fluid.  Works on stored
// values of any mode: the coefficients sum to one and f_i, f_ibar share the
// same rest weight.  wall = 2 w_i rho0 (e_ibar . u_w)/cs^2.
__device__ __forceinline__ double bouzidi(double q, double fi, double fi1, double fi2, double fib,
                                          double fib1, bool have1, bool have2, double wall) {
    if (q <= 0.5) {
        if (have1 && have2)
            return q * (2.0 * q + 1.0) * fi + (1.0 - 4.0 * q * q) * fi1 - q * (1.0 - 2.0 * q) * fi2 + wall;
        if (have1) return 2.0 * q * fi + (1.0 - 2.0 * q) * fi1 + wall;
        return fi + wall;
    }
    const double a = 1.0 / (q * (2.0 * q + 1.0));
    if (have1) return a * fi + (2.0 * q - 1.0) / q * fib - (2.0 * q - 1.0) / (2.0 * q + 1.0) * fib1 + a * wall;
    return 1.0 / (2.0 * q) * fi + (2.0 * q - 1.0) / (2.0 * q) * fib + wall / (2.0 * q);
}

// Thermal curved wall, Sec. 2.3 Eqs. (11)-(12), on stored values whose rest
// part is w T_store (T_store = T_sh for shifted storage, 0 for plain):
// g_ibar = -g_i + c (g_i(x_f - e_i) + g_ibar) + c4 2 w (T_w - T_store),
// c = (2q-1)/(2q+1), c4 = 2/(2q+1); anti-bounce-back without x_f - e_i.
__device__ __forceinline__ double thermal_link(double q, double gi, double gi1, double gib, bool have1,
                                               double w, double Tw_rel) {
    if (!have1) return -gi + 2.0 * w * Tw_rel;
    const double c = (2.0 * q - 1.0) / (2.0 * q + 1.0);
    const double c4 = 2.0 / (2.0 * q + 1.0);
    return (-gi + c * gi1 + c * gib) + c4 * (2.0 * w * Tw_rel);
}

}  // namespace ptlbm
