// link.h -- device-side evaluation of one fluid-particle link, shared by the
// link pass (particles.hip) and the pull of the lattice kernel
// (lattice.hip), so that both compute the same bits.
//
// Method: Xu & Li, arXiv 2308.16597, Sec. 2.3 (Eqs. (9)-(12)) and the wall
// velocity of Sec. 2.4.
#pragma once

#include "launch.h"

namespace ptlbm {

__device__ __forceinline__ bool in_rows(int y, const LP& lp) { return y >= 0 && y < lp.ny; }

// A link's values: its fraction q, the post-collision f_i(x_f) it was built
// from, the unknown f_ibar(x_f) of t_n+1 by interpolated bounce-back
// (Eqs. (9)-(10), with the linear and halfway fallbacks) and, for axis
// links, g_ibar(x_f) by the thermal curved wall (Eqs. (11)-(12)) -- both in
// the storage's units, before rounding to the storage type -- the lever
// x_w - X_c and the wall velocity u_w at x_w = x_f + q e_i.
struct LinkEval {
    double q, fi, fnew, gnew, rx, ry, uwx, uwy;
};

// One link: fluid node (x, y), direction i towards particle P, from the
// post-collision state A of t_n in its layout.  QFIRST: gather only what the
// branch of q needs (q <= 1/2: f_i at x_f, x_f - e_i, x_f - 2 e_i; q > 1/2:
// f_i at x_f and f_ibar at x_f, x_f - e_i); otherwise gather both branches'
// populations without waiting for q (the direct pass, whose threads take
// their links one after another).  Stencil nodes that are not fluid at t_n
// are read but not used (have1, have2), so no value written into a solid
// node's slots enters the result.
template <int MODE, bool QFIRST = true>
__device__ __forceinline__ LinkEval eval_link(const RunStep& rs, const PState& P, const Shape& sh, int x, int y,
                                              int i) {
    using S = Store<MODE>;
    const LP& lp = rs.lp;
    // population arrays picked straight from the run's pointer table (a
    // local copy indexed by the link direction would live in scratch)
    auto F = [&](int a) { return (const PT_GLOBAL ST<MODE>*)rs.A[a]; };
    const PT_GLOBAL int32_t* __restrict__ Ocur = gl(rs.Ocur);
    const int pitch = lp.pitch;
    const int ib = OPPd(i), ex = EXd(i), ey = EYd(i);
    const int x1 = col_of(x - ex, lp), y1 = y - ey;
    const int x2 = col_of(x - 2 * ex, lp), y2 = y - 2 * ey;
    const bool in1 = in_rows(y1, lp) && x1 >= 0, in2 = in_rows(y2, lp) && x2 >= 0;
    const size_t k = (size_t)y * pitch + x;
    const size_t k1 = in1 ? (size_t)y1 * pitch + x1 : k;
    const size_t k2 = in2 ? (size_t)y2 * pitch + x2 : k;
    const int32_t o1 = Ocur[k1], o2 = Ocur[k2];
    // where the post-collision state keeps f_a*(node): slot a at the node
    // (two sets), slot abar at the node (in place, reversed), or slot a at
    // the node + e_a (in place, pushed; slot abar at the node at a wall)
    const int lay = lp.aa ? 1 + rs.parity : 0;
    // q first (arithmetic only), then the gathers of its branch
    const double dx = min_image_x((double)x - P.x, lp);
    const double dy = (double)y - P.y;
    const double q = link_q_shape(sh, dx, dy, i);
    const bool lo = q <= 0.5;
    const bool get_lo = !QFIRST || lo, get_hi = !QFIRST || !lo;
    double fi, fib = 0.0, fi1 = 0.0, fib1 = 0.0, fi2 = 0.0, gi = 0.0, gib = 0.0, gi1 = 0.0;
    if (lay != 2) {
        const int si = lay ? ib : i, sib = lay ? i : ib;
        const size_t tk = tix<ST<MODE>>(k), tk1 = tix<ST<MODE>>(k1), tk2 = tix<ST<MODE>>(k2);
        fi = (double)S::ld(F(si) + tk);
        if (get_lo) {
            fi1 = (double)S::ld(F(si) + tk1);
            fi2 = (double)S::ld(F(si) + tk2);
        }
        if (get_hi) {
            fib = (double)S::ld(F(sib) + tk);
            fib1 = (double)S::ld(F(sib) + tk1);
        }
        if (i <= 4) {
            gi = (double)S::ld(F(9 + si) + tk);
            gib = (double)S::ld(F(9 + sib) + tk);
            gi1 = (double)S::ld(F(9 + si) + tk1);
        }
    } else {
        int sl;
        size_t at;
        at = pushed_at(lp, x, y, i, sl);
        fi = (double)S::ld(F(sl) + tix<ST<MODE>>(at));
        if (i <= 4) gi = (double)S::ld(F(9 + sl) + tix<ST<MODE>>(at));
        at = pushed_at(lp, x, y, ib, sl);
        if (get_hi) fib = (double)S::ld(F(sl) + tix<ST<MODE>>(at));
        if (i <= 4) gib = (double)S::ld(F(9 + sl) + tix<ST<MODE>>(at));
        if (in1) {
            at = pushed_at(lp, x1, y1, i, sl);
            if (get_lo) fi1 = (double)S::ld(F(sl) + tix<ST<MODE>>(at));
            if (i <= 4) gi1 = (double)S::ld(F(9 + sl) + tix<ST<MODE>>(at));
            if (get_hi) {
                at = pushed_at(lp, x1, y1, ib, sl);
                fib1 = (double)S::ld(F(sl) + tix<ST<MODE>>(at));
            }
        }
        if (in2 && get_lo) {
            at = pushed_at(lp, x2, y2, i, sl);
            fi2 = (double)S::ld(F(sl) + tix<ST<MODE>>(at));
        }
    }
    const bool have1 = in1 && o1 == -1;
    const bool have2 = have1 && in2 && o2 == -1;
    const double rx = dx + q * ex, ry = dy + q * ey;   // x_w - X_c
    const double uwx = P.ux - P.om * ry, uwy = P.uy + P.om * rx;
    const double w9i = i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0;
    const double wall = 6.0 * w9i * lp.rho0 * (-(ex * uwx) - ey * uwy);
    const double fnew = bouzidi(q, fi, fi1, fi2, fib, fib1, have1, have2, wall);
    LinkEval e;
    e.q = q;
    e.fi = fi;
    e.fnew = fnew;
    e.gnew = i <= 4 ? thermal_link(q, gi, gi1, gib, have1, lp.w5_k, lp.particle_T - lp.T_sh) : 0.0;
    e.rx = rx;
    e.ry = ry;
    e.uwx = uwx;
    e.uwy = uwy;
    return e;
}

}  // namespace ptlbm
