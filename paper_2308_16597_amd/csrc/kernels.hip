// kernels.hip -- the gfx950 kernels of one step of the particle-resolved
// thermal lattice Boltzmann method (Xu & Li, arXiv 2308.16597).
//
// Per step, in launch order (cur = time level n, ring = particle slot of t_n):
//   k_compact       one block per particle: clear the owner map and node
//                   flags of two steps ago over the old window, then collect
//                   the particle's links from the owner map of t_n into LDS in
//                   the fixed slot order of Sec. 3 (one slot per lattice line
//                   and direction), wave ballot + LDS prefix scan, one global
//                   atomic per block to reserve a contiguous segment.
//   k_link_pass     one wavefront per particle: q, wall velocity, Bouzidi
//                   bounce-back (Eqs. (9)-(10)) and the thermal wall
//                   (Eqs. (11)-(12)) written into the solid slots of the
//                   post-collision state, momentum exchange (Eqs. (13)-(14))
//                   reduced in FP64 in a fixed order.
//   k_particles     one wavefront per particle: repulsion (Eq. (15)) summed in
//                   ascending partner order, net weight, Newton-Euler update.
//   k_mask_mark     one block per particle: owner map of t_n+1 by atomic min.
//   k_refill        one block per particle: node flags of (t_n, t_n+1) and
//                   refilling + collision of newborn nodes (Sec. 2.5).
//   k_stream_collide  one thread per node: fused pull-stream + D2Q9/D2Q5 MRT
//                   collision with buoyancy (Sec. 2.1) of every node fluid at
//                   both time levels.
// Built with -ffp-contract=off: the solid test and link fractions must round
// exactly as the CPU oracle rounds them.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace ptlbm {

constexpr int LAT_BLOCK = 256;
constexpr int PBLOCK = 256;
constexpr double kPi = 3.14159265358979323846;
constexpr int OUTSIDE = -2;

template <int MODE> using ST = typename Store<MODE>::T;

template <int MODE> __host__ __device__ Pops<ST<MODE>> pops_of(void* const (&a)[14]) {
    Pops<ST<MODE>> p;
    for (int i = 0; i < 9; ++i) p.f[i] = (ST<MODE>*)a[i];
    for (int i = 0; i < 5; ++i) p.g[i] = (ST<MODE>*)a[9 + i];
    return p;
}

// ------------------------------------------------------ lattice kernels ----

template <int MODE>
__global__ __launch_bounds__(LAT_BLOCK) void k_stream_collide(Pops<ST<MODE>> A, Pops<ST<MODE>> B,
                                                              const uint8_t* __restrict__ flag, LP lp,
                                                              unsigned* status) {
    using S = Store<MODE>;
    using R = typename S::R;
    const int x = blockIdx.x * LAT_BLOCK + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= lp.nx) return;
    const size_t k = (size_t)y * lp.pitch + x;
    if (flag[k] != 0) return;
    R s[9], t[5];
    pull_node<S>(A, lp, x, y, s, t);
    const CC<R> c(lp);
    R rho, ux, uy, T;
    collide<R>(c, s, t, rho, ux, uy, T);
    if (!(isfinite(rho) && isfinite(T) && isfinite(ux) && isfinite(uy))) atomicOr(status, ST_NONFINITE);
    store_node<S>(B, lp, k, s, t);
}

// Equilibrium of the given macroscopic fields (host layout j*nx + i; NULL
// pointers select the uniform rest state), collided once: the
// post-collision state of t_0.
template <int MODE, class FT>
__global__ __launch_bounds__(LAT_BLOCK) void k_init(Pops<ST<MODE>> A, const int32_t* __restrict__ owner,
                                                    const FT* rho_f, const FT* ux_f, const FT* uy_f,
                                                    const FT* T_f, double rho_u, double T_u, LP lp) {
    using S = Store<MODE>;
    using R = typename S::R;
    const int x = blockIdx.x * LAT_BLOCK + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= lp.nx) return;
    const size_t k = (size_t)y * lp.pitch + x;
    const size_t h = (size_t)y * lp.nx + x;
    R s[9], t[5];
    if (owner[k] >= 0) {
        for (int i = 0; i < 9; ++i) s[i] = (R)0;
        for (int i = 0; i < 5; ++i) t[i] = (R)0;
    } else {
        const R rho = rho_f ? (R)rho_f[h] : (R)rho_u;
        const R ux = ux_f ? (R)ux_f[h] : (R)0;
        const R uy = uy_f ? (R)uy_f[h] : (R)0;
        const R T = T_f ? (R)T_f[h] : (R)T_u;
        feq_dev<R>(rho, (R)lp.rho0, ux, uy, s);
        geq_dev<R>(T, (R)lp.T_sh, ux, uy, (R)lp.w5_0, (R)lp.w5_k, t);
        const CC<R> c(lp);
        R r_, u_, v_, T_;
        collide<R>(c, s, t, r_, u_, v_, T_);
    }
    store_node<S>(A, lp, k, s, t);
}

// Pre-collision macroscopics from the post-collision state: rho and T are
// collision invariants and the momentum gained the force, so
// u = (j+ - F/2)/rho.  NaN inside solids.  Output: 4 planes of nx*ny (OT).
template <int MODE, class OT>
__global__ __launch_bounds__(LAT_BLOCK) void k_macros(Pops<ST<MODE>> A, const int32_t* __restrict__ owner,
                                                      OT* out, LP lp) {
    using S = Store<MODE>;
    using R = typename S::R;
    const int x = blockIdx.x * LAT_BLOCK + threadIdx.x;
    const int y = blockIdx.y;
    if (x >= lp.nx) return;
    const size_t k = (size_t)y * lp.pitch + x;
    const size_t n = (size_t)lp.nx * lp.ny, h = (size_t)y * lp.nx + x;
    if (owner[k] >= 0) {
        const OT nan = (OT)NAN;
        out[h] = nan;
        out[n + h] = nan;
        out[2 * n + h] = nan;
        out[3 * n + h] = nan;
        return;
    }
    R s[9], t[5];
#pragma unroll
    for (int i = 0; i < 9; ++i) s[i] = S::ld(A.f[i] + k) - (S::shifted ? (R)0 : w9<R>(i) * (R)lp.rho0);
#pragma unroll
    for (int i = 0; i < 5; ++i) t[i] = S::ld(A.g[i] + k);
    R drho = (R)0, jx = (R)0, jy = (R)0, dT = (R)0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        drho += s[i];
        jx += (R)EXd(i) * s[i];
        jy += (R)EYd(i) * s[i];
    }
#pragma unroll
    for (int i = 0; i < 5; ++i) dT += t[i];
    const R rho = (R)lp.rho0 + drho;
    const R T = (R)lp.T_sh + dT;
    const R Fx = (R)lp.body_fx;
    const R Fy = rho * (R)lp.gbeta * (T - (R)lp.T_ref);
    out[h] = (OT)rho;
    out[n + h] = (OT)((jx - (R)0.5 * Fx) / rho);
    out[2 * n + h] = (OT)((jy - (R)0.5 * Fy) / rho);
    out[3 * n + h] = (OT)T;
}

// ----------------------------------------------------- particle kernels ----

__device__ __forceinline__ bool in_rows(int y, const LP& lp) { return y >= 0 && y < lp.ny; }

// One slot of the fixed link mapping (Sec. 3): slot -> (direction, lattice
// line through the window); walks the line and returns the link of that
// line, if any (at most one per line and direction).  Window of nxw x nyw
// nodes, values in LDS: -1 fluid, particle index, or OUTSIDE.
//   directions 1, 3: the nyw rows;  2, 4: the nxw columns;
//   5, 7 (lines a - b = c) and 6, 8 (lines a + b = c): nxw + nyw - 3 lines
//   each (the two single-node corner lines cannot hold a link).
__device__ __forceinline__ bool find_link(const int* __restrict__ win, int nxw, int nyw, int p, int s,
                                          int& a_out, int& b_out, int& d_out) {
    int d, l;
    const int nd = nxw + nyw - 3;
    if (s < nyw) { d = 1; l = s; }
    else if (s < nyw + nxw) { d = 2; l = s - nyw; }
    else if (s < 2 * nyw + nxw) { d = 3; l = s - nyw - nxw; }
    else if (s < 2 * (nyw + nxw)) { d = 4; l = s - 2 * nyw - nxw; }
    else {
        const int r = s - 2 * (nyw + nxw);
        d = 5 + r / nd;
        l = r % nd;
    }
    const int ex = EXd(d), ey = EYd(d);
    int a, b, da, db, len;
    if (ey == 0) { a = 0; b = l; da = 1; db = 0; len = nxw; }          // row b
    else if (ex == 0) { a = l; b = 0; da = 0; db = 1; len = nyw; }     // column a
    else if (ex == ey) {                                              // a - b = c
        const int c = l - (nyw - 2);
        a = c > 0 ? c : 0;
        b = a - c;
        da = 1; db = 1;
        len = min(nxw - a, nyw - b);
    } else {                                                          // a + b = c
        const int c = l + 1;
        b = c < nyw - 1 ? c : nyw - 1;
        a = c - b;
        da = 1; db = -1;
        len = min(nxw - a, b + 1);
    }
    for (int m = 0; m < len; ++m, a += da, b += db) {
        const int ta = a + ex, tb = b + ey;
        if (ta < 0 || ta >= nxw || tb < 0 || tb >= nyw) continue;
        if (win[b * nxw + a] == -1 && win[tb * nxw + ta] == p) {
            a_out = a;
            b_out = b;
            d_out = d;
            return true;
        }
    }
    return false;
}

__global__ __launch_bounds__(PBLOCK) void k_compact(const int32_t* __restrict__ Ocur, int32_t* Onext,
                                                    uint8_t* flag, const PState* __restrict__ Pc,
                                                    const PState* __restrict__ Po, uint2* links, int2* seg,
                                                    unsigned* counter, unsigned* status, LP lp) {
    extern __shared__ uint2 smem_u2[];
    __shared__ int wave_cnt[PBLOCK / 64];
    __shared__ unsigned seg_start, seg_count;
    const int p = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int nx = lp.nx, pitch = lp.pitch;

    // Owner map and flags left by t_n-1 (two time levels ago) in the buffer
    // that will hold t_n+1.
    const PState po = Po[p];
    if (particle_ok(po, lp)) {
        const Win w = window_of(po);
        if (w.nxw <= lp.nwin && w.nyw <= lp.nwin) {
            for (int idx = tid; idx < w.nxw * w.nyw; idx += PBLOCK) {
                const int yy = w.y0 + idx / w.nxw;
                if (!in_rows(yy, lp)) continue;
                const size_t k = (size_t)yy * pitch + wrap_x(w.x0 + idx % w.nxw, nx);
                Onext[k] = -1;
                flag[k] = 0;
            }
        }
    }

    const PState P = Pc[p];
    const Win w = window_of(P);
    if (!particle_ok(P, lp) || w.nxw > lp.nwin || w.nyw > lp.nwin) {
        if (tid == 0) {
            seg[p] = make_int2(0, 0);
            atomicOr(status, ST_BAD_PARTICLE);
        }
        return;
    }
    int* win = (int*)smem_u2;
    uint2* lk = smem_u2 + (lp.nwin * lp.nwin + 1) / 2;
    for (int idx = tid; idx < w.nxw * w.nyw; idx += PBLOCK) {
        const int yy = w.y0 + idx / w.nxw;
        win[idx] = in_rows(yy, lp) ? Ocur[(size_t)yy * pitch + wrap_x(w.x0 + idx % w.nxw, nx)] : OUTSIDE;
    }
    __syncthreads();

    const int nslots = 2 * (w.nxw + w.nyw) + 4 * (w.nxw + w.nyw - 3);
    int base = 0;
    for (int s0 = 0; s0 < nslots; s0 += PBLOCK) {
        const int s = s0 + tid;
        int a = 0, b = 0, d = 0;
        const bool valid = s < nslots && find_link(win, w.nxw, w.nyw, p, s, a, b, d);
        const unsigned long long m = __ballot(valid);
        const int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wave_cnt[wv] = __popcll(m);
        __syncthreads();
        int off = base, tot = 0;
        for (int i = 0; i < PBLOCK / 64; ++i) {
            off += i < wv ? wave_cnt[i] : 0;
            tot += wave_cnt[i];
        }
        if (valid) {
            const unsigned xx = (unsigned)wrap_x(w.x0 + a, nx), yy = (unsigned)(w.y0 + b);
            lk[off + pre] = make_uint2(xx | (yy << 16), (unsigned)d | ((unsigned)p << 4));
        }
        base += tot;
        __syncthreads();
    }
    if (tid == 0) {
        unsigned start = atomicAdd(counter, (unsigned)base);
        unsigned cnt = (unsigned)base;
        if ((unsigned long long)start + cnt > (unsigned long long)lp.link_cap) {
            atomicOr(status, ST_LINK_OVERFLOW);
            cnt = 0;
        }
        seg_start = start;
        seg_count = cnt;
        seg[p] = make_int2((int)start, (int)cnt);
    }
    __syncthreads();
    for (unsigned i = tid; i < seg_count; i += PBLOCK) links[seg_start + i] = lk[i];
}

template <int MODE>
__global__ __launch_bounds__(256) void k_link_pass(Pops<ST<MODE>> A, const int32_t* __restrict__ Ocur,
                                                   const PState* __restrict__ Pc, const uint2* __restrict__ links,
                                                   const int2* __restrict__ seg, double* Fh, LP lp) {
    using S = Store<MODE>;
    const int lane = threadIdx.x & 63;
    const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (p >= lp.np) return;
    const PState P = Pc[p];
    const int2 sg = seg[p];
    const int nx = lp.nx, pitch = lp.pitch;
    const double shf = S::shifted ? lp.rho0 : 0.0;  // rest density carried by the stored f
    double fx = 0.0, fy = 0.0, tz = 0.0;
    for (int l = lane; l < sg.y; l += 64) {
        const uint2 L = links[sg.x + l];
        const int x = (int)(L.x & 0xffffu), y = (int)(L.x >> 16), i = (int)(L.y & 15u);
        const int ib = OPPd(i), ex = EXd(i), ey = EYd(i);
        const double dx = min_image_x((double)x - P.x, nx);
        const double dy = (double)y - P.y;
        const double q = link_q(dx, dy, P.r, i);
        const double rx = dx + q * ex, ry = dy + q * ey;   // x_w - X_c
        const double uwx = P.ux - P.om * ry, uwy = P.uy + P.om * rx;
        const int x1 = wrap_x(x - ex, nx), y1 = y - ey;
        const int x2 = wrap_x(x - 2 * ex, nx), y2 = y - 2 * ey;
        const bool have1 = in_rows(y1, lp) && Ocur[(size_t)y1 * pitch + x1] == -1;
        const bool have2 = have1 && in_rows(y2, lp) && Ocur[(size_t)y2 * pitch + x2] == -1;
        const size_t k = (size_t)y * pitch + x;
        const size_t k1 = have1 ? (size_t)y1 * pitch + x1 : k;
        const size_t k2 = have2 ? (size_t)y2 * pitch + x2 : k;
        const double w = i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0;
        const double fi = (double)S::ld(A.f[i] + k), fib = (double)S::ld(A.f[ib] + k);
        const double fi1 = (double)S::ld(A.f[i] + k1), fib1 = (double)S::ld(A.f[ib] + k1);
        const double fi2 = (double)S::ld(A.f[i] + k2);
        const double wall = 6.0 * w * lp.rho0 * (-(ex * uwx) - ey * uwy);
        const double fnew = bouzidi(q, fi, fi1, fi2, fib, fib1, have1, have2, wall);
        const size_t kb = (size_t)(y + ey) * pitch + wrap_x(x + ex, nx);
        S::st(A.f[ib] + kb, (typename S::R)fnew);
        if (i <= 4) {
            const double gi = (double)S::ld(A.g[i] + k), gib = (double)S::ld(A.g[ib] + k);
            const double gi1 = (double)S::ld(A.g[i] + k1);
            const double gnew = thermal_link(q, gi, gi1, gib, have1, lp.w5_k, lp.particle_T - lp.T_sh);
            S::st(A.g[ib] + kb, (typename S::R)gnew);
        }
        // Eq. (13) on full populations (stored value + rest part w rho0)
        const double Fi = fi + w * shf, Fb = (double)(typename S::R)fnew + w * shf;
        const double dFx = Fi * (ex - uwx) - Fb * (-ex - uwx);
        const double dFy = Fi * (ey - uwy) - Fb * (-ey - uwy);
        fx += dFx;
        fy += dFy;
        tz += rx * dFy - ry * dFx;   // Eq. (14), z component
    }
    for (int off = 32; off > 0; off >>= 1) {
        fx += __shfl_xor(fx, off);
        fy += __shfl_xor(fy, off);
        tz += __shfl_xor(tz, off);
    }
    if (lane == 0) {
        Fh[4 * p + 0] = fx;
        Fh[4 * p + 1] = fy;
        Fh[4 * p + 2] = tz;
    }
}

// Spring repulsion of Eq. (15) on particle (xp, yp, rp) from (xq, yq, rq):
// surface gap along the centre line, force scale pi rp rq (rho_p - rho_f) g.
__device__ __forceinline__ void repulsion_pair(const LP& lp, double xp, double yp, double rp, double xq,
                                               double yq, double rq, double& fx, double& fy) {
    const double dx = min_image_x(xp - xq, lp.nx);
    const double dy = yp - yq;
    const double dist = sqrt(dx * dx + dy * dy);
    const double gap = dist - rp - rq;
    const double C = kPi * (rp * rq) * (lp.rho_ratio - 1.0) * lp.rho0 * lp.gravity;
    const double t = (gap - lp.rep_range) / lp.rep_range;
    const double mag = C / lp.rep_eps * (t * t);
    fx = mag * (dx / dist);
    fy = mag * (dy / dist);
}

__global__ __launch_bounds__(64) void k_particles(const PState* __restrict__ Pc, PState* Pn,
                                                  const double* __restrict__ Fh, unsigned* counter,
                                                  unsigned* status, LP lp) {
    const int p = blockIdx.x, lane = threadIdx.x;
    const PState P = Pc[p];
    const int np = lp.np;
    double Rx = 0.0, Ry = 0.0;
    if (lp.repulsion) {
        // partners in ascending index order (chunks of 64, then bits of the ballot)
        for (int q0 = 0; q0 < np; q0 += 64) {
            const int q = q0 + lane;
            bool near = false;
            if (q < np && q != p) {
                const PState Q = Pc[q];
                const double dx = min_image_x(P.x - Q.x, lp.nx);
                const double dy = P.y - Q.y;
                near = sqrt(dx * dx + dy * dy) - P.r - Q.r <= lp.rep_range;
            }
            unsigned long long m = __ballot(near);
            while (m) {
                const int b = __ffsll((long long)m) - 1;
                m &= m - 1ull;
                const PState Q = Pc[q0 + b];
                double fx, fy;
                repulsion_pair(lp, P.x, P.y, P.r, Q.x, Q.y, Q.r, fx, fy);
                Rx += fx;
                Ry += fy;
            }
        }
        double wy = 0.0;
        if (!lp.periodic_y) {
            const double C = kPi * (P.r * P.r) * (lp.rho_ratio - 1.0) * lp.rho0 * lp.gravity;
            const double gb = (P.y + 0.5) - P.r;
            if (gb <= lp.rep_range) {
                const double t = (gb - lp.rep_range) / lp.rep_range;
                wy += C / lp.rep_eps * (t * t);
            }
            const double gt = ((lp.ny - 0.5) - P.y) - P.r;
            if (gt <= lp.rep_range) {
                const double t = (gt - lp.rep_range) / lp.rep_range;
                wy -= C / lp.rep_eps * (t * t);
            }
        }
        Rx += 0.0;
        Ry += wy;
    }
    if (lane != 0) return;
    if (p == 0) {
        counter[1] = counter[0];
        counter[0] = 0u;
    }
    const double Fg = -(lp.rho_ratio - 1.0) * lp.rho0 * kPi * P.r * P.r * lp.gravity;
    const double Fx = Fh[4 * p + 0] + Rx;
    const double Fy = (Fh[4 * p + 1] + Ry) + Fg;
    const double Tz = Fh[4 * p + 2];
    // Newton-Euler (Sec. 2.2): explicit velocities, trapezoidal positions.
    const double mass = lp.rho_ratio * lp.rho0 * kPi * P.r * P.r;
    const double inertia = 0.5 * mass * P.r * P.r;
    PState N = P;
    N.ux = P.ux + Fx / mass;
    N.uy = P.uy + Fy / mass;
    N.om = P.om + Tz / inertia;
    N.x = P.x + 0.5 * (P.ux + N.ux);
    N.y = P.y + 0.5 * (P.uy + N.uy);
    N.th = P.th + 0.5 * (P.om + N.om);
    if (N.x < 0.0) N.x += lp.nx;
    else if (N.x >= lp.nx) N.x -= lp.nx;
    const double ddx = min_image_x(N.x - P.x, lp.nx), ddy = N.y - P.y;
    if (!(ddx * ddx + ddy * ddy <= 0.25)) atomicOr(status, ST_OVERSPEED);
    Pn[p] = N;
}

__global__ __launch_bounds__(PBLOCK) void k_mask_mark(int32_t* O, const PState* __restrict__ Pp, LP lp) {
    const int p = blockIdx.x;
    const PState P = Pp[p];
    if (!particle_ok(P, lp)) return;
    const Win w = window_of(P);
    if (w.nxw > lp.nwin || w.nyw > lp.nwin) return;
    const double r2 = P.r * P.r;
    for (int idx = threadIdx.x; idx < w.nxw * w.nyw; idx += PBLOCK) {
        const int yy = w.y0 + idx / w.nxw;
        if (!in_rows(yy, lp)) continue;
        const int xx = wrap_x(w.x0 + idx % w.nxw, lp.nx);
        const double dx = min_image_x((double)xx - P.x, lp.nx);
        const double dy = (double)yy - P.y;
        if (dx * dx + dy * dy <= r2) atomicMin((unsigned*)&O[(size_t)yy * lp.pitch + xx], (unsigned)p);
    }
}

// Refilling of the newborn node (x, y) of particle P (state at t_n+1),
// Sec. 2.5: e_c maximises n . e_c (n parallel to x - X_c; ties to the lowest
// index); pre-collision f at x + m e_c (m = 1..3, nodes fluid at t_n and
// t_n+1) rebuilt by pulling from A; Eq. (16) extrapolation (lower order when
// fewer points are fluid, equilibrium at rho0 with none); momentum set so
// that u = u_w; g = g^eq(T_w, u_w) (Eq. (17)); then collided into B.
template <int MODE>
__device__ void refill_node(const Pops<ST<MODE>>& A, const Pops<ST<MODE>>& B, const int32_t* Ocur,
                            const int32_t* Onext, const PState& P, int x, int y, const LP& lp) {
    using S = Store<MODE>;
    using R = typename S::R;
    const double dx = min_image_x((double)x - P.x, lp.nx);
    const double dy = (double)y - P.y;
    int c = 1;
    double best = dx * EXd(1) + dy * EYd(1);
    for (int d = 2; d < 9; ++d) {
        const double v = dx * EXd(d) + dy * EYd(d);
        if (v > best) {
            best = v;
            c = d;
        }
    }
    R sm[3][9];
    int K = 0;
    for (int m = 1; m <= 3; ++m) {
        const int ym = y + m * EYd(c);
        if (!in_rows(ym, lp)) break;
        const int xm = wrap_x(x + m * EXd(c), lp.nx);
        const size_t km = (size_t)ym * lp.pitch + xm;
        if (Ocur[km] != -1 || Onext[km] != -1) break;
        R tt[5];
        pull_node<S>(A, lp, xm, ym, sm[m - 1], tt);
        K = m;
    }
    const double uwx = P.ux - P.om * dy, uwy = P.uy + P.om * dx;
    R s[9], t[5];
    if (K == 3) {
        for (int a = 0; a < 9; ++a) s[a] = (R)3 * sm[0][a] - (R)3 * sm[1][a] + sm[2][a];
    } else if (K == 2) {
        for (int a = 0; a < 9; ++a) s[a] = (R)2 * sm[0][a] - sm[1][a];
    } else if (K == 1) {
        for (int a = 0; a < 9; ++a) s[a] = sm[0][a];
    } else {
        feq_dev<R>((R)lp.rho0, (R)lp.rho0, (R)uwx, (R)uwy, s);
    }
    R drho = (R)0, jx = (R)0, jy = (R)0;
    for (int a = 0; a < 9; ++a) {
        drho += s[a];
        jx += (R)EXd(a) * s[a];
        jy += (R)EYd(a) * s[a];
    }
    const R rho = (R)lp.rho0 + drho;
    const R Tw = (R)lp.particle_T;
    const R Fx = (R)lp.body_fx, Fy = rho * (R)lp.gbeta * (Tw - (R)lp.T_ref);
    const R djx = (rho * (R)uwx - (R)0.5 * Fx) - jx;
    const R djy = (rho * (R)uwy - (R)0.5 * Fy) - jy;
    for (int a = 0; a < 9; ++a) s[a] += ((R)EXd(a) * djx + (R)EYd(a) * djy) * (R)(1.0 / 6.0);
    geq_dev<R>(Tw, (R)lp.T_sh, (R)uwx, (R)uwy, (R)lp.w5_0, (R)lp.w5_k, t);
    const CC<R> cc(lp);
    R r_, u_, v_, T_;
    collide<R>(cc, s, t, r_, u_, v_, T_);
    store_node<S>(B, lp, (size_t)y * lp.pitch + x, s, t);
}

template <int MODE>
__global__ __launch_bounds__(PBLOCK) void k_refill(Pops<ST<MODE>> A, Pops<ST<MODE>> B,
                                                   const int32_t* __restrict__ Ocur,
                                                   const int32_t* __restrict__ Onext, uint8_t* flag,
                                                   const PState* __restrict__ Pc,
                                                   const PState* __restrict__ Pn, LP lp) {
    const int p = blockIdx.x;
    const PState P0 = Pc[p], P1 = Pn[p];
    if (!particle_ok(P0, lp) || !particle_ok(P1, lp)) return;
    const Win w0 = window_of(P0);
    Win w1 = window_of(P1);
    if (w1.x0 - w0.x0 > lp.nx / 2) w1.x0 -= lp.nx;
    else if (w0.x0 - w1.x0 > lp.nx / 2) w1.x0 += lp.nx;
    const int xa = min(w0.x0, w1.x0), xb = max(w0.x0 + w0.nxw, w1.x0 + w1.nxw);
    const int ya = min(w0.y0, w1.y0), yb = max(w0.y0 + w0.nyw, w1.y0 + w1.nyw);
    const int bw = xb - xa, bh = yb - ya;
    if (bw > lp.nwin + 2 || bh > lp.nwin + 2) return;
    for (int idx = threadIdx.x; idx < bw * bh; idx += PBLOCK) {
        const int yy = ya + idx / bw;
        if (!in_rows(yy, lp)) continue;
        const int xx = wrap_x(xa + idx % bw, lp.nx);
        const size_t k = (size_t)yy * lp.pitch + xx;
        const int32_t on = Ocur[k], onx = Onext[k];
        flag[k] = (uint8_t)((on >= 0 ? 2 : 0) | (onx >= 0 ? 1 : 0));
        if (on == p && onx == -1) refill_node<MODE>(A, B, Ocur, Onext, P1, xx, yy, lp);
    }
}

__global__ void k_link_q(const PState* __restrict__ Pc, const uint2* __restrict__ links, int n, int32_t* node,
                         int32_t* dir, int32_t* part, double* qo, LP lp) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    const uint2 L = links[l];
    const int x = (int)(L.x & 0xffffu), y = (int)(L.x >> 16), i = (int)(L.y & 15u), p = (int)(L.y >> 4);
    const PState P = Pc[p];
    const double dx = min_image_x((double)x - P.x, lp.nx);
    const double dy = (double)y - P.y;
    node[l] = y * lp.nx + x;
    dir[l] = i;
    part[l] = p;
    qo[l] = link_q(dx, dy, P.r, i);
}

// -------------------------------------------------------------- launchers ----

static dim3 lattice_grid(const LP& lp) { return dim3((lp.nx + LAT_BLOCK - 1) / LAT_BLOCK, lp.ny); }

#define PTLBM_DISPATCH(mode, CALL)                                      \
    switch (mode) {                                                     \
        case LBM_STORE_F64: { constexpr int M = LBM_STORE_F64; CALL; } break;             \
        case LBM_STORE_F32: { constexpr int M = LBM_STORE_F32; CALL; } break;             \
        case LBM_STORE_SHIFT_F32: { constexpr int M = LBM_STORE_SHIFT_F32; CALL; } break; \
        case LBM_STORE_SHIFT_F16: { constexpr int M = LBM_STORE_SHIFT_F16; CALL; } break; \
        case LBM_STORE_SHIFT_BF16: { constexpr int M = LBM_STORE_SHIFT_BF16; CALL; } break; \
        default: return hipErrorInvalidValue;                           \
    }

hipError_t launch_stream_collide(const DevState& d, int cur, hipStream_t st) {
    PTLBM_DISPATCH(d.mode, (k_stream_collide<M><<<lattice_grid(d.lp), LAT_BLOCK, 0, st>>>(
                               pops_of<M>(d.S[cur]), pops_of<M>(d.S[1 - cur]), d.flag, d.lp, d.status)));
    return hipGetLastError();
}

hipError_t launch_init(const DevState& d, int cur, const void* rho, const void* ux, const void* uy,
                       const void* T, bool f64, double rho_u, double T_u, hipStream_t st) {
    if (f64) {
        PTLBM_DISPATCH(d.mode, (k_init<M, double><<<lattice_grid(d.lp), LAT_BLOCK, 0, st>>>(
                                   pops_of<M>(d.S[cur]), d.O[cur], (const double*)rho, (const double*)ux,
                                   (const double*)uy, (const double*)T, rho_u, T_u, d.lp)));
    } else {
        PTLBM_DISPATCH(d.mode, (k_init<M, float><<<lattice_grid(d.lp), LAT_BLOCK, 0, st>>>(
                                   pops_of<M>(d.S[cur]), d.O[cur], (const float*)rho, (const float*)ux,
                                   (const float*)uy, (const float*)T, rho_u, T_u, d.lp)));
    }
    return hipGetLastError();
}

hipError_t launch_macros(const DevState& d, int cur, void* out, hipStream_t st) {
    if (d.mode == LBM_STORE_F64) {
        k_macros<LBM_STORE_F64, double><<<lattice_grid(d.lp), LAT_BLOCK, 0, st>>>(
            pops_of<LBM_STORE_F64>(d.S[cur]), d.O[cur], (double*)out, d.lp);
    } else {
        PTLBM_DISPATCH(d.mode, (k_macros<M, float><<<lattice_grid(d.lp), LAT_BLOCK, 0, st>>>(
                                   pops_of<M>(d.S[cur]), d.O[cur], (float*)out, d.lp)));
    }
    return hipGetLastError();
}

static size_t compact_smem(const LP& lp) {
    const size_t win = ((size_t)lp.nwin * lp.nwin + 1) & ~(size_t)1;
    return win * sizeof(int) + (size_t)(12 * lp.nwin - 12) * sizeof(uint2);
}

hipError_t launch_compact(const DevState& d, int cur, int ring, hipStream_t st) {
    if (d.lp.np == 0) return hipSuccess;
    k_compact<<<d.lp.np, PBLOCK, compact_smem(d.lp), st>>>(d.O[cur], d.O[1 - cur], d.flag, d.P[ring],
                                                           d.P[ring_old(ring)], d.links, d.seg, d.counter,
                                                           d.status, d.lp);
    return hipGetLastError();
}

hipError_t launch_link_pass(const DevState& d, int cur, int ring, hipStream_t st) {
    if (d.lp.np == 0) return hipSuccess;
    PTLBM_DISPATCH(d.mode, (k_link_pass<M><<<(d.lp.np + 3) / 4, 256, 0, st>>>(
                               pops_of<M>(d.S[cur]), d.O[cur], d.P[ring], d.links, d.seg, d.Fh, d.lp)));
    return hipGetLastError();
}

hipError_t launch_particles(const DevState& d, int ring, hipStream_t st) {
    if (d.lp.np == 0) return hipSuccess;
    k_particles<<<d.lp.np, 64, 0, st>>>(d.P[ring], d.P[ring_next(ring)], d.Fh, d.counter, d.status, d.lp);
    return hipGetLastError();
}

hipError_t launch_mask_mark(const DevState& d, int owner_idx, const PState* P, hipStream_t st) {
    if (d.lp.np == 0) return hipSuccess;
    k_mask_mark<<<d.lp.np, PBLOCK, 0, st>>>(d.O[owner_idx], P, d.lp);
    return hipGetLastError();
}

hipError_t launch_refill(const DevState& d, int cur, int ring, hipStream_t st) {
    if (d.lp.np == 0) return hipSuccess;
    PTLBM_DISPATCH(d.mode, (k_refill<M><<<d.lp.np, PBLOCK, 0, st>>>(
                               pops_of<M>(d.S[cur]), pops_of<M>(d.S[1 - cur]), d.O[cur], d.O[1 - cur], d.flag,
                               d.P[ring], d.P[ring_next(ring)], d.lp)));
    return hipGetLastError();
}

hipError_t launch_link_q(const DevState& d, int ring, int nlinks, int32_t* node, int32_t* dir, int32_t* part,
                         double* q, hipStream_t st) {
    if (nlinks <= 0) return hipSuccess;
    k_link_q<<<(nlinks + 255) / 256, 256, 0, st>>>(d.P[ring], d.links, nlinks, node, dir, part, q, d.lp);
    return hipGetLastError();
}

}  // namespace ptlbm
