// lattice.h -- device-side building blocks of the lattice update: storage
// policies, the fused D2Q9 + D2Q5 MRT collision in deviation variables and
// the pull step with flat walls; also the lattice constants every kernel
// takes and the helpers shared by the kernel files.
//
// Method: Xu & Li, arXiv 2308.16597, Sec. 2 (equations cited at each piece).
// Readings of points the paper leaves open are the same as in the library's
// header: Lallemand-Luo D2Q9 moment basis, Guo-type forcing in moment space,
// D2Q5 with n_e^eq = a T, halfway flat walls, Bouzidi fallbacks.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lbm.h"

namespace ptlbm {

// Device-memory pointers typed as such: every access through them compiles
// to a global (not flat) memory instruction, also when the pointer itself
// was read from a run table in memory rather than from kernel arguments.
#define PT_GLOBAL __attribute__((address_space(1)))
template <class T> __device__ __forceinline__ PT_GLOBAL T* gl(T* p) { return (PT_GLOBAL T*)p; }

// --------------------------------------------------------------- storage ----
// Populations are kept as deviations from the rest state inside the kernels:
//   s_i = f_i - w_i rho0,   t_k = g_k - w_k T_sh.
// Plain modes store f and g themselves (the kernels subtract/add w_i rho0;
// T_sh is 0 for them); SHIFT_ modes store the deviations directly.

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
    return __uint_as_float(((uint32_t)b) << 16);
}
// Round to nearest even: gfx950 converts in one instruction
// (v_cvt_pk_bf16_f32); a NaN stays a NaN.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

template <int MODE> struct Store;
template <> struct Store<LBM_STORE_F64> {
    using T = double; using R = double; static constexpr bool shifted = false;
    __device__ static R ld(const PT_GLOBAL T* p) { return *p; }
    __device__ static R ld_nt(const PT_GLOBAL T* p) { return __builtin_nontemporal_load(p); }
    __device__ static void st(PT_GLOBAL T* p, R v) { *p = v; }
    __device__ static void st_nt(PT_GLOBAL T* p, R v) { __builtin_nontemporal_store(v, p); }
};
template <> struct Store<LBM_STORE_F32> {
    using T = float; using R = float; static constexpr bool shifted = false;
    __device__ static R ld(const PT_GLOBAL T* p) { return *p; }
    __device__ static R ld_nt(const PT_GLOBAL T* p) { return __builtin_nontemporal_load(p); }
    __device__ static void st(PT_GLOBAL T* p, R v) { *p = v; }
    __device__ static void st_nt(PT_GLOBAL T* p, R v) { __builtin_nontemporal_store(v, p); }
};
template <> struct Store<LBM_STORE_SHIFT_F32> {
    using T = float; using R = float; static constexpr bool shifted = true;
    __device__ static R ld(const PT_GLOBAL T* p) { return *p; }
    __device__ static R ld_nt(const PT_GLOBAL T* p) { return __builtin_nontemporal_load(p); }
    __device__ static void st(PT_GLOBAL T* p, R v) { *p = v; }
    __device__ static void st_nt(PT_GLOBAL T* p, R v) { __builtin_nontemporal_store(v, p); }
};
template <> struct Store<LBM_STORE_SHIFT_F16> {
    using T = _Float16; using R = float; static constexpr bool shifted = true;
    __device__ static R ld(const PT_GLOBAL T* p) { return (float)*p; }
    __device__ static R ld_nt(const PT_GLOBAL T* p) { return (float)__builtin_nontemporal_load(p); }
    __device__ static void st(PT_GLOBAL T* p, R v) { *p = (_Float16)v; }
    __device__ static void st_nt(PT_GLOBAL T* p, R v) { __builtin_nontemporal_store((_Float16)v, p); }
};
template <> struct Store<LBM_STORE_SHIFT_BF16> {
    using T = uint16_t; using R = float; static constexpr bool shifted = true;
    __device__ static R ld(const PT_GLOBAL T* p) { return bf16_to_f32(*p); }
    __device__ static R ld_nt(const PT_GLOBAL T* p) { return bf16_to_f32(__builtin_nontemporal_load(p)); }
    __device__ static void st(PT_GLOBAL T* p, R v) { *p = f32_to_bf16_rne(v); }
    __device__ static void st_nt(PT_GLOBAL T* p, R v) { __builtin_nontemporal_store(f32_to_bf16_rne(v), p); }
};

template <class T> struct Pops {
    PT_GLOBAL T* f[9];
    PT_GLOBAL T* g[5];
};

// Collision and wall constants in the compute type R, derived in FP64 (in
// the order the kernels would take them).  FP64 kernels derive them from
// their arguments; FP32 arithmetic reads a copy rounded once on the host and
// spends no instruction on them.
template <class R> struct CC {
    R rho0, gbeta, T_ref, body_fx;
    R s_e, s_eps, s_q, s_nu;        // D2Q9 rates
    R h_e, h_eps, h_q, h_nu;        // 1 - s/2 of the same rates (forcing terms)
    R s_a, s_Te, s_Tp, a_T;         // D2Q5 rates and equilibrium constant
    R w5_0, w5_k, T_sh;
    R fsw[9];                       // rest state w_i rho0
    R u_wall[2];                    // wall_ux rho0 / 6 of the moving walls [bottom, top]
    R g_wall[2];                    // 2 w5_k (wall_T - T_sh) [bottom, top]
    R g_side[2];                    // 2 w5_k (side_T - T_sh) [left, right]
};

// Lattice constants handed to every kernel (host-filled, FP64).
struct LP {
    int nx, ny, pitch, periodic_x, periodic_y;   // periodic_x = 0: closed cavity
    double rho0, gbeta, T_ref, body_fx;
    double s_e, s_eps, s_q, s_nu;      // D2Q9 rates (the j rates are immaterial)
    double s_a, s_Te, s_Tp, a_T;       // D2Q5 rates and equilibrium constant
    double w5_0, w5_k;                 // D2Q5 weights
    double wall_T[2], wall_ux[2];      // [bottom, top]
    double side_T[2];                  // [left, right] side walls of the cavity
    double T_sh;                       // storage shift of g (0 for plain modes)
    double particle_T, rho_ratio, gravity, rep_eps, rep_range;
    int repulsion, np, nwin;           // particles, window edge capacity
    int link_cap;
    int direct;                        // link pass by direct addressing (ablation)
    int aa;                            // in-place (AA) streaming in one population set
    int lpp;                           // lanes per particle of the per-particle kernels (64, 256)
    int ncx, ncy, ncells;              // neighbour-search cell grid
    // the constants above rounded for FP32 arithmetic, in device memory
    // next to the run's buffers (read with scalar loads; kept out of the
    // kernel arguments, which they would make 20 % larger)
    const PT_GLOBAL CC<float>* cf;
};

// The constants of lp for FP64 arithmetic, derived in the order the kernels
// would take (host and device compute the same bits).
__host__ __device__ inline CC<double> make_cc(const LP& lp) {
    CC<double> c;
    c.rho0 = lp.rho0;
    c.gbeta = lp.gbeta;
    c.T_ref = lp.T_ref;
    c.body_fx = lp.body_fx;
    c.s_e = lp.s_e;
    c.s_eps = lp.s_eps;
    c.s_q = lp.s_q;
    c.s_nu = lp.s_nu;
    c.h_e = 1.0 - 0.5 * lp.s_e;
    c.h_eps = 1.0 - 0.5 * lp.s_eps;
    c.h_q = 1.0 - 0.5 * lp.s_q;
    c.h_nu = 1.0 - 0.5 * lp.s_nu;
    c.s_a = lp.s_a;
    c.s_Te = lp.s_Te;
    c.s_Tp = lp.s_Tp;
    c.a_T = lp.a_T;
    c.w5_0 = lp.w5_0;
    c.w5_k = lp.w5_k;
    c.T_sh = lp.T_sh;
    for (int i = 0; i < 9; ++i) c.fsw[i] = (i == 0 ? 4.0 / 9.0 : (i < 5 ? 1.0 / 9.0 : 1.0 / 36.0)) * lp.rho0;
    for (int w = 0; w < 2; ++w) {
        c.u_wall[w] = lp.wall_ux[w] * lp.rho0 * (1.0 / 6.0);
        c.g_wall[w] = 2.0 * lp.w5_k * (lp.wall_T[w] - lp.T_sh);
        c.g_side[w] = 2.0 * lp.w5_k * (lp.side_T[w] - lp.T_sh);
    }
    return c;
}

// The same rounded once to FP32 (on the host for lp.cf).
__host__ __device__ inline CC<float> round_cc(const CC<double>& c) {
    CC<float> f;
    f.rho0 = (float)c.rho0;
    f.gbeta = (float)c.gbeta;
    f.T_ref = (float)c.T_ref;
    f.body_fx = (float)c.body_fx;
    f.s_e = (float)c.s_e;
    f.s_eps = (float)c.s_eps;
    f.s_q = (float)c.s_q;
    f.s_nu = (float)c.s_nu;
    f.h_e = (float)c.h_e;
    f.h_eps = (float)c.h_eps;
    f.h_q = (float)c.h_q;
    f.h_nu = (float)c.h_nu;
    f.s_a = (float)c.s_a;
    f.s_Te = (float)c.s_Te;
    f.s_Tp = (float)c.s_Tp;
    f.a_T = (float)c.a_T;
    f.w5_0 = (float)c.w5_0;
    f.w5_k = (float)c.w5_k;
    f.T_sh = (float)c.T_sh;
    for (int i = 0; i < 9; ++i) f.fsw[i] = (float)c.fsw[i];
    for (int w = 0; w < 2; ++w) {
        f.u_wall[w] = (float)c.u_wall[w];
        f.g_wall[w] = (float)c.g_wall[w];
        f.g_side[w] = (float)c.g_side[w];
    }
    return f;
}

// The run's constants in the compute type R.  FP64: derived from the
// kernel arguments where used.  FP32: one copy taken from lp.cf, before any
// store and any divergent branch of the kernel, so that the loads are
// scalar; the pull, collision and store helpers receive it.
template <class R> __device__ __forceinline__ CC<R> lp_cc(const LP& lp);
template <> __device__ __forceinline__ CC<double> lp_cc<double>(const LP& lp) { return make_cc(lp); }
template <> __device__ __forceinline__ CC<float> lp_cc<float>(const LP& lp) { return *(const CC<float>*)lp.cf; }
// The same values derived from the kernel arguments alone (for kernels that
// would otherwise hold the copy in scalar registers across their stores).
template <class R> __device__ __forceinline__ CC<R> args_cc(const LP& lp);
template <> __device__ __forceinline__ CC<double> args_cc<double>(const LP& lp) { return make_cc(lp); }
template <> __device__ __forceinline__ CC<float> args_cc<float>(const LP& lp) { return round_cc(make_cc(lp)); }

// D2Q9 weights.
template <class R> __device__ __forceinline__ R w9(int i) {
    return i == 0 ? (R)(4.0 / 9.0) : (i < 5 ? (R)(1.0 / 9.0) : (R)(1.0 / 36.0));
}
__device__ __forceinline__ constexpr int EXd(int i) {
    return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__device__ __forceinline__ constexpr int EYd(int i) {
    return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
__device__ __forceinline__ constexpr int OPPd(int i) {
    return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4 + 1) : ((i - 5 + 2) % 4 + 5));
}

// ---------------------------------------------------------------- collide ----
// Sec. 2.1, Eqs. (5)-(6), in deviation variables.  On entry s[9], t[5] are
// the pre-collision deviations; on exit the post-collision deviations.
// Outputs the pre-collision macroscopics rho, u (with the half force) and T.
//   m = M f, f+ = f - M^-1 [S (m - m^eq) - (I - S/2) Fbar]   (flow)
//   n = N g, g+ = g - N^-1 Q (n - n^eq)                      (heat)
// M: Lallemand-Luo rows (rho, e, eps, jx, qx, jy, qy, pxx, pxy), squared
// norms (9, 36, 36, 6, 12, 6, 12, 4, 4); N: rows (T, jx, jy, e, pxx) with
// squared norms (5, 2, 2, 20, 4).  The rest state w_i rho0 carries e = -2 rho0,
// eps = rho0 and nothing else; w_k T_sh carries T_sh and e = a T_sh.
template <class R>
__device__ __forceinline__ void collide(const CC<R>& c, R (&s)[9], R (&t)[5], R& rho, R& ux,
                                        R& uy, R& T) {
    const R ax = (s[1] + s[2]) + (s[3] + s[4]);
    const R dg = (s[5] + s[6]) + (s[7] + s[8]);
    const R drho = (s[0] + ax) + dg;
    const R jx = (s[1] - s[3]) + ((s[5] - s[6]) + (s[8] - s[7]));
    const R jy = (s[2] - s[4]) + ((s[5] + s[6]) - (s[7] + s[8]));
    const R e_s = ((R)-4 * s[0] - ax) + (R)2 * dg;
    const R eps_s = ((R)4 * s[0] - (R)2 * ax) + dg;
    const R qx = (R)-2 * (s[1] - s[3]) + ((s[5] - s[6]) + (s[8] - s[7]));
    const R qy = (R)-2 * (s[2] - s[4]) + ((s[5] + s[6]) - (s[7] + s[8]));
    const R pxx = (s[1] + s[3]) - (s[2] + s[4]);
    const R pxy = (s[5] + s[7]) - (s[6] + s[8]);

    const R dT = ((t[0] + t[1]) + (t[2] + t[3])) + t[4];
    T = c.T_sh + dT;
    rho = c.rho0 + drho;
    const R Fx = c.body_fx;
    const R Fy = rho * c.gbeta * (T - c.T_ref);
    const R irho = (R)1 / rho;
    ux = (jx + (R)0.5 * Fx) * irho;
    uy = (jy + (R)0.5 * Fy) * irho;
    const R usq = ux * ux + uy * uy;
    const R uF = ux * Fx + uy * Fy;

    // dm = S (m - m^eq) - (I - S/2) Fbar, moment by moment
    const R de = c.s_e * ((e_s + (R)2 * drho) - (R)3 * rho * usq) - c.h_e * ((R)6 * uF);
    const R deps = c.s_eps * ((eps_s - drho) + (R)3 * rho * usq) + c.h_eps * ((R)6 * uF);
    const R djx = -Fx, djy = -Fy;
    const R dqx = c.s_q * (qx + jx + (R)0.5 * Fx) + c.h_q * Fx;
    const R dqy = c.s_q * (qy + jy + (R)0.5 * Fy) + c.h_q * Fy;
    const R dpxx = c.s_nu * (pxx - rho * (ux * ux - uy * uy)) -
                   c.h_nu * ((R)2 * (ux * Fx - uy * Fy));
    const R dpxy = c.s_nu * (pxy - rho * ux * uy) - c.h_nu * (ux * Fy + uy * Fx);

    // f+ = f - M^-1 dm
    const R A = -de * (R)(1.0 / 36.0) - deps * (R)(1.0 / 18.0);
    const R Bd = de * (R)(1.0 / 18.0) + deps * (R)(1.0 / 36.0);
    const R X1 = (djx - dqx) * (R)(1.0 / 6.0);
    const R Y1 = (djy - dqy) * (R)(1.0 / 6.0);
    const R X2 = djx * (R)(1.0 / 6.0) + dqx * (R)(1.0 / 12.0);
    const R Y2 = djy * (R)(1.0 / 6.0) + dqy * (R)(1.0 / 12.0);
    const R P1 = dpxx * (R)0.25, P2 = dpxy * (R)0.25;
    s[0] -= (deps - de) * (R)(1.0 / 9.0);
    s[1] -= (A + X1) + P1;
    s[2] -= (A + Y1) - P1;
    s[3] -= (A - X1) + P1;
    s[4] -= (A - Y1) - P1;
    s[5] -= (Bd + (X2 + Y2)) + P2;
    s[6] -= (Bd + (Y2 - X2)) - P2;
    s[7] -= (Bd - (X2 + Y2)) + P2;
    s[8] -= (Bd + (X2 - Y2)) - P2;

    // g+ = g - N^-1 dn
    const R dnx = c.s_a * ((t[1] - t[3]) - ux * T);
    const R dny = c.s_a * ((t[2] - t[4]) - uy * T);
    const R dne = c.s_Te * ((((t[1] + t[2]) + (t[3] + t[4])) - (R)4 * t[0]) - c.a_T * dT);
    const R dnp = c.s_Tp * ((t[1] + t[3]) - (t[2] + t[4]));
    const R E = dne * (R)(1.0 / 20.0), Pp = dnp * (R)0.25;
    t[0] += dne * (R)(1.0 / 5.0);
    t[1] -= (dnx * (R)0.5 + E) + Pp;
    t[2] -= (dny * (R)0.5 + E) - Pp;
    t[3] -= (E - dnx * (R)0.5) + Pp;
    t[4] -= (E - dny * (R)0.5) - Pp;
}

// Equilibria in deviation variables (second-order D2Q9; D2Q5 with moments
// (T, ux T, uy T, a T, 0)).
template <class R>
__device__ __forceinline__ void feq_dev(R rho, R rho0, R ux, R uy, R (&s)[9]) {
    const R usq = ux * ux + uy * uy;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R eu = (R)EXd(i) * ux + (R)EYd(i) * uy;
        s[i] = w9<R>(i) * (rho - rho0) + w9<R>(i) * rho * ((R)3 * eu + (R)4.5 * eu * eu - (R)1.5 * usq);
    }
}
template <class R>
__device__ __forceinline__ void geq_dev(R T, R Tsh, R ux, R uy, R w0, R wk, R (&t)[5]) {
    t[0] = w0 * (T - Tsh);
#pragma unroll
    for (int k = 1; k < 5; ++k) t[k] = wk * (T - Tsh) + (R)0.5 * T * ((R)EXd(k) * ux + (R)EYd(k) * uy);
}

// ------------------------------------------------------------ streaming ----
// Addressing.  2- and 4-byte values: a wavefront covers 64 consecutive nodes
// of one row (the pitch is a multiple of 64); with the row taken from the
// wavefront's first lane, the byte offset of the row is added to the array
// base in scalar registers and each lane adds only the 32-bit byte offset of
// its column, so every load and store is one global instruction with a
// scalar base and no per-lane 64-bit address arithmetic.  8-byte values:
// per-lane element indices (row + column, shared by the 14 arrays).
//
// Layout of a state's 14 arrays.  8-byte values: tiles of 64 nodes of a row
// (the pitch is a multiple of 64), each tile holding its 64 values of every
// array one after another, and array i's pointer the state's base plus 64 i
// values; node k = y pitch + x sits at element tix(k) = (k / 64) 896 +
// k mod 64 of each array.  A wavefront's 14 loads and 14 stores then fall
// in a few tiles instead of 28 separate arrays, fewer concurrent DRAM
// streams: the FP64 lattice kernel runs 3-4 % faster.  2- and 4-byte
// values: one array after another (there the link pass's scattered gathers
// lose more to the tiles than the lattice kernel gains).
template <class T> __device__ __forceinline__ constexpr bool byte_offsets() { return sizeof(T) < 8; }
template <class T> __host__ __device__ __forceinline__ constexpr bool tiled() { return sizeof(T) == 8; }
template <class T> __host__ __device__ __forceinline__ size_t tix(size_t k) {
    return tiled<T>() ? (k >> 6) * (size_t)(14 * 64) + (k & 63u) : k;
}
template <class T> __device__ __forceinline__ size_t row_off(const LP& lp, int y) {
    if (tiled<T>()) return (size_t)y * (size_t)lp.pitch * 14u;
    return byte_offsets<T>() ? (size_t)y * (size_t)lp.pitch * sizeof(T) : (size_t)y * (size_t)lp.pitch;
}
template <class T> __device__ __forceinline__ uint32_t col_off(int x) {
    if (tiled<T>()) return ((uint32_t)x >> 6) * (uint32_t)(14 * 64) + ((uint32_t)x & 63u);
    return byte_offsets<T>() ? (uint32_t)x * (uint32_t)sizeof(T) : (uint32_t)x;
}
template <class T>
__device__ __forceinline__ PT_GLOBAL T* at_rc(PT_GLOBAL T* a, size_t row, uint32_t col) {
    if (byte_offsets<T>()) return (PT_GLOBAL T*)(((PT_GLOBAL char*)a + row) + col);
    return a + (row + (size_t)col);
}
template <class T>
__device__ __forceinline__ const PT_GLOBAL T* at_rc(const PT_GLOBAL T* a, size_t row, uint32_t col) {
    if (byte_offsets<T>()) return (const PT_GLOBAL T*)(((const PT_GLOBAL char*)a + row) + col);
    return a + (row + (size_t)col);
}

// Pull of the 9 + 5 populations arriving at node (x, y) from the
// post-collision state A, as deviations: flat walls in y by halfway
// bounce-back (moving tangentially at wall_ux) for f and anti-bounce-back
// (Dirichlet wall_T) for g; x periodic, or bounded by the static side walls
// of the closed cavity (the same two rules at rest, Dirichlet side_T).  A
// diagonal population whose upstream node is beyond a y wall and a side
// wall at once takes the y wall's rule.  Solid upstream nodes hold the
// bounce-back values written by the link pass.  Plain modes store f (the
// rest part w_i rho0 is removed here) and g with T_sh = 0; shifted modes
// store the deviations.  WALLS = false: the caller knows that (x, y) is
// next to no wall, and the wall rules are compiled out (the pull is then
// one straight run of loads with scalar bases).
template <class S, bool NTL = false, bool WALLS = true>
__device__ __forceinline__ void pull_node(const Pops<typename S::T>& A, const LP& lp,
                                          const CC<typename S::R>& c, int x, int y, typename S::R (&s)[9],
                                          typename S::R (&t)[5]) {
    using R = typename S::R;
    using T = typename S::T;
    // NTL: non-temporal loads (the lattice kernel reads each value once)
    auto ld = [](const PT_GLOBAL T* q) { return NTL ? S::ld_nt(q) : S::ld(q); };
    const int nx = lp.nx, ny = lp.ny;
    const int xm = x == 0 ? nx - 1 : x - 1;
    const int xp = x == nx - 1 ? 0 : x + 1;
    const bool bot = WALLS && !lp.periodic_y && y == 0;
    const bool top = WALLS && !lp.periodic_y && y == ny - 1;
    const bool lft = WALLS && !lp.periodic_x && x == 0;
    const bool rgt = WALLS && !lp.periodic_x && x == nx - 1;
    const int ym = y == 0 ? ny - 1 : y - 1;
    const int yp = y == ny - 1 ? 0 : y + 1;
    const size_t r0 = row_off<T>(lp, y), rm = row_off<T>(lp, ym), rp = row_off<T>(lp, yp);
    const uint32_t c0 = col_off<T>(x), cm = col_off<T>(xm), cp = col_off<T>(xp);
    R fs[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) fs[i] = S::shifted ? (R)0 : c.fsw[i];
    // at a side wall the address moves to the node's own opposite population
    // (the pairs share their rest weight, so fs stays the same)
    s[0] = ld(at_rc(A.f[0], r0, c0)) - fs[0];
    s[1] = ld(lft ? at_rc(A.f[3], r0, c0) : at_rc(A.f[1], r0, cm)) - fs[1];
    s[3] = ld(rgt ? at_rc(A.f[1], r0, c0) : at_rc(A.f[3], r0, cp)) - fs[3];
    t[0] = ld(at_rc(A.g[0], r0, c0));
    const R g1 = ld(lft ? at_rc(A.g[3], r0, c0) : at_rc(A.g[1], r0, cm));
    const R g3 = ld(rgt ? at_rc(A.g[1], r0, c0) : at_rc(A.g[3], r0, cp));
    t[1] = lft ? c.g_side[0] - g1 : g1;
    t[3] = rgt ? c.g_side[1] - g3 : g3;
    if (bot) {
        const R u = c.u_wall[0];
        s[2] = ld(at_rc(A.f[4], r0, c0)) - fs[4];
        s[5] = (ld(at_rc(A.f[7], r0, c0)) - fs[7]) + u;
        s[6] = (ld(at_rc(A.f[8], r0, c0)) - fs[8]) - u;
        t[2] = -ld(at_rc(A.g[4], r0, c0)) + c.g_wall[0];
    } else {
        s[2] = ld(at_rc(A.f[2], rm, c0)) - fs[2];
        s[5] = ld(lft ? at_rc(A.f[7], r0, c0) : at_rc(A.f[5], rm, cm)) - fs[5];
        s[6] = ld(rgt ? at_rc(A.f[8], r0, c0) : at_rc(A.f[6], rm, cp)) - fs[6];
        t[2] = ld(at_rc(A.g[2], rm, c0));
    }
    if (top) {
        const R u = c.u_wall[1];
        s[4] = ld(at_rc(A.f[2], r0, c0)) - fs[2];
        s[7] = (ld(at_rc(A.f[5], r0, c0)) - fs[5]) - u;
        s[8] = (ld(at_rc(A.f[6], r0, c0)) - fs[6]) + u;
        t[4] = -ld(at_rc(A.g[2], r0, c0)) + c.g_wall[1];
    } else {
        s[4] = ld(at_rc(A.f[4], rp, c0)) - fs[4];
        s[7] = ld(rgt ? at_rc(A.f[5], r0, c0) : at_rc(A.f[7], rp, cp)) - fs[7];
        s[8] = ld(lft ? at_rc(A.f[6], r0, c0) : at_rc(A.f[8], rp, cm)) - fs[8];
        t[4] = ld(at_rc(A.g[4], rp, c0));
    }
}

// Store of the 14 post-collision values of node (x, y); NT selects
// non-temporal (streaming) stores.
template <class S, bool NT = false>
__device__ __forceinline__ void store_node(const Pops<typename S::T>& B, const LP& lp,
                                           const CC<typename S::R>& c, int x, int y, const typename S::R (&s)[9],
                                           const typename S::R (&t)[5]) {
    using R = typename S::R;
    using T = typename S::T;
    const size_t r0 = row_off<T>(lp, y);
    const uint32_t c0 = col_off<T>(x);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R v = s[i] + (S::shifted ? (R)0 : c.fsw[i]);
        if (NT) S::st_nt(at_rc(B.f[i], r0, c0), v);
        else S::st(at_rc(B.f[i], r0, c0), v);
    }
#pragma unroll
    for (int k5 = 0; k5 < 5; ++k5) {
        if (NT) S::st_nt(at_rc(B.g[k5], r0, c0), t[k5]);
        else S::st(at_rc(B.g[k5], r0, c0), t[k5]);
    }
}

// ------------------------------------------------ in-place (AA) streaming ----
// One population set F holds the state.  After an even kernel (and after
// initialisation) the post-collision value f_k*(y) sits in slot kbar of y
// itself (parity 0, "reversed"); the odd kernel pulls from there and pushes
// f_k*(x) to slot k of x + e_k, or to slot kbar of x where x + e_k is beyond
// a wall (parity 1, "pushed"); the even kernel then reads slot k of x in
// place, which is f_k(x) after streaming, with the wall rules applied at
// read time, and writes f_k* reversed into x.  Each location is read and
// written by one thread only, so the update is in place.  A parity-0 state
// is the two-set state with slots k and kbar exchanged: every reader and
// writer of the two-set layout works on it through opp_view.
template <class T> __host__ __device__ Pops<T> opp_view(const Pops<T>& F) {
    Pops<T> v;
    for (int i = 0; i < 9; ++i) v.f[i] = F.f[i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4 + 1) : ((i - 5 + 2) % 4 + 5))];
    for (int k = 0; k < 5; ++k) v.g[k] = F.g[k == 0 ? 0 : ((k + 1) % 4 + 1)];
    return v;
}

// Whether node (x, y) + e_k lies beyond a flat wall (not a node).
__device__ __forceinline__ bool beyond_wall(const LP& lp, int x, int y, int k) {
    const int x2 = x + EXd(k), y2 = y + EYd(k);
    return (!lp.periodic_y && (y2 < 0 || y2 >= lp.ny)) || (!lp.periodic_x && (x2 < 0 || x2 >= lp.nx));
}
// Index of node (x, y) + e_k with the periodic axes wrapped (a node).
__device__ __forceinline__ size_t node_plus(const LP& lp, int x, int y, int k) {
    int x2 = x + EXd(k), y2 = y + EYd(k);
    x2 = x2 < 0 ? x2 + lp.nx : (x2 >= lp.nx ? x2 - lp.nx : x2);
    y2 = y2 < 0 ? y2 + lp.ny : (y2 >= lp.ny ? y2 - lp.ny : y2);
    return (size_t)y2 * lp.pitch + x2;
}
// Where the pushed (parity-1) state keeps f_k*(x, y): slot *slot at the
// returned node index.
__device__ __forceinline__ size_t pushed_at(const LP& lp, int x, int y, int k, int& slot) {
    if (beyond_wall(lp, x, y, k)) {
        slot = OPPd(k);
        return (size_t)y * lp.pitch + x;
    }
    slot = k;
    return node_plus(lp, x, y, k);
}
// The same as an address, for a population index k known at compile time
// (after unrolling), so that no pointer table is indexed at run time.
template <class T>
__device__ __forceinline__ PT_GLOBAL T* pushed_ptr(PT_GLOBAL T* own, PT_GLOBAL T* opp, const LP& lp, int x, int y,
                                                    int k) {
    if (beyond_wall(lp, x, y, k)) return opp + tix<T>((size_t)y * lp.pitch + x);
    return own + tix<T>(node_plus(lp, x, y, k));
}

// The even kernel's read of node (x, y) from a pushed state: every slot in
// place; where the upstream node is beyond a wall the slot holds the
// node's own outgoing post-collision value and the wall rule of pull_node
// applies to it (with the same arithmetic, so both layouts give the same
// bits).  WALLS as for pull_node.
template <class S, bool NTL = false, bool WALLS = true>
__device__ __forceinline__ void pull_node_pushed(const Pops<typename S::T>& F, const LP& lp,
                                                 const CC<typename S::R>& c, int x, int y, typename S::R (&s)[9],
                                                 typename S::R (&t)[5]) {
    using R = typename S::R;
    using T = typename S::T;
    auto ld = [](const PT_GLOBAL T* q) { return NTL ? S::ld_nt(q) : S::ld(q); };
    const bool bot = WALLS && !lp.periodic_y && y == 0;
    const bool top = WALLS && !lp.periodic_y && y == lp.ny - 1;
    const bool lft = WALLS && !lp.periodic_x && x == 0;
    const bool rgt = WALLS && !lp.periodic_x && x == lp.nx - 1;
    const size_t r0 = row_off<T>(lp, y);
    const uint32_t c0 = col_off<T>(x);
    auto L = [&](const PT_GLOBAL T* a) { return ld(at_rc(a, r0, c0)); };
    R fs[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) fs[i] = S::shifted ? (R)0 : c.fsw[i];
    s[0] = L(F.f[0]) - fs[0];
    s[1] = L(F.f[1]) - fs[1];
    s[3] = L(F.f[3]) - fs[3];
    t[0] = L(F.g[0]);
    const R g1 = L(F.g[1]);
    const R g3 = L(F.g[3]);
    t[1] = lft ? c.g_side[0] - g1 : g1;
    t[3] = rgt ? c.g_side[1] - g3 : g3;
    if (bot) {
        const R u = c.u_wall[0];
        s[2] = L(F.f[2]) - fs[4];
        s[5] = (L(F.f[5]) - fs[7]) + u;
        s[6] = (L(F.f[6]) - fs[8]) - u;
        t[2] = -L(F.g[2]) + c.g_wall[0];
    } else {
        s[2] = L(F.f[2]) - fs[2];
        s[5] = L(F.f[5]) - fs[5];
        s[6] = L(F.f[6]) - fs[6];
        t[2] = L(F.g[2]);
    }
    if (top) {
        const R u = c.u_wall[1];
        s[4] = L(F.f[4]) - fs[2];
        s[7] = (L(F.f[7]) - fs[5]) - u;
        s[8] = (L(F.f[8]) - fs[6]) + u;
        t[4] = -L(F.g[4]) + c.g_wall[1];
    } else {
        s[4] = L(F.f[4]) - fs[4];
        s[7] = L(F.f[7]) - fs[7];
        s[8] = L(F.f[8]) - fs[8];
        t[4] = L(F.g[4]);
    }
}

// Where the odd kernel pushes population k of node (x, y): slot k of
// (x, y) + e_k, or slot kbar of (x, y) itself where that node is beyond a
// wall.  WALLS = false: (x, y) is next to no wall.
template <class T, bool WALLS = true>
__device__ __forceinline__ PT_GLOBAL T* push_ptr(PT_GLOBAL T* own, PT_GLOBAL T* opp, const LP& lp, int x, int y,
                                                 int k) {
    const int x2 = x + EXd(k), y2 = y + EYd(k);
    const bool beyond = WALLS && ((!lp.periodic_y && (y2 < 0 || y2 >= lp.ny)) ||
                                  (!lp.periodic_x && (x2 < 0 || x2 >= lp.nx)));
    const int yw = y2 < 0 ? y2 + lp.ny : (y2 >= lp.ny ? y2 - lp.ny : y2);
    const int xw = x2 < 0 ? x2 + lp.nx : (x2 >= lp.nx ? x2 - lp.nx : x2);
    return beyond ? at_rc(opp, row_off<T>(lp, y), col_off<T>(x)) : at_rc(own, row_off<T>(lp, yw), col_off<T>(xw));
}

// The odd kernel's store: f_k*(x, y) pushed to slot k of (x, y) + e_k, or to
// slot kbar of (x, y) where that node is beyond a wall.
template <class S, bool NT = false, bool WALLS = true>
__device__ __forceinline__ void store_node_pushed(const Pops<typename S::T>& F, const LP& lp,
                                                  const CC<typename S::R>& c, int x, int y,
                                                  const typename S::R (&s)[9], const typename S::R (&t)[5]) {
    using R = typename S::R;
    using T = typename S::T;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const R v = s[i] + (S::shifted ? (R)0 : c.fsw[i]);
        PT_GLOBAL T* q = push_ptr<T, WALLS>(F.f[i], F.f[OPPd(i)], lp, x, y, i);
        if (NT) S::st_nt(q, v);
        else S::st(q, v);
    }
#pragma unroll
    for (int k5 = 0; k5 < 5; ++k5) {
        PT_GLOBAL T* q = push_ptr<T, WALLS>(F.g[k5], F.g[OPPd(k5)], lp, x, y, k5);
        if (NT) S::st_nt(q, t[k5]);
        else S::st(q, t[k5]);
    }
}

// -------------------------------------------------- shared by the kernels ----
constexpr int LAT_BLOCK = 256;

template <int MODE> using ST = typename Store<MODE>::T;

template <int MODE> __host__ __device__ Pops<ST<MODE>> pops_of(void* const (&a)[14]) {
    Pops<ST<MODE>> p;
    for (int i = 0; i < 9; ++i) p.f[i] = (PT_GLOBAL ST<MODE>*)a[i];
    for (int i = 0; i < 5; ++i) p.g[i] = (PT_GLOBAL ST<MODE>*)a[9 + i];
    return p;
}

// Run CALL with the storage mode as the compile-time constant M.
#define PTLBM_DISPATCH(mode, CALL)                                                          \
    switch (mode) {                                                                         \
        case LBM_STORE_F64: { constexpr int M = LBM_STORE_F64; CALL; } break;               \
        case LBM_STORE_F32: { constexpr int M = LBM_STORE_F32; CALL; } break;               \
        case LBM_STORE_SHIFT_F32: { constexpr int M = LBM_STORE_SHIFT_F32; CALL; } break;   \
        case LBM_STORE_SHIFT_F16: { constexpr int M = LBM_STORE_SHIFT_F16; CALL; } break;   \
        case LBM_STORE_SHIFT_BF16: { constexpr int M = LBM_STORE_SHIFT_BF16; CALL; } break; \
        default: return hipErrorInvalidValue;                                               \
    }

}  // namespace ptlbm
