// lattice.hip -- the gfx950 lattice kernels of the particle-resolved thermal
// lattice Boltzmann method (Xu & Li, arXiv 2308.16597): the fused
// pull-stream + D2Q9/D2Q5 MRT collision of every node of one step (Sec. 2.1,
// Eqs. (5)-(6)), for one run or batched over many, and the initialisation
// and read-back of macroscopic fields.
// Built with -ffp-contract=off, like the particle kernels.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace ptlbm {

// ------------------------------------------------------ lattice kernels ----

// Node of lane `threadIdx.x` in block `bid` of the flat grid.  ROW: the row
// is the same for the whole wavefront (the pitch is a multiple of 64) and is
// taken from its first lane, so that it lives in scalar registers and every
// access has a scalar base (the pitched lattice has fewer than 2^32 nodes:
// both edges are below 2^16).  Otherwise each lane divides for itself.
template <bool ROW>
__device__ __forceinline__ void lattice_node(const LP& lp, unsigned bid, int& x, int& y) {
    if (ROW) {
        const unsigned w0 = (unsigned)__builtin_amdgcn_readfirstlane((int)threadIdx.x);   // first lane of the wave
        const unsigned n0 = bid * (unsigned)LAT_BLOCK + w0;
        y = (int)(n0 / (unsigned)lp.pitch);
        x = (int)(n0 - (unsigned)y * (unsigned)lp.pitch) + (int)(threadIdx.x - w0);
    } else {
        const size_t n0 = (size_t)bid * LAT_BLOCK + threadIdx.x;
        y = (int)(n0 / (unsigned)lp.pitch);
        x = (int)(n0 - (size_t)y * lp.pitch);
    }
}

// Scalar row bases and a wall-free pull for the nodes next to no wall pay
// off where the kernel's arithmetic limits it (FP32 arithmetic on 2- and
// 4-byte values: 45 % fewer instructions per node); with 8-byte values the
// kernel moves the same bytes 2.5 % faster with per-lane addresses and the
// wall rules evaluated in every node (both measured at 4000^2).
template <int MODE> constexpr bool row_addressing() { return sizeof(ST<MODE>) < 8; }

// A node next to a wall: a side wall of the closed cavity or a flat wall in
// y.  The pulls and pushes take the wall rules there; everywhere else they
// are compiled out.
__device__ __forceinline__ bool next_to_wall(const LP& lp, int x, int y) {
    return (!lp.periodic_x && (x == 0 || x == lp.nx - 1)) || (!lp.periodic_y && (y == 0 || y == lp.ny - 1));
}

template <class R>
__device__ __forceinline__ void check_finite(const RunStep& rs, int x, int y, R rho, R ux, R uy, R T) {
    if (isfinite(rho) && isfinite(T) && isfinite(ux) && isfinite(uy)) return;
    if (gl(rs.Ocur)[(size_t)y * rs.lp.pitch + x] != -1) return;
    // one report per wavefront, none once the bit is set: a run that has
    // gone non-finite must not serialise on its status word
    const unsigned long long m = __ballot(1);
    if ((threadIdx.x & 63) == (unsigned)(__ffsll((long long)m) - 1) && !(gl(rs.status)[0] & ST_NONFINITE))
        atomicOr(rs.status, ST_NONFINITE);
}

// Fused pull-stream + collide of every node of the lattice, one thread per
// node of the pitched layout (flat 1-D grid, rows padded to the pitch).
// Every node is written, so each wavefront stores whole cache lines: nodes
// that are solid at t_n+1 receive values nobody reads (their slots facing the
// fluid are rewritten by the next link pass), and newborn nodes are
// overwritten by the refill kernel that runs after this one.  The stores are
// non-temporal: B is not read again before the next step.  A non-finite
// macroscopic value is an error at a node fluid at t_n (a node solid at t_n
// pulls from inside the particle); the owner map is read only for a node
// whose value is non-finite, so the check costs no traffic while the run is
// sound.  The kernel reads nothing that the particle kernels of the same
// step write, so those may run concurrently with it.  The nodes next to no
// wall (all but a few wavefronts) take a pull without wall rules.
template <int MODE, bool WALLS>
__device__ __forceinline__ void two_sets_node(const RunStep& rs, const CC<typename Store<MODE>::R>& c, int x,
                                              int y) {
    using S = Store<MODE>;
    using R = typename S::R;
    const LP& lp = rs.lp;
    const Pops<ST<MODE>> A = pops_of<MODE>(rs.A), B = pops_of<MODE>(rs.B);
    R s[9], t[5];
    pull_node<S, true, WALLS>(A, lp, c, x, y, s, t);
    R rho, ux, uy, T;
    collide<R>(c, s, t, rho, ux, uy, T);
    store_node<S, true>(B, lp, c, x, y, s, t);
    check_finite<R>(rs, x, y, rho, ux, uy, T);
}

template <int MODE>
__device__ __forceinline__ void stream_collide_body(const RunStep& rs, unsigned bid) {
    constexpr bool ROW = row_addressing<MODE>();
    int x, y;
    lattice_node<ROW>(rs.lp, bid, x, y);
    if (x >= rs.lp.nx || y >= rs.lp.ny) return;
    const CC<typename Store<MODE>::R> c = lp_cc<typename Store<MODE>::R>(rs.lp);
    if (!ROW || next_to_wall(rs.lp, x, y)) two_sets_node<MODE, true>(rs, c, x, y);
    else two_sets_node<MODE, false>(rs, c, x, y);
}

// The same step in place (AA streaming, one population set F = A = B).
// ODD: from a reversed (parity-0) state, the pull of pull_node through
// opp_view, the post-collision values pushed to the neighbours (parity 1
// after it).  EVEN: from a pushed state, every slot read in place
// (pull_node_pushed) and written back reversed into the node (parity 0).
// Same collision, same wall rules, same values as the two-set kernel.
template <int MODE, bool ODD, bool WALLS>
__device__ __forceinline__ void in_place_node(const RunStep& rs, const CC<typename Store<MODE>::R>& c, int x,
                                              int y) {
    using S = Store<MODE>;
    using R = typename S::R;
    const LP& lp = rs.lp;
    const Pops<ST<MODE>> F = pops_of<MODE>(rs.A);
    R s[9], t[5];
    if (ODD) pull_node<S, true, WALLS>(opp_view(F), lp, c, x, y, s, t);
    else pull_node_pushed<S, true, WALLS>(F, lp, c, x, y, s, t);
    R rho, ux, uy, T;
    collide<R>(c, s, t, rho, ux, uy, T);
    if (ODD) store_node_pushed<S, true, WALLS>(F, lp, c, x, y, s, t);
    else store_node<S, true>(opp_view(F), lp, c, x, y, s, t);
    check_finite<R>(rs, x, y, rho, ux, uy, T);
}

template <int MODE, bool ODD>
__device__ __forceinline__ void stream_collide_aa_body(const RunStep& rs, unsigned bid) {
    constexpr bool ROW = row_addressing<MODE>();
    int x, y;
    lattice_node<ROW>(rs.lp, bid, x, y);
    if (x >= rs.lp.nx || y >= rs.lp.ny) return;
    const CC<typename Store<MODE>::R> c = lp_cc<typename Store<MODE>::R>(rs.lp);
    if (!ROW || next_to_wall(rs.lp, x, y)) in_place_node<MODE, ODD, true>(rs, c, x, y);
    else in_place_node<MODE, ODD, false>(rs, c, x, y);
}

// Equilibrium of the given macroscopic fields (host layout j*nx + i over
// rows y0.., NULL pointers select the uniform rest state), collided once:
// the post-collision state of t_0, in the two-set layout or, in place, in
// the layout of the given parity.
template <int MODE, class FT>
__global__ __launch_bounds__(LAT_BLOCK) void k_init(Pops<ST<MODE>> A, const int32_t* __restrict__ owner,
                                                    const FT* rho_f, const FT* ux_f, const FT* uy_f,
                                                    const FT* T_f, double rho_u, double T_u, int y0, int parity,
                                                    LP lp) {
    using S = Store<MODE>;
    using R = typename S::R;
    const int x = blockIdx.x * LAT_BLOCK + threadIdx.x;
    const int y = y0 + (int)blockIdx.y;
    if (x >= lp.nx) return;
    const size_t k = (size_t)y * lp.pitch + x;
    const size_t h = (size_t)blockIdx.y * lp.nx + x;
    const CC<R> c = lp_cc<R>(lp);
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
        R r_, u_, v_, T_;
        collide<R>(c, s, t, r_, u_, v_, T_);
    }
    if (!lp.aa) store_node<S>(A, lp, c, x, y, s, t);
    else if (parity == 0) store_node<S>(opp_view(A), lp, c, x, y, s, t);
    else store_node_pushed<S>(A, lp, c, x, y, s, t);
}

// Pre-collision macroscopics from the post-collision state: rho and T are
// collision invariants and the momentum gained the force, so
// u = (j+ - F/2)/rho.  NaN inside solids.  Output: 4 planes of nx * rows
// (OT) for rows y0..; the state in either layout.
template <int MODE, class OT>
__global__ __launch_bounds__(LAT_BLOCK) void k_macros(Pops<ST<MODE>> A, const int32_t* __restrict__ owner,
                                                      OT* out, int y0, int rows, int parity, LP lp) {
    using S = Store<MODE>;
    using R = typename S::R;
    const int x = blockIdx.x * LAT_BLOCK + threadIdx.x;
    const int y = y0 + (int)blockIdx.y;
    if (x >= lp.nx) return;
    const size_t k = (size_t)y * lp.pitch + x;
    const size_t n = (size_t)lp.nx * rows, h = (size_t)blockIdx.y * lp.nx + x;
    if (lp.aa && parity == 0) A = opp_view(A);
    if (owner[k] >= 0) {
        const OT nan = (OT)NAN;
        out[h] = nan;
        out[n + h] = nan;
        out[2 * n + h] = nan;
        out[3 * n + h] = nan;
        return;
    }
    R s[9], t[5];
    if (lp.aa && parity == 1) {   // pushed: f_k* sits at the neighbour (or reversed at a wall)
#pragma unroll
        for (int i = 0; i < 9; ++i)
            s[i] = S::ld(pushed_ptr(A.f[i], A.f[OPPd(i)], lp, x, y, i)) -
                   (S::shifted ? (R)0 : w9<R>(i) * (R)lp.rho0);
#pragma unroll
        for (int i = 0; i < 5; ++i) t[i] = S::ld(pushed_ptr(A.g[i], A.g[OPPd(i)], lp, x, y, i));
    } else {
#pragma unroll
        for (int i = 0; i < 9; ++i) s[i] = S::ld(A.f[i] + tix<ST<MODE>>(k)) - (S::shifted ? (R)0 : w9<R>(i) * (R)lp.rho0);
#pragma unroll
        for (int i = 0; i < 5; ++i) t[i] = S::ld(A.g[i] + tix<ST<MODE>>(k));
    }
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

// The lattice step kernel for one run (RunStep by value) and batched (block
// b works on block bmap[b].y of run bmap[b].x, whose RunStep is
// tab[bmap[b].x]); both run the same body.
// Wavefronts per SIMD: with 8-byte values the lattice kernels move their
// bytes fastest at 5 (two sets), 4 (in place, odd) and 5 (in place, even),
// the occupancies their register counts gave before the scalar row
// addressing of the narrow types (at 4000^2: 611 us at 5 against 624 us
// at 6 for the two-set kernel); the narrow types are not limited.
template <int MODE> constexpr int lattice_waves(bool odd = false) {
    return sizeof(ST<MODE>) == 8 ? (odd ? 4 : 5) : 8;
}

template <int MODE>
__global__ __launch_bounds__(LAT_BLOCK) __attribute__((amdgpu_waves_per_eu(1, lattice_waves<MODE>())))
void k_stream_collide(RunStep rs) {
    stream_collide_body<MODE>(rs, blockIdx.x);
}
template <int MODE>
__global__ __launch_bounds__(LAT_BLOCK) void k_stream_collide_b(const RunStep* __restrict__ tab,
                                                                const uint2* __restrict__ bmap) {
    const uint2 m = bmap[blockIdx.x];
    stream_collide_body<MODE>(tab[m.x], m.y);
}
template <int MODE, bool ODD>
__global__ __launch_bounds__(LAT_BLOCK) __attribute__((amdgpu_waves_per_eu(1, lattice_waves<MODE>(ODD))))
void k_stream_collide_aa(RunStep rs) {
    stream_collide_aa_body<MODE, ODD>(rs, blockIdx.x);
}
// batched in place: each run at its own parity (one branch per block)
template <int MODE>
__global__ __launch_bounds__(LAT_BLOCK) void k_stream_collide_aa_b(const RunStep* __restrict__ tab,
                                                                   const uint2* __restrict__ bmap) {
    const uint2 m = bmap[blockIdx.x];
    if (tab[m.x].parity == 0) stream_collide_aa_body<MODE, true>(tab[m.x], m.y);
    else stream_collide_aa_body<MODE, false>(tab[m.x], m.y);
}

// -------------------------------------------------------------- launchers ----

static dim3 lattice_grid(const LP& lp, int rows) { return dim3((lp.nx + LAT_BLOCK - 1) / LAT_BLOCK, rows); }

hipError_t launch_lattice(const RunStep& R, int mode, unsigned nblocks, hipStream_t st) {
    if (!R.lp.aa) {
        PTLBM_DISPATCH(mode, (k_stream_collide<M><<<nblocks, LAT_BLOCK, 0, st>>>(R)));
    } else if (R.parity == 0) {
        PTLBM_DISPATCH(mode, (k_stream_collide_aa<M, true><<<nblocks, LAT_BLOCK, 0, st>>>(R)));
    } else {
        PTLBM_DISPATCH(mode, (k_stream_collide_aa<M, false><<<nblocks, LAT_BLOCK, 0, st>>>(R)));
    }
    return hipGetLastError();
}

hipError_t launch_lattice_batch(const RunStep* tab, const uint2* bmap, unsigned nblocks, int mode, bool aa,
                                hipStream_t st) {
    if (aa) {
        PTLBM_DISPATCH(mode, (k_stream_collide_aa_b<M><<<nblocks, LAT_BLOCK, 0, st>>>(tab, bmap)));
    } else {
        PTLBM_DISPATCH(mode, (k_stream_collide_b<M><<<nblocks, LAT_BLOCK, 0, st>>>(tab, bmap)));
    }
    return hipGetLastError();
}

hipError_t launch_init(const DevState& d, int cur, int y0, int rows, const void* rho, const void* ux,
                       const void* uy, const void* T, bool f64, double rho_u, double T_u, hipStream_t st) {
    if (f64) {
        PTLBM_DISPATCH(d.mode, (k_init<M, double><<<lattice_grid(d.lp, rows), LAT_BLOCK, 0, st>>>(
                                   pops_of<M>(d.S[cur]), d.O[cur], (const double*)rho, (const double*)ux,
                                   (const double*)uy, (const double*)T, rho_u, T_u, y0, cur, d.lp)));
    } else {
        PTLBM_DISPATCH(d.mode, (k_init<M, float><<<lattice_grid(d.lp, rows), LAT_BLOCK, 0, st>>>(
                                   pops_of<M>(d.S[cur]), d.O[cur], (const float*)rho, (const float*)ux,
                                   (const float*)uy, (const float*)T, rho_u, T_u, y0, cur, d.lp)));
    }
    return hipGetLastError();
}

hipError_t launch_macros(const DevState& d, int cur, int y0, int rows, void* out, hipStream_t st) {
    if (d.mode == LBM_STORE_F64) {
        k_macros<LBM_STORE_F64, double><<<lattice_grid(d.lp, rows), LAT_BLOCK, 0, st>>>(
            pops_of<LBM_STORE_F64>(d.S[cur]), d.O[cur], (double*)out, y0, rows, cur, d.lp);
    } else {
        PTLBM_DISPATCH(d.mode, (k_macros<M, float><<<lattice_grid(d.lp, rows), LAT_BLOCK, 0, st>>>(
                                   pops_of<M>(d.S[cur]), d.O[cur], (float*)out, y0, rows, cur, d.lp)));
    }
    return hipGetLastError();
}

}  // namespace ptlbm
