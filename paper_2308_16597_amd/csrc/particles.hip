// particles.hip -- the gfx950 particle kernels of one step of the
// particle-resolved thermal lattice Boltzmann method (Xu & Li, arXiv
// 2308.16597), and the dispatch of all six step kernels (the lattice kernel
// itself is in lattice.hip).
//
// One step n -> n+1 (cur = time level n, ring = particle slot of t_n); the
// links of t_n were collected at the end of the step before:
// (the per-particle kernels below give a particle a wavefront, or a whole
// block when its window is wide and the particles are few)
//   k_link_pass     one block per particle (128, 256 or 512 threads by the
//                   particle size), a thread per link: q, wall
//                   velocity, Bouzidi bounce-back (Eqs. (9)-(10)) and the
//                   thermal wall (Eqs. (11)-(12)) written where the lattice
//                   kernel pulls them; the momentum exchange (Eqs. (13)-(14))
//                   summed over the particle in FP64 in a fixed order.
//   k_particles     per particle: clear its t_n-1 marks in the
//                   owner-map buffer of t_n+1; repulsion (Eq. (15)) summed
//                   in ascending partner order over a cell grid, net weight,
//                   Newton-Euler update.
//   k_mask_mark     per particle: owner map of t_n+1 by atomic
//                   min; newborn-node candidates.
//   k_stream_collide  one thread per node: fused pull-stream + D2Q9/D2Q5 MRT
//                   collision with buoyancy (Sec. 2.1) of the whole lattice
//                   (two kernels in place, lattice.hip).
//   k_refill        per particle: refilling + collision of the newborn nodes
//                   (Sec. 2.5): the values computed (from the state of t_n
//                   and the owner maps) and stored over the lattice kernel's
//                   output; a single run computes them on the second stream
//                   (in place before the lattice kernel; with two sets and
//                   2- or 4-byte values beside it) and stores them after it.
//   k_links         per particle: the links of t_n+1 from its
//                   owner map, collected into LDS in the fixed slot order of
//                   Sec. 3 (one slot per lattice line and direction), ballot
//                   + prefix count, compacted to the front of the
//                   particle's own segment of 12 N - 12 entries.
// k_particles, k_mask_mark, k_links and the refill's compute half write
// nothing k_stream_collide reads or writes (with two sets), so a single run
// launches them on a second stream, concurrent with the lattice kernel.
// Built with -ffp-contract=off: the solid test and link fractions must round
// exactly as the CPU oracle rounds them.
#include <hip/hip_runtime.h>

#include "link.h"

namespace ptlbm {

constexpr double kPi = 3.14159265358979323846;
constexpr int OUTSIDE = -2;

// ----------------------------------------------------- particle kernels ----
// The per-particle kernels run one wavefront per particle (4 particles per
// block), so that a particle's window, slots, neighbours and newborn nodes
// stay inside one wavefront and need no block-wide barrier; particles whose
// windows are 32 nodes wide or more get the whole block of 256 lanes when
// there are few of them (lp.lpp), with block barriers between the phases.


// Lanes of one particle: a wavefront (4 particles per block of 256) or, for
// particles whose windows are large (lp.lpp == 256), the whole block.
struct PartLanes {
    int p;       // particle
    int lane;    // lane within the particle's lanes
    int nl;      // lanes per particle
    bool blk;    // the block is the particle's
};
__device__ __forceinline__ PartLanes part_lanes(const LP& lp, unsigned bid) {
    PartLanes q;
    q.blk = lp.lpp > 64;
    q.nl = q.blk ? 256 : 64;
    q.lane = q.blk ? (int)threadIdx.x : (int)(threadIdx.x & 63);
    q.p = q.blk ? (int)bid : (int)bid * 4 + (int)(threadIdx.x >> 6);
    return q;
}
// Block slot of a launch whose grid is a multiple of 8 blocks: consecutive
// blocks go to the 8 XCDs in turn (each with its own L2), and XCD k (the
// blocks b = k mod 8) takes the k-th eighth of the slots.
__device__ __forceinline__ unsigned xcd_slot(unsigned bid) {
    return (bid & 7u) * (gridDim.x >> 3) + (bid >> 3);
}
// Orders the LDS accesses of the lanes of one wavefront.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// ... of a particle's lanes (the block in block mode; every lane of the
// block must reach it).
__device__ __forceinline__ void part_sync(bool blk) {
    if (blk) __syncthreads();
    else wave_lds_sync();
}
// Compaction step over the particle's lanes: v is this lane's flag; returns
// the number of flagged lanes before it (in lane order) and sets total.
// In block mode every lane of the block takes part.
__device__ __forceinline__ unsigned part_prefix(bool v, bool blk, unsigned& total) {
    __shared__ unsigned wcnt[4];
    const unsigned long long m = __ballot(v);
    const unsigned wl = threadIdx.x & 63;
    const unsigned mine = (unsigned)__popcll(m & ((1ull << wl) - 1ull));
    if (!blk) {
        total = (unsigned)__popcll(m);
        return mine;
    }
    const int w = (int)(threadIdx.x >> 6);
    if (wl == 0) wcnt[w] = (unsigned)__popcll(m);
    __syncthreads();
    unsigned before = 0, all = 0;
    for (int j = 0; j < 4; ++j) {
        before += j < w ? wcnt[j] : 0u;
        all += wcnt[j];
    }
    __syncthreads();   // wcnt is reused by the next step
    total = all;
    return before + mine;
}

// The fixed link mapping of Sec. 3: a particle's window of nxw x nyw nodes
// (x from INT(x_c - r) - 1 to INT(x_c + r) + 1, likewise y) is crossed by
// lattice lines; every (direction, line) pair owns one slot, and each slot
// holds at most one link (a line enters a disk once):
//   directions 1, 3: the nyw rows b;  2, 4: the nxw columns a;
//   5, 7: the lines a - b = c;  6, 8: the lines a + b = c, nxw + nyw - 3 each
//   (the two single-node corner lines cannot hold a link).
// 6 (nxw + nyw) - 12 slots, 12 N - 12 for a square window of edge N.
__device__ __forceinline__ int link_slot(int d, int a, int b, int nxw, int nyw) {
    const int nd = nxw + nyw - 3;
    switch (d) {
        case 1: return b;
        case 2: return nyw + a;
        case 3: return nyw + nxw + b;
        case 4: return 2 * nyw + nxw + a;
        case 5: return 2 * (nyw + nxw) + (a - b + nyw - 2);
        case 6: return 2 * (nyw + nxw) + nd + (a + b - 1);
        case 7: return 2 * (nyw + nxw) + 2 * nd + (a - b + nyw - 2);
        default: return 2 * (nyw + nxw) + 3 * nd + (a + b - 1);
    }
}
__device__ __forceinline__ int slot_direction(int s, int nxw, int nyw) {
    const int nd = nxw + nyw - 3, base = 2 * (nyw + nxw);
    if (s < nyw) return 1;
    if (s < nyw + nxw) return 2;
    if (s < 2 * nyw + nxw) return 3;
    if (s < base) return 4;
    return 5 + (s - base) / nd;
}

// LDS of one particle of k_links: the owner map over the window, the slot
// array, then the compacted link list.  links_slots is also the length of
// each particle's segment of the link array.
__host__ __device__ inline size_t links_win_ints(int nwin) { return (size_t)nwin * nwin; }
__host__ __device__ inline size_t links_slots(int nwin) { return (size_t)(12 * nwin - 12); }
__host__ __device__ inline size_t links_list_offset(int nwin) {
    return ((links_win_ints(nwin) + links_slots(nwin)) * 4 + 7) / 8 * 8;
}
__host__ __device__ inline size_t links_wave_lds(int nwin) {
    return links_list_offset(nwin) + links_slots(nwin) * sizeof(uint2);
}

// Link collection (Sec. 3) from the owner map of t_n, the lanes of one
// particle (it runs at the end of the step before, once that map is built):
//  (a) load the window of the owner map of t_n into LDS;
//  (b) every fluid node of the window tests its 8 neighbours in parallel; a
//      neighbour owned by this particle is a link, written into its fixed
//      slot; the slots are then compacted in slot order (ballot + prefix
//      count within each wavefront, and across the wavefronts of a block);
//  (c) the list goes to the particle's fixed segment of the link array,
//      12 N - 12 entries from p (12 N - 12): no atomics between particles.
__device__ __forceinline__ void links_body(const RunStep& rs, const PartLanes& pl) {
    extern __shared__ uint2 smem[];
    const LP& lp = rs.lp;
    const PT_GLOBAL int32_t* __restrict__ Ocur = gl(rs.Ocur);
    const PState* __restrict__ Pc = rs.Pc;
    uint2* links = rs.links;
    int2* seg = rs.seg;
    unsigned* status = rs.status;
    const int lane = pl.lane, nl = pl.nl, p = pl.p;
    const int w = pl.blk ? 0 : (int)(threadIdx.x >> 6);   // the particle's LDS area in the block
    const bool have_p = p < lp.np;
    const int pitch = lp.pitch;

    const size_t wl = links_wave_lds(lp.nwin) / sizeof(uint2);
    int* win = (int*)(smem + (size_t)w * wl);
    unsigned* slot = (unsigned*)(win + links_win_ints(lp.nwin));
    uint2* lk = smem + (size_t)w * wl + links_list_offset(lp.nwin) / sizeof(uint2);
    PState P{};
    Win wn{};
    bool ok = false;
    if (have_p) {
        P = ld_state(Pc + p);
        wn = window_of(P);
        ok = particle_ok(P, lp) && wn.nxw <= lp.nwin && wn.nyw <= lp.nwin;
        if (!ok && lane == 0) atomicOr(status, ST_BAD_PARTICLE);
    }
    unsigned count = 0;
    if (ok) {
        const int nw = wn.nxw * wn.nyw;
        const int nslots = 6 * (wn.nxw + wn.nyw) - 12;
        for (int base = 0; base < nw; base += 8 * nl) {   // 8 loads in flight per lane
            int v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = base + u * nl + lane;
                const int b = idx / wn.nxw, a = idx - b * wn.nxw;
                const int yy = wn.y0 + b, xx = col_of(wn.x0 + a, lp);
                v[u] = (idx < nw && in_rows(yy, lp) && xx >= 0) ? Ocur[(size_t)yy * pitch + xx] : OUTSIDE;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int idx = base + u * nl + lane;
                if (idx < nw) win[idx] = v[u];
            }
        }
        for (int s = lane; s < nslots; s += nl) slot[s] = 0xffffffffu;
        part_sync(pl.blk);
        for (int idx = lane; idx < nw; idx += nl) {
            const int b = idx / wn.nxw, a = idx - b * wn.nxw;
            if (win[idx] != -1) continue;
            const unsigned code = (unsigned)col_of(wn.x0 + a, lp) | ((unsigned)(wn.y0 + b) << 16);
#pragma unroll
            for (int d = 1; d < 9; ++d) {
                const int ta = a + EXd(d), tb = b + EYd(d);
                if (ta < 0 || ta >= wn.nxw || tb < 0 || tb >= wn.nyw) continue;
                if (win[tb * wn.nxw + ta] == p) slot[link_slot(d, a, b, wn.nxw, wn.nyw)] = code;
            }
        }
        part_sync(pl.blk);
        for (int s0 = 0; s0 < nslots; s0 += nl) {
            const int s = s0 + lane;
            const unsigned code = s < nslots ? slot[s] : 0xffffffffu;
            const bool v = code != 0xffffffffu;
            unsigned total;
            const unsigned before = part_prefix(v, pl.blk, total);
            if (v) {
                const unsigned d = (unsigned)slot_direction(s, wn.nxw, wn.nyw);
                lk[count + before] = make_uint2(code, d | ((unsigned)p << 4));
            }
            count += total;
        }
        part_sync(pl.blk);
    }
    if (!have_p) return;
    const size_t start = (size_t)p * links_slots(lp.nwin);
    for (unsigned i = lane; i < count; i += nl) st_u2(links + start + i, lk[i]);
    if (lane == 0) st_i2(seg + p, make_int2((int)start, (int)count));
}

// The link pass, one block per particle, a thread per link of its segment
// (Sec. 2.3-2.4): q from the circle, wall point x_w = x_f + q e_i and its
// rigid-body velocity u_w, Bouzidi bounce-back f_ibar (Eqs. (9)-(10), with
// the linear and halfway fallbacks) and, for axis links, the thermal wall
// g_ibar (Eqs. (11)-(12)), both written into the solid slots x_f + e_i of
// the post-collision state A that the pull of x_f reads; the link's
// momentum exchange f_i^+ (e_i - u_w) - f_ibar (e_ibar - u_w) and its torque
// about X_c, summed in FP64 over the particle in a fixed order into Fh[p]:
// the segment in chunks of 64 slots, each chunk by a butterfly in one
// wavefront, the chunk sums in chunk order.  The order does not depend on
// the block size, which follows the particle size (pass_threads), so a
// run gives the same bits alone and in a batch.  The gathers of a link are
// issued together, after its (arithmetic-only) link fraction.
constexpr int PASS_CHUNKS = (12 * 100 - 12 + 63) / 64;   // the window edge is at most 100

// One link in the link pass: the values of eval_link (link.h) stored where
// the next pull reads them -- slot ibar of the solid node x_f + e_i (two
// sets), slot i there (in place, before the odd kernel), slot ibar of x_f
// itself (in place, before the even one) -- and the link's momentum
// exchange, Eqs. (13)-(14), added to (hx, hy, hz).
template <int MODE, bool QFIRST = true>
__device__ __forceinline__ void link_pass_link(const RunStep& rs, const PState& P, const Shape& sh, int x, int y,
                                               int i, double& hx, double& hy, double& hz) {
    using S = Store<MODE>;
    const LP& lp = rs.lp;
    auto Fw = [&](int a) { return (PT_GLOBAL ST<MODE>*)rs.A[a]; };
    const LinkEval e = eval_link<MODE, QFIRST>(rs, P, sh, x, y, i);
    const int ib = OPPd(i), ex = EXd(i), ey = EYd(i);
    const int lay = lp.aa ? 1 + rs.parity : 0;
    const size_t k = (size_t)y * lp.pitch + x;
    const size_t kb = (size_t)(y + ey) * lp.pitch + col_of(x + ex, lp);   // a node of P
    const size_t ko = lay == 2 ? k : kb;
    const int so = lay == 1 ? i : ib;
    S::st(Fw(so) + tix<ST<MODE>>(ko), (typename S::R)e.fnew);
    if (i <= 4) S::st(Fw(9 + so) + tix<ST<MODE>>(ko), (typename S::R)e.gnew);
    // Eq. (13) on full populations (stored value + rest part w rho0)
    const double w9i = i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0;
    const double shf = S::shifted ? lp.rho0 : 0.0;
    const double Fi = e.fi + w9i * shf, Fb = (double)(typename S::R)e.fnew + w9i * shf;
    const double dFx = Fi * (ex - e.uwx) - Fb * (-ex - e.uwx);
    const double dFy = Fi * (ey - e.uwy) - Fb * (-ey - e.uwy);
    hx += dFx;
    hy += dFy;
    hz += e.rx * dFy - e.ry * dFx;   // Eq. (14), z component
}

template <int MODE, int NT>
__device__ __forceinline__ void link_pass_body(const RunStep& rs, unsigned bid) {
    __shared__ double part[PASS_CHUNKS][3];
    const int p = (int)bid;
    if (p >= rs.lp.np) return;   // the whole block
    const int2 sg = ld_i2(rs.seg + p);
    const PState P = ld_state(rs.Pc + p);
    const Shape sh = shape_of(P);
    const int lane = (int)threadIdx.x & 63, w = (int)threadIdx.x >> 6;
    const int nchunks = (sg.y + 63) / 64;
    for (int c = w; c < nchunks; c += NT / 64) {   // the same trip count in all lanes of a wave
        double hx = 0.0, hy = 0.0, hz = 0.0;
        const int t = 64 * c + lane;
        if (t < sg.y) {
            const uint2 L = ld_u2(rs.links + sg.x + t);
            link_pass_link<MODE>(rs, P, sh, (int)(L.x & 0xffffu), (int)(L.x >> 16), (int)(L.y & 15u), hx, hy, hz);
        }
        for (int off = 32; off > 0; off >>= 1) {
            hx += __shfl_xor(hx, off);
            hy += __shfl_xor(hy, off);
            hz += __shfl_xor(hz, off);
        }
        if (lane == 0) {
            part[c][0] = hx;
            part[c][1] = hy;
            part[c][2] = hz;
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sx = 0.0, sy = 0.0, sz = 0.0;
        for (int j = 0; j < nchunks; ++j) {
            sx += part[j][0];
            sy += part[j][1];
            sz += part[j][2];
        }
        PT_GLOBAL double* Fa = gl(rs.Fa);
        Fa[4 * p + 0] = sx;
        Fa[4 * p + 1] = sy;
        Fa[4 * p + 2] = sz;
    }
}

// The direct-addressing link pass, kept as the ablation of Sec. 3's
// comparison: one thread per lattice node, no link collection; a fluid node
// tests its 8 neighbours in the owner map and handles each link it finds as
// above, adding the link's force and torque to the particle's sums with
// FP64 atomics (so their summation order, and the last bits, vary from run
// to run).  Most threads find no link: the load imbalance the indirect
// scheme removes.
template <int MODE>
__device__ __forceinline__ void link_pass_direct_body(const RunStep& rs, unsigned bid) {
    const LP& lp = rs.lp;
    const size_t n0 = (size_t)bid * LAT_BLOCK + threadIdx.x;
    const int y = (int)(n0 / (unsigned)lp.pitch);
    const int x = (int)(n0 - (size_t)y * lp.pitch);
    if (x >= lp.nx || y >= lp.ny) return;
    const PT_GLOBAL int32_t* __restrict__ Ocur = gl(rs.Ocur);
    if (Ocur[(size_t)y * lp.pitch + x] != -1) return;
    int own[9];
#pragma unroll
    for (int d = 1; d < 9; ++d) {
        const int yy = y + EYd(d), xx = col_of(x + EXd(d), lp);
        own[d] = in_rows(yy, lp) && xx >= 0 ? Ocur[(size_t)yy * lp.pitch + xx] : -1;
    }
    for (int d = 1; d < 9; ++d) {
        if (own[d] < 0) continue;
        const PState P = ld_state(rs.Pc + own[d]);
        double hx = 0.0, hy = 0.0, hz = 0.0;
        link_pass_link<MODE, false>(rs, P, shape_of(P), x, y, d, hx, hy, hz);
        double* Fa = rs.Fa + 4 * (size_t)own[d];
        atomicAdd(Fa + 0, hx);
        atomicAdd(Fa + 1, hy);
        atomicAdd(Fa + 2, hz);
    }
}

// Spring repulsion of Eq. (15) on particle P from Q: surface gap along the
// centre line (the centre distance minus each shape's extent along it),
// force scale pi r_p r_q (rho_p - rho_f) g with equal-area radii.  Returns
// whether the gap is within the range s (else no force).
__device__ __forceinline__ bool repulsion_pair(const LP& lp, const PState& P, const Shape& sp, const PState& Q,
                                               double& fx, double& fy) {
    const double dx = min_image_x(P.x - Q.x, lp);
    const double dy = P.y - Q.y;
    const double dist = sqrt(dx * dx + dy * dy);
    const Shape sq = shape_of(Q);
    const double ep = radial_extent(sp, dx / dist, dy / dist);
    const double eq = radial_extent(sq, dx / dist, dy / dist);
    const double gap = dist - ep - eq;
    if (gap > lp.rep_range) return false;
    const double C = kPi * (area_radius(sp) * area_radius(sq)) * (lp.rho_ratio - 1.0) * lp.rho0 * lp.gravity;
    const double t = (gap - lp.rep_range) / lp.rep_range;
    const double mag = C / lp.rep_eps * (t * t);
    fx = mag * (dx / dist);
    fy = mag * (dy / dist);
    return true;
}

// Uniform cell grid for the neighbour search: cells at least 2 r_max + s
// wide, BINCAP particles per cell.
__device__ __forceinline__ int cell_of(const PState& P, const LP& lp) {
    int cx = (int)(P.x / lp.nx * lp.ncx);
    int cy = (int)floor((P.y + 0.5) / lp.ny * lp.ncy);
    cx = min(max(cx, 0), lp.ncx - 1);
    cy = min(max(cy, 0), lp.ncy - 1);
    return cy * lp.ncx + cx;
}

__device__ __forceinline__ void bin_insert(const PState& P, int p, unsigned* bins, unsigned* cnt,
                                           unsigned* status, const LP& lp) {
    if (!particle_ok(P, lp)) return;
    const int c = cell_of(P, lp);
    const unsigned slot = atomicAdd(&cnt[c], 1u);
    if (slot < (unsigned)BINCAP) bins[(size_t)c * BINCAP + slot] = (unsigned)p;
    else atomicOr(status, ST_BIN_OVERFLOW);
}

__global__ __launch_bounds__(256) void k_bin_init(const PState* __restrict__ P, unsigned* bins, unsigned* cnt,
                                                  unsigned* status, LP lp) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < lp.np) bin_insert(P[p], p, bins, cnt, status, lp);
}

// Particle update, per particle (Sec. 2.2, 2.4; the repulsion and the
// update on its first wavefront):
//  - the momentum-exchange force and torque of the link pass, Fh[p];
//  - repulsion: partners from the cell grid of t_n (lane = one slot of the
//    3 x 3 cells around the particle), summed in ascending partner index (the
//    order of a plain loop over all partners); walls; net weight;
//  - Newton-Euler; the new state goes into the cell grid of t_n+1.
__device__ __forceinline__ void particles_body(const RunStep& rs, const PartLanes& pl) {
    const LP& lp = rs.lp;
    const PState* __restrict__ Pc = rs.Pc;
    const PT_GLOBAL unsigned* __restrict__ bins_cur = gl(rs.bins_cur);
    const PT_GLOBAL unsigned* __restrict__ cnt_cur = gl(rs.cnt_cur);
    unsigned* status = rs.status;
    const int p = pl.p;
    if (p >= lp.np) return;
    // the loads that need nothing else first, issued together
    const PState po = ld_state(rs.Pold + p);
    const PState P = ld_state(Pc + p);
    PT_GLOBAL double* Fa = gl(rs.Fa);
    const double hx = Fa[4 * p + 0], hy = Fa[4 * p + 1], hz = Fa[4 * p + 2];   // from the link pass
    {   // the owner-map buffer that will hold t_n+1 still holds t_n-1: clear
        // this particle's marks there (its window at t_n-1)
        const Win wo = window_of(po);
        PT_GLOBAL int32_t* Onext = gl(rs.Onext);
        if (particle_ok(po, lp) && wo.nxw <= lp.nwin && wo.nyw <= lp.nwin)
            for (int idx = pl.lane; idx < wo.nxw * wo.nyw; idx += pl.nl) {
                const int b = idx / wo.nxw, a = idx - b * wo.nxw;
                const int yy = wo.y0 + b, xx = col_of(wo.x0 + a, lp);
                if (in_rows(yy, lp) && xx >= 0) Onext[(size_t)yy * lp.pitch + xx] = -1;
            }
    }
    if (threadIdx.x >= 64 && pl.blk) return;   // the rest on the first wavefront
    const int lane = threadIdx.x & 63;
    const Shape sh = shape_of(P);
    double Rx = 0.0, Ry = 0.0;
    if (lp.repulsion && particle_ok(P, lp)) {
        const int c0 = cell_of(P, lp);
        const int cx = c0 % lp.ncx, cy = c0 / lp.ncx;
        bool near = false;
        int q = 0x7fffffff;
        double fx = 0.0, fy = 0.0;
        if (lane < 9 * BINCAP) {
            const int j = lane / BINCAP, sl = lane - j * BINCAP;
            const int dcx = j % 3 - 1, dcy = j / 3 - 1;
            const int yy = cy + dcy;
            int xx = cx + dcx;
            bool cell_ok = yy >= 0 && yy < lp.ncy;
            if (!lp.periodic_x) {
                if (xx < 0 || xx >= lp.ncx) cell_ok = false;   // beyond a side wall
            } else {
                if (lp.ncx == 1 && dcx != 0) cell_ok = false;   // the 3 x-neighbours coincide
                if (lp.ncx == 2 && dcx == 1) cell_ok = false;
                xx = xx < 0 ? xx + lp.ncx : (xx >= lp.ncx ? xx - lp.ncx : xx);
            }
            if (cell_ok) {
                const int c = yy * lp.ncx + xx;
                const unsigned cnt = cnt_cur[c];
                const int qq = (int)bins_cur[(size_t)c * BINCAP + sl];   // with the count: one round trip
                if ((unsigned)sl < min(cnt, (unsigned)BINCAP)) {
                    if (qq != p && repulsion_pair(lp, P, sh, ld_state(Pc + qq), fx, fy)) {
                        near = true;
                        q = qq;
                    }
                }
            }
        }
        const unsigned long long m = __ballot(near);
        int rank = 0;
        for (unsigned long long mm = m; mm; mm &= mm - 1ull) {
            const int qb = __shfl(q, __ffsll((long long)mm) - 1);
            rank += (qb < q) ? 1 : 0;
        }
        const int nn = __popcll(m);
        for (int r = 0; r < nn; ++r) {
            const unsigned long long sel = __ballot(near && rank == r);
            const int b = __ffsll((long long)sel) - 1;
            Rx += __shfl(fx, b);
            Ry += __shfl(fy, b);
        }
    }
    if (lp.repulsion) {   // the flat walls: Eq. (15) with the wall plane as the partner surface
        const double R = area_radius(sh);
        const double C = kPi * (R * R) * (lp.rho_ratio - 1.0) * lp.rho0 * lp.gravity;
        double ex, ey;   // the shape's half-extents normal to the walls
        half_extents(sh, ex, ey);
        double wx = 0.0, wy = 0.0;
        if (!lp.periodic_x) {
            const double gap_l = (P.x + 0.5) - ex;
            if (gap_l <= lp.rep_range) {
                const double t = (gap_l - lp.rep_range) / lp.rep_range;
                wx += C / lp.rep_eps * (t * t);
            }
            const double gap_r = ((lp.nx - 0.5) - P.x) - ex;
            if (gap_r <= lp.rep_range) {
                const double t = (gap_r - lp.rep_range) / lp.rep_range;
                wx -= C / lp.rep_eps * (t * t);
            }
        }
        if (!lp.periodic_y) {
            const double gb = (P.y + 0.5) - ey;
            if (gb <= lp.rep_range) {
                const double t = (gb - lp.rep_range) / lp.rep_range;
                wy += C / lp.rep_eps * (t * t);
            }
            const double gt = ((lp.ny - 0.5) - P.y) - ey;
            if (gt <= lp.rep_range) {
                const double t = (gt - lp.rep_range) / lp.rep_range;
                wy -= C / lp.rep_eps * (t * t);
            }
        }
        Rx += wx;
        Ry += wy;
    }
    if (lane != 0) return;
    PT_GLOBAL double* Fh = gl(rs.Fh);
    Fh[4 * p + 0] = hx;
    Fh[4 * p + 1] = hy;
    Fh[4 * p + 2] = hz;
    if (lp.direct) {   // the direct pass adds into Fa: start the next step at zero
        Fa[4 * p + 0] = 0.0;
        Fa[4 * p + 1] = 0.0;
        Fa[4 * p + 2] = 0.0;
    }
    const double Fg = -(lp.rho_ratio - 1.0) * lp.rho0 * kPi * P.r * P.b * lp.gravity;   // pi a b
    const double Fx = hx + Rx;
    const double Fy = (hy + Ry) + Fg;
    const double Tz = hz;
    // Newton-Euler (Sec. 2.2): explicit velocities, trapezoidal positions;
    // M = rho_p pi a b, I = M r^2 / 2 (disk) or M (a^2 + b^2) / 4 (ellipse).
    const double mass = lp.rho_ratio * lp.rho0 * kPi * P.r * P.b;
    const double inertia = sh.circle ? 0.5 * mass * P.r * P.r : 0.25 * mass * (P.r * P.r + P.b * P.b);
    PState N = P;
    N.ux = P.ux + Fx / mass;
    N.uy = P.uy + Fy / mass;
    N.om = P.om + Tz / inertia;
    N.x = P.x + 0.5 * (P.ux + N.ux);
    N.y = P.y + 0.5 * (P.uy + N.uy);
    N.th = P.th + 0.5 * (P.om + N.om);
    if (lp.periodic_x) {
        if (N.x < 0.0) N.x += lp.nx;
        else if (N.x >= lp.nx) N.x -= lp.nx;
    }
    const double ddx = min_image_x(N.x - P.x, lp), ddy = N.y - P.y;
    if (!(ddx * ddx + ddy * ddy <= 0.25)) atomicOr(status, ST_OVERSPEED);
    st_state(rs.Pn + p, N);
    bin_insert(N, p, rs.bins_next, rs.cnt_next, status, lp);
}

// Owner map of t_n+1, per particle, over the
// union of the particle's windows at t_n and t_n+1: a node inside the disk at
// t_n+1 gets owner = the lowest index whose disk holds it (atomic min, exact
// solid test); a node inside the disk at t_n but not at t_n+1 is a newborn
// candidate (k_refill keeps it if this particle owned it at t_n and no
// particle covers it at t_n+1).  Also clears the cell-grid counts read this
// step.
__device__ __forceinline__ void mask_body(const RunStep& rs, unsigned bid, const PartLanes& pl) {
    const LP& lp = rs.lp;
    int32_t* O = rs.Onext;
    const PState* __restrict__ Pp = rs.Pn;
    const PState* __restrict__ Pprev = rs.Pc;
    PT_GLOBAL unsigned* cand = gl(rs.cand);
    PT_GLOBAL unsigned* ncand = gl(rs.ncand);
    unsigned* status = rs.status;
    if (rs.cnt_cur) {   // every thread of the run's grid clears a share of the counts
        const int nblocks = pl.blk ? lp.np : (lp.np + 3) / 4;
        for (int c = (int)bid * 256 + threadIdx.x; c < lp.ncells; c += nblocks * 256) gl(rs.cnt_cur)[c] = 0u;
    }
    const int lane = pl.lane, p = pl.p;
    if (p >= lp.np) return;
    const PState P = ld_state(Pp + p);
    const PState Q0 = Pprev != nullptr ? ld_state(Pprev + p) : PState{};   // issued with P
    if (!particle_ok(P, lp)) return;
    Win w = window_of(P);
    if (w.nxw > lp.nwin || w.nyw > lp.nwin) return;
    int xa = w.x0, xb = w.x0 + w.nxw, ya = w.y0, yb = w.y0 + w.nyw;
    PState Q{};
    const bool with_prev = Pprev != nullptr && particle_ok(Q0, lp);
    if (with_prev) {
        Q = Q0;
        Win v = window_of(Q);
        if (lp.periodic_x) {   // the two windows on the same side of the seam
            if (v.x0 - w.x0 > lp.nx / 2) v.x0 -= lp.nx;
            else if (w.x0 - v.x0 > lp.nx / 2) v.x0 += lp.nx;
        }
        xa = min(xa, v.x0);
        xb = max(xb, v.x0 + v.nxw);
        ya = min(ya, v.y0);
        yb = max(yb, v.y0 + v.nyw);
    }
    const int bw = xb - xa, bh = yb - ya;
    if (bw > lp.nwin + 2 || bh > lp.nwin + 2) return;
    const Shape sp = shape_of(P), sq = shape_of(Q);
    unsigned nc = 0;
    const unsigned ccap = (unsigned)(4 * lp.nwin);
    for (int base = 0; base < bw * bh; base += pl.nl) {
        const int idx = base + lane;
        bool nb = false;
        unsigned code = 0;
        if (idx < bw * bh) {
            const int b = idx / bw, a = idx - b * bw;
            const int yy = ya + b;
            const int xx = col_of(xa + a, lp);
            if (in_rows(yy, lp) && xx >= 0) {
                const double dx = min_image_x((double)xx - P.x, lp);
                const double dy = (double)yy - P.y;
                const size_t k = (size_t)yy * lp.pitch + xx;
                if (inside_shape(sp, dx, dy)) {
                    atomicMin((unsigned*)&O[k], (unsigned)p);
                } else if (with_prev) {
                    const double qx = min_image_x((double)xx - Q.x, lp);
                    const double qy = (double)yy - Q.y;
                    nb = inside_shape(sq, qx, qy);
                    code = (unsigned)xx | ((unsigned)yy << 16);
                }
            }
        }
        unsigned total;
        const unsigned before = part_prefix(nb, pl.blk, total);
        if (nb) {
            const unsigned at = nc + before;
            if (at < ccap) cand[(size_t)p * ccap + at] = code;
        }
        nc += total;
    }
    if (lane == 0) {
        if (nc > ccap) {
            atomicOr(status, ST_CAND_OVERFLOW);
            nc = ccap;
        }
        if (with_prev) ncand[p] = nc;
        gl(rs.nborn)[p] = 0u;
    }
}

// Refilling of the newborn node (x, y) of particle p (state P at t_n+1),
// Sec. 2.5: e_c maximises n . e_c (n parallel to x - X_c; ties to the lowest
// index); pre-collision f at x + m e_c (m = 1..3, nodes fluid at t_n and
// t_n+1) rebuilt by pulling from A; Eq. (16) extrapolation (lower order when
// fewer points are fluid, equilibrium at rho0 with none); momentum set so
// that u = u_w; g = g^eq(T_w, u_w) (Eq. (17)).  COLLIDE: then collided (the
// node's post-collision values of t_n+1 in s, t); otherwise s, t hold the
// refilled values before the collision.  Returns false (nothing to refill)
// unless p owned the node at t_n and it is fluid at t_n+1.  lay: the layout
// of A (0 two sets, 1 in place reversed, 2 in place pushed).  SEQ_PULLS:
// only the stencil nodes the extrapolation uses are pulled, one at a time
// into the running sum, so that few values are live at once; otherwise all
// in-lattice ones at once, before any is used.  Either way the same values
// enter the same sums.
template <int MODE, bool COLLIDE, bool SEQ_PULLS>
__device__ bool refill_node(const Pops<ST<MODE>>& A, int lay, const PT_GLOBAL int32_t* Ocur,
                            const PT_GLOBAL int32_t* Onext, const PState& P, const Shape& sh, int p, int x,
                            int y, const LP& lp, const CC<typename Store<MODE>::R>& cc,
                            typename Store<MODE>::R (&s)[9], typename Store<MODE>::R (&t)[5]) {
    using S = Store<MODE>;
    using R = typename S::R;
    const size_t k0 = (size_t)y * lp.pitch + x;
    const double dx = min_image_x((double)x - P.x, lp);
    const double dy = (double)y - P.y;
    // n along the gradient of the shape's implicit function: (dx, dy) for a
    // disk, (b^2 u, a^2 v) in body coordinates for an ellipse
    double gx = dx, gy = dy;
    if (!sh.circle) {
        const double u = dx * sh.c + dy * sh.s, v = dy * sh.c - dx * sh.s;
        const double gu = (sh.b * sh.b) * u, gv = (sh.a * sh.a) * v;
        gx = gu * sh.c - gv * sh.s;
        gy = gu * sh.s + gv * sh.c;
    }
    int c = 1;
    double best = gx * EXd(1) + gy * EYd(1);
    for (int d = 2; d < 9; ++d) {
        const double v = gx * EXd(d) + gy * EYd(d);
        if (v > best) {
            best = v;
            c = d;
        }
    }
    const double uwx = P.ux - P.om * dy, uwy = P.uy + P.om * dx;
    // Eq. (16): 3 f1 - 3 f2 + f3, 2 f1 - f2 or f1 from the K fluid points
    // (K = 0: the equilibrium at rho0 and u_w)
    if constexpr (SEQ_PULLS) {
        // owner tests first, then one stencil node at a time into the sum
        bool fl[3];
        for (int m = 0; m < 3; ++m) {
            const int ym = y + (m + 1) * EYd(c), xm = col_of(x + (m + 1) * EXd(c), lp);
            const size_t km = (size_t)ym * lp.pitch + xm;
            fl[m] = in_rows(ym, lp) && xm >= 0 && Ocur[km] == -1 && Onext[km] == -1;
        }
        if (!(Ocur[k0] == p && Onext[k0] == -1)) return false;
        const int K = !fl[0] ? 0 : (!fl[1] ? 1 : (!fl[2] ? 2 : 3));
        if (K == 0) feq_dev<R>((R)lp.rho0, (R)lp.rho0, (R)uwx, (R)uwy, s);
#pragma nounroll
        for (int m = 0; m < K; ++m) {
            const int ym = y + (m + 1) * EYd(c), xm = col_of(x + (m + 1) * EXd(c), lp);
            R sm[9], tt[5];
            if (lay == 0) pull_node<S>(A, lp, cc, xm, ym, sm, tt);
            else if (lay == 1) pull_node<S>(opp_view(A), lp, cc, xm, ym, sm, tt);
            else pull_node_pushed<S>(A, lp, cc, xm, ym, sm, tt);
            if (m == 0) {
                const R c0 = K == 3 ? (R)3 : (K == 2 ? (R)2 : (R)1);
                for (int a = 0; a < 9; ++a) s[a] = K == 1 ? sm[a] : c0 * sm[a];
            } else if (m == 1) {
                for (int a = 0; a < 9; ++a) s[a] = K == 3 ? s[a] - (R)3 * sm[a] : s[a] - sm[a];
            } else {
                for (int a = 0; a < 9; ++a) s[a] = s[a] + sm[a];
            }
        }
    } else {
        // owner tests and the pulls of every in-lattice stencil node, all
        // issued before any is used
        int xs[3], ys[3];
        bool fl[3];
        R sm[3][9];
        const bool mine = Ocur[k0] == p && Onext[k0] == -1;
        for (int m = 0; m < 3; ++m) {
            ys[m] = y + (m + 1) * EYd(c);
            xs[m] = col_of(x + (m + 1) * EXd(c), lp);
            fl[m] = false;
            if (in_rows(ys[m], lp) && xs[m] >= 0) {
                const size_t km = (size_t)ys[m] * lp.pitch + xs[m];
                fl[m] = Ocur[km] == -1 && Onext[km] == -1;
                R tt[5];
                if (lay == 0) pull_node<S>(A, lp, cc, xs[m], ys[m], sm[m], tt);
                else if (lay == 1) pull_node<S>(opp_view(A), lp, cc, xs[m], ys[m], sm[m], tt);
                else pull_node_pushed<S>(A, lp, cc, xs[m], ys[m], sm[m], tt);
            }
        }
        if (!mine) return false;
        const int K = !fl[0] ? 0 : (!fl[1] ? 1 : (!fl[2] ? 2 : 3));
        if (K == 3) {
            for (int a = 0; a < 9; ++a) s[a] = (R)3 * sm[0][a] - (R)3 * sm[1][a] + sm[2][a];
        } else if (K == 2) {
            for (int a = 0; a < 9; ++a) s[a] = (R)2 * sm[0][a] - sm[1][a];
        } else if (K == 1) {
            for (int a = 0; a < 9; ++a) s[a] = sm[0][a];
        } else {
            feq_dev<R>((R)lp.rho0, (R)lp.rho0, (R)uwx, (R)uwy, s);
        }
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
    if (COLLIDE) {
        R r_, u_, v_, T_;
        collide<R>(cc, s, t, r_, u_, v_, T_);
    }
    return true;
}

// Refill of particle p's newborn nodes, the particle's lanes and one
// lane per candidate from k_mask_mark.  REFILL_TWO_SETS: after the lattice
// kernel, pulling from A, colliding and storing into B.  Split:
// REFILL_COMPUTE (the refilled values of each candidate into rbuf, 16
// doubles: 14 values and a flag; collided unless LATE),
// REFILL_STORE (into the node's slots of the new state) after the
// lattice kernel.  In place the split is needed: the lattice kernel
// overwrites what the stencil pulls read, so the values are computed before
// it.  An overlapped two-set step of a single run computes them at the end
// of the side stream, beside the lattice kernel, and only the store (LATE:
// the collision and the store) waits on the main stream.  The values are the
// same bits in every form.
enum RefillPart { REFILL_TWO_SETS = 0, REFILL_COMPUTE, REFILL_STORE };
// LATE (the compute half of a single two-set FP64 run with a wavefront per
// particle, k_refill_w<0, true>): the compute half pulls only the stencil
// nodes it uses, one at a time, and leaves the collision to the store half,
// so that it fits the register slot that one retiring FP64 lattice
// wavefront frees.  Otherwise the compute half pulls every stencil node at
// once and collides (in place it runs alone, before the lattice kernel, and
// the narrower lattice kernels leave it room).  The whole refill pulls one
// node at a time with 8-byte values.  The same arithmetic either way.
template <int MODE, int PART, bool LATE>
__device__ __forceinline__ void refill_body(const RunStep& rs, const PartLanes& pl) {
    using S = Store<MODE>;
    using R = typename S::R;
    const LP& lp = rs.lp;
    const int lane = pl.lane, p = pl.p;
    if (p >= lp.np) return;
    const unsigned ccap = (unsigned)(4 * lp.nwin);
    const unsigned n = min(gl(rs.ncand)[p], ccap);
    if (n == 0) return;
    const Pops<ST<MODE>> A = pops_of<MODE>(rs.A), B = pops_of<MODE>(rs.B);
    PT_GLOBAL double* buf = gl(rs.rbuf);
    const PState P1 = ld_state(rs.Pn + p);
    const Shape sh = shape_of(P1);
    unsigned refilled = 0;   // this lane's newborn nodes
    for (unsigned i = lane; i < n; i += pl.nl) {
        const unsigned code = gl(rs.cand)[(size_t)p * ccap + i];
        const int x = (int)(code & 0xffffu), y = (int)(code >> 16);
        const size_t slot = ((size_t)p * ccap + i) * 16;
        R s[9], t[5];
        if (PART == REFILL_STORE) {
            if (buf[slot + 14] == 0.0) continue;
            for (int a = 0; a < 9; ++a) s[a] = (R)buf[slot + a];
            for (int a = 0; a < 5; ++a) t[a] = (R)buf[slot + 9 + a];
            if (LATE) {
                R r_, u_, v_, T_;
                collide<R>(args_cc<R>(lp), s, t, r_, u_, v_, T_);
            }
            if (!lp.aa) store_node<S>(B, lp, args_cc<R>(lp), x, y, s, t);
            else if (rs.parity == 0) store_node_pushed<S>(A, lp, args_cc<R>(lp), x, y, s, t);   // the odd kernel ran
            else store_node<S>(opp_view(A), lp, args_cc<R>(lp), x, y, s, t);
            continue;
        }
        const int lay = lp.aa ? 1 + rs.parity : 0;
        constexpr bool COLLIDE = PART == REFILL_TWO_SETS || !LATE;   // LATE: the store half collides
        constexpr bool SEQ = LATE || (PART == REFILL_TWO_SETS && MODE == 0);
        const bool mine = refill_node<MODE, COLLIDE, SEQ>(A, lay, gl(rs.Ocur), gl(rs.Onext), P1, sh, p, x, y, lp,
                                                          args_cc<R>(lp), s, t);
        refilled += mine ? 1u : 0u;
        if (PART == REFILL_TWO_SETS) {
            if (mine) store_node<S>(B, lp, args_cc<R>(lp), x, y, s, t);
        } else {
            if (mine) {
                for (int a = 0; a < 9; ++a) buf[slot + a] = (double)s[a];
                for (int a = 0; a < 5; ++a) buf[slot + 9 + a] = (double)t[a];
            }
            buf[slot + 14] = mine ? 1.0 : 0.0;
        }
    }
    if (PART == REFILL_STORE) return;
    // newborn nodes of the particle this step (its count, zeroed by k_mask_mark)
    for (int off = 32; off > 0; off >>= 1) refilled += __shfl_xor(refilled, off);
    if ((threadIdx.x & 63) == 0 && refilled) atomicAdd(rs.nborn + p, refilled);
}

// ------------------------------------------------------- step kernels ----
// Each step kernel exists twice: for one run (its RunStep passed by value,
// read from the kernel-argument segment) and batched over several runs (one
// grid; block b works on block bmap[b].y of run bmap[b].x, whose RunStep is
// tab[bmap[b].x]).  Both call the same body, so a run computes the same bits
// alone and in a batch.

__global__ __launch_bounds__(256) void k_links(RunStep rs) { links_body(rs, part_lanes(rs.lp, blockIdx.x)); }
__global__ __launch_bounds__(256) void k_links_b(const RunStep* __restrict__ tab, const uint2* __restrict__ bmap) {
    const uint2 m = bmap[blockIdx.x];
    links_body(tab[m.x], part_lanes(tab[m.x].lp, m.y));
}

// At most 80 VGPRs (6 wavefronts per SIMD instead of 5 at the 88 it would
// take, no scratch): the pass waits on scattered gathers, and the extra
// wavefronts hide more of them (dense FP16 +3.3 %, paper scale +0.1-0.4 %).
template <int MODE, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(6))) void k_link_pass(RunStep rs) {
    // the particles in band order, an eighth per XCD (xcd_slot): those
    // whose gathers share cache lines are taken on one XCD, one after
    // another.  Any order gives the same bits.
    const unsigned s = xcd_slot(blockIdx.x);
    if (s >= (unsigned)rs.lp.np) return;
    link_pass_body<MODE, NT>(rs, rs.order[s]);
}
template <int MODE>
__global__ __launch_bounds__(LAT_BLOCK) void k_link_pass_direct(RunStep rs) {
    link_pass_direct_body<MODE>(rs, blockIdx.x);
}
template <int MODE>
__global__ __launch_bounds__(256) void k_link_pass_b(const RunStep* __restrict__ tab,
                                                     const uint2* __restrict__ bmap) {
    const uint2 m = bmap[blockIdx.x];
    link_pass_body<MODE, 256>(tab[m.x], m.y);
}

__global__ __launch_bounds__(256) void k_particles(RunStep rs) { particles_body(rs, part_lanes(rs.lp, blockIdx.x)); }
__global__ __launch_bounds__(256) void k_particles_b(const RunStep* __restrict__ tab,
                                                     const uint2* __restrict__ bmap) {
    const uint2 m = bmap[blockIdx.x];
    particles_body(tab[m.x], part_lanes(tab[m.x].lp, m.y));
}

__global__ __launch_bounds__(256) void k_mask_mark(RunStep rs) {
    mask_body(rs, blockIdx.x, part_lanes(rs.lp, blockIdx.x));
}
__global__ __launch_bounds__(256) void k_mask_mark_b(const RunStep* __restrict__ tab,
                                                     const uint2* __restrict__ bmap) {
    const uint2 m = bmap[blockIdx.x];
    mask_body(tab[m.x], m.y, part_lanes(tab[m.x].lp, m.y));
}

template <int MODE, int PART, bool LATE = false>
__global__ __launch_bounds__(256) void k_refill(RunStep rs) {
    refill_body<MODE, PART, LATE>(rs, part_lanes(rs.lp, blockIdx.x));
}
// The compute half with a block of one wavefront per particle (particles
// whose lanes are a wavefront): beside the lattice kernel a block of 256
// threads must wait until four of its wavefronts' register slots are free
// on one compute unit at once, a block of 64 only for one.  LATE with
// 8-byte values.
template <int MODE, bool LATE>
__global__ __launch_bounds__(64) void k_refill_w(RunStep rs) {
    PartLanes pl;
    pl.p = (int)blockIdx.x;
    pl.lane = (int)threadIdx.x;
    pl.nl = 64;
    pl.blk = false;
    refill_body<MODE, REFILL_COMPUTE, LATE>(rs, pl);
}
template <int MODE, int PART>
__global__ __launch_bounds__(256) void k_refill_b(const RunStep* __restrict__ tab, const uint2* __restrict__ bmap) {
    const uint2 m = bmap[blockIdx.x];
    refill_body<MODE, PART, false>(tab[m.x], part_lanes(tab[m.x].lp, m.y));
}

__global__ void k_link_q(const PState* __restrict__ Pc, const uint2* __restrict__ links, int n, int32_t* node,
                         int32_t* dir, int32_t* part, double* qo, LP lp) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n) return;
    const uint2 L = links[l];
    const int x = (int)(L.x & 0xffffu), y = (int)(L.x >> 16), i = (int)(L.y & 15u), p = (int)(L.y >> 4);
    const PState P = Pc[p];
    const double dx = min_image_x((double)x - P.x, lp);
    const double dy = (double)y - P.y;
    node[l] = y * lp.nx + x;
    dir[l] = i;
    part[l] = p;
    qo[l] = link_q_shape(shape_of(P), dx, dy, i);
}

// -------------------------------------------------------------- launchers ----

// A block per particle pays off when the windows are large and there are
// too few particles to fill the GPU with wavefronts (with thousands of
// particles the wavefronts already do, and whole blocks would take more of
// the GPU from the lattice kernel running beside them).
// The link collection keeps one particle's window, slots and list in LDS
// (links_wave_lds); four wavefront-particles share a block's LDS, so where
// four of them would exceed 64 KiB (windows of about 50 nodes and more) a
// particle takes the whole block instead.
int lanes_per_particle(int nwin, int np) {
    if (nwin >= 32 && np <= 1024) return 256;
    return 4 * links_wave_lds(nwin) > kLinksLdsLimit ? 256 : 64;
}
// Threads of a single run's link-pass block: 128 where that covers about
// three quarters of the segment (12 N - 12 slots for window edge N; a disk
// of diameter d has about 0.7 of that many links), so that few lanes idle;
// 512 for large particles when they are few (at most 1024 blocks: the
// block's lanes are the parallelism), else 256.  Measured at 4096^2 with
// 64 000 disks d = 10: 128 against 256 threads, 338 vs 457 us (FP16); 129
// ellipses 50 x 25: 512 against 256, 13.2 vs 15.6 us; 4800 disks d = 40:
// 512 no faster than 256 (156 vs 152 us).
int pass_threads(int nwin, int np) {
    const int typical = (3 * (12 * nwin - 12)) / 4;
    if (typical <= 128) return 128;
    return typical > 256 && np <= 1024 ? 512 : 256;
}

size_t links_block_lds(const LP& lp) { return (size_t)(lp.lpp > 64 ? 1 : 4) * links_wave_lds(lp.nwin); }

unsigned run_blocks(int c, const LP& lp) {
    switch (c) {
        case GC_LINKS:
        case GC_WAVE: return (unsigned)(lp.lpp > 64 ? lp.np : (lp.np + 3) / 4);
        case GC_PASS: return (unsigned)lp.np;   // a block per particle
        default: return (unsigned)(((size_t)lp.pitch * lp.ny + LAT_BLOCK - 1) / LAT_BLOCK);
    }
}

// Grid of the single-run link pass: a whole number of blocks per XCD, as
// xcd_slot assumes (the blocks beyond the particle count return).
static unsigned xcd_grid(unsigned nb) { return 8u * ((nb + 7u) / 8u); }

hipError_t launch_step(int k, const RunStep& R, int mode, hipStream_t st) {
    if (R.lp.direct && R.lp.np > 0) {   // direct addressing: no collection, a thread per node
        if (k == SK_COLLECT) return hipSuccess;
        if (k == SK_PASS) {
            PTLBM_DISPATCH(mode, (k_link_pass_direct<M><<<run_blocks(GC_LAT, R.lp), LAT_BLOCK, 0, st>>>(R)));
            return hipGetLastError();
        }
    }
    const unsigned nb = run_blocks(grid_class(k), R.lp);
    if (nb == 0) return hipSuccess;
    switch (k) {
        case SK_COLLECT:   // R: the RunStep of the step whose links are collected
            k_links<<<nb, 256, links_block_lds(R.lp), st>>>(R);
            break;
        case SK_PASS: {
            const unsigned nb8 = xcd_grid(nb);
            switch (pass_threads(R.lp.nwin, R.lp.np)) {
                case 128: PTLBM_DISPATCH(mode, (k_link_pass<M, 128><<<nb8, 128, 0, st>>>(R))); break;
                case 256: PTLBM_DISPATCH(mode, (k_link_pass<M, 256><<<nb8, 256, 0, st>>>(R))); break;
                default: PTLBM_DISPATCH(mode, (k_link_pass<M, 512><<<nb8, 512, 0, st>>>(R))); break;
            }
            break;
        }
        case SK_PARTICLES: k_particles<<<nb, 256, 0, st>>>(R); break;
        case SK_MASK:   // in place, the refill is computed here, before the lattice kernel
            k_mask_mark<<<nb, 256, 0, st>>>(R);
            if (R.lp.aa) {
                PTLBM_DISPATCH(mode, (k_refill<M, REFILL_COMPUTE><<<nb, 256, 0, st>>>(R)));
            }
            break;
        case SK_LATTICE: return launch_lattice(R, mode, nb, st);
        case SK_REFILL:
            if (R.lp.aa) {
                PTLBM_DISPATCH(mode, (k_refill<M, REFILL_STORE><<<nb, 256, 0, st>>>(R)));
            } else {
                PTLBM_DISPATCH(mode, (k_refill<M, REFILL_TWO_SETS><<<nb, 256, 0, st>>>(R)));
            }
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_refill_part(const RunStep& R, int mode, bool store, hipStream_t st) {
    const unsigned nb = run_blocks(GC_WAVE, R.lp);
    if (nb == 0) return hipSuccess;
    const bool late = mode == 0 && R.lp.lpp <= 64;   // k_refill_w<0, true> and its store
    if (store && late) {
        k_refill<0, REFILL_STORE, true><<<nb, 256, 0, st>>>(R);
    } else if (store) {
        PTLBM_DISPATCH(mode, (k_refill<M, REFILL_STORE><<<nb, 256, 0, st>>>(R)));
    } else if (late) {
        k_refill_w<0, true><<<(unsigned)R.lp.np, 64, 0, st>>>(R);
    } else if (R.lp.lpp <= 64) {
        PTLBM_DISPATCH(mode, (k_refill_w<M, false><<<(unsigned)R.lp.np, 64, 0, st>>>(R)));
    } else {
        PTLBM_DISPATCH(mode, (k_refill<M, REFILL_COMPUTE><<<nb, 256, 0, st>>>(R)));
    }
    return hipGetLastError();
}

hipError_t launch_step_batch(int k, const BatchLaunch& b, hipStream_t st) {
    const int c = grid_class(k);
    const unsigned nb = b.nblk[c];
    if (nb == 0) return hipSuccess;
    const uint2* bm = b.bmap[c];
    switch (k) {
        case SK_COLLECT: k_links_b<<<nb, 256, b.lds, st>>>(b.tab_next, bm); break;
        case SK_PASS: PTLBM_DISPATCH(b.mode, (k_link_pass_b<M><<<nb, 256, 0, st>>>(b.tab, bm))); break;
        case SK_PARTICLES: k_particles_b<<<nb, 256, 0, st>>>(b.tab, bm); break;
        case SK_MASK:
            k_mask_mark_b<<<nb, 256, 0, st>>>(b.tab, bm);
            if (b.aa) {
                PTLBM_DISPATCH(b.mode, (k_refill_b<M, REFILL_COMPUTE><<<nb, 256, 0, st>>>(b.tab, bm)));
            }
            break;
        case SK_LATTICE: return launch_lattice_batch(b.tab, bm, nb, b.mode, b.aa, st);
        case SK_REFILL:
            if (b.aa) {
                PTLBM_DISPATCH(b.mode, (k_refill_b<M, REFILL_STORE><<<nb, 256, 0, st>>>(b.tab, bm)));
            } else {
                PTLBM_DISPATCH(b.mode, (k_refill_b<M, REFILL_TWO_SETS><<<nb, 256, 0, st>>>(b.tab, bm)));
            }
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mask_setup(const RunStep& R, hipStream_t st) {
    RunStep S = R;
    S.Pc = nullptr;       // no previous time level: no newborn candidates
    S.cnt_cur = nullptr;  // no cell counts to clear
    const unsigned nb = run_blocks(GC_WAVE, S.lp);
    if (nb == 0) return hipSuccess;
    k_mask_mark<<<nb, 256, 0, st>>>(S);
    return hipGetLastError();
}

hipError_t launch_bin_init(const DevState& d, const PState* P, int bin_parity, hipStream_t st) {
    if (d.lp.np == 0) return hipSuccess;
    k_bin_init<<<(d.lp.np + 255) / 256, 256, 0, st>>>(P, d.bins[bin_parity], d.bcnt[bin_parity], d.status,
                                                       d.lp);
    return hipGetLastError();
}

hipError_t launch_link_q(const DevState& d, int ring, const uint2* links, int nlinks, int32_t* node,
                         int32_t* dir, int32_t* part, double* q, hipStream_t st) {
    if (nlinks <= 0) return hipSuccess;
    k_link_q<<<(nlinks + 255) / 256, 256, 0, st>>>(d.P[ring], links, nlinks, node, dir, part, q, d.lp);
    return hipGetLastError();
}

}  // namespace ptlbm
