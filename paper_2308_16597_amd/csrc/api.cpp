// api.cpp -- the C ABI declared in include/lbm.h: parameter validation,
// device memory layout, particle seeding, step sequencing and read-back.
// All arithmetic of the method runs in the kernels of lattice.hip and
// particles.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "sim.h"

using namespace ptlbm;

static_assert(LBM_NPHASES == SK_COUNT, "one timed phase per step kernel");

namespace {

thread_local std::string g_create_error;

constexpr size_t kAlign = 256;
constexpr size_t kArrayAlign = 65536;
constexpr size_t kStagger = 4096;   // start offset between consecutive population arrays

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t elem_size(int mode) {
    switch (mode) {
        case LBM_STORE_F64: return 8;
        case LBM_STORE_F32:
        case LBM_STORE_SHIFT_F32: return 4;
        case LBM_STORE_SHIFT_F16:
        case LBM_STORE_SHIFT_BF16: return 2;
        default: return 0;
    }
}

// Largest window edge for a diameter: INT(x + r) - INT(x - r) + 3 <= floor(2r) + 4.
int window_cap(double max_diameter) { return (int)std::floor(max_diameter) + 4; }

Layout make_layout(const lbm_params& p) {
    Layout L;
    // rows padded to 64 nodes: at 4000 x 4000 in FP64, unpadded rows (still
    // 128-byte aligned) made the lattice kernel 3.7 % slower (662 vs 638 us)
    L.pitch = (int)round_up((size_t)p.nx, 64);
    L.npitched = (size_t)L.pitch * p.ny;
    const size_t es = elem_size(p.storage);
    // a state: 14 arrays, each 64 KiB aligned and staggered by 4 KiB (2- and
    // 4-byte values), or the same bytes as one block of 64-node tiles
    // (8-byte values, lattice.h)
    L.array_stride = round_up(L.npitched * es, kArrayAlign) + kStagger;
    L.state_bytes = round_up(14 * L.array_stride, kArrayAlign);
    size_t off = 0;
    const bool aa = p.streaming == LBM_STREAM_IN_PLACE;
    L.off_S[0] = off; off += L.state_bytes;
    L.off_S[1] = L.off_S[0];
    if (!aa) {
        L.off_S[1] = off;
        off += L.state_bytes;
    }
    L.off_O[0] = off; off = round_up(off + L.npitched * 4, kArrayAlign);
    L.off_O[1] = off; off = round_up(off + L.npitched * 4, kArrayAlign);
    const size_t cap = (size_t)(p.max_particles > 0 ? p.max_particles : 0);
    L.nwin = window_cap(p.max_diameter > 0 ? p.max_diameter : 2.0);
    L.link_cap = cap * (size_t)(12 * L.nwin - 12);
    L.off_P = off; off = round_up(off + 3 * cap * sizeof(PState), kAlign);
    L.off_Fh = off; off = round_up(off + cap * 4 * sizeof(double), kAlign);
    L.off_Fa = off; off = round_up(off + cap * 4 * sizeof(double), kAlign);
    L.off_seg = off; off = round_up(off + cap * sizeof(int2), kAlign);
    L.off_links = off; off = round_up(off + L.link_cap * sizeof(uint2), kAlign);
    // read_links: the gathered list, then node, direction, particle, q
    L.off_lscratch = off;
    off = round_up(off + L.link_cap * (sizeof(uint2) + 3 * sizeof(int32_t) + sizeof(double)) + 16, kAlign);
    L.off_status = off; off = round_up(off + 64, kAlign);
    L.off_cc = off; off = round_up(off + sizeof(CC<float>), kAlign);
    // neighbour-search cells at least 2 r_max + s wide
    const double cell = (p.max_diameter > 0 ? p.max_diameter : 2.0) + (p.rep_range > 0 ? p.rep_range : 0.0);
    L.ncx = std::max(1, (int)std::floor(p.nx / cell));
    L.ncy = std::max(1, (int)std::floor(p.ny / cell));
    const size_t ncells = cap > 0 ? (size_t)L.ncx * L.ncy : 0;
    for (int b = 0; b < 2; ++b) {
        L.off_bins[b] = off; off = round_up(off + ncells * BINCAP * sizeof(unsigned), kAlign);
        L.off_bcnt[b] = off; off = round_up(off + ncells * sizeof(unsigned), kAlign);
    }
    L.off_cand = off; off = round_up(off + cap * 4 * (size_t)L.nwin * sizeof(unsigned), kAlign);
    L.off_ncand = off; off = round_up(off + cap * sizeof(unsigned), kAlign);
    L.off_nborn = off; off = round_up(off + cap * sizeof(unsigned), kAlign);
    L.off_order = off; off = round_up(off + cap * sizeof(unsigned), kAlign);
    // refilled values of the newborn candidates, computed beside the lattice
    // kernel and stored after it (16 doubles each)
    L.off_rbuf = off; off = round_up(off + cap * 4 * (size_t)L.nwin * 16 * sizeof(double), kAlign);
    // field upload / read-back: the second population set of the two-set
    // layout; in place a scratch of 4 FP64 planes over an eighth of the rows
    L.field_rows = p.ny;
    if (aa) {
        L.field_rows = (p.ny + 7) / 8;
        L.off_fscratch = off; off = round_up(off + 4 * (size_t)p.nx * L.field_rows * sizeof(double), kAlign);
    }
    L.total = off;
    return L;
}

}  // namespace

namespace ptlbm {

int fail(lbm_sim* h, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (h) h->err = buf;
    else g_create_error = buf;
    return code;
}

int hip_fail(lbm_sim* h, hipError_t e, const char* what) {
    return fail(h, LBM_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace ptlbm

namespace {

bool validate(const lbm_params* p, std::string& why) {
    char buf[256];
    auto bad = [&](const char* m) { why = m; return false; };
    if (!p) return bad("null parameters");
    if (p->abi_version != LBM_ABI_VERSION) {
        snprintf(buf, sizeof buf, "abi_version %d, library has %d", p->abi_version, LBM_ABI_VERSION);
        why = buf;
        return false;
    }
    if (p->nx < 8 || p->ny < 8 || p->nx > 65535 || p->ny > 65535) return bad("nx and ny must lie in [8, 65535]");
    if (p->periodic_x != 0 && p->periodic_x != 1) return bad("periodic_x must be 0 or 1");
    if (p->periodic_y != 0 && p->periodic_y != 1) return bad("periodic_y must be 0 or 1");
    if (elem_size(p->storage) == 0) return bad("unknown storage mode");
    if (p->streaming != LBM_STREAM_TWO_SETS && p->streaming != LBM_STREAM_IN_PLACE)
        return bad("unknown streaming layout");
    if (!(p->rho0 > 0) || !(p->nu > 0) || !(p->alpha > 0)) return bad("rho0, nu and alpha must be > 0");
    if (!(p->a_T > -4.0 && p->a_T <= 1.0)) return bad("a_T must lie in (-4, 1]");
    const double rates[5] = {p->s_e, p->s_eps, p->s_q, p->sT_e, p->sT_p};
    for (double r : rates)
        if (!(r < 2.0) || std::isnan(r)) return bad("relaxation rates must be < 2 (<= 0 selects the default)");
    if (p->max_particles < 0) return bad("max_particles must be >= 0");
    if (p->max_particles > 0) {
        if (p->periodic_y) return bad("particles need flat walls in y (periodic_y = 0)");
        if (!(p->max_diameter > 2.0)) return bad("max_diameter must be > 2");
        if (window_cap(p->max_diameter) > p->nx) return bad("particle window wider than the lattice");
        if (window_cap(p->max_diameter) > 100) return bad("max_diameter must be <= 96");
        if ((double)p->max_particles * (12.0 * window_cap(p->max_diameter) - 12) > 2.0e9)
            return bad("too many link slots");
        if (!(p->rep_eps > 0) || !(p->rep_range > 0)) return bad("rep_eps and rep_range must be > 0");
        if (!(p->rho_ratio > 0)) return bad("rho_ratio must be > 0");
    }
    const double vals[] = {p->gravity,  p->beta,       p->T_ref,      p->body_fx,    p->wall_T[0],
                           p->wall_T[1], p->wall_ux[0], p->wall_ux[1], p->T_fluid0,   p->particle_T,
                           p->T_shift,  p->side_T[0],  p->side_T[1]};
    for (double v : vals)
        if (!std::isfinite(v)) return bad("parameters must be finite");
    return true;
}

void fill_lp(lbm_sim* h) {
    const lbm_params& p = h->p;
    LP& lp = h->d.lp;
    lp.nx = p.nx;
    lp.ny = p.ny;
    lp.pitch = h->L.pitch;
    lp.periodic_x = p.periodic_x;
    lp.periodic_y = p.periodic_y;
    lp.rho0 = p.rho0;
    lp.gbeta = p.gravity * p.beta;
    lp.T_ref = p.T_ref;
    lp.body_fx = p.body_fx;
    const double s_nu = 1.0 / (p.nu * 3.0 + 0.5);
    lp.s_nu = s_nu;
    lp.s_e = p.s_e > 0 ? p.s_e : s_nu;
    lp.s_eps = p.s_eps > 0 ? p.s_eps : s_nu;
    lp.s_q = p.s_q > 0 ? p.s_q : 1.0 / (0.5 + (3.0 / 16.0) / (1.0 / s_nu - 0.5));
    const double a = p.a_T;
    lp.a_T = a;
    lp.w5_0 = (1.0 - a) / 5.0;
    lp.w5_k = (4.0 + a) / 20.0;
    const double cs2T = (4.0 + a) / 10.0;
    const double s_a = 1.0 / (p.alpha / cs2T + 0.5);
    lp.s_a = s_a;
    const double s_T = 1.0 / (0.5 + 0.25 / (1.0 / s_a - 0.5));
    lp.s_Te = p.sT_e > 0 ? p.sT_e : s_T;
    lp.s_Tp = p.sT_p > 0 ? p.sT_p : s_T;
    for (int w = 0; w < 2; ++w) {
        lp.wall_T[w] = p.wall_T[w];
        lp.wall_ux[w] = p.wall_ux[w];
        lp.side_T[w] = p.periodic_x ? 0.0 : p.side_T[w];
    }
    const bool shifted = p.storage >= LBM_STORE_SHIFT_F32;
    lp.T_sh = shifted ? p.T_shift : 0.0;
    lp.particle_T = p.particle_T;
    lp.rho_ratio = p.rho_ratio;
    lp.gravity = p.gravity;
    lp.rep_eps = p.rep_eps;
    lp.rep_range = p.rep_range;
    lp.repulsion = p.repulsion;
    lp.np = 0;
    lp.nwin = h->L.nwin;
    lp.link_cap = (int)h->L.link_cap;
    lp.direct = 0;
    lp.aa = p.streaming == LBM_STREAM_IN_PLACE ? 1 : 0;
    lp.lpp = lanes_per_particle(h->L.nwin, 0);
    lp.ncx = h->L.ncx;
    lp.ncy = h->L.ncy;
    lp.ncells = p.max_particles > 0 ? h->L.ncx * h->L.ncy : 0;
    lp.cf = (const PT_GLOBAL CC<float>*)(h->base + h->L.off_cc);
}

int create_common(const lbm_params* p, void* dev_ptr, size_t bytes, void* stream, lbm_handle* out) {
    if (!out) return fail(nullptr, LBM_EINVAL, "null output handle");
    *out = nullptr;
    std::string why;
    if (!validate(p, why)) return fail(nullptr, LBM_EINVAL, "%s", why.c_str());
    lbm_sim* h = new lbm_sim();
    h->p = *p;
    h->L = make_layout(*p);
    if (dev_ptr) {
        if (((uintptr_t)dev_ptr % kAlign) != 0) {
            delete h;
            return fail(nullptr, LBM_EINVAL, "arena not 256-byte aligned");
        }
        if (bytes < h->L.total) {
            const size_t need = h->L.total;
            delete h;
            return fail(nullptr, LBM_EBUDGET, "arena of %zu bytes, the run needs %zu", bytes, need);
        }
        h->base = (char*)dev_ptr;
    } else {
        const size_t total = h->L.total;
        hipError_t e = hipMalloc((void**)&h->base, total);
        if (e != hipSuccess) {
            delete h;
            (void)hipGetLastError();
            return fail(nullptr, e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "hipMalloc of %zu bytes: %s",
                        total, hipGetErrorString(e));
        }
        h->own_mem = true;
    }
    if (stream) {
        h->stream = (hipStream_t)stream;
    } else {
        hipError_t e = hipStreamCreate(&h->stream);
        if (e != hipSuccess) {
            if (h->own_mem) (void)hipFree(h->base);
            delete h;
            return fail(nullptr, LBM_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
        }
        h->own_stream = true;
    }
    {
        hipError_t e = hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_side, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_mask, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&h->ev_order, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreate(&h->ev_t0);
        if (e == hipSuccess) e = hipEventCreate(&h->ev_t1);
        if (e != hipSuccess) {
            lbm_destroy(h);
            return fail(nullptr, LBM_EDEVICE, "side stream / events: %s", hipGetErrorString(e));
        }
    }
    DevState& d = h->d;
    d.mode = p->storage;
    const Layout& L = h->L;
    for (int s = 0; s < 2; ++s)
        for (int i = 0; i < 14; ++i)   // 8-byte values in tiles of 64 nodes (lattice.h), others array by array
            d.S[s][i] = h->base + L.off_S[s] + (size_t)i * (elem_size(p->storage) == 8 ? 64 * 8 : L.array_stride);
    d.O[0] = (int32_t*)(h->base + L.off_O[0]);
    d.O[1] = (int32_t*)(h->base + L.off_O[1]);
    const size_t cap = (size_t)(p->max_particles > 0 ? p->max_particles : 0);
    for (int r = 0; r < 3; ++r) d.P[r] = (PState*)(h->base + L.off_P) + r * cap;
    d.Fh = (double*)(h->base + L.off_Fh);
    d.Fa = (double*)(h->base + L.off_Fa);
    d.seg = (int2*)(h->base + L.off_seg);
    d.links = (uint2*)(h->base + L.off_links);
    d.status = (unsigned*)(h->base + L.off_status);
    for (int b = 0; b < 2; ++b) {
        d.bins[b] = (unsigned*)(h->base + L.off_bins[b]);
        d.bcnt[b] = (unsigned*)(h->base + L.off_bcnt[b]);
    }
    d.cand = (unsigned*)(h->base + L.off_cand);
    d.ncand = (unsigned*)(h->base + L.off_ncand);
    d.nborn = (unsigned*)(h->base + L.off_nborn);
    d.order = (unsigned*)(h->base + L.off_order);
    d.rbuf = L.off_rbuf ? (double*)(h->base + L.off_rbuf) : nullptr;
    fill_lp(h);
    {
        const CC<float> cc = round_cc(make_cc(d.lp));
        hipError_t e = hipMemcpy(h->base + L.off_cc, &cc, sizeof cc, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            hip_fail(h, e, "upload of the lattice constants");
            g_create_error = h->err;
            lbm_destroy(h);
            return LBM_EDEVICE;
        }
    }
    *out = h;
    int rc = lbm_set_particles(h, 0, nullptr);
    if (rc != LBM_OK) {
        g_create_error = h->err;
        lbm_destroy(h);
        *out = nullptr;
    }
    return rc;
}

int check_status(lbm_sim* h) {
    unsigned st = 0;
    HIPCHK(h, hipMemcpyAsync(&st, h->d.status, sizeof st, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    if (st == 0) return LBM_OK;
    std::string m = "device reported:";
    if (st & ST_NONFINITE) m += " non-finite populations;";
    if (st & ST_OVERSPEED) m += " a particle moved more than 0.5 in one step;";
    if (st & ST_LINK_OVERFLOW) m += " more links for one particle than its segment holds;";
    if (st & ST_BAD_PARTICLE) m += " particle state not finite or outside the lattice;";
    if (st & ST_BIN_OVERFLOW) m += " more than 7 particles in one neighbour-search cell;";
    if (st & ST_CAND_OVERFLOW) m += " too many newborn nodes for one particle in one step;";
    return fail(h, LBM_EUNSTABLE, "%s", m.c_str());
}

}  // namespace

namespace ptlbm {

RunStep make_runstep(const lbm_sim* h, int c, int r, int bp) {
    const DevState& d = h->d;
    RunStep R{};
    R.lp = d.lp;
    R.parity = c;
    for (int i = 0; i < 14; ++i) {
        R.A[i] = d.S[c][i];
        R.B[i] = d.S[1 - c][i];
    }
    R.Ocur = d.O[c];
    R.Onext = d.O[1 - c];
    R.Pold = d.P[ring_old(r)];
    R.Pc = d.P[r];
    R.Pn = d.P[ring_next(r)];
    R.Fh = d.Fh;
    R.Fa = d.Fa;
    R.links = d.links;
    R.seg = d.seg;
    R.status = d.status;
    R.bins_cur = d.bins[bp];
    R.cnt_cur = d.bcnt[bp];
    R.bins_next = d.bins[1 - bp];
    R.cnt_next = d.bcnt[1 - bp];
    R.cand = d.cand;
    R.ncand = d.ncand;
    R.nborn = d.nborn;
    R.order = d.order;
    R.rbuf = d.rbuf;
    return R;
}

RunStep current_runstep(const lbm_sim* h) { return make_runstep(h, h->cur, h->ring, h->bin_parity); }
RunStep next_runstep(const lbm_sim* h) {
    return make_runstep(h, 1 - h->cur, ring_next(h->ring), 1 - h->bin_parity);
}

void advance_state(lbm_sim* h) {
    h->cur = 1 - h->cur;
    h->ring = ring_next(h->ring);
    h->bin_parity = 1 - h->bin_parity;
    h->steps += 1;
}

}  // namespace ptlbm

namespace {

// One step.  With timing events: the six kernels in sequence on the
// handle's stream, an event before each.  Otherwise the particle kernels
// (update, owner map of t_n+1, links of t_n+1) run on the side stream while
// the lattice kernel runs on the main one, with one wait on each side (an
// event operation costs the main stream a few microseconds of idle time),
// and the refill's values are computed last on the side stream and only
// stored on the main one:
//   main: link pass -> [fork] -> lattice -> wait(side) -> refill store
//   side: wait(fork) -> particles -> mask -> links of t_n+1 -> refill values -> [side]
// (FP64 at 4000^2 with 4800 particles: 21.44 k MLUPS with the whole refill
// after the lattice kernel, 21.62 k split with a compute half that waited for
// register room beside the lattice kernel, 22.24 k with the compute half
// that fits one retiring lattice wavefront's registers, k_refill_w.)
// In place the refill's values are computed with the owner map, before the
// lattice kernel overwrites the state they are pulled from, so the lattice
// kernel waits for that part of the side stream:
//   main: link pass -> [fork] -> wait(mask) -> lattice -> refill store -> wait(side)
//   side: wait(fork) -> particles -> mask + refill values -> [mask] -> links of t_n+1 -> [side]

int enqueue_step(lbm_sim* h, hipEvent_t* ev, hipEvent_t* lat = nullptr) {
    hipStream_t st = h->stream;
    const RunStep R = current_runstep(h);
    const RunStep Rn = next_runstep(h);
    const int mode = h->d.mode;
    if (ev || h->np == 0) {
        for (int k = 0; k < SK_COUNT; ++k) {
            if (ev) HIPCHK(h, hipEventRecord(ev[k], st));
            HIPCHK(h, launch_step(k, k == SK_COLLECT ? Rn : R, mode, st));
        }
        if (ev) HIPCHK(h, hipEventRecord(ev[SK_COUNT], st));
    } else {
        hipStream_t sd = h->side;
        HIPCHK(h, launch_step(SK_PASS, R, mode, st));
        HIPCHK(h, hipEventRecord(h->ev_fork, st));
        const bool aa = h->d.lp.aa != 0;
        // two sets: the lattice kernel needs nothing from the side stream and
        // is enqueued first; in place it waits for the refilled values (it
        // overwrites what the refill reads)
        if (!aa) {
            if (lat) HIPCHK(h, hipEventRecord(lat[0], st));
            HIPCHK(h, launch_step(SK_LATTICE, R, mode, st));
            if (lat) HIPCHK(h, hipEventRecord(lat[1], st));
        }
        HIPCHK(h, hipStreamWaitEvent(sd, h->ev_fork, 0));
        HIPCHK(h, launch_step(SK_PARTICLES, R, mode, sd));
        HIPCHK(h, launch_step(SK_MASK, R, mode, sd));   // in place: and the refilled values
        if (aa) HIPCHK(h, hipEventRecord(h->ev_mask, sd));
        HIPCHK(h, launch_step(SK_COLLECT, Rn, mode, sd));
        // two sets: the refilled values last on the side stream, beside the
        // lattice kernel (their kernel needs many registers; the link
        // collection must not wait for it)
        const bool split = !aa;
        if (split) HIPCHK(h, launch_refill_part(R, mode, false, sd));
        HIPCHK(h, hipEventRecord(h->ev_side, sd));
        if (aa) {
            HIPCHK(h, hipStreamWaitEvent(st, h->ev_mask, 0));
            if (lat) HIPCHK(h, hipEventRecord(lat[0], st));
            HIPCHK(h, launch_step(SK_LATTICE, R, mode, st));
            if (lat) HIPCHK(h, hipEventRecord(lat[1], st));
            HIPCHK(h, launch_step(SK_REFILL, R, mode, st));
            HIPCHK(h, hipStreamWaitEvent(st, h->ev_side, 0));
        } else {
            HIPCHK(h, hipStreamWaitEvent(st, h->ev_side, 0));
            if (split) HIPCHK(h, launch_refill_part(R, mode, true, st));
            else HIPCHK(h, launch_step(SK_REFILL, R, mode, st));
        }
    }
    advance_state(h);
    return LBM_OK;
}

// Device scratch for field uploads and read-backs of L.field_rows rows: the
// idle population set of the two-set layout, a buffer of its own in place.
void* scratch_of(lbm_sim* h) {
    return h->d.lp.aa ? (void*)(h->base + h->L.off_fscratch) : h->d.S[1 - h->cur][0];
}

void drop_cycle_graphs(lbm_sim* h) {
    for (hipGraphExec_t& g : h->cycle_graph) {
        if (g) (void)hipGraphExecDestroy(g);
        g = nullptr;
    }
}

// Capture six overlapped steps from the current state into the graph slot
// of that state (nothing runs; the state is restored afterwards).  A graph
// is kept per state (at most 6 are reachable from one start), so step
// counts that are not multiples of 6 do not recapture on the next call.
int capture_cycle(lbm_sim* h) {
    const int cur = h->cur, ring = h->ring, bp = h->bin_parity;
    const int state = state_index(cur, ring, bp);
    hipGraphExec_t& slot = h->cycle_graph[state];
    if (slot) (void)hipGraphExecDestroy(slot);
    slot = nullptr;
    const int64_t steps = h->steps;
    HIPCHK(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed));
    int rc = LBM_OK;
    for (int j = 0; j < 6 && rc == LBM_OK; ++j) rc = enqueue_step(h, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->stream, &g);
    h->cur = cur;
    h->ring = ring;
    h->bin_parity = bp;
    h->steps = steps;
    if (rc != LBM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&slot, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        slot = nullptr;
        return hip_fail(h, e, "capture of the step cycle");
    }
    h->cycle_generation[state] = h->generation;
    return LBM_OK;
}

}  // namespace

extern "C" {

int32_t lbm_abi_version(void) { return LBM_ABI_VERSION; }

void lbm_params_default(lbm_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->abi_version = LBM_ABI_VERSION;
    p->nx = 64;
    p->ny = 64;
    p->periodic_x = 1;
    p->periodic_y = 0;
    p->storage = LBM_STORE_F64;
    p->rho0 = 1.0;
    p->nu = 0.1;
    p->alpha = 0.1;
    p->a_T = -2.0;
    p->particle_T = 1.0;
    p->rho_ratio = 1.5;
    p->repulsion = 1;
    p->rep_eps = 1e-3;
    p->rep_range = 3.0;
    p->T_shift = 0.5;
    p->max_particles = 0;
    p->max_diameter = 0.0;
}

size_t lbm_bytes_required(const lbm_params* p) {
    std::string why;
    if (!validate(p, why)) return 0;
    return make_layout(*p).total;
}

int lbm_create(const lbm_params* p, void* hip_stream, lbm_handle* out) {
    return create_common(p, nullptr, 0, hip_stream, out);
}

int lbm_create_in_arena(const lbm_params* p, void* dev_ptr, size_t bytes, void* hip_stream, lbm_handle* out) {
    if (!dev_ptr) return fail(nullptr, LBM_EINVAL, "null arena");
    return create_common(p, dev_ptr, bytes, hip_stream, out);
}

void lbm_destroy(lbm_handle h) {
    if (!h) return;
    forget_batches(h);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    if (h->side) (void)hipStreamSynchronize(h->side);
    drop_cycle_graphs(h);
    if (h->own_mem && h->base) (void)hipFree(h->base);
    for (hipEvent_t e : {h->ev_fork, h->ev_side, h->ev_mask, h->ev_order, h->ev_t0, h->ev_t1})
        if (e) (void)hipEventDestroy(e);
    if (h->side) (void)hipStreamDestroy(h->side);
    if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
    delete h;
}

const char* lbm_last_error(lbm_handle h) { return h ? h->err.c_str() : g_create_error.c_str(); }

int lbm_rsa_seed(int32_t nx, int32_t ny, int32_t n, double diameter, double min_gap, uint64_t seed,
                 double* rows7) {
    if (n < 0 || !(diameter > 0) || nx < 1 || ny < 1 || (n > 0 && !rows7))
        return fail(nullptr, LBM_EINVAL, "invalid seeding arguments");
    const double r = 0.5 * diameter;
    const double ylo = (-0.5 + min_gap) + r;
    const double yhi = ((ny - 0.5) - min_gap) - r;
    if (n > 0 && yhi < ylo) return fail(nullptr, LBM_ESEED, "channel too narrow for the particles");
    // SplitMix64 (Steele, Lea & Flood 2014)
    uint64_t state = seed;
    auto next_u64 = [&]() {
        state += 0x9E3779B97F4A7C15ull;
        uint64_t z = state;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    auto uniform = [&]() { return (double)(next_u64() >> 11) * (1.0 / 9007199254740992.0); };
    // neighbour search on cells at least one exclusion distance wide
    const double cell = 2.0 * r + (min_gap > 0 ? min_gap : 0.0);
    const int ncx = std::max(1, (int)std::floor(nx / cell));
    const int ncy = std::max(1, (int)std::floor(ny / cell));
    std::vector<std::vector<int>> grid((size_t)ncx * ncy);
    std::vector<double> xs, ys;
    xs.reserve(n);
    ys.reserve(n);
    const double half = 0.5 * nx;
    long long attempts = 0;
    while ((int)xs.size() < n) {
        if (attempts >= 1000LL * n)
            return fail(nullptr, LBM_ESEED, "placed %zu of %d particles in %lld attempts", xs.size(), n, attempts);
        ++attempts;
        const double x = uniform() * nx;
        const double y = ylo + uniform() * (yhi - ylo);
        const int cx = std::min((int)(x / nx * ncx), ncx - 1);
        const int cy = std::min(std::max((int)((y + 0.5) / ny * ncy), 0), ncy - 1);
        bool ok = true;
        for (int dcy = -1; dcy <= 1 && ok; ++dcy) {
            const int yy = cy + dcy;
            if (yy < 0 || yy >= ncy) continue;
            for (int dcx = -1; dcx <= 1 && ok; ++dcx) {
                const int xx = ((cx + dcx) % ncx + ncx) % ncx;
                for (int q : grid[(size_t)yy * ncx + xx]) {
                    double dx = x - xs[q];
                    if (dx > half) dx = dx - nx;
                    else if (dx < -half) dx = dx + nx;
                    const double dy = y - ys[q];
                    const double gap = (std::sqrt(dx * dx + dy * dy) - r) - r;
                    if (gap < min_gap) {
                        ok = false;
                        break;
                    }
                }
            }
        }
        if (ok) {
            grid[(size_t)cy * ncx + cx].push_back((int)xs.size());
            xs.push_back(x);
            ys.push_back(y);
        }
    }
    for (int i = 0; i < n; ++i) {
        double* row = rows7 + 7 * (size_t)i;
        row[0] = xs[i];
        row[1] = ys[i];
        row[2] = r;
        row[3] = row[4] = row[5] = row[6] = 0.0;
    }
    return LBM_OK;
}

int lbm_seed_particles(lbm_handle h, int32_t n, double diameter, double min_gap, uint64_t seed) {
    if (!h) return LBM_EINVAL;
    if (n < 0) return fail(h, LBM_EINVAL, "negative particle count");
    if (!h->p.periodic_x) return fail(h, LBM_EINVAL, "seeding is for periodic channels; place cavity particles with lbm_set_particles");
    std::vector<double> rows((size_t)n * 7 + 1);
    int rc = lbm_rsa_seed(h->p.nx, h->p.ny, n, diameter, min_gap, seed, rows.data());
    if (rc != LBM_OK) return fail(h, rc, "%s", g_create_error.c_str());
    return lbm_set_particles(h, n, rows.data());
}

namespace {

// rows of `cols` values: 7 = (x, y, r, ux, uy, theta, omega) for circles,
// 8 = (x, y, a, b, ux, uy, theta, omega) for ellipses.
int set_particles_rows(lbm_handle h, int32_t n, const double* rows, int cols) {
    if (!h) return LBM_EINVAL;
    if (n < 0 || n > h->p.max_particles) return fail(h, LBM_EINVAL, "particle count %d outside [0, %d]", n, h->p.max_particles);
    if (n > 0 && !rows) return fail(h, LBM_EINVAL, "null particle rows");
    std::vector<PState> P((size_t)n);
    const double rmax = 0.5 * h->p.max_diameter;
    for (int i = 0; i < n; ++i) {
        const double* row = rows + (size_t)cols * i;
        for (int c = 0; c < cols; ++c)
            if (!std::isfinite(row[c])) return fail(h, LBM_EINVAL, "particle %d: non-finite value", i);
        double in[7];
        double b = row[2];
        if (cols == 7) {
            for (int c = 0; c < 7; ++c) in[c] = row[c];
        } else {
            in[0] = row[0];
            in[1] = row[1];
            in[2] = row[2];
            b = row[3];
            for (int c = 3; c < 7; ++c) in[c] = row[c + 1];
        }
        if (!(in[2] > 1.0) || in[2] > rmax) return fail(h, LBM_EINVAL, "particle %d: radius %g outside (1, %g]", i, in[2], rmax);
        if (!(b > 1.0) || b > in[2]) return fail(h, LBM_EINVAL, "particle %d: semi-axis b = %g outside (1, a]", i, b);
        if (in[1] < -0.5 || in[1] > h->p.ny - 0.5) return fail(h, LBM_EINVAL, "particle %d: centre outside the channel", i);
        double x = in[0];
        if (h->p.periodic_x) {
            x = std::fmod(in[0], (double)h->p.nx);
            if (x < 0) x += h->p.nx;
        } else if (x < -0.5 || x > h->p.nx - 0.5) {
            return fail(h, LBM_EINVAL, "particle %d: centre outside the cavity", i);
        }
        P[i] = PState{x, in[1], in[2], in[3], in[4], in[5], in[6], b};
    }
    DevState& d = h->d;
    hipStream_t st = h->stream;
    HIPCHK(h, hipStreamSynchronize(st));
    forget_batches(h);
    h->np = n;
    h->generation += 1;
    d.lp.np = n;
    d.lp.lpp = lanes_per_particle(h->L.nwin, n);
    h->cur = 0;
    h->ring = 0;
    h->bin_parity = 0;
    const size_t nb = h->L.npitched;
    HIPCHK(h, hipMemsetAsync(d.O[0], 0xff, nb * 4, st));
    HIPCHK(h, hipMemsetAsync(d.O[1], 0xff, nb * 4, st));
    HIPCHK(h, hipMemsetAsync(d.status, 0, 64, st));
    if (n > 0) {
        for (int r = 0; r < 3; ++r)
            HIPCHK(h, hipMemcpyAsync(d.P[r], P.data(), sizeof(PState) * n, hipMemcpyHostToDevice, st));
        // the order the link pass takes the particles in: row bands one
        // neighbour cell high, left to right within a band, so that blocks
        // that run close in time gather from the same cache lines
        const double band = h->p.max_diameter + std::max(h->p.rep_range, 0.0);
        std::vector<unsigned> order((size_t)n);
        std::vector<long long> key((size_t)n);
        for (int i = 0; i < n; ++i) {
            order[i] = (unsigned)i;
            key[i] = (long long)std::floor((P[i].y + 0.5) / band) * (2LL * h->p.nx + 2) +
                     (long long)std::floor(P[i].x + 0.5);
        }
        std::stable_sort(order.begin(), order.end(), [&](unsigned a, unsigned b) { return key[a] < key[b]; });
        HIPCHK(h, hipMemcpyAsync(d.order, order.data(), sizeof(unsigned) * n, hipMemcpyHostToDevice, st));
        HIPCHK(h, hipStreamSynchronize(st));   // the host vector goes out of scope
        HIPCHK(h, hipMemsetAsync(d.Fh, 0, sizeof(double) * 4 * n, st));
        HIPCHK(h, hipMemsetAsync(d.Fa, 0, sizeof(double) * 4 * n, st));
        HIPCHK(h, hipMemsetAsync(d.seg, 0, sizeof(int2) * n, st));
        for (int b = 0; b < 2; ++b)
            HIPCHK(h, hipMemsetAsync(d.bcnt[b], 0, sizeof(unsigned) * (size_t)d.lp.ncells, st));
        HIPCHK(h, hipMemsetAsync(d.ncand, 0, sizeof(unsigned) * n, st));
        HIPCHK(h, hipMemsetAsync(d.nborn, 0, sizeof(unsigned) * n, st));
        // owner map of t_0 into O[0] from the particles in ring slot 0
        HIPCHK(h, launch_mask_setup(make_runstep(h, 1, 2, 0), st));
        HIPCHK(h, launch_bin_init(d, d.P[0], 0, st));
        HIPCHK(h, launch_step(SK_COLLECT, current_runstep(h), d.mode, st));   // links of t_0
    }
    HIPCHK(h, launch_init(d, 0, 0, h->p.ny, nullptr, nullptr, nullptr, nullptr, true, h->p.rho0, h->p.T_fluid0, st));
    HIPCHK(h, hipStreamSynchronize(st));
    h->steps = 0;
    return LBM_OK;
}

}  // namespace

int lbm_set_particles(lbm_handle h, int32_t n, const double* rows7) { return set_particles_rows(h, n, rows7, 7); }

int lbm_set_particles_ellipse(lbm_handle h, int32_t n, const double* rows8) {
    return set_particles_rows(h, n, rows8, 8);
}

int lbm_set_addressing(lbm_handle h, int32_t mode) {
    if (!h) return LBM_EINVAL;
    if (mode != LBM_LINKS_INDIRECT && mode != LBM_LINKS_DIRECT)
        return fail(h, LBM_EINVAL, "unknown link addressing %d", mode);
    HIPCHK(h, hipStreamSynchronize(h->stream));
    forget_batches(h);
    h->generation += 1;   // captured graphs hold the old constants
    DevState& d = h->d;
    d.lp.direct = mode == LBM_LINKS_DIRECT ? 1 : 0;
    if (h->np > 0) {
        // a direct pass adds into zeroed sums; an indirect step needs the
        // links of the current state
        HIPCHK(h, hipMemsetAsync(d.Fa, 0, sizeof(double) * 4 * h->np, h->stream));
        if (!d.lp.direct) HIPCHK(h, launch_step(SK_COLLECT, current_runstep(h), d.mode, h->stream));
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_set_equilibrium(lbm_handle h, const double* rho, const double* ux, const double* uy, const double* T) {
    if (!h) return LBM_EINVAL;
    if (!rho || !ux || !uy || !T) return fail(h, LBM_EINVAL, "null field");
    const size_t nx = (size_t)h->p.nx;
    const bool f64 = h->p.storage == LBM_STORE_F64;
    const size_t es = f64 ? 8 : 4;
    char* scr = (char*)scratch_of(h);
    const double* src[4] = {rho, ux, uy, T};
    HIPCHK(h, hipStreamSynchronize(h->stream));
    std::vector<float> tmp;
    // in chunks of L.field_rows rows (the whole lattice with two sets)
    for (int y0 = 0; y0 < h->p.ny; y0 += h->L.field_rows) {
        const int rows = std::min(h->L.field_rows, h->p.ny - y0);
        const size_t n = nx * rows, off = nx * y0;
        if (f64) {
            for (int c = 0; c < 4; ++c)
                HIPCHK(h, hipMemcpyAsync(scr + c * n * 8, src[c] + off, n * 8, hipMemcpyHostToDevice, h->stream));
        } else {
            tmp.resize(4 * n);
            for (int c = 0; c < 4; ++c)
                for (size_t k = 0; k < n; ++k) tmp[c * n + k] = (float)src[c][off + k];
            HIPCHK(h, hipMemcpyAsync(scr, tmp.data(), 4 * n * 4, hipMemcpyHostToDevice, h->stream));
        }
        HIPCHK(h, launch_init(h->d, h->cur, y0, rows, scr, scr + n * es, scr + 2 * n * es, scr + 3 * n * es, f64,
                              0.0, 0.0, h->stream));
        HIPCHK(h, hipStreamSynchronize(h->stream));
    }
    h->steps = 0;
    return LBM_OK;
}

int lbm_step(lbm_handle h, int32_t nsteps) {
    if (!h) return LBM_EINVAL;
    if (nsteps < 0) return fail(h, LBM_EINVAL, "negative step count");
    if (nsteps == 0) return LBM_OK;
    HIPCHK(h, hipEventRecord(h->ev_t0, h->stream));
    int32_t s = 0;
    // whole 6-step cycles (the step state repeats every 6 steps) replay the
    // graph captured for the current state, captured once there are two
    // cycles to run or kept from an earlier call
    const int state = state_index(h->cur, h->ring, h->bin_parity);
    const bool have = h->cycle_graph[state] && h->cycle_generation[state] == h->generation;
    if (nsteps >= 12 || (have && nsteps >= 6)) {
        if (!have) {
            int rc = capture_cycle(h);
            if (rc != LBM_OK) return rc;
        }
        for (; nsteps - s >= 6; s += 6) {
            HIPCHK(h, hipGraphLaunch(h->cycle_graph[state], h->stream));
            h->steps += 6;   // six steps return the state to where it was
        }
    }
    for (; s < nsteps; ++s) {
        int rc = enqueue_step(h, nullptr);
        if (rc != LBM_OK) return rc;
    }
    HIPCHK(h, hipEventRecord(h->ev_t1, h->stream));
    h->timed_steps = nsteps;
    return LBM_OK;
}

int lbm_sync(lbm_handle h) {
    if (!h) return LBM_EINVAL;
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return check_status(h);
}

int lbm_read_fields(lbm_handle h, double* rho, double* ux, double* uy, double* T, int32_t* owner) {
    if (!h) return LBM_EINVAL;
    int rc = lbm_sync(h);
    if (rc != LBM_OK && rc != LBM_EUNSTABLE) return rc;
    const size_t nx = (size_t)h->p.nx;
    const bool f64 = h->p.storage == LBM_STORE_F64;
    void* scr = scratch_of(h);
    double* outs[4] = {rho, ux, uy, T};
    std::vector<float> tmp;
    // in chunks of L.field_rows rows (the whole lattice with two sets)
    for (int y0 = 0; y0 < h->p.ny; y0 += h->L.field_rows) {
        const int rows = std::min(h->L.field_rows, h->p.ny - y0);
        const size_t n = nx * rows, off = nx * y0;
        HIPCHK(h, launch_macros(h->d, h->cur, y0, rows, scr, h->stream));
        if (f64) {
            for (int c = 0; c < 4; ++c)
                if (outs[c])
                    HIPCHK(h, hipMemcpyAsync(outs[c] + off, (char*)scr + c * n * 8, n * 8, hipMemcpyDeviceToHost,
                                             h->stream));
            HIPCHK(h, hipStreamSynchronize(h->stream));
        } else {
            tmp.resize(n);
            for (int c = 0; c < 4; ++c) {
                if (!outs[c]) continue;
                HIPCHK(h, hipMemcpyAsync(tmp.data(), (char*)scr + c * n * 4, n * 4, hipMemcpyDeviceToHost, h->stream));
                HIPCHK(h, hipStreamSynchronize(h->stream));
                for (size_t k = 0; k < n; ++k) outs[c][off + k] = tmp[k];
            }
        }
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    // the owner map row by row out of the pitched layout, as a blocking copy
    // (the asynchronous 2-D copy into pageable memory came back as zeros
    // under a profiler)
    if (owner)
        HIPCHK(h, hipMemcpy2D(owner, (size_t)h->p.nx * 4, h->d.O[h->cur], (size_t)h->L.pitch * 4,
                              (size_t)h->p.nx * 4, h->p.ny, hipMemcpyDeviceToHost));
    return rc;
}

int lbm_read_particles(lbm_handle h, double* rows10, int32_t* n) {
    if (!h) return LBM_EINVAL;
    if (n) *n = h->np;
    if (!rows10 || h->np == 0) return LBM_OK;
    int rc = lbm_sync(h);
    if (rc != LBM_OK && rc != LBM_EUNSTABLE) return rc;
    std::vector<PState> P(h->np);
    std::vector<double> F((size_t)4 * h->np);
    HIPCHK(h, hipMemcpyAsync(P.data(), h->d.P[h->ring], sizeof(PState) * h->np, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipMemcpyAsync(F.data(), h->d.Fh, sizeof(double) * 4 * h->np, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (int i = 0; i < h->np; ++i) {
        double* o = rows10 + 10 * (size_t)i;
        o[0] = P[i].x; o[1] = P[i].y; o[2] = P[i].r; o[3] = P[i].ux; o[4] = P[i].uy;
        o[5] = P[i].th; o[6] = P[i].om;
        o[7] = F[4 * i]; o[8] = F[4 * i + 1]; o[9] = F[4 * i + 2];
    }
    return rc;
}

int lbm_read_links(lbm_handle h, int32_t* node, int32_t* dir, int32_t* particle, double* q, int64_t cap,
                   int64_t* n_out) {
    if (!h) return LBM_EINVAL;
    int rc = lbm_sync(h);
    if (rc != LBM_OK) return rc;
    if (n_out) *n_out = 0;
    if (h->np == 0) return LBM_OK;
    DevState& d = h->d;
    if (d.lp.direct) {   // direct addressing collects nothing: collect now
        RunStep R = current_runstep(h);
        R.lp.direct = 0;
        HIPCHK(h, launch_step(SK_COLLECT, R, d.mode, h->stream));
    }
    // the links of the current state were collected at the end of the last
    // step (or by lbm_set_particles), each particle's at the front of its
    // own segment; gather them into one list on the host
    const size_t per = (size_t)(12 * h->L.nwin - 12), np = (size_t)h->np;
    std::vector<int2> seg(np);
    HIPCHK(h, hipMemcpyAsync(seg.data(), d.seg, np * sizeof(int2), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    size_t nl = 0;
    for (const int2& sg : seg) nl += (size_t)sg.y;
    if (n_out) *n_out = (int64_t)nl;
    if (!(node || dir || particle || q) || nl == 0) return LBM_OK;
    if ((int64_t)nl > cap) return fail(h, LBM_EINVAL, "cap %lld < %zu links", (long long)cap, nl);
    std::vector<uint2> all(np * per), list;
    list.reserve(nl);
    HIPCHK(h, hipMemcpyAsync(all.data(), d.links, all.size() * sizeof(uint2), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    for (size_t p = 0; p < np; ++p)
        for (int i = 0; i < seg[p].y; ++i) list.push_back(all[(size_t)seg[p].x + i]);
    char* ls = h->base + h->L.off_lscratch;
    uint2* dl = (uint2*)ls;
    ls += round_up(nl * sizeof(uint2), 8);
    int32_t* dn = (int32_t*)ls;
    int32_t* dd = dn + nl;
    int32_t* dp = dd + nl;
    double* dq = (double*)(ls + round_up(nl * 12, 8));
    HIPCHK(h, hipMemcpyAsync(dl, list.data(), nl * sizeof(uint2), hipMemcpyHostToDevice, h->stream));
    HIPCHK(h, launch_link_q(d, h->ring, dl, (int)nl, dn, dd, dp, dq, h->stream));
    if (node) HIPCHK(h, hipMemcpyAsync(node, dn, nl * 4, hipMemcpyDeviceToHost, h->stream));
    if (dir) HIPCHK(h, hipMemcpyAsync(dir, dd, nl * 4, hipMemcpyDeviceToHost, h->stream));
    if (particle) HIPCHK(h, hipMemcpyAsync(particle, dp, nl * 4, hipMemcpyDeviceToHost, h->stream));
    if (q) HIPCHK(h, hipMemcpyAsync(q, dq, nl * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(h, hipStreamSynchronize(h->stream));
    return check_status(h);
}

int lbm_time_phases(lbm_handle h, int32_t nsteps, double* ms_out) {
    if (!h || !ms_out || nsteps <= 0) return h ? fail(h, LBM_EINVAL, "invalid arguments") : LBM_EINVAL;
    hipEvent_t ev[LBM_NPHASES + 1];
    for (auto& e : ev) HIPCHK(h, hipEventCreate(&e));
    double acc[LBM_NPHASES + 1] = {0};
    int rc = LBM_OK;
    for (int32_t s = 0; s < nsteps && rc == LBM_OK; ++s) {
        rc = enqueue_step(h, ev);
        if (rc != LBM_OK) break;
        hipError_t e = hipEventSynchronize(ev[LBM_NPHASES]);
        if (e != hipSuccess) {
            rc = hip_fail(h, e, "hipEventSynchronize");
            break;
        }
        for (int ph = 0; ph < LBM_NPHASES; ++ph) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[ph], ev[ph + 1]);
            acc[ph] += ms;
        }
        float tot = 0.f;
        (void)hipEventElapsedTime(&tot, ev[0], ev[LBM_NPHASES]);
        acc[LBM_NPHASES] += tot;
    }
    for (auto& e : ev) (void)hipEventDestroy(e);
    if (rc != LBM_OK) return rc;
    for (int ph = 0; ph <= LBM_NPHASES; ++ph) ms_out[ph] = acc[ph] / nsteps;
    // the same number of steps as lbm_step runs them (particle kernels
    // concurrent with the lattice kernel), the lattice kernel bracketed
    std::vector<hipEvent_t> le(2 * (size_t)nsteps + 2, nullptr);
    for (auto& e : le)
        if (rc == LBM_OK && hipEventCreate(&e) != hipSuccess) rc = fail(h, LBM_EDEVICE, "hipEventCreate");
    if (rc == LBM_OK && hipEventRecord(le[0], h->stream) != hipSuccess) rc = fail(h, LBM_EDEVICE, "hipEventRecord");
    for (int32_t s = 0; s < nsteps && rc == LBM_OK; ++s) rc = enqueue_step(h, nullptr, &le[2 + 2 * (size_t)s]);
    if (rc == LBM_OK && hipEventRecord(le[1], h->stream) != hipSuccess) rc = fail(h, LBM_EDEVICE, "hipEventRecord");
    if (rc == LBM_OK && hipEventSynchronize(le[1]) != hipSuccess) rc = fail(h, LBM_EDEVICE, "hipEventSynchronize");
    if (rc == LBM_OK) {
        double lat = 0.0;
        float ms = 0.f;
        for (int32_t s = 0; s < nsteps; ++s) {
            (void)hipEventElapsedTime(&ms, le[2 + 2 * (size_t)s], le[3 + 2 * (size_t)s]);
            lat += ms;
        }
        (void)hipEventElapsedTime(&ms, le[0], le[1]);
        ms_out[LBM_NPHASES + 1] = h->np > 0 ? lat / nsteps : ms_out[LBM_PHASE_LATTICE];
        ms_out[LBM_NPHASES + 2] = ms / nsteps;
    }
    for (auto& e : le)
        if (e) (void)hipEventDestroy(e);
    if (rc != LBM_OK) return rc;
    return check_status(h);
}

int lbm_stats(lbm_handle h, double* out) {
    if (!h || !out) return LBM_EINVAL;
    std::vector<int2> seg((size_t)h->np);
    std::vector<unsigned> nb((size_t)h->np);
    if (h->np > 0) {
        HIPCHK(h, hipMemcpyAsync(seg.data(), h->d.seg, seg.size() * sizeof(int2), hipMemcpyDeviceToHost,
                                 h->stream));
        HIPCHK(h, hipMemcpyAsync(nb.data(), h->d.nborn, nb.size() * sizeof(unsigned), hipMemcpyDeviceToHost,
                                 h->stream));
    }
    HIPCHK(h, hipStreamSynchronize(h->stream));
    double nl = 0.0, newborn = 0.0;
    for (const int2& sg : seg) nl += sg.y;
    for (unsigned v : nb) newborn += v;
    double ms = 0.0;
    if (h->timed_steps > 0) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, h->ev_t0, h->ev_t1) == hipSuccess) ms = (double)t / h->timed_steps;
        else (void)hipGetLastError();
    }
    const double nodes = (double)h->p.nx * h->p.ny;
    // algorithmic bytes of a lattice update: 9 + 5 populations read and written
    const double bytes_per_step = nodes * 28.0 * (double)elem_size(h->p.storage);
    out[LBM_STAT_STEPS] = (double)h->steps;
    out[LBM_STAT_LINKS] = nl;
    out[LBM_STAT_NEWBORN] = newborn;
    out[LBM_STAT_MS_PER_STEP] = ms;
    out[LBM_STAT_GBPS] = ms > 0.0 ? bytes_per_step / (ms * 1e-3) / 1e9 : 0.0;
    out[LBM_STAT_PARTICLES] = (double)h->np;
    out[LBM_STAT_NODES] = nodes;
    out[LBM_STAT_DEVICE_BYTES] = (double)h->L.total;
    return LBM_OK;
}

int lbm_check_budget(const lbm_params* p, size_t budget_bytes) {
    std::string why;
    if (!validate(p, why)) return fail(nullptr, LBM_EINVAL, "%s", why.c_str());
    const size_t need = make_layout(*p).total;
    if (need > budget_bytes) return fail(nullptr, LBM_EBUDGET, "the run needs %zu bytes, the budget is %zu", need, budget_bytes);
    return LBM_OK;
}

int lbm_time_copy(lbm_handle h, int32_t reps, double* ms_out) {
    if (!h || !ms_out || reps <= 0) return h ? fail(h, LBM_EINVAL, "invalid arguments") : LBM_EINVAL;
    // the current state A is read; B (the set the next step writes whole)
    // receives the copy; in place the single set is copied onto itself
    const RunStep R = current_runstep(h);
    const size_t bytes = h->L.npitched * elem_size(h->p.storage);   // a multiple of 16: rows of 64 nodes
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = LBM_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = fail(h, LBM_EDEVICE, "hipEventCreate");
    double best = 0.0;
    // the faster of 8- and 16-byte lanes (which is faster depends on the GPU
    // and the value size)
    for (int lane : {8, 16}) {
        if (rc == LBM_OK && launch_copy(R, bytes, lane, h->stream) != hipSuccess) rc = fail(h, LBM_EDEVICE, "copy launch");
        if (rc == LBM_OK && hipEventRecord(e0, h->stream) != hipSuccess) rc = fail(h, LBM_EDEVICE, "hipEventRecord");
        for (int32_t r = 0; r < reps && rc == LBM_OK; ++r)
            if (launch_copy(R, bytes, lane, h->stream) != hipSuccess) rc = fail(h, LBM_EDEVICE, "copy launch");
        if (rc == LBM_OK && hipEventRecord(e1, h->stream) != hipSuccess) rc = fail(h, LBM_EDEVICE, "hipEventRecord");
        if (rc == LBM_OK && hipEventSynchronize(e1) != hipSuccess) rc = fail(h, LBM_EDEVICE, "hipEventSynchronize");
        float ms = 0.f;
        if (rc == LBM_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = fail(h, LBM_EDEVICE, "hipEventElapsedTime");
        if (rc == LBM_OK && (best == 0.0 || ms / reps < best)) best = (double)ms / reps;
    }
    if (rc == LBM_OK) *ms_out = best;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}

size_t lbm_collect_lds_bytes(const lbm_params* p) {
    std::string why;
    if (!validate(p, why) || p->max_particles <= 0) return 0;
    const int nwin = window_cap(p->max_diameter);
    LP lp{};
    lp.nwin = nwin;
    size_t worst = 0;
    for (int n : {1, p->max_particles}) {
        lp.lpp = lanes_per_particle(nwin, n);
        worst = std::max(worst, links_block_lds(lp));
    }
    return worst;
}

}  // extern "C"
