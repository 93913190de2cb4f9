// sim.h -- the handle behind the C ABI (lbm_handle) and the host helpers
// shared by api.cpp (single runs) and serve.cpp (batched runs).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "launch.h"
#include "lbm.h"

namespace ptlbm {

// Offsets of every buffer inside the handle's one device allocation.
struct Layout {
    int pitch = 0;
    size_t npitched = 0, array_stride = 0, state_bytes = 0;
    size_t off_S[2] = {0, 0}, off_O[2] = {0, 0}, off_P = 0, off_Fh = 0, off_Fa = 0, off_seg = 0,
           off_links = 0, off_lscratch = 0, off_counter = 0, off_status = 0, off_bins[2] = {0, 0},
           off_bcnt[2] = {0, 0}, off_cand = 0, off_ncand = 0, off_nborn = 0, off_order = 0, off_rbuf = 0, off_fscratch = 0, off_cc = 0,
           total = 0;
    int field_rows = 0;   // rows per chunk of the field upload / read-back scratch
    int nwin = 0;
    size_t link_cap = 0;
    int ncx = 1, ncy = 1;
};

}  // namespace ptlbm

struct lbm_sim {
    lbm_params p{};
    ptlbm::Layout L;
    ptlbm::DevState d{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t side = nullptr;  // particle kernels, concurrent with the lattice kernel
    hipEvent_t ev_fork = nullptr, ev_side = nullptr;
    hipEvent_t ev_mask = nullptr;  // in place: the owner map and refilled values of t_n+1 are ready
    hipEvent_t ev_order = nullptr; // orders another stream after the work on this handle's stream
    char* base = nullptr;
    bool own_mem = false;
    int cur = 0;         // time level holding the current (post-collision) state; in place its parity
    int ring = 0;        // particle slot of the current time level
    int bin_parity = 0;  // cell grid holding the particles of the current time level
    int np = 0;
    int64_t steps = 0;
    uint64_t generation = 0;  // bumped whenever the particle count changes
    // six overlapped steps captured from each step state (state_index), for
    // the particle generation they were captured in
    hipGraphExec_t cycle_graph[12] = {};
    uint64_t cycle_generation[12] = {};
    // device time of the last lbm_step call (lbm_stats)
    hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;
    int32_t timed_steps = 0;
    std::string err;
};

namespace ptlbm {

// Record an error message on the handle (or, with h NULL, for the calling
// thread) and return code.
int fail(lbm_sim* h, int code, const char* fmt, ...);
int hip_fail(lbm_sim* h, hipError_t e, const char* what);

// The buffers of the step taken from time level c, ring slot r, cell-grid
// parity bp; the current step of h; the state after one more step.
RunStep make_runstep(const lbm_sim* h, int c, int r, int bp);
RunStep current_runstep(const lbm_sim* h);
RunStep next_runstep(const lbm_sim* h);
void advance_state(lbm_sim* h);
// Step-cycle position of h: the state repeats every 6 steps.
inline int state_index(int cur, int ring, int bp) { return cur * 6 + ring * 2 + bp; }

// Drop every cached batch that refers to h (serve.cpp).
void forget_batches(const lbm_sim* h);

}  // namespace ptlbm

#define HIPCHK(h, expr)                                                   \
    do {                                                                  \
        hipError_t e_ = (expr);                                           \
        if (e_ != hipSuccess) return ptlbm::hip_fail(h, e_, #expr);       \
    } while (0)
