// launch.h -- host-side launchers of the gfx950 kernels (lattice.hip,
// particles.hip) and the structures they take, used
// by the C ABI implementation (api.cpp).  Every launcher enqueues on the
// given stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.h"
#include "particles.h"

namespace ptlbm {

struct DevState {
    LP lp;
    int mode;
    void* S[2][14];              // population arrays of the two time levels (one set, twice, in place)
    int32_t* O[2];               // owner maps
    PState* P[3];                // particle ring (old, current, next rotate)
    double* Fh;                  // per-particle momentum-exchange force/torque (x, y, z, pad)
    double* Fa;                  // the link pass's sums (x, y, z, pad), read by k_particles
    uint2* links;                // link array: particle p's links at p (12 nwin - 12)
    int2* seg;                   // per-particle {start, count}
    unsigned* status;            // device error bits
    unsigned* bins[2];           // cell grid (BINCAP particle slots per cell), two time levels
    unsigned* bcnt[2];           // particles per cell
    unsigned* cand;              // newborn-node candidates, 4 nwin per particle (x | y << 16)
    unsigned* ncand;             // candidates per particle
    unsigned* nborn;             // newborn nodes refilled per particle in the last step
    unsigned* order;             // particles in row-band order (the link pass's block order)
    double* rbuf;                // refilled post-collision values per candidate (16 each)
};

// Everything the step kernels need of one run at one step: its lattice
// constants and its buffers resolved for the time level (cur), the particle
// ring slot and the cell-grid parity of that step.  Passed by value to a
// single-run launch; an array of them (one per run) drives a batched launch.
struct RunStep {
    LP lp;
    int parity;                  // in place: 0 reversed state (odd kernel next), 1 pushed (even next)
    void* A[14];                 // post-collision state of t_n
    void* B[14];                 // state of t_n+1 being written (A itself in place)
    int32_t* Ocur;               // owner map of t_n
    int32_t* Onext;              // owner map of t_n+1 (holds t_n-1 until cleared)
    const PState* Pold;          // particles at t_n-1
    const PState* Pc;            // particles at t_n
    PState* Pn;                  // particles at t_n+1
    double* Fh;
    double* Fa;
    uint2* links;
    int2* seg;
    unsigned* status;
    const unsigned* bins_cur;
    unsigned* cnt_cur;           // read by k_particles, cleared by k_mask_mark
    unsigned* bins_next;
    unsigned* cnt_next;
    unsigned* cand;
    unsigned* ncand;
    unsigned* nborn;
    const unsigned* order;
    double* rbuf;
};

// The six step kernels, in the order of a sequential step; SK_COLLECT
// gathers the links of the next step and takes the next step's RunStep.
enum StepKernel { SK_PASS = 0, SK_PARTICLES, SK_MASK, SK_LATTICE, SK_REFILL, SK_COLLECT, SK_COUNT };
// Grid classes of the step kernels: how many blocks one run needs.
enum GridClass { GC_LINKS = 0, GC_PASS, GC_WAVE, GC_LAT, GC_COUNT };
inline GridClass grid_class(int k) {
    return k == SK_COLLECT ? GC_LINKS : k == SK_PASS ? GC_PASS : k == SK_LATTICE ? GC_LAT : GC_WAVE;
}

// A batched launch: one grid over several runs.  bmap[c][b] = {run, block
// of that run} for block b of a class-c kernel; tab holds one RunStep per
// run for the step being launched, tab_next those of the step after it
// (for SK_COLLECT).
struct BatchLaunch {
    const RunStep* tab;
    const RunStep* tab_next;
    const uint2* bmap[GC_COUNT];
    unsigned nblk[GC_COUNT];
    size_t lds;                  // dynamic LDS bytes of the link collection's blocks
    int mode;
    bool aa;                     // every run of the batch streams in place
};

enum StatusBits : unsigned {
    ST_NONFINITE = 1u,      // non-finite macroscopic value
    ST_OVERSPEED = 2u,      // particle moved more than 0.5 per step
    ST_LINK_OVERFLOW = 4u,  // more links for one particle than its segment holds
    ST_BAD_PARTICLE = 8u,   // particle state unusable (not finite / far outside)
    ST_BIN_OVERFLOW = 16u,  // more than BINCAP particles in one neighbour-search cell
    ST_CAND_OVERFLOW = 32u, // more newborn nodes for one particle than its candidate list holds
};

// Blocks one run needs for a kernel of class c.  The per-particle kernels
// give each particle a wavefront (4 per block), or the whole block of 256
// (lp.lpp) when its window is 32 nodes wide or more and there are at most
// 1024 particles.
unsigned run_blocks(int c, const LP& lp);
// Dynamic LDS of one block of the link collection is kept within this.
constexpr size_t kLinksLdsLimit = 65536;
int lanes_per_particle(int nwin, int np);
int pass_threads(int nwin, int np);
size_t links_block_lds(const LP& lp);

hipError_t launch_step(int k, const RunStep& R, int mode, hipStream_t st);
// The lattice kernel alone (lattice.hip), for one run or batched (two-set
// or in place, at each run's parity).
hipError_t launch_lattice(const RunStep& R, int mode, unsigned nblocks, hipStream_t st);
// A plain copy of the run's 14 population arrays A -> B, array_bytes each
// (a multiple of 16), lane_bytes (8 or 16) per lane: the HBM ceiling
// (copy.hip).
hipError_t launch_copy(const RunStep& R, size_t array_bytes, int lane_bytes, hipStream_t st);
hipError_t launch_lattice_batch(const RunStep* tab, const uint2* bmap, unsigned nblocks, int mode, bool aa,
                                hipStream_t st);
// The two halves of the split refill of one run (store = false: compute).
hipError_t launch_refill_part(const RunStep& R, int mode, bool store, hipStream_t st);
hipError_t launch_step_batch(int k, const BatchLaunch& b, hipStream_t st);
// Owner map of R.Pn into R.Onext with no previous time level (set-up).
hipError_t launch_mask_setup(const RunStep& R, hipStream_t st);

// Initial state and macroscopic read-back over rows y0 .. y0 + rows - 1 (the
// host fields and the output are nx x rows planes).
hipError_t launch_init(const DevState& d, int cur, int y0, int rows, const void* rho, const void* ux,
                       const void* uy, const void* T, bool fields_f64, double rho_u, double T_u, hipStream_t st);
hipError_t launch_macros(const DevState& d, int cur, int y0, int rows, void* out, hipStream_t st);
hipError_t launch_bin_init(const DevState& d, const PState* P, int bin_parity, hipStream_t st);
hipError_t launch_link_q(const DevState& d, int ring, const uint2* links, int nlinks, int32_t* node,
                         int32_t* dir, int32_t* part, double* q, hipStream_t st);

// Ring slots: current = ring, next = (ring + 1) % 3, old = (ring + 2) % 3.
inline int ring_next(int r) { return (r + 1) % 3; }
inline int ring_old(int r) { return (r + 2) % 3; }

}  // namespace ptlbm
