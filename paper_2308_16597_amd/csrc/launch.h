// launch.h -- host-side launchers of the gfx950 kernels (kernels.hip), used
// by the C ABI implementation (api.cpp).  Every launcher enqueues on the
// given stream and returns the launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.h"

namespace ptlbm {

struct DevState {
    LP lp;
    int mode;
    void* S[2][14];              // population arrays of the two time levels
    int32_t* O[2];               // owner maps
    PState* P[3];                // particle ring (old, current, next rotate)
    double* Fh;                  // per-particle momentum-exchange force/torque (x, y, z, pad)
    double4* contrib;            // per-link momentum exchange (Fx, Fy, Tz, pad)
    uint2* links;                // compacted link array
    int2* seg;                   // per-particle {start, count}
    unsigned* counter;           // [0] link counter, [1] links of the last step
    unsigned* status;            // device error bits
    unsigned* bins[2];           // cell grid (BINCAP particle slots per cell), two time levels
    unsigned* bcnt[2];           // particles per cell
    unsigned* cand;              // newborn-node candidates, 4 nwin per particle (x | y << 16)
    unsigned* ncand;             // candidates per particle
};

enum StatusBits : unsigned {
    ST_NONFINITE = 1u,      // non-finite macroscopic value
    ST_OVERSPEED = 2u,      // particle moved more than 0.5 per step
    ST_LINK_OVERFLOW = 4u,  // link array too small
    ST_BAD_PARTICLE = 8u,   // particle state unusable (not finite / far outside)
    ST_BIN_OVERFLOW = 16u,  // more than BINCAP particles in one neighbour-search cell
    ST_CAND_OVERFLOW = 32u, // more newborn nodes for one particle than its candidate list holds
};

hipError_t launch_stream_collide(const DevState& d, int cur, hipStream_t st);
hipError_t launch_init(const DevState& d, int cur, const void* rho, const void* ux, const void* uy,
                       const void* T, bool fields_f64, double rho_u, double T_u, hipStream_t st);
hipError_t launch_macros(const DevState& d, int cur, void* out, hipStream_t st);
hipError_t launch_links(const DevState& d, int cur, int ring, hipStream_t st);
hipError_t launch_link_pass(const DevState& d, int cur, int ring, hipStream_t st);
hipError_t launch_particles(const DevState& d, int ring, int bin_parity, hipStream_t st);
hipError_t launch_bin_init(const DevState& d, const PState* P, int bin_parity, hipStream_t st);
hipError_t launch_mask_mark(const DevState& d, int owner_idx, const PState* P, const PState* Pprev,
                            unsigned* cnt_clear, hipStream_t st);
hipError_t launch_refill(const DevState& d, int cur, int ring, hipStream_t st);
hipError_t launch_link_q(const DevState& d, int ring, int nlinks, int32_t* node, int32_t* dir,
                         int32_t* part, double* q, hipStream_t st);

// Ring slots: current = ring, next = (ring + 1) % 3, old = (ring + 2) % 3.
inline int ring_next(int r) { return (r + 1) % 3; }
inline int ring_old(int r) { return (r + 2) % 3; }

}  // namespace ptlbm
