// copy.hip -- the bandwidth ceiling of the lattice update: a plain copy of a
// run's 14 population arrays, the bytes one stream-collide (Sec. 2.1) reads
// and writes, with no arithmetic (lbm_time_copy).
#include <hip/hip_runtime.h>

#include "launch.h"

namespace ptlbm {

// A -> B, one V (8 or 16 bytes: 1 to 8 nodes of each array; every array
// holds the padded lattice, whose size is a multiple of 16 bytes) per lane
// and array, non-temporal loads and stores.
template <class V>
__global__ __launch_bounds__(LAT_BLOCK) void k_copy14(RunStep rs, size_t nchunks) {
    const size_t c = (size_t)blockIdx.x * LAT_BLOCK + threadIdx.x;
    if (c >= nchunks) return;
#pragma unroll
    for (int i = 0; i < 14; ++i) {
        const PT_GLOBAL V* a = (const PT_GLOBAL V*)rs.A[i];
        PT_GLOBAL V* b = (PT_GLOBAL V*)rs.B[i];
        __builtin_nontemporal_store(__builtin_nontemporal_load(a + c), b + c);
    }
}
// The tiled 8-byte state (lattice.h) is one block of 14 arrays' bytes from
// A[0] on: copied as one array, one V per lane.
template <class V>
__global__ __launch_bounds__(LAT_BLOCK) void k_copy_block(RunStep rs, size_t nchunks) {
    const size_t c = (size_t)blockIdx.x * LAT_BLOCK + threadIdx.x;
    if (c >= nchunks) return;
    __builtin_nontemporal_store(__builtin_nontemporal_load((const PT_GLOBAL V*)rs.A[0] + c), (PT_GLOBAL V*)rs.B[0] + c);
}

hipError_t launch_copy(const RunStep& R, size_t array_bytes, int lane_bytes, hipStream_t st) {
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
    const size_t nchunks = array_bytes / (size_t)lane_bytes;
    const unsigned nblocks = (unsigned)((nchunks + LAT_BLOCK - 1) / LAT_BLOCK);
    const size_t es = array_bytes / ((size_t)R.lp.pitch * (size_t)R.lp.ny);
    if (es == 8) {   // tiled: the 14 arrays' bytes as one block
        const size_t nflat = 14 * nchunks;
        const unsigned nbf = (unsigned)((nflat + LAT_BLOCK - 1) / LAT_BLOCK);
        if (lane_bytes == 16) k_copy_block<u32x4><<<nbf, LAT_BLOCK, 0, st>>>(R, nflat);
        else k_copy_block<u32x2><<<nbf, LAT_BLOCK, 0, st>>>(R, nflat);
    } else if (lane_bytes == 16) {
        k_copy14<u32x4><<<nblocks, LAT_BLOCK, 0, st>>>(R, nchunks);
    } else {
        k_copy14<u32x2><<<nblocks, LAT_BLOCK, 0, st>>>(R, nchunks);
    }
    return hipGetLastError();
}

}  // namespace ptlbm
