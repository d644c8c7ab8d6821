// wave.h -- wavefront-level scans, lane sums and the uniform-value helper
// shared by the dose and adjoint kernels (wave64, gfx950).
#pragma once

#include "fspb_internal.h"

namespace fspb {

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ int wave_incl_scan_int(int x, int lane) {
    for (int o = 1; o < kWave; o <<= 1) {
        int y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    return x;
}

// Shuffles addressed from an explicit lane index.  In the adjoint's unit
// loop the lane comes through an empty asm statement (opaque_lane), so that
// the compiler recomputes the lane addresses at each use instead of keeping
// a dozen of them in registers across the loop (where they were spilled).
__device__ __forceinline__ int opaque_lane(int lane) {
    asm volatile("" : "+v"(lane));
    return lane;
}
__device__ __forceinline__ int lane_incl_scan_int(int x, int lane) {
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __builtin_amdgcn_ds_bpermute((lane - o) << 2, x);
        if (lane >= o) x += y;
    }
    return x;
}
__device__ __forceinline__ int lane_xor_sum_bits(int x, int lane, bool fp) {
    for (int o = 32; o > 0; o >>= 1) {
        const int y = __builtin_amdgcn_ds_bpermute((lane ^ o) << 2, x);
        x = fp ? __float_as_int(__int_as_float(x) + __int_as_float(y)) : x + y;
    }
    return x;
}

}  // namespace fspb
