// gamma.h -- launch wrappers of the gamma-index kernels (gamma.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace fspb {

constexpr int kMaxGammaOffsets = 4096;   // offsets of the search sphere held in LDS

struct GammaArgs {
    int nx, ny, nz;
    float inv_dD2;   // 1 / dD^2
    float cap2;      // cap^2
    int n_off;
};

struct GammaPart {
    double sum;      // sum of gamma over the statistics region
    long long n;     // voxels in the region
    long long pass;  // of which gamma < 1
    float max;       // max gamma over the grid
    float pad;
};

// off: (dx, dy, dz, bits of |o|^2 / dd^2) sorted by length, (0,0,0) first.
void launch_gamma(const float* ref, const float* ev, const int4* off, const GammaArgs& a,
                  float* gamma, hipStream_t s);
void launch_grid_max(const float* x, long n, float* part, int n_part, float* out, hipStream_t s);
void launch_gamma_stats(const float* gamma, const float* ref, long n, float iso, GammaPart* part,
                        int n_part, GammaPart* out, hipStream_t s);

}  // namespace fspb
