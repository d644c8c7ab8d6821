// mlp.h -- layout constants and launch wrappers of the learned surrogate:
// the MLP (202 -> 64 -> 64 -> 6, tanh-GELU) on the gfx950 matrix cores, its
// input rows (density patch along the source-voxel ray, depth, angle), and
// the fused gather + inference kernel.
#pragma once

#include "kernels.h"

namespace fspb {

constexpr int kMlpIn = 202, kMlpHid = 64, kMlpOut = 6;
constexpr int kMlpInPad = 224;  // layer-1 inputs padded to a multiple of 32
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpIn * kMlpHid;
constexpr int kOffW2 = kOffB1 + kMlpHid;
constexpr int kOffB2 = kOffW2 + kMlpHid * kMlpHid;
constexpr int kOffW3 = kOffB2 + kMlpHid;
constexpr int kOffB3 = kOffW3 + kMlpHid * kMlpOut;
constexpr int kMlpParams = kOffB3 + kMlpOut;   // 17542
// BF16 copy sizes (elements)
constexpr int kW1tN = kMlpHid * kMlpInPad, kW2N = kMlpHid * kMlpHid, kW3tN = 16 * kMlpHid,
              kW3rN = kMlpHid * 32;

// Input row of the surrogate: 200 patch densities (8 planes x 5 x 5), depth
// t and angle theta of the nearest beamlet.  Fixed input scaling:
//   patch: rho - 1;  depth: t / 10 cm - 1;  angle: 10 theta.
constexpr int kPatchPlanes = 8, kPatchSide = 5, kPatchN = 200;
constexpr float kPatchPitch = 0.5f;   // cm between lattice points in a plane

struct MlpWeights {
    const __bf16* w1t;
    const __bf16* w2t;
    const __bf16* w2r;
    const __bf16* w3t;
    const __bf16* w3r;
    const float* b1;
    const float* b2;
    const float* b3;
    __bf16* w1t_rw;
    __bf16* w2t_rw;
    __bf16* w2r_rw;
    __bf16* w3t_rw;
    __bf16* w3r_rw;
};

struct AdamParams {
    float lr, beta1, beta2, eps;
    float bc1, bc2;   // 1 - beta^step
};

// Network outputs are standardised targets: z = y * std + mean, where z is
// (log u1x, log u1y, log u2x, log u2y, w1, w2).
struct SurrogateScale {
    float mean[kMlpOut], stdev[kMlpOut];
};

// A row falls back to the density-corrected parameters when it is invalid
// (no nearest-beamlet pair), when a patch density leaves [rho_lo, rho_hi],
// when the larger of max |rho - rho(voxel)| over the two planes next to the
// voxel and |rho_hat(voxel) - rho(voxel)| exceeds het_max, or when a
// predicted parameter (u, w) leaves [band_lo, band_hi].
struct SurrogateGuard {
    float rho_lo, rho_hi, het_max;
    float band_lo[kMlpOut], band_hi[kMlpOut];
};

int mlp_tiles(long n_rows);
void launch_mlp_forward(const __bf16* X, long n_rows, const MlpWeights& W, float* Y, hipStream_t s);
void launch_mlp_train(const __bf16* X, const float* T, long n_rows, const MlpWeights& W,
                      float* grad, float* loss, hipStream_t s);
void launch_mlp_adam(const float* grad, int n_parts, const MlpWeights& W, float* master, float* m,
                     float* v, const AdamParams& ap, hipStream_t s);
void launch_mlp_sync(const float* master, const MlpWeights& W, hipStream_t s);
void launch_mlp_grad_sum(const float* grad, int n_parts, float* out, hipStream_t s);
void launch_mlp_loss_sum(const float* parts, int n_parts, float* out, hipStream_t s);

// Training rows: rows[k] = (voxel, beam).  X [n][224] BF16 scaled inputs,
// T [n][6] density-corrected parameters of the nearest beamlet (u in 1/cm),
// valid [n].  Needs a density-corrected geometry.
void launch_surrogate_samples(const DoseArgs& a, const float* rho, const int2* rows, long n,
                              __bf16* X, float* T, int* valid, hipStream_t s);
// Every (voxel, beam) row: prm[2 (b n_vox + v)] = (u1x, u1y, u2x, u2y) log2 e,
// prm[2 (b n_vox + v) + 1] = (w1, w2, fallback flag, 0).
// Two passes: classify every row (fallback records written, the others
// listed in live[0 .. *n_live), live holding n_vox * n_beams entries), then
// the gather and network over the list; quad (n_vox records) receives the
// CT's 2x2 neighbourhoods the gathers read.
void launch_surrogate_infer(const DoseArgs& a, const float* rho, const float* rhohat,
                            const MlpWeights& W, const SurrogateScale& sc,
                            const SurrogateGuard& g, float4* prm, float4* quad, unsigned* live,
                            unsigned* n_live, hipStream_t s);

}  // namespace fspb
