// kernels.h -- launch wrappers of the gfx950 kernels (host-callable).
#pragma once

#include "fspb_internal.h"

namespace fspb {

// Beam parameters in FP64 for the beamlet-setup kernel.
struct BeamIn {
    double gantry, couch, iso[3], sad, wx, wy, cx, cy;
    int nbx, nby, first, pad;
};

struct TraceGrid {
    double o[3], inv[3];
    int n[3];
    double del[3];   // voxel sizes (the plane positions of the exact path)
};

struct TraceParams {
    double step, rho_surface, theta_step;
    double p0[3];
    int n_theta, n_A, k_stride;
};

// Per-beamlet ray-trace results kept for inspection.
struct TraceInfo {
    int n_samples, k_entry;
    double s_entry, margin;
};

// Smoothed density and per-voxel factors from rho.  With copy non-null the
// first kernel also copies rho there (after_copy, if non-null, is recorded
// once that kernel is queued) and the factors read the copy.  tmp1 is used
// only by the single-axis passes (radii over 24 voxels).
void launch_smooth(const float* rho, float* copy, hipEvent_t after_copy, float* tmp0, float* tmp1,
                   float* rhohat, float4* fac, int nx, int ny, int nz, const float* w3,
                   const int r[3], const float* dtabs, const DensTabs& dt, hipStream_t s);
void launch_setup(const BeamIn* beams, int n_beams, int n_beamlets, const double lo[3],
                  const double hi[3], double step, Frame64* out, hipStream_t s);
void launch_trace(const Frame64* frames, int n_beamlets, const float* rho, const TraceGrid& g,
                  const TraceParams& tp, const float* dtabs, const DensTabs& dt, float2* tT,
                  float4* tTW, float2* tW2, BeamletDesc* desc, TraceInfo* info, hipStream_t s);

// Exact (Siddon) depth tables instead of the uniform samples: per beamlet,
// one 32-byte record per voxel segment past the entrance,
//   sid[2(off + m)]     = (t_m, T_m, rho_m, W1_m)   depth and integrals at
//                                                  the segment start, T slope
//   sid[2(off + m) + 1] = (b1_m, W2_m, b2_m, 0)     weight-drift slopes
// with off = beamlet * stride; the descriptor's K counts the records.
void launch_siddon(const Frame64* frames, int n_beamlets, const float* rho, const TraceGrid& g,
                   const TraceParams& tp, int stride, const float* dtabs, const DensTabs& dt,
                   float4* sid, BeamletDesc* desc, TraceInfo* info, hipStream_t s);

// Dose kernels (dose.hip).
struct DoseArgs {
    PlanConst P;
    const BeamDesc* beams;
    const BeamletDesc* bl;
    const float4* fac;
    const float4* dtab;
    const float4* atab;
    const float2* tT;
    const float4* tTW;
    const float2* tW2;
    const float4* sid;     // exact depth tables (null unless the plan uses them)
};

// Forward-kernel tile configuration: brick shape (index into the built
// shapes) and waves per workgroup: 1, 2 or 4 read the water table from
// global memory; kLdsWaves stages it in LDS once per workgroup when it fits
// in kLdsWaterMax bytes (else the launch uses 4 waves and global reads).
constexpr int kNumShapes = 4;
constexpr int kLdsWaves = 8;
constexpr int kLdsWaterMax = 65536;
struct TileCfg {
    int shape = 0;            // 4 x 4 x 4 bricks
    int waves_per_block = kLdsWaves;
    int per_beam = 0;         // 1: the per-beam schedule (below)
};
long brick_count(const PlanConst& P, int shape);
void shape_dims(int shape, int d[3]);

void launch_forward(const DoseArgs& a, bool dc, TileCfg cfg, const int* order,
                    const float* fluence, float* dose, hipStream_t s);
// Dose with the learned surrogate's per-(voxel, beam) parameters (see
// dose.hip, mode kSurr); needs a density-corrected geometry.
// Forward with the exact (Siddon) depth tables.
void launch_forward_siddon(const DoseArgs& a, bool dc, TileCfg cfg, const int* order,
                           const float* fluence, float* dose, hipStream_t s);
void launch_forward_surrogate(const DoseArgs& a, TileCfg cfg, const int* order,
                              const float* fluence, const float4* prm, float* dose, hipStream_t s);
void launch_count(const DoseArgs& a, TileCfg cfg, const int* order, const float* fluence,
                  int* counts, hipStream_t s);
// Evaluated pairs summed per brick of the tile's shape: brick_counts[b] for
// every brick b (brick_count(P, cfg.shape) values, each written once).
void launch_count_bricks(const DoseArgs& a, TileCfg cfg, const int* order, const float* fluence,
                         int* brick_counts, hipStream_t s);
void launch_brick_cost(const DoseArgs& a, TileCfg cfg, int* cost, hipStream_t s);
// order[0..n) = bricks by decreasing cost[brick] (one workgroup, no host round trip)
void launch_order_bricks(const int* cost, long n, int* order, hipStream_t s);

// The per-beam schedule of the forward.  Work items are (brick, beam) pairs,
// item = beam * n_bricks + brick.  They are sorted by beam, then by the
// depth of the brick along the beam's central axis (BeamDesc.nbins bins, at
// most kSplitKeys keys in all), and the sorted list is cut into
// 8 kSplitSegments segments of about equal estimated work; XCD x (workgroup
// q runs on XCD q mod 8) runs segments x, x + 8, ...: within a segment it
// sweeps one beam's slabs front to back, so the depth-table lines of its
// concurrent bricks stay in its L2, and its segments spread over the beams
// and depths so that the XCDs' shares of work match.  Each item writes its
// beam's partial dose to planes[beam][voxel]; sum_planes adds the planes in
// beam order, which is the order the brick-major forward adds its beams in,
// so both give bitwise the same dose for one brick shape.
// With 8-wave workgroups (the water table in LDS) the workgroups are
// persistent instead: each wave takes its XCD's next position from the XCD's
// counter, item after item, until the XCD's run is done.
constexpr int kSplitKeys = 4096;
constexpr int kSplitItemsPerWave = 1;   // consecutive items a wavefront takes
constexpr int kSplitSegments = 2;       // segments per XCD
constexpr int kSplitQueueInts = 16;     // ints per XCD counter (64 bytes apart)
struct SplitSched {
    int* order;     // [n_items] sorted items
    int* chunk;     // [8 kSplitSegments + 1] segment boundaries in order[]
    int* queue;     // [8 kSplitQueueInts] the XCDs' position counters
    int* cost;      // [n_items] scratch: estimated work per item
    int* key;       // [n_items] scratch: sort key per item
    int* hist_n;    // [slices][kSplitKeys] scratch: items per key and slice
    unsigned int* hist_w;   // [slices][kSplitKeys] scratch: work per key and slice
};
// Longest segment, and the most items an XCD runs (the launch covers it).
long split_seg_cap(long n_items);
long split_run_cap(long n_items);
// Slices of the item list the sort's histograms are taken over (at most 64).
int split_sort_slices(long n_items);
void launch_split_schedule(const DoseArgs& a, TileCfg cfg, const SplitSched& sc, hipStream_t s);
void launch_forward_split(const DoseArgs& a, bool dc, TileCfg cfg, const SplitSched& sc,
                          const float* fluence, float* planes, float* dose, int n_cu,
                          hipStream_t s);
// Per-plan fluence and dose pointers of a batch, passed by value as a kernel
// argument (so a captured graph keeps them).
constexpr int kMaxBatchPlans = 64;
struct BatchPtrs {
    const float* fluence[kMaxBatchPlans];
    float* dose[kMaxBatchPlans];
};
// water: the water table every plan of the batch uses (n samples per plane),
// or null when the plans' tables differ (then no LDS staging); dc: the
// correction mode shared by every plan (kPlain, kDcTwoDrift, kDcOneDrift)
void launch_forward_batch(int dc, TileCfg cfg, const DoseArgs* plans, const int2* items,
                          const int* wave_begin, int n_waves, const BatchPtrs& ptrs,
                          unsigned long long* ts_done, unsigned long long* ts_start,
                          const float4* water, int water_n, hipStream_t s);
void launch_fill_u64(unsigned long long* p, long n, unsigned long long v, hipStream_t s);
// The adjoint (and its pair count per beamlet) in units (beamlet, slab of
// `slab` grid planes k): part holds adjoint_slabs(P, slab) * n_beamlets
// partial sums, at most kAdjMaxSlabs * n_beamlets (slab >= adjoint_min_slab),
// queue 8 * kAdjQueueInts ints (the XCDs' unit counters, zeroed by the
// launch); n_cu: the device's compute units.  adjoint_slab(P) is the default
// thickness.
constexpr int kAdjQueueInts = 16;
constexpr int kAdjMaxSlabs = 64;
int adjoint_min_slab(const PlanConst& P);
int adjoint_slab(const PlanConst& P);
int adjoint_slabs(const PlanConst& P, int slab);
void launch_adjoint(const DoseArgs& a, bool dc, int n_beamlets, const float* w, float* grad,
                    float* part, int* queue, int slab, int n_cu, hipStream_t s);
void launch_adjoint_count(const DoseArgs& a, int n_beamlets, int* counts, float* part,
                          int* queue, int slab, int n_cu, hipStream_t s);
void launch_sum_counts(const int* counts, long n, unsigned long long* partial, int n_partial,
                       unsigned long long* total, hipStream_t s);

}  // namespace fspb
