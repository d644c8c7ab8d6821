// fspb_internal.h -- device data layouts shared by the gfx950 kernels and the
// host side of libfspb.  Not part of the public ABI (see include/fspb.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fspb {

constexpr float kLog2e = 1.4426950408889634f;
constexpr int kWave = 64;

// FP64 frame of one beamlet, written by the beamlet-setup kernel and read by
// the ray trace.  Geometry of Eq. 2: source r_s, unit direction, lateral axes.
struct Frame64 {
    double src[3];
    double d[3];
    double ex[3];
    double ey[3];
    double theta;      // angle to the beam's central axis
    double s_in;       // distance from the source to the grid-box entry
    double s_cover;    // deepest box point along the axis (table coverage)
    double sad, x0, y0;
    int n_samples;     // samples from s_in (0 if the axis misses the box)
    int beam;
};

// FP32 descriptor of one beamlet for the pair kernels.  All positions are
// relative to the plan reference point P0 (the grid centre):
//   t  = q.d  + c_t   depth below the entrance (s - s_entry)
//   xp = q.ex + c_x   lateral offsets from the axis
//   yp = q.ey + c_y
// with q = r - P0.  96 bytes, read with scalar loads (wave-uniform index);
// everything the uniform-table pair arithmetic reads sits in the first 80
// bytes (one 64-byte and one 16-byte scalar load).  A larger descriptor
// costs the forward more in scalar loads than the arithmetic it could save.
struct alignas(16) BeamletDesc {
    float d[3];
    float c_t;
    float ex[3];
    float c_x;
    float ey[3];
    float c_y;
    float s_entry;     // |r_a| = t + s_entry
    float sad;
    float nx2, ny2;    // -2 x0, -2 y0: beamlet half widths at the isocentre
                       // plane (Eq. 4), in the form the profile arithmetic uses
    float th_frac;     // A-table theta interpolation weight
    int a_off;         // first A-table record of the beamlet's theta rows (r, r+1): r n_A
    int tab_off;       // first sample of this beamlet's depth tables
    int j_last;        // last usable depth-table interval, max(K - 2, 0)
    int hit;
    float theta;       // angle to the beam's central axis
    int beam;          // index of the beam the beamlet belongs to
    int K;             // depth-table length (0 if the beamlet misses the body)
};
static_assert(sizeof(BeamletDesc) == 96, "BeamletDesc layout");
static_assert(sizeof(BeamletDesc) % 16 == 0, "BeamletDesc is read as float4 records");

// Per-beam data for candidate-beamlet culling.  A voxel at q (relative to
// P0) projects onto the isocentre plane at (a, b) = (v.ex, v.ey) * sad/(v.cax)
// with v = q - src.  Beamlet (n, m) sits at (a0 + m wx, b0 + n wy).
struct alignas(16) BeamDesc {
    float src[3];
    float sad;
    float cax[3];
    float pad_scale;   // R * SAD / cos(theta_max): lateral reach in the iso plane times depth
    float ex[3];
    float a0;
    float ey[3];
    float b0;
    float wx, wy;
    int nbx, nby;
    int first;         // index of the beam's first beamlet
    // depth bins of the per-beam schedule: a point at depth z = (q - src).cax
    // along the central axis falls in bin (z - zlo) zinv, of nbins
    float zlo, zinv;
    int nbins;
};
static_assert(sizeof(BeamDesc) == 96, "BeamDesc layout");

// Density-correction modes of the pair kernels (their template argument DC).
// Section 2.1 gives both weight components one drift integral of a single
// b(rho); the library accepts a separate b_i per component.  When the
// commissioned b2 is c b1 at every table sample (c = 1: the single b of the
// paper), the second drift is c W1 and a pair reads one depth record (tTW)
// instead of two (tTW and tW2); that load is what limits the corrected
// forward.  With c = +-1 both modes give bitwise the same dose.
enum { kPlain = 0, kDcTwoDrift = 1, kDcOneDrift = 2 };

// Plan-wide constants passed by value to the pair kernels.
struct PlanConst {
    int nx, ny, nz, n_beams;
    float dx, dy, dz, R2;
    float qx0, qy0, qz0;  // centre of voxel (0,0,0) minus P0
    float inv_d;          // 1 / ray sample step
    float dt_inv, dt_off, at_inv, at_off;  // table coordinate = value * inv + off
    int dt_n, at_n, a_cols, dc;
    float w2c;            // b2 = w2c b1 at every table sample when w2_one
    int w2_one;           // (the second weight drift is then w2c W1)
};

// Density-table grid (host copy of start/step/n for the factor kernel and
// the ray trace).
struct DTab {
    float start, step, inv_step;
    int n, off;           // off: first value in the packed device array
};

struct DensTabs {
    DTab fu1, fu2, fw1, fw2, b1, b2;
    float rho_min, rho_max;
};

// Linear lookup with clamped coordinate in a packed density table.
__device__ __forceinline__ float dens_lookup(const float* __restrict__ v, DTab t, float x) {
    float c = (x - t.start) * t.inv_step;
    c = fminf(fmaxf(c, 0.0f), (float)(t.n - 1));
    int i = (int)c;
    i = max(min(i, t.n - 2), 0);
    float f = (t.n > 1) ? c - (float)i : 0.0f;
    float a = v[t.off + i];
    float b = v[t.off + min(i + 1, t.n - 1)];
    return fmaf(f, b - a, a);
}

}  // namespace fspb
