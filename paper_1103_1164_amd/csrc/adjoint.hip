// adjoint.hip -- the transpose of the dose superposition (Eq. 1 over Eqs.
// 2-4) and the per-beamlet count of the pairs of Algorithm A1 step 8, for
// gfx950.
//
// Beamlet-major.  A work unit is (beamlet, slab of grid planes k): the grid
// rows (j, k) of the slab that can meet the beamlet's ROI cylinder.  A
// workgroup solves, one row per thread, the x-interval of each row that can
// hold pairs (in single precision, widened past the pair test's rounding),
// compacts the non-empty intervals with block scans, and deals their voxels
// to its lanes, 64 consecutive voxels per wave; a bitmap of row starts gives
// each lane its row.  Each lane runs the forward's exact pair test (the same
// fmas in the same order) and evaluates the pair with the forward's
// arithmetic.  Units are taken from per-XCD queues slab by slab; per-unit
// sums are added in slab order, so the gradient is deterministic.
#include "kernels.h"
#include "pair.h"
#include "persistent.h"
#include "wave.h"

#include <algorithm>

namespace fspb {

enum { kAdjGrad = 0, kAdjCount = 1 };

// The adjoint of the forward (Eq. 1 transposed): g_b = sum_v w_v D_b(v) over
// the voxels v paired with beamlet b (Algorithm A1, step 8).  The work is cut
// into units (beamlet b, slab s): the grid rows (j, k), k in slab s, that can
// meet b's ROI cylinder.  Each XCD owns a contiguous run of beamlets, whose
// cylinders overlap, and walks its units slab by slab: the voxel weights and
// factors of one slab then serve the whole run from that XCD's L2.  A unit's
// sum goes to part[s n_beamlets + b]; adj_sum_slabs adds the slabs in order,
// so the result does not depend on which workgroup took which unit.
//
// Workgroups are persistent: each takes units from its XCD's queue (an
// atomic counter, zeroed before the launch) until the run is done.
constexpr int kAdjBlocks = 256;          // 64-item blocks per window of items
constexpr float kAdjPad = 0.05f;         // voxels added to each interval end
constexpr float kAdjTSlack = 1e-3f;      // depth below the entrance still scanned

int adjoint_min_slab(const PlanConst& P) { return (P.nz + kAdjMaxSlabs - 1) / kAdjMaxSlabs; }
int adjoint_slab(const PlanConst& P) {
    // about 5 MiB of voxel data (16-byte factors, 4-byte weight) per slab
    const long plane = (long)P.nx * P.ny * 20;
    const long k = ((5L << 20) + plane / 2) / std::max(plane, 1L);
    return (int)std::min<long>(P.nz, std::max<long>({2L, k, (long)adjoint_min_slab(P)}));
}
int adjoint_slabs(const PlanConst& P, int slab) { return (P.nz + slab - 1) / slab; }

// Per-beamlet constants of the row intervals (single precision).  Along a
// grid row, voxel i = 0..nx-1, the pair coordinates are affine in i:
// xp = X0 + a1 i, yp = Y0 + a2 i, t = T0 + a3 i.  R2s is the squared ROI
// radius widened past the pair test's rounding (relative 1e-3 and 1e-5 of
// the grid's extent): every voxel the test accepts lies inside.
struct RowSolve {
    float a1, a2, a3, invA, R2s;
    int j_lo, j_hi, k_lo, k_hi;   // rows (j, k) that can meet the cylinder
};

__device__ __forceinline__ int clamp_index(float x, int lo, int hi) {
    return (int)fminf(fmaxf(x, (float)lo), (float)hi);
}

template <class BD>
__device__ __forceinline__ RowSolve row_solve(const BD& d, const PlanConst& P) {
    RowSolve r;
    r.a1 = P.dx * d.ex[0];
    r.a2 = P.dx * d.ey[0];
    r.a3 = P.dx * d.d[0];
    const float A = fmaf(r.a1, r.a1, r.a2 * r.a2);
    // below 1e-20 the offsets change by less than 1e-10 * nx along a row
    r.invA = A > 1e-20f ? 1.0f / A : 0.0f;
    const float ex_ = P.nx * P.dx, ey_ = P.ny * P.dy, ez_ = P.nz * P.dz;
    const float diag = sqrtf(ex_ * ex_ + ey_ * ey_ + ez_ * ez_);
    const float R = sqrtf(P.R2);
    const float Rs = fmaf(R, 1.0f + 5e-4f, 1e-5f * (diag + R));
    r.R2s = Rs * Rs;
    // every pair lies within Rs of the axis segment from the entrance
    // (t = 0) to t = the grid's diagonal: its y and z extents, widened by Rs
    // and a voxel, bound the rows
    float qe[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)   // the entrance: q.d = -c_t, q.ex = -c_x, q.ey = -c_y
        qe[c] = -(d.c_t * d.d[c] + d.c_x * d.ex[c] + d.c_y * d.ey[c]);
    const float y0 = fminf(qe[1], qe[1] + diag * d.d[1]) - Rs;
    const float y1 = fmaxf(qe[1], qe[1] + diag * d.d[1]) + Rs;
    const float z0 = fminf(qe[2], qe[2] + diag * d.d[2]) - Rs;
    const float z1 = fmaxf(qe[2], qe[2] + diag * d.d[2]) + Rs;
    r.j_lo = clamp_index(floorf((y0 - P.qy0) / P.dy) - 1.0f, 0, P.ny - 1);
    r.j_hi = clamp_index(ceilf((y1 - P.qy0) / P.dy) + 1.0f, -1, P.ny - 1);
    r.k_lo = clamp_index(floorf((z0 - P.qz0) / P.dz) - 1.0f, 0, P.nz - 1);
    r.k_hi = clamp_index(ceilf((z1 - P.qz0) / P.dz) + 1.0f, -1, P.nz - 1);
    return r;
}

// Voxels [ilo, ihi] of a row whose coordinates at i = 0 are (T0, X0, Y0):
// a superset of those the pair test accepts (inside the widened cylinder,
// depth >= -kAdjTSlack, each end widened by kAdjPad voxels and 1e-6 of its
// magnitude, past the rounding of this arithmetic); false when empty.
__device__ __forceinline__ bool row_interval(const RowSolve& r, const PlanConst& P, float T0,
                                             float X0, float Y0, int& ilo, int& ihi) {
    float flo = -1.0f, fhi = (float)P.nx;
    if (r.invA == 0.0f) {
        if (fmaf(X0, X0, Y0 * Y0) > r.R2s) return false;
    } else {
        // closest approach to the axis at i = ic, half chord h
        const float ic = -fmaf(X0, r.a1, Y0 * r.a2) * r.invA;
        const float Xc = fmaf(ic, r.a1, X0), Yc = fmaf(ic, r.a2, Y0);
        const float rem = r.R2s - fmaf(Xc, Xc, Yc * Yc);
        if (rem < 0.0f) return false;
        const float h = sqrtf(rem * r.invA);
        const float pad = fmaf(1e-6f, fabsf(ic) + h, kAdjPad);
        flo = fmaxf(flo, ic - h - pad);
        fhi = fminf(fhi, ic + h + pad);
    }
    if (r.a3 != 0.0f) {
        const float b = (-kAdjTSlack - T0) / r.a3;
        const float pad = fmaf(1e-6f, fabsf(b), kAdjPad);
        if (r.a3 > 0.0f) flo = fmaxf(flo, b - pad);
        else fhi = fminf(fhi, b + pad);
    } else if (T0 < -kAdjTSlack) {
        return false;
    }
    if (!(flo <= fhi)) return false;
    ilo = clamp_index(ceilf(flo), 0, P.nx);
    ihi = clamp_index(floorf(fhi), -1, P.nx - 1);
    return ihi >= ilo;
}

// MODE kAdjGrad: g partials; kAdjCount: pair counts (ints in part).  NW waves per
// workgroup; with LW the water table is staged in LDS once per workgroup.
template <int DC, int NW, bool LW, int MODE>
__global__ __launch_bounds__(NW * kWave) __attribute__((amdgpu_waves_per_eu(6)))
void dose_adjoint(DoseArgs a, int n_beamlets, int per, int slab, int n_slabs,
                  const float* __restrict__ w, float* __restrict__ part, int* __restrict__ queue) {
    constexpr int NT = NW * kWave;
    constexpr int kWinItems = kAdjBlocks * kWave;
    // the unit's rows that meet the cylinder, compacted in row order
    __shared__ int s_off[NT];               // first item of the row
    __shared__ float4 s_row[NT];            // (i - item, v - item, rt, rx); bits of ints in x, y
    __shared__ float s_ry[NT];
    __shared__ int s_brow[kAdjBlocks];      // the row holding item w0 + 64 b
    __shared__ unsigned s_start[2 * kAdjBlocks];   // bit e: a row starts at item w0 + e
    __shared__ int s_wsum[NW];
    __shared__ int s_wcnt[NW];
    __shared__ float s_red[NW];
    __shared__ int s_q[2];
    extern __shared__ float4 s_water[];
    const int xcd = blockIdx.x & 7;
    const int b_first = xcd * per;
    const int run = min(per, n_beamlets - b_first);
    if (run <= 0) return;   // whole workgroup
    const int n_units = run * n_slabs;
    int* const q = queue + xcd * kAdjQueueInts;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    if (tid == 0) s_q[0] = atomicAdd(q, 1);
    if (LW) {
        const int n = a.P.dt_n;
        const FSPB_GLOBAL float4* __restrict__ g = as_global(a.dtab);
        for (int i = tid; i < 3 * n; i += NT) {
            const int plane = i / n, j = i - plane * n;
            s_water[3 * j + plane] = g[i];
        }
    }
    __syncthreads();
    const PlanConst& P = a.P;
    const FSPB_GLOBAL float4* __restrict__ facs = as_global(a.fac);
    const FSPB_GLOBAL float* __restrict__ wv = as_global(w);
    for (int it = 0;; ++it) {
        const int u = s_q[it & 1];
        if (u >= n_units) break;   // whole workgroup
        if (tid == 0) s_q[(it + 1) & 1] = atomicAdd(q, 1);   // the next unit, early
        const int s = u / run, b = b_first + (u - s * run);
        // the beamlet's descriptor in scalar registers (read once per unit)
        const BeamletDesc d = as_const(a.bl)[b];
        float acc = 0.0f;
        int cnt = 0;
        if (d.hit) {
            const RowSolve r = row_solve(d, P);
            const int k_lo = max(r.k_lo, s * slab), k_hi = min(r.k_hi, s * slab + slab - 1);
            const int nj = r.j_hi - r.j_lo + 1;
            const int n_rows = (nj > 0 && k_hi >= k_lo) ? nj * (k_hi - k_lo + 1) : 0;
            for (int r0 = 0; r0 < n_rows; r0 += NT) {
                const int rr = r0 + tid;
                int lo = 0, len = 0, vrow = 0;
                float rt = 0.0f, rx = 0.0f, ry = 0.0f;
                if (rr < n_rows) {
                    const int j = r.j_lo + rr % nj, k = k_lo + rr / nj;
                    float qx, qy, qz;
                    voxel_q(P, 0, j, k, qx, qy, qz);
                    // the row's share of the pair coordinates: the voxel's
                    // are fma(qx, d[0], rt) etc., as pair_coords computes them
                    rt = fmaf(qy, d.d[1], fmaf(qz, d.d[2], d.c_t));
                    rx = fmaf(qy, d.ex[1], fmaf(qz, d.ex[2], d.c_x));
                    ry = fmaf(qy, d.ey[1], fmaf(qz, d.ey[2], d.c_y));
                    int ilo, ihi;
                    if (row_interval(r, P, fmaf(qx, d.d[0], rt), fmaf(qx, d.ex[0], rx),
                                     fmaf(qx, d.ey[0], ry), ilo, ihi)) {
                        lo = ilo;
                        len = ihi - ilo + 1;
                    }
                    vrow = (k * P.ny + j) * P.nx;
                }
                // block scans: the rows' first items and their compacted slots
                const int incl = lane_incl_scan_int(len, opaque_lane(lane));
                const unsigned long long ne = __ballot(len > 0);
                const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(ne >> 32),
                                                           __builtin_amdgcn_mbcnt_lo((unsigned)ne, 0));
                if (lane == kWave - 1) s_wsum[wid] = incl;
                if (lane == 0) s_wcnt[wid] = __popcll(ne);
                __syncthreads();
                int base = 0, total = 0, rbase = 0, nrows = 0;
                for (int w2 = 0; w2 < NW; ++w2) {
                    if (w2 < wid) {
                        base += s_wsum[w2];
                        rbase += s_wcnt[w2];
                    }
                    total += s_wsum[w2];
                    nrows += s_wcnt[w2];
                }
                if (len > 0) {
                    const int c = rbase + rank, off = base + incl - len;
                    s_off[c] = off;
                    s_row[c] = make_float4(__int_as_float(lo - off), __int_as_float(vrow + lo - off),
                                           rt, rx);
                    s_ry[c] = ry;
                }
                for (int w0 = 0; w0 < total; w0 += kWinItems) {
                    __syncthreads();   // the compacted rows are written; the last window is read
                    for (int e = tid; e < 2 * kAdjBlocks; e += NT) s_start[e] = 0u;
                    for (int bk = tid; bk < kAdjBlocks; bk += NT)
                        if (w0 + bk * kWave >= total) s_brow[bk] = nrows - 1;
                    __syncthreads();
                    // row c holds items [s_off[c], s_off[c + 1])
                    for (int c = tid; c < nrows; c += NT) {
                        const int x0 = s_off[c] - w0;
                        const int x1 = (c + 1 < nrows ? s_off[c + 1] : total) - w0;   // exclusive
                        if (x0 >= 0 && x0 < kWinItems) atomicOr(&s_start[x0 >> 5], 1u << (x0 & 31));
                        int bk = x0 > 0 ? (x0 + kWave - 1) / kWave : 0;
                        for (; bk < kAdjBlocks && bk * kWave < x1; ++bk) s_brow[bk] = c;
                    }
                    __syncthreads();
                    const int wend = min(total - w0, kWinItems);
                    for (int e0 = wid * kWave; e0 < wend; e0 += NT) {
                        // the row of the block's first item, plus the rows
                        // starting at block positions 1..lane
                        const int blk = e0 / kWave;
                        const unsigned m0 = uniform((int)s_start[2 * blk]);
                        const unsigned m1 = uniform((int)s_start[2 * blk + 1]);
                        const int c = s_brow[blk] +
                                      (int)__builtin_amdgcn_mbcnt_hi(m1 >> 1,
                                                                     __builtin_amdgcn_mbcnt_lo((m0 >> 1) | (m1 << 31), 0));
                        const int e = w0 + e0 + lane;
                        if (e >= total) continue;
                        const float4 rc = s_row[c];
                        const int i = e + __float_as_int(rc.x);
                        const float qx = fmaf((float)i, P.dx, P.qx0);
                        const float t = fmaf(qx, d.d[0], rc.z);
                        const float xp = fmaf(qx, d.ex[0], rc.w);
                        const float yp = fmaf(qx, d.ey[0], s_ry[c]);
                        if ((t >= 0.0f) & (fmaf(xp, xp, yp * yp) <= P.R2)) {
                            if (MODE == kAdjCount) {
                                ++cnt;
                                continue;
                            }
                            const unsigned v = (unsigned)(e + __float_as_int(rc.y));
                            float4 fac = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
                            if (DC) fac = facs[v];
                            const float wx = wv[v];
                            const float kmag = magnification(t, d);
                            const float pd =
                                LW ? pair_dose<DC>(t, xp, yp, kmag, d, fac, P,
                                                   WaterLds{(const FSPB_LDS float4*)s_water},
                                                   as_global(a.atab), as_global(a.tT),
                                                   as_global(a.tTW), as_global(a.tW2))
                                   : pair_dose<DC>(t, xp, yp, kmag, d, fac, P,
                                                   WaterGlobal{as_global(a.dtab), P.dt_n},
                                                   as_global(a.atab), as_global(a.tT),
                                                   as_global(a.tTW), as_global(a.tW2));
                            acc = fmaf(wx, pd, acc);
                        }
                    }
                }
                __syncthreads();
            }
        }
        // the unit's sum: waves, then a fixed pairwise tree over them
        if (MODE == kAdjCount) acc = __int_as_float(lane_xor_sum_bits(cnt, opaque_lane(lane), false));
        else acc = __int_as_float(lane_xor_sum_bits(__float_as_int(acc), opaque_lane(lane), true));
        if (lane == 0) s_red[wid] = acc;
        __syncthreads();
        if (tid == 0) {
            if (MODE == kAdjCount) {
                int sum = 0;
#pragma unroll
                for (int w2 = 0; w2 < NW; ++w2) sum += __float_as_int(s_red[w2]);
                reinterpret_cast<int*>(part)[(long)s * n_beamlets + b] = sum;
            } else {
                float sum[NW];
#pragma unroll
                for (int w2 = 0; w2 < NW; ++w2) sum[w2] = s_red[w2];
#pragma unroll
                for (int h = NW / 2; h > 0; h >>= 1)
#pragma unroll
                    for (int w2 = 0; w2 < h; ++w2) sum[w2] = sum[w2] + sum[w2 + h];
                part[(long)s * n_beamlets + b] = sum[0];
            }
        }
        __syncthreads();   // s_red and s_q[it & 1] are read; s_q[(it + 1) & 1] is written
    }
}

// g_b (or the pair count of b): the units' sums in slab order.
template <class T>
__global__ void adj_sum_slabs(const T* __restrict__ part, int n_slabs, int n, T* __restrict__ out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    T acc = 0;
    for (int s = 0; s < n_slabs; ++s) acc += part[(long)s * n + b];
    out[b] = acc;
}

__global__ void fill_i32(int* __restrict__ p, int n, int v) {
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) p[q] = v;
}


void launch_adjoint(const DoseArgs& a, bool dc, int n_beamlets, const float* w, float* grad,
                    float* part, int* queue, int slab, int n_cu, hipStream_t s) {
    // with the water table in LDS, 8-wave workgroups; else 4-wave workgroups
    // reading it from global memory
    const size_t water_bytes = sizeof(float4) * 3 * (size_t)a.P.dt_n;
    const bool lw = water_bytes <= (size_t)kLdsWaterMax;
    const int n_slabs = adjoint_slabs(a.P, slab);
    const int per = (n_beamlets + 7) / 8;
    hipLaunchKernelGGL(fill_i32, dim3(1), dim3(128), 0, s, queue, 8 * kAdjQueueInts, 0);
#define FSPB_ADJ(DCV, NWV, LWV)                                                               \
    do {                                                                                      \
        auto k = dose_adjoint<DCV, NWV, LWV, kAdjGrad>;                                          \
        const size_t lds = LWV ? water_bytes : 0;                                             \
        hipLaunchKernelGGL(k, dim3(persistent_grid(k, NWV * kWave, lds, n_cu)),                \
                           dim3(NWV * kWave), lds, s, a, n_beamlets, per, slab, n_slabs, w,    \
                           part, queue);                                                      \
    } while (0)
    const int mode = !dc ? kPlain : a.P.w2_one ? kDcOneDrift : kDcTwoDrift;
    if (lw && mode == kDcOneDrift)
        FSPB_ADJ(kDcOneDrift, 8, true);
    else if (lw && mode == kDcTwoDrift)
        FSPB_ADJ(kDcTwoDrift, 8, true);
    else if (lw)
        FSPB_ADJ(kPlain, 8, true);
    else if (mode == kDcOneDrift)
        FSPB_ADJ(kDcOneDrift, 4, false);
    else if (mode == kDcTwoDrift)
        FSPB_ADJ(kDcTwoDrift, 4, false);
    else
        FSPB_ADJ(kPlain, 4, false);
#undef FSPB_ADJ
    hipLaunchKernelGGL(adj_sum_slabs<float>, dim3((n_beamlets + 255) / 256), dim3(256), 0, s,
                       (const float*)part, n_slabs, n_beamlets, grad);
}

void launch_adjoint_count(const DoseArgs& a, int n_beamlets, int* counts, float* part,
                          int* queue, int slab, int n_cu, hipStream_t s) {
    const int n_slabs = adjoint_slabs(a.P, slab);
    const int per = (n_beamlets + 7) / 8;
    hipLaunchKernelGGL(fill_i32, dim3(1), dim3(128), 0, s, queue, 8 * kAdjQueueInts, 0);
    auto k = dose_adjoint<kPlain, 8, false, kAdjCount>;
    hipLaunchKernelGGL(k, dim3(persistent_grid(k, 8 * kWave, 0, n_cu)), dim3(8 * kWave), 0, s, a,
                       n_beamlets, per, slab, n_slabs, nullptr, part, queue);
    hipLaunchKernelGGL(adj_sum_slabs<int>, dim3((n_beamlets + 255) / 256), dim3(256), 0, s,
                       (const int*)part, n_slabs, n_beamlets, counts);
}

}  // namespace fspb
