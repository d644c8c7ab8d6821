// dose.hip -- the dose superposition (Eq. 1 over Eqs. 2-4; Algorithm A2
// kernel 5) and the evaluated-pair count, for gfx950.
//
// Forward: voxel-major.  A wavefront owns a 64-voxel brick (4x4x4 by default,
// one voxel per lane); with 8-wave workgroups the commissioned water table is
// first staged in LDS.  For each beam it bounds the projection of the box of
// its voxel centres onto the isocentre plane by a rectangle of beamlets whose
// 5 cm ROI cylinder can reach the brick.  The rectangle is filtered 64
// beamlets at a time (one per lane) against the brick's bounding sphere and
// the survivors are compacted; the wave then walks them with wave-uniform
// beamlet descriptors (scalar loads), each lane testing its own voxel exactly
// and evaluating the pair in FP32 (with one of two exact forms of the Eq. 4
// profile product, chosen per wave; see pair.h).  Each voxel is written once:
// no atomics, and the result does not depend on scheduling.
// (The transpose is in adjoint.hip.)
#include "kernels.h"
#include "pair.h"
#include "persistent.h"
#include "wave.h"

#include <stdint.h>

#include <algorithm>

namespace fspb {

// ---------------------------------------------------------------------------
// Forward pass over one brick, three modes sharing the candidate search:
//   kDose   D(r) = sum_i f_i D_i(r) over beamlets with f_i != 0
//   kCount  number of evaluated pairs per voxel
//   kCountBrick  the same summed over the brick's voxels: one value per brick
//   kSurr   the dose with the learned surrogate's parameters: per (voxel,
//           beam) row prm[2 (b n_vox + v) + 0..1] = ((u1x, u1y, u2x, u2y)
//           log2 e, (w1, w2, fallback, 0)); a row whose fallback flag is set
//           takes the density-corrected pair instead
// A brick is BX x BY x BZ = 64 voxels, one per lane.
//   kSid    the dose with the exact (Siddon) depth tables
enum { kDose = 0, kCount = 1, kCountBrick = 2, kSurr = 3, kSid = 4 };

template <int BX, int BY, int BZ>
__device__ __forceinline__ int bricks_x(const PlanConst& P) { return (P.nx + BX - 1) / BX; }
template <int BX, int BY, int BZ>
__device__ __forceinline__ int bricks_y(const PlanConst& P) { return (P.ny + BY - 1) / BY; }
template <int BX, int BY, int BZ>
__device__ __forceinline__ int bricks_total(const PlanConst& P) {
    return bricks_x<BX, BY, BZ>(P) * bricks_y<BX, BY, BZ>(P) * ((P.nz + BZ - 1) / BZ);
}

template <int DC, int MODE, int BX, int BY, int BZ, bool PIPE = false, class WT>
__device__ __forceinline__ void brick_pass(const DoseArgs& a, const int brick,
                                           const float* fluence_, float* dose_, int* out_int_,
                                           const WT& water, const float4* prm_ = nullptr,
                                           int b_lo = 0, int b_hi = -1) {
    static_assert(MODE != kSurr || DC, "the surrogate replaces the density-corrected parameters");
    static_assert(BX * BY * BZ == kWave, "a brick holds one voxel per lane");
    // The table offsets are held in vector registers: an FMA may read only one
    // scalar operand, and t * inv + off with both scalars would cost a move
    // per pair.
    PlanConst P = a.P;
    asm volatile("" : "+v"(P.dt_off), "+v"(P.at_off));
    const FSPB_CONST BeamDesc* __restrict__ beams = as_const(a.beams);
    const FSPB_CONST BeamletDesc* __restrict__ bl = as_const(a.bl);
    const FSPB_GLOBAL float4* __restrict__ bl4 = as_global(reinterpret_cast<const float4*>(a.bl));
    const FSPB_GLOBAL float4* __restrict__ facs = as_global(a.fac);
    const FSPB_GLOBAL float4* __restrict__ atab = as_global(a.atab);
    const FSPB_GLOBAL float2* __restrict__ tT = as_global(a.tT);
    const FSPB_GLOBAL float4* __restrict__ tTW = as_global(a.tTW);
    const FSPB_GLOBAL float2* __restrict__ tW2 = as_global(a.tW2);
    const FSPB_GLOBAL float4* __restrict__ sid = as_global(a.sid);
    const FSPB_GLOBAL float* __restrict__ fluence = as_global(fluence_);
    FSPB_GLOBAL float* __restrict__ dose = as_global_rw(dose_);
    FSPB_GLOBAL int* __restrict__ out_int = as_global_rw(out_int_);
    const int lane = threadIdx.x & (kWave - 1);
    const int nbx = bricks_x<BX, BY, BZ>(P), nby = bricks_y<BX, BY, BZ>(P);
    const int bx = brick % nbx;
    const int by = (brick / nbx) % nby;
    const int bz = brick / (nbx * nby);
    const int i = bx * BX + (lane % BX), j = by * BY + ((lane / BX) % BY),
              k = bz * BZ + lane / (BX * BY);
    const bool valid = (i < P.nx) && (j < P.ny) && (k < P.nz);
    const long v = ((long)k * P.ny + j) * P.nx + i;
    float qx, qy, qz;
    voxel_q(P, i, j, k, qx, qy, qz);
    float4 fac = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
    if (DC && (MODE == kDose || MODE == kSurr || MODE == kSid) && valid) fac = facs[v];
    // bounding sphere of the brick's voxel centres
    float cqx, cqy, cqz;
    voxel_q(P, bx * BX, by * BY, bz * BZ, cqx, cqy, cqz);
    const float hx = 0.5f * (BX - 1) * P.dx, hy = 0.5f * (BY - 1) * P.dy, hz = 0.5f * (BZ - 1) * P.dz;
    cqx += hx;
    cqy += hy;
    cqz += hz;
    const float rb = sqrtf(hx * hx + hy * hy + hz * hz) * 1.0001f + 1e-3f;
    const float Rc = sqrtf(P.R2) + rb;
    const float Rc2 = Rc * Rc;

    float acc = 0.0f;
    int cnt = 0;
    const FSPB_GLOBAL float4* __restrict__ prm = as_global(prm_);
    const long n_vox = (long)P.nx * P.ny * P.nz;
    if (b_hi < 0) b_hi = P.n_beams;
    for (int b = b_lo; b < b_hi; ++b) {
        const FSPB_CONST BeamDesc& B = beams[b];
        // Rectangle of beamlets whose ROI can reach the brick, from the box of
        // its voxel centres.  In the beam's frame (offsets X, Y along ex, ey
        // and Z along the central axis, measured from the source) the box
        // spans centre +- (hX, hY, hZ), and a point projects onto the
        // isocentre plane at SAD (X, Y) / Z.  While Z > 0 over the box, X / Z
        // is largest at the largest X together with the smallest Z if that X
        // is >= 0 (else the largest Z), and smallest likewise: the bounds
        // hold for every voxel, with no reduction across the wave.  A voxel
        // inside beamlet (n,m)'s ROI lies within R / cos(theta) of its axis
        // in the plane normal to the central axis: scaled to the isocentre
        // plane, at most pad_scale / Z.  A box that reaches Z <= 0 (a source
        // next to the grid) takes the whole field.
        const float vx = cqx - B.src[0], vy = cqy - B.src[1], vz = cqz - B.src[2];
        const float Zc = fmaf(vx, B.cax[0], fmaf(vy, B.cax[1], vz * B.cax[2]));
        const float Xc = fmaf(vx, B.ex[0], fmaf(vy, B.ex[1], vz * B.ex[2]));
        const float Yc = fmaf(vx, B.ey[0], fmaf(vy, B.ey[1], vz * B.ey[2]));
        const float hZ = fmaf(hx, fabsf(B.cax[0]), fmaf(hy, fabsf(B.cax[1]), hz * fabsf(B.cax[2])));
        const float hX = fmaf(hx, fabsf(B.ex[0]), fmaf(hy, fabsf(B.ex[1]), hz * fabsf(B.ex[2])));
        const float hY = fmaf(hx, fabsf(B.ey[0]), fmaf(hy, fabsf(B.ey[1]), hz * fabsf(B.ey[2])));
        const float zlo = Zc - hZ;
        int m_lo = 0, m_hi = B.nbx - 1, n_lo = 0, n_hi = B.nby - 1;
        if (zlo > 0.0f) {
            const float rlo = fast_rcp(zlo), rhi = fast_rcp(Zc + hZ);
            const float slo = B.sad * rlo, shi = B.sad * rhi;
            const float X1 = Xc + hX, X0 = Xc - hX, Y1 = Yc + hY, Y0 = Yc - hY;
            const float amax = X1 * (X1 >= 0.0f ? slo : shi), amin = X0 * (X0 <= 0.0f ? slo : shi);
            const float bmax = Y1 * (Y1 >= 0.0f ? slo : shi), bmin = Y0 * (Y0 <= 0.0f ? slo : shi);
            const float pad = fmaf(B.pad_scale * rlo, 1.0001f, 1e-3f);
            const float iwx = fast_rcp(B.wx), iwy = fast_rcp(B.wy);
            const float fm0 = fmaxf((amin - pad - B.a0) * iwx, -1.0f);
            const float fm1 = fminf((amax + pad - B.a0) * iwx, (float)B.nbx);
            const float fn0 = fmaxf((bmin - pad - B.b0) * iwy, -1.0f);
            const float fn1 = fminf((bmax + pad - B.b0) * iwy, (float)B.nby);
            m_lo = max((int)ceilf(fm0), 0);
            m_hi = min((int)floorf(fm1), B.nbx - 1);
            n_lo = max((int)ceilf(fn0), 0);
            n_hi = min((int)floorf(fn1), B.nby - 1);
        }
        m_lo = uniform(m_lo);
        m_hi = uniform(m_hi);
        n_lo = uniform(n_lo);
        n_hi = uniform(n_hi);
        const int first = uniform(B.first), nbl_x = uniform(B.nbx);
        const int nm = m_hi - m_lo + 1;
        const int total = (nm > 0 && n_hi >= n_lo) ? nm * (n_hi - n_lo + 1) : 0;
        // surrogate row of this voxel and beam, read only when some beamlet
        // of the beam can reach the brick
        float4 s_ul = make_float4(0.0f, 0.0f, 0.0f, 0.0f), s_w = s_ul;
        bool own = false;
        if (MODE == kSurr && valid && total > 0) {
            s_ul = prm[2 * ((long)b * n_vox + v)];
            s_w = prm[2 * ((long)b * n_vox + v) + 1];
            own = s_w.z == 0.0f;
        }
        float accb = 0.0f;
        for (int base = 0; base < total; base += kWave) {
            // 64 candidates at once: one per lane, tested against the brick's
            // bounding sphere with the beamlet's true axis
            const int c = base + lane;
            bool pass = false;
            int ib = 0;
            float fi = 1.0f;
            if (c < total) {
                ib = first + (n_lo + c / nm) * nbl_x + (m_lo + c % nm);
                if (MODE == kDose || fluence_) fi = fluence[ib];
                if (fi != 0.0f) {
                    const FSPB_GLOBAL float4* dp = bl4 + (sizeof(BeamletDesc) / 16) * ib;
                    const float4 r0 = dp[0], r1 = dp[1], r2 = dp[2];
                    float tc = fmaf(cqx, r0.x, fmaf(cqy, r0.y, fmaf(cqz, r0.z, r0.w)));
                    float xc = fmaf(cqx, r1.x, fmaf(cqy, r1.y, fmaf(cqz, r1.z, r1.w)));
                    float yc = fmaf(cqx, r2.x, fmaf(cqy, r2.y, fmaf(cqz, r2.z, r2.w)));
                    pass = (tc >= -rb) && (fmaf(xc, xc, yc * yc) <= Rc2);
                }
            }
            const unsigned long long mask = __ballot(pass);
            const int ncand = __popcll(mask);
            if (ncand == 0) continue;
            // compact: the r-th passing candidate moves to lane r
            const int rank = __builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0));
            const int dst = pass ? rank : ncand + (lane - rank);
            const int pk_ib = __builtin_amdgcn_ds_permute(dst << 2, ib);
            const int pk_f = __builtin_amdgcn_ds_permute(dst << 2, __float_as_int(fi));
            if constexpr (PIPE && (MODE == kDose || MODE == kSurr) && DC != kDcTwoDrift) {
                // Software pipeline over the candidates (PIPE).  A pair's depth
                // record (t_eq and W1 at its sample, from a table larger than
                // an XCD's L2) and the A record indexed by that t_eq are two
                // dependent loads; waiting on both in turn per candidate left
                // the SIMDs idle.  So the depth record of candidate e+1 is
                // read while candidate e is evaluated: its depth comes from
                // its descriptor, fetched (scalar loads) two candidates
                // ahead, and the record is read on every lane before the pair
                // test, at an index kept inside the beamlet's rows
                // (depth_record).  It is issued after candidate e's A load,
                // so that the wait for the A record (loads complete in
                // order) does not wait for it too.  The arithmetic is
                // pair_dose's (pair_dose_given's for the surrogate's own
                // rows), so the dose is bitwise the same.  The brick-major
                // and batch kernels with the water table in LDS take it.  With the water table in global memory its three
                // loads follow the prefetch and so wait for it; the per-beam
                // kernels, whose items each walk a short candidate list,
                // measured slower with it; both keep the loop below.
                BeamletDesc dA = bl[__builtin_amdgcn_readlane(pk_ib, 0)];
                BeamletDesc dB = bl[__builtin_amdgcn_readlane(pk_ib, min(1, ncand - 1))];
                float t_cur = pair_depth(dA, qx, qy, qz);
                float4 rec = depth_record<DC>(t_cur, dA, P, tT, tTW);
                for (int e = 0; e < ncand; ++e) {
                    const BeamletDesc d = dA;
                    const float fe = __int_as_float(__builtin_amdgcn_readlane(pk_f, e));
                    float xp, yp;
                    const bool act = pair_test_given_depth(d, P, qx, qy, qz, t_cur, xp, yp) & valid;
                    // the record is consumed on every lane, so that no load into
                    // its registers is pending when the next one is issued
                    float f, teq, W1, fa, kmag, cd;
                    float4 ae;
                    pair_depth_lerp<DC>(t_cur, rec, P, f, teq);
                    if (act) pair_first_half<DC>(t_cur, rec, f, teq, d, P, atab, W1, fa, ae, kmag, cd);
                    t_cur = pair_depth(dB, qx, qy, qz);
                    rec = depth_record<DC>(t_cur, dB, P, tT, tTW);
                    dA = dB;
                    dB = bl[__builtin_amdgcn_readlane(pk_ib, min(e + 2, ncand - 1))];
                    // the surrogate's rows: the network's parameters where the
                    // row is its own, else the corrected pair (as below)
                    if (MODE == kSurr && (act & own))
                        accb = fmaf(fe, pair_given_from_A(xp, yp, kmag, d, s_ul, s_w, fa, ae), accb);
                    else if (act)
                        accb = fmaf(fe, pair_second_half<DC>(xp, yp, kmag, cd, d, fac, P, water, W1, fa, ae),
                                    accb);
                }
                continue;
            }
            // software pipeline: the next candidate's descriptor is fetched
            // (scalar loads) while the current one is evaluated; the fluences
            // travel in a vector register (a scalar load per candidate would
            // add to the descriptor stream through the shared scalar cache)
            BeamletDesc dn = bl[__builtin_amdgcn_readlane(pk_ib, 0)];
            for (int e = 0; e < ncand; ++e) {
                const BeamletDesc d = dn;
                const float fe = __int_as_float(__builtin_amdgcn_readlane(pk_f, e));
                dn = bl[__builtin_amdgcn_readlane(pk_ib, min(e + 1, ncand - 1))];
                float t, xp, yp;
                // evaluated on every lane (no short circuit) so that the whole
                // descriptor is fetched in one scalar batch before the branch
                const bool act = pair_coords(d, P, qx, qy, qz, t, xp, yp) & valid;
                if (MODE == kCount || MODE == kCountBrick) {
                    cnt += act ? 1 : 0;
                    continue;
                }
                const float kmag = magnification(t, d);
                // a candidate with no active lane skips the block (empty exec mask)
                if (MODE == kSurr) {
                    if (act & own)
                        accb = fmaf(fe, pair_dose_given(t, xp, yp, kmag, d, s_ul, s_w, P, atab, tTW),
                                    accb);
                    else if (act)
                        accb = fmaf(fe, pair_dose<DC>(t, xp, yp, kmag, d, fac, P, water, atab, tT, tTW, tW2),
                                    accb);
                } else if (MODE == kSid) {
                    if (act)
                        accb = fmaf(fe, pair_dose_siddon<DC>(t, xp, yp, kmag, d, fac, P, water, atab, sid),
                                    accb);
                } else if (act) {
                    accb = fmaf(fe, pair_dose<DC>(t, xp, yp, kmag, d, fac, P, water, atab, tT, tTW, tW2),
                                accb);
                }
            }
        }
        acc += accb;
    }
    if (MODE == kCountBrick) {
        // lanes outside the grid counted nothing; lane 0 (the brick's corner
        // voxel) is always inside it
        for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, kWave);
        if (lane == 0) out_int[brick] = cnt;
    } else if (valid) {
        if (MODE == kCount)
            out_int[v] = cnt;
        else
            dose[v] = acc;
    }
}

// One plan: wave w of the grid takes the brick in slot w of `order` (bricks in
// decreasing order of estimated work, so expensive bricks start early and
// cheap ones fill the tail; consecutive workgroups are dealt round-robin to
// the 8 XCDs).  With LW the workgroup (kLdsWaves waves) first copies the
// water table into LDS as 48-byte records: the pairs then read it there and
// the vector-memory data path carries only the per-beamlet and A lookups
// (with 8 waves per workgroup four workgroups, a full CU, fit in LDS for
// tables up to 853 samples).

template <int DC, int MODE, int BX, int BY, int BZ, bool LW>
__global__ __launch_bounds__(LW ? kLdsWaves * kWave : 256, LW ? 8 : 1) void dose_forward(
    DoseArgs a, const int* __restrict__ order, const float* __restrict__ fluence,
    float* __restrict__ dose, int* __restrict__ out_int, const float4* __restrict__ prm) {
    extern __shared__ float4 s_water[];
    if (LW) {
        const int n = a.P.dt_n;
        const FSPB_GLOBAL float4* __restrict__ g = as_global(a.dtab);
        for (int q = threadIdx.x; q < 3 * n; q += blockDim.x) {
            const int plane = q / n, j = q - plane * n;
            s_water[3 * j + plane] = g[q];
        }
        __syncthreads();
    }
    const int slot = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (slot >= bricks_total<BX, BY, BZ>(a.P)) return;
    const int brick = order ? order[slot] : slot;
    if (LW)
        brick_pass<DC, MODE, BX, BY, BZ, true>(a, brick, fluence, dose, out_int,
                                               WaterLds{(const FSPB_LDS float4*)s_water}, prm);
    else
        brick_pass<DC, MODE, BX, BY, BZ>(a, brick, fluence, dose, out_int,
                                         WaterGlobal{as_global(a.dtab), a.P.dt_n}, prm);
}

// The per-beam schedule (see kernels.h).  XCD x (workgroups q with
// q mod 8 = x) runs the concatenation of its segments x, x + 8, x + 16, ...
// of the sorted items; wave w of its m-th workgroup takes positions
// (m wpb + w) ipw .. + ipw - 1 of that concatenation (consecutive items: the
// same beam, neighbouring slabs).  For each, the item's beam alone is
// evaluated for its brick and written to that beam's plane.  The water
// table is read from global memory (1, 2 or 4 waves per workgroup).
template <int DC, int BX, int BY, int BZ>
__global__ __launch_bounds__(256) void dose_forward_split(
    DoseArgs a, const int* __restrict__ order, const int* __restrict__ chunk, int ipw,
    const float* __restrict__ fluence, float* __restrict__ planes, long stride) {
    const int wpb = blockDim.x / kWave;
    const int x = blockIdx.x & 7, m = blockIdx.x >> 3;
    int total = 0;
    for (int k = 0; k < kSplitSegments; ++k) total += chunk[x + 8 * k + 1] - chunk[x + 8 * k];
    if (m * wpb * ipw >= total) return;
    const int nb = bricks_total<BX, BY, BZ>(a.P);
    const int v0 = (m * wpb + (int)(threadIdx.x / kWave)) * ipw;
    const int v1 = min(v0 + ipw, total);
    for (int v = v0; v < v1; ++v) {
        // position v of the concatenation -> position in order[]
        int j = v, pos = 0;
        for (int k = 0; k < kSplitSegments; ++k) {
            const int s0 = chunk[x + 8 * k], len = chunk[x + 8 * k + 1] - s0;
            if (j < len) {
                pos = s0 + j;
                break;
            }
            j -= len;
        }
        const int item = uniform(order[pos]);
        const int b = item / nb, brick = item - b * nb;
        brick_pass<DC, kDose, BX, BY, BZ>(a, brick, fluence, planes + (long)b * stride, nullptr,
                                          WaterGlobal{as_global(a.dtab), a.P.dt_n}, nullptr, b,
                                          b + 1);
    }
}

// The per-beam schedule with the water table in LDS: persistent workgroups
// of kLdsWaves waves stage the table once.  Each wave then takes positions of
// its XCD's concatenation of segments from the XCD's counter (zeroed before
// the launch), one item at a time, asking for the next position while the
// current item runs, until the XCD's run is done.  A wave's items are those
// of the static schedule, in the same order along the list, and each is
// evaluated by the same brick pass, so the planes are bitwise the same.
template <int DC, int BX, int BY, int BZ>
__global__ __launch_bounds__(kLdsWaves * kWave) __attribute__((amdgpu_waves_per_eu(6))) void dose_forward_split_q(
    DoseArgs a, const int* __restrict__ order, const int* __restrict__ chunk,
    const float* __restrict__ fluence, float* __restrict__ planes, long stride,
    int* __restrict__ queue) {
    extern __shared__ float4 s_water[];
    const int x = blockIdx.x & 7;
    int total = 0;
    for (int k = 0; k < kSplitSegments; ++k) total += chunk[x + 8 * k + 1] - chunk[x + 8 * k];
    if (total == 0) return;   // the whole workgroup: nothing to stage
    {
        const int n = a.P.dt_n;
        const FSPB_GLOBAL float4* __restrict__ g = as_global(a.dtab);
        for (int q = threadIdx.x; q < 3 * n; q += blockDim.x) {
            const int plane = q / n, j = q - plane * n;
            s_water[3 * j + plane] = g[q];
        }
        __syncthreads();
    }
    const int nb = bricks_total<BX, BY, BZ>(a.P);
    const int lane = threadIdx.x & (kWave - 1);
    int* const q = queue + x * kSplitQueueInts;
    int got = 0;
    if (lane == 0) got = atomicAdd(q, 1);
    int v = __builtin_amdgcn_readlane(got, 0);
    while (v < total) {
        if (lane == 0) got = atomicAdd(q, 1);   // the next position, early
        int j = v, pos = 0;
        for (int k = 0; k < kSplitSegments; ++k) {
            const int s0 = chunk[x + 8 * k], len = chunk[x + 8 * k + 1] - s0;
            if (j < len) {
                pos = s0 + j;
                break;
            }
            j -= len;
        }
        const int item = uniform(order[pos]);
        const int b = item / nb, brick = item - b * nb;
        brick_pass<DC, kDose, BX, BY, BZ>(a, brick, fluence, planes + (long)b * stride, nullptr,
                                          WaterLds{(const FSPB_LDS float4*)s_water}, nullptr, b,
                                          b + 1);
        v = __builtin_amdgcn_readlane(got, 0);
    }
}

__global__ void zero_queue(int* __restrict__ p, int n) {
    for (int q = threadIdx.x; q < n; q += blockDim.x) p[q] = 0;
}

// dose[v] = sum over beams of planes[b][v] (plane b at planes + b stride,
// stride a multiple of 4), added in beam order from 0.  Four voxels a thread
// when dose is 16-byte aligned (the caller's buffer need not be).
__global__ __launch_bounds__(256) void sum_planes(const float* __restrict__ planes, int n_beams,
                                                  long n_vox, long stride, float* __restrict__ dose) {
    const long t0 = (long)blockIdx.x * blockDim.x + threadIdx.x, step = (long)gridDim.x * blockDim.x;
    const bool vec = (reinterpret_cast<uintptr_t>(dose) & 15) == 0;
    const long n4 = vec ? n_vox / 4 : 0;
    const float4* __restrict__ p4 = reinterpret_cast<const float4*>(planes);
    float4* __restrict__ d4 = reinterpret_cast<float4*>(dose);
    for (long q = t0; q < n4; q += step) {
        float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        for (int b = 0; b < n_beams; ++b) {
            const float4 v = p4[(long)b * (stride / 4) + q];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
        d4[q] = acc;
    }
    for (long q = 4 * n4 + t0; q < n_vox; q += step) {
        float acc = 0.0f;
        for (int b = 0; b < n_beams; ++b) acc += planes[(long)b * stride + q];
        dose[q] = acc;
    }
}

// Many plans in one persistent launch: wave q walks its own static list of
// (plan, brick) items, built on the host by longest-processing-time-first
// assignment.  ts_done[plan * n_waves + q] receives the wall clock after the
// wave's last item of that plan; ts_start[q] the wave's start.  No atomics.
// With LW every plan uses the same water table (water, n samples), which
// the workgroup stages in LDS as dose_forward does.
template <int DC, int BX, int BY, int BZ, bool LW>
__global__ __launch_bounds__(LW ? kLdsWaves * kWave : 256, LW ? 8 : 1) void dose_forward_batch(
    const DoseArgs* __restrict__ plans, const int2* __restrict__ items,
    const int* __restrict__ wave_begin, int n_waves, BatchPtrs ptrs,
    unsigned long long* __restrict__ ts_done, unsigned long long* __restrict__ ts_start,
    const float4* __restrict__ water, int water_n) {
    extern __shared__ float4 s_water[];
    if (LW) {
        const FSPB_GLOBAL float4* __restrict__ g = as_global(water);
        for (int r = threadIdx.x; r < 3 * water_n; r += blockDim.x) {
            const int plane = r / water_n, j = r - plane * water_n;
            s_water[3 * j + plane] = g[r];
        }
        __syncthreads();
    }
    const int q = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (q >= n_waves) return;
    const int lane = threadIdx.x & (kWave - 1);
    if (ts_start && lane == 0) ts_start[q] = wall_clock64();
    const int it0 = uniform(wave_begin[q]), it1 = uniform(wave_begin[q + 1]);
    for (int it = it0; it < it1; ++it) {
        const int p = uniform(items[it].x), brick = uniform(items[it].y);
        if (LW)
            brick_pass<DC, kDose, BX, BY, BZ, true>(plans[p], brick, ptrs.fluence[p], ptrs.dose[p],
                                                    nullptr, WaterLds{(const FSPB_LDS float4*)s_water});
        else
            brick_pass<DC, kDose, BX, BY, BZ>(plans[p], brick, ptrs.fluence[p], ptrs.dose[p],
                                              nullptr,
                                              WaterGlobal{as_global(plans[p].dtab), plans[p].P.dt_n});
        if (ts_done && lane == 0) ts_done[(long)p * n_waves + q] = wall_clock64();
    }
}

__global__ void fill_u64(unsigned long long* __restrict__ p, long n, unsigned long long v) {
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x)
        p[q] = v;
}


// ---------------------------------------------------------------------------
// Brick schedule: bricks in decreasing order of estimated work (candidate
// beamlets), by a counting sort in one workgroup.  Bricks of equal cost may
// come out in any order: each voxel's sum does not depend on the schedule.
constexpr int kOrderBins = 4096;

__global__ __launch_bounds__(1024) void order_bricks(const int* __restrict__ cost, int n,
                                                     int* __restrict__ order) {
    __shared__ int hist[kOrderBins];
    __shared__ int s_wsum[16];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    for (int b = tid; b < kOrderBins; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    // bin 0 holds the most expensive bricks; costs are read eight at a time
    // so that their loads overlap (a single workgroup does all the work)
    auto bin = [&](int q) { return kOrderBins - 1 - min(max(cost[q], 0), kOrderBins - 1); };
    constexpr int kBatch = 8;
    const int span = kBatch * blockDim.x;
    for (int q0 = tid; q0 < n; q0 += span) {
        int bq[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int q = q0 + u * (int)blockDim.x;
            bq[u] = q < n ? bin(q) : -1;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
            if (bq[u] >= 0) atomicAdd(&hist[bq[u]], 1);
    }
    __syncthreads();
    // exclusive scan of the 4096 bins, 4 consecutive bins a thread
    const int b0 = 4 * tid;
    const int c0 = hist[b0], c1 = hist[b0 + 1], c2 = hist[b0 + 2], c3 = hist[b0 + 3];
    const int local = c0 + c1 + c2 + c3;
    const int incl = wave_incl_scan_int(local, lane);
    if (lane == kWave - 1) s_wsum[wid] = incl;
    __syncthreads();
    int off = 0;
    for (int w = 0; w < wid; ++w) off += s_wsum[w];
    const int ex = off + incl - local;
    hist[b0] = ex;
    hist[b0 + 1] = ex + c0;
    hist[b0 + 2] = ex + c0 + c1;
    hist[b0 + 3] = ex + c0 + c1 + c2;
    __syncthreads();
    for (int q0 = tid; q0 < n; q0 += span) {
        int bq[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int q = q0 + u * (int)blockDim.x;
            bq[u] = q < n ? bin(q) : -1;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u)
            if (bq[u] >= 0) order[atomicAdd(&hist[bq[u]], 1)] = q0 + u * (int)blockDim.x;
    }
}

void launch_order_bricks(const int* cost, long n, int* order, hipStream_t s) {
    hipLaunchKernelGGL(order_bricks, dim3(1), dim3(1024), 0, s, cost, (int)n, order);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sum_counts_partial(const int* __restrict__ c, long n,
                                                          unsigned long long* __restrict__ part) {
    __shared__ unsigned long long s[256];
    unsigned long long acc = 0;
    for (long q = (long)blockIdx.x * 256 + threadIdx.x; q < n; q += (long)gridDim.x * 256)
        acc += (unsigned long long)c[q];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ void sum_counts_final(const unsigned long long* __restrict__ part, int n,
                                 unsigned long long* __restrict__ total) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        unsigned long long acc = 0;
        for (int q = 0; q < n; ++q) acc += part[q];
        *total = acc;
    }
}

// ---------------------------------------------------------------------------
// Brick shapes the kernels are built for (index = TileCfg::shape).
struct Shape {
    int x, y, z;
};
static const Shape kShapes[kNumShapes] = {{4, 4, 4}, {8, 4, 2}, {4, 8, 2}, {8, 2, 4}};

long brick_count(const PlanConst& P, int shape) {
    const Shape& S = kShapes[shape];
    return (long)((P.nx + S.x - 1) / S.x) * ((P.ny + S.y - 1) / S.y) * ((P.nz + S.z - 1) / S.z);
}

void shape_dims(int shape, int d[3]) {
    d[0] = kShapes[shape].x;
    d[1] = kShapes[shape].y;
    d[2] = kShapes[shape].z;
}

template <int DC, int MODE>
static void launch_mode(const DoseArgs& a, TileCfg cfg, const int* order, const float* fluence,
                        float* dose, int* out_int, hipStream_t s, const float4* prm = nullptr) {
    const size_t water_bytes = sizeof(float4) * 3 * (size_t)a.P.dt_n;
    const bool lds = cfg.waves_per_block == kLdsWaves;
    const bool lw = lds && MODE != kCount && MODE != kCountBrick && water_bytes <= (size_t)kLdsWaterMax;
    const int wpb = lds && !lw ? 4 : cfg.waves_per_block;
    const long nb = brick_count(a.P, cfg.shape);
    dim3 grid((unsigned)((nb + wpb - 1) / wpb)), block(kWave * wpb);
#define FSPB_SHAPE(ID, X, Y, Z)                                                                \
    case ID:                                                                                   \
        if (lw)                                                                                \
            hipLaunchKernelGGL((dose_forward<DC, MODE, X, Y, Z, true>), grid, block,           \
                               water_bytes, s, a, order, fluence, dose, out_int, prm);         \
        else                                                                                   \
            hipLaunchKernelGGL((dose_forward<DC, MODE, X, Y, Z, false>), grid, block, 0, s, a, \
                               order, fluence, dose, out_int, prm);                            \
        break;
    switch (cfg.shape) {
        FSPB_SHAPE(0, 4, 4, 4)
        FSPB_SHAPE(1, 8, 4, 2)
        FSPB_SHAPE(2, 4, 8, 2)
        FSPB_SHAPE(3, 8, 2, 4)
    }
#undef FSPB_SHAPE
}

void launch_forward(const DoseArgs& a, bool dc, TileCfg cfg, const int* order,
                    const float* fluence, float* dose, hipStream_t s) {
    if (dc && a.P.w2_one)
        launch_mode<kDcOneDrift, kDose>(a, cfg, order, fluence, dose, nullptr, s);
    else if (dc)
        launch_mode<kDcTwoDrift, kDose>(a, cfg, order, fluence, dose, nullptr, s);
    else
        launch_mode<kPlain, kDose>(a, cfg, order, fluence, dose, nullptr, s);
}

void launch_forward_siddon(const DoseArgs& a, bool dc, TileCfg cfg, const int* order,
                           const float* fluence, float* dose, hipStream_t s) {
    // the exact-table records carry both drifts
    if (dc)
        launch_mode<kDcTwoDrift, kSid>(a, cfg, order, fluence, dose, nullptr, s);
    else
        launch_mode<kPlain, kSid>(a, cfg, order, fluence, dose, nullptr, s);
}

void launch_forward_surrogate(const DoseArgs& a, TileCfg cfg, const int* order,
                              const float* fluence, const float4* prm, float* dose, hipStream_t s) {
    if (a.P.w2_one)
        launch_mode<kDcOneDrift, kSurr>(a, cfg, order, fluence, dose, nullptr, s, prm);
    else
        launch_mode<kDcTwoDrift, kSurr>(a, cfg, order, fluence, dose, nullptr, s, prm);
}

void launch_count(const DoseArgs& a, TileCfg cfg, const int* order, const float* fluence,
                  int* counts, hipStream_t s) {
    launch_mode<kPlain, kCount>(a, cfg, order, fluence, nullptr, counts, s);
}

void launch_count_bricks(const DoseArgs& a, TileCfg cfg, const int* order, const float* fluence,
                         int* brick_counts, hipStream_t s) {
    launch_mode<kPlain, kCountBrick>(a, cfg, order, fluence, nullptr, brick_counts, s);
}

// Scheduling estimate, one thread per brick: the brick's bounding sphere is
// projected onto each beam's isocentre plane (at its nearest depth, so the
// projection is not too small) and padded by the ROI reach; the estimate is
// the number of beamlet centres in the padded square.  Only the order of
// the bricks depends on it.
template <int BX, int BY, int BZ>
__global__ __launch_bounds__(256) void brick_cost_kernel(DoseArgs a, int* __restrict__ cost) {
    const PlanConst& P = a.P;
    const int brick = blockIdx.x * blockDim.x + threadIdx.x;
    if (brick >= bricks_total<BX, BY, BZ>(P)) return;
    const int nbx = bricks_x<BX, BY, BZ>(P), nby = bricks_y<BX, BY, BZ>(P);
    const int bx = brick % nbx, by = (brick / nbx) % nby, bz = brick / (nbx * nby);
    float cqx, cqy, cqz;
    voxel_q(P, bx * BX, by * BY, bz * BZ, cqx, cqy, cqz);
    const float hx = 0.5f * (BX - 1) * P.dx, hy = 0.5f * (BY - 1) * P.dy, hz = 0.5f * (BZ - 1) * P.dz;
    cqx += hx;
    cqy += hy;
    cqz += hz;
    const float rb = sqrtf(hx * hx + hy * hy + hz * hz);
    int c = 0;
    for (int b = 0; b < P.n_beams; ++b) {
        const BeamDesc& B = a.beams[b];
        const float vx = cqx - B.src[0], vy = cqy - B.src[1], vz = cqz - B.src[2];
        const float z = vx * B.cax[0] + vy * B.cax[1] + vz * B.cax[2];
        const float zn = fmaxf(z - rb, 1e-3f);
        const float pa = (vx * B.ex[0] + vy * B.ex[1] + vz * B.ex[2]) * B.sad / z;
        const float pb = (vx * B.ey[0] + vy * B.ey[1] + vz * B.ey[2]) * B.sad / z;
        const float half = (rb * B.sad + B.pad_scale) / zn;
        const int m_lo = max((int)ceilf((pa - half - B.a0) / B.wx), 0);
        const int m_hi = min((int)floorf((pa + half - B.a0) / B.wx), B.nbx - 1);
        const int n_lo = max((int)ceilf((pb - half - B.b0) / B.wy), 0);
        const int n_hi = min((int)floorf((pb + half - B.b0) / B.wy), B.nby - 1);
        if (m_hi >= m_lo && n_hi >= n_lo) c += (m_hi - m_lo + 1) * (n_hi - n_lo + 1);
    }
    cost[brick] = c;
}

// ---------------------------------------------------------------------------
// The per-beam schedule (kernels.h).  item_cost: one thread per (brick, beam)
// item: the estimate of brick_cost_kernel for that beam alone, and the sort
// key beam * nbins + depth bin of the brick centre along the beam's axis.
template <int BX, int BY, int BZ>
__global__ __launch_bounds__(256) void item_cost_kernel(DoseArgs a, int* __restrict__ cost,
                                                        int* __restrict__ key) {
    const PlanConst& P = a.P;
    const int nb = bricks_total<BX, BY, BZ>(P);
    const long item = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (item >= (long)nb * P.n_beams) return;
    const int b = (int)(item / nb), brick = (int)(item - (long)b * nb);
    const int nbx = bricks_x<BX, BY, BZ>(P), nby = bricks_y<BX, BY, BZ>(P);
    const int bx = brick % nbx, by = (brick / nbx) % nby, bz = brick / (nbx * nby);
    float cqx, cqy, cqz;
    voxel_q(P, bx * BX, by * BY, bz * BZ, cqx, cqy, cqz);
    const float hx = 0.5f * (BX - 1) * P.dx, hy = 0.5f * (BY - 1) * P.dy, hz = 0.5f * (BZ - 1) * P.dz;
    cqx += hx;
    cqy += hy;
    cqz += hz;
    const float rb = sqrtf(hx * hx + hy * hy + hz * hz);
    const BeamDesc& B = a.beams[b];
    const float vx = cqx - B.src[0], vy = cqy - B.src[1], vz = cqz - B.src[2];
    const float z = vx * B.cax[0] + vy * B.cax[1] + vz * B.cax[2];
    const float zn = fmaxf(z - rb, 1e-3f);
    const float pa = (vx * B.ex[0] + vy * B.ex[1] + vz * B.ex[2]) * B.sad / z;
    const float pb = (vx * B.ey[0] + vy * B.ey[1] + vz * B.ey[2]) * B.sad / z;
    const float half = (rb * B.sad + B.pad_scale) / zn;
    const int m_lo = max((int)ceilf((pa - half - B.a0) / B.wx), 0);
    const int m_hi = min((int)floorf((pa + half - B.a0) / B.wx), B.nbx - 1);
    const int n_lo = max((int)ceilf((pb - half - B.b0) / B.wy), 0);
    const int n_hi = min((int)floorf((pb + half - B.b0) / B.wy), B.nby - 1);
    int c = (m_hi >= m_lo && n_hi >= n_lo) ? (m_hi - m_lo + 1) * (n_hi - n_lo + 1) : 0;
    // a brick in front of the entrance of the beamlet whose axis passes
    // nearest to it (in the air before the body) evaluates next to no pairs
    if (c > 0) {
        const int m = min(max((int)floorf((pa - B.a0) / B.wx + 0.5f), 0), B.nbx - 1);
        const int n = min(max((int)floorf((pb - B.b0) / B.wy + 0.5f), 0), B.nby - 1);
        const BeamletDesc& d = a.bl[B.first + n * B.nbx + m];
        const float tc = cqx * d.d[0] + cqy * d.d[1] + cqz * d.d[2] + d.c_t;
        if (!d.hit || tc + rb < 0.0f) c = 0;
    }
    // an item with no candidate still writes its plane: one unit of work
    cost[item] = 1 + c;
    const int bin = min(max((int)((z - B.zlo) * B.zinv), 0), B.nbins - 1);
    key[item] = b * B.nbins + bin;
}

// Counting sort of the items by key (ties in any order; the dose does not
// depend on it) in three passes, then the cut of the sorted list into
// segments of about equal work at key boundaries.  Pass 1: workgroup g counts
// the keys (and sums the work) of its slice of items into hist[g][key];
// pass 2 (one workgroup): per key, each slice's first slot in the sorted list
// and the cuts; pass 3: workgroup g writes its slice's items to their slots.
// Inside a slice, lane l of every wave walks block l of 64 contiguous blocks,
// the waves interleaved within it, so that the lanes of one wave hold items
// far apart (neighbouring items mostly share a key, and same-address LDS
// atomics serialise).
constexpr int kSortThreads = 512;

__device__ __forceinline__ void slice_range(int n, int n_slices, int g, int& lo, int& hi) {
    const int per = (n + n_slices - 1) / n_slices;
    lo = min(g * per, n);
    hi = min(lo + per, n);
}

template <class F>
__device__ __forceinline__ void for_slice_items(int lo, int hi, F f) {
    const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    const int blk = (hi - lo + kWave - 1) / kWave;
    for (int j = wid; j < blk; j += nw) {
        const int q = lo + lane * blk + j;
        if (q < hi) f(q);
    }
}

__global__ __launch_bounds__(kSortThreads) void items_hist(const int* __restrict__ cost,
                                                          const int* __restrict__ key, int n,
                                                          int* __restrict__ hist_n,
                                                          unsigned int* __restrict__ hist_w) {
    __shared__ int cnt[kSplitKeys];
    __shared__ unsigned int csum[kSplitKeys];
    for (int k = threadIdx.x; k < kSplitKeys; k += blockDim.x) {
        cnt[k] = 0;
        csum[k] = 0u;
    }
    __syncthreads();
    int lo, hi;
    slice_range(n, gridDim.x, blockIdx.x, lo, hi);
    for_slice_items(lo, hi, [&](int q) {
        const int k = key[q];
        atomicAdd(&cnt[k], 1);
        atomicAdd(&csum[k], (unsigned int)cost[q]);
    });
    __syncthreads();
    for (int k = threadIdx.x; k < kSplitKeys; k += blockDim.x) {
        hist_n[(long)blockIdx.x * kSplitKeys + k] = cnt[k];
        hist_w[(long)blockIdx.x * kSplitKeys + k] = csum[k];
    }
}

// One workgroup of 1024 threads, four keys a thread.  hist_n[g][k] becomes
// the first slot of slice g's items of key k.
__global__ __launch_bounds__(1024) void items_scan(int* __restrict__ hist_n,
                                                   const unsigned int* __restrict__ hist_w,
                                                   int n_slices, int n, int cap,
                                                   int* __restrict__ chunk) {
    __shared__ int kstart[kSplitKeys];
    __shared__ unsigned long long wpre[kSplitKeys];   // inclusive prefix of the work
    __shared__ int s_wsum[16];
    __shared__ unsigned long long s_wcost[16];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wid = tid / kWave;
    // the thread's four keys of every slice, 16 slices of 16-byte loads at a
    // time (issued together: the loads, not the adds, take the time)
    const int k0 = 4 * tid;
    const int4* __restrict__ hn4 = reinterpret_cast<const int4*>(hist_n);
    const uint4* __restrict__ hw4 = reinterpret_cast<const uint4*>(hist_w);
    constexpr int kB = 16;
    int c[4] = {0, 0, 0, 0};
    unsigned long long w[4] = {0, 0, 0, 0};
    for (int g0 = 0; g0 < n_slices; g0 += kB) {
        int4 vn[kB];
        uint4 vw[kB];
#pragma unroll
        for (int q = 0; q < kB; ++q) {
            const long at = (long)min(g0 + q, n_slices - 1) * (kSplitKeys / 4) + tid;
            vn[q] = hn4[at];
            vw[q] = hw4[at];
        }
#pragma unroll
        for (int q = 0; q < kB; ++q) {
            if (g0 + q < n_slices) {
                c[0] += vn[q].x;
                c[1] += vn[q].y;
                c[2] += vn[q].z;
                c[3] += vn[q].w;
                w[0] += vw[q].x;
                w[1] += vw[q].y;
                w[2] += vw[q].z;
                w[3] += vw[q].w;
            }
        }
    }
    int local = 0;
    unsigned long long lw = 0;
    for (int u = 0; u < 4; ++u) {
        local += c[u];
        lw += w[u];
    }
    int incl = local;
    unsigned long long wincl = lw;
    for (int o = 1; o < kWave; o <<= 1) {
        const int y = __shfl_up(incl, o, kWave);
        const unsigned long long wy = __shfl_up(wincl, o, kWave);
        if (lane >= o) {
            incl += y;
            wincl += wy;
        }
    }
    if (lane == kWave - 1) {
        s_wsum[wid] = incl;
        s_wcost[wid] = wincl;
    }
    __syncthreads();
    int off = 0;
    unsigned long long woff = 0;
    for (int q = 0; q < wid; ++q) {
        off += s_wsum[q];
        woff += s_wcost[q];
    }
    int ex = off + incl - local;
    unsigned long long wex = woff + wincl - lw;
    int run[4];
    for (int u = 0; u < 4; ++u) {
        kstart[k0 + u] = ex;
        run[u] = ex;
        ex += c[u];
        wex += w[u];
        wpre[k0 + u] = wex;
    }
    // each slice's first slot of these keys (the counts are read again)
    int4* __restrict__ hn4w = reinterpret_cast<int4*>(hist_n);
    for (int g0 = 0; g0 < n_slices; g0 += kB) {
        int4 vn[kB];
#pragma unroll
        for (int q = 0; q < kB; ++q)
            vn[q] = hn4[(long)min(g0 + q, n_slices - 1) * (kSplitKeys / 4) + tid];
#pragma unroll
        for (int q = 0; q < kB; ++q) {
            if (g0 + q < n_slices) {
                hn4w[(long)(g0 + q) * (kSplitKeys / 4) + tid] =
                    make_int4(run[0], run[1], run[2], run[3]);
                run[0] += vn[q].x;
                run[1] += vn[q].y;
                run[2] += vn[q].z;
                run[3] += vn[q].w;
            }
        }
    }
    __syncthreads();
    // cuts: segment g (of 8 kSplitSegments, run by XCD g mod 8) ends at the
    // first key whose inclusive work reaches (g + 1) / (8 kSplitSegments) of
    // the total, each segment at most `cap` items
    constexpr int kSeg = 8 * kSplitSegments;
    if (tid == 0) {
        const unsigned long long total = wpre[kSplitKeys - 1];
        chunk[0] = 0;
        int prev = 0;
        for (int g = 1; g < kSeg; ++g) {
            const unsigned long long target = total * (unsigned long long)g / (unsigned long long)kSeg;
            int lo = 0, hi = kSplitKeys - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (wpre[mid] >= target) hi = mid;
                else lo = mid + 1;
            }
            int pos = lo + 1 < kSplitKeys ? kstart[lo + 1] : n;   // items of keys 0..lo
            pos = min(pos, prev + cap);
            pos = max(pos, n - (kSeg - g) * cap);
            pos = max(pos, prev);
            chunk[g] = pos;
            prev = pos;
        }
        chunk[kSeg] = n;
    }
}

__global__ __launch_bounds__(kSortThreads) void items_scatter(const int* __restrict__ key, int n,
                                                             const int* __restrict__ hist_n,
                                                             int* __restrict__ order) {
    __shared__ int slot[kSplitKeys];
    for (int k = threadIdx.x; k < kSplitKeys; k += blockDim.x)
        slot[k] = hist_n[(long)blockIdx.x * kSplitKeys + k];
    __syncthreads();
    int lo, hi;
    slice_range(n, gridDim.x, blockIdx.x, lo, hi);
    for_slice_items(lo, hi, [&](int q) { order[atomicAdd(&slot[key[q]], 1)] = q; });
}

// Longest segment: 1.5 times an even share of the items.
long split_seg_cap(long n_items) {
    return (3 * n_items + 16 * kSplitSegments - 1) / (16 * kSplitSegments);
}
long split_run_cap(long n_items) { return kSplitSegments * split_seg_cap(n_items); }
int split_sort_slices(long n_items) { return (int)std::min<long>(64, (n_items + 2047) / 2048); }

void launch_split_schedule(const DoseArgs& a, TileCfg cfg, const SplitSched& sc, hipStream_t s) {
    const long n = brick_count(a.P, cfg.shape) * a.P.n_beams;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    switch (cfg.shape) {
        case 0: hipLaunchKernelGGL((item_cost_kernel<4, 4, 4>), grid, block, 0, s, a, sc.cost, sc.key); break;
        case 1: hipLaunchKernelGGL((item_cost_kernel<8, 4, 2>), grid, block, 0, s, a, sc.cost, sc.key); break;
        case 2: hipLaunchKernelGGL((item_cost_kernel<4, 8, 2>), grid, block, 0, s, a, sc.cost, sc.key); break;
        case 3: hipLaunchKernelGGL((item_cost_kernel<8, 2, 4>), grid, block, 0, s, a, sc.cost, sc.key); break;
    }
    const int slices = split_sort_slices(n);
    hipLaunchKernelGGL(items_hist, dim3(slices), dim3(kSortThreads), 0, s, (const int*)sc.cost,
                       (const int*)sc.key, (int)n, sc.hist_n, sc.hist_w);
    hipLaunchKernelGGL(items_scan, dim3(1), dim3(1024), 0, s, sc.hist_n,
                       (const unsigned int*)sc.hist_w, slices, (int)n, (int)split_seg_cap(n),
                       sc.chunk);
    hipLaunchKernelGGL(items_scatter, dim3(slices), dim3(kSortThreads), 0, s, (const int*)sc.key,
                       (int)n, (const int*)sc.hist_n, sc.order);
}

template <int DC>
static void launch_split_dc(const DoseArgs& a, TileCfg cfg, const SplitSched& sc,
                            const float* fluence, float* planes, long stride, int n_cu,
                            hipStream_t s) {
    const size_t water_bytes = sizeof(float4) * 3 * (size_t)a.P.dt_n;
    const bool lds = cfg.waves_per_block == kLdsWaves;
    const bool lw = lds && water_bytes <= (size_t)kLdsWaterMax;
    const int wpb = lds && !lw ? 4 : cfg.waves_per_block;
    const long n = brick_count(a.P, cfg.shape) * a.P.n_beams;
    const int ipw = kSplitItemsPerWave;
    const long per_xcd = (split_run_cap(n) + (long)wpb * ipw - 1) / ((long)wpb * ipw);
    dim3 grid((unsigned)(8 * per_xcd)), block(kWave * wpb);
    if (lw) hipLaunchKernelGGL(zero_queue, dim3(1), dim3(128), 0, s, sc.queue, 8 * kSplitQueueInts);
#define FSPB_SHAPE(ID, X, Y, Z)                                                                   \
    case ID:                                                                                      \
        if (lw) {                                                                                 \
            auto k = dose_forward_split_q<DC, X, Y, Z>;                                           \
            hipLaunchKernelGGL(k, dim3(persistent_grid(k, kLdsWaves * kWave, water_bytes, n_cu)), \
                               block, water_bytes, s, a, (const int*)sc.order,                    \
                               (const int*)sc.chunk, fluence, planes, stride, sc.queue);          \
        } else {                                                                                  \
            hipLaunchKernelGGL((dose_forward_split<DC, X, Y, Z>), grid, block, 0, s, a,           \
                               (const int*)sc.order, (const int*)sc.chunk, ipw, fluence, planes,  \
                               stride);                                                           \
        }                                                                                         \
        break;
    switch (cfg.shape) {
        FSPB_SHAPE(0, 4, 4, 4)
        FSPB_SHAPE(1, 8, 4, 2)
        FSPB_SHAPE(2, 4, 8, 2)
        FSPB_SHAPE(3, 8, 2, 4)
    }
#undef FSPB_SHAPE
}

void launch_forward_split(const DoseArgs& a, bool dc, TileCfg cfg, const SplitSched& sc,
                          const float* fluence, float* planes, float* dose, int n_cu,
                          hipStream_t s) {
    const long nv = (long)a.P.nx * a.P.ny * a.P.nz;
    const long stride = (nv + 63) / 64 * 64;
    if (dc && a.P.w2_one)
        launch_split_dc<kDcOneDrift>(a, cfg, sc, fluence, planes, stride, n_cu, s);
    else if (dc)
        launch_split_dc<kDcTwoDrift>(a, cfg, sc, fluence, planes, stride, n_cu, s);
    else
        launch_split_dc<kPlain>(a, cfg, sc, fluence, planes, stride, n_cu, s);
    const int blocks = (int)std::min<long>((nv / 4 + 255) / 256 + 1, 8192);
    hipLaunchKernelGGL(sum_planes, dim3(blocks), dim3(256), 0, s, (const float*)planes,
                       a.P.n_beams, nv, stride, dose);
}

void launch_brick_cost(const DoseArgs& a, TileCfg cfg, int* cost, hipStream_t s) {
    const long nb = brick_count(a.P, cfg.shape);
    const dim3 grid((unsigned)((nb + 255) / 256)), block(256);
    switch (cfg.shape) {
        case 0: hipLaunchKernelGGL((brick_cost_kernel<4, 4, 4>), grid, block, 0, s, a, cost); break;
        case 1: hipLaunchKernelGGL((brick_cost_kernel<8, 4, 2>), grid, block, 0, s, a, cost); break;
        case 2: hipLaunchKernelGGL((brick_cost_kernel<4, 8, 2>), grid, block, 0, s, a, cost); break;
        case 3: hipLaunchKernelGGL((brick_cost_kernel<8, 2, 4>), grid, block, 0, s, a, cost); break;
    }
}

void launch_forward_batch(int dc, TileCfg cfg, const DoseArgs* plans, const int2* items,
                          const int* wave_begin, int n_waves, const BatchPtrs& ptrs,
                          unsigned long long* ts_done, unsigned long long* ts_start,
                          const float4* water, int water_n, hipStream_t s) {
    const size_t water_bytes = sizeof(float4) * 3 * (size_t)water_n;
    const bool lds = cfg.waves_per_block == kLdsWaves;
    const bool lw = lds && water && water_bytes <= (size_t)kLdsWaterMax;
    const int wpb = lds && !lw ? 4 : cfg.waves_per_block;
    const size_t sh = lw ? water_bytes : 0;
    dim3 grid((unsigned)((n_waves + wpb - 1) / wpb)), block(kWave * wpb);
#define FSPB_BATCH(DCV, LWV, X, Y, Z)                                                         \
    hipLaunchKernelGGL((dose_forward_batch<DCV, X, Y, Z, LWV>), grid, block, sh, s, plans,    \
                       items, wave_begin, n_waves, ptrs, ts_done, ts_start, water, water_n)
#define FSPB_SHAPE(ID, X, Y, Z)                                                               \
    case ID:                                                                                  \
        if (dc == kDcOneDrift && lw)                                                          \
            FSPB_BATCH(kDcOneDrift, true, X, Y, Z);                                           \
        else if (dc == kDcOneDrift)                                                           \
            FSPB_BATCH(kDcOneDrift, false, X, Y, Z);                                          \
        else if (dc && lw)                                                                    \
            FSPB_BATCH(kDcTwoDrift, true, X, Y, Z);                                           \
        else if (dc)                                                                          \
            FSPB_BATCH(kDcTwoDrift, false, X, Y, Z);                                          \
        else if (lw)                                                                          \
            FSPB_BATCH(kPlain, true, X, Y, Z);                                                \
        else                                                                                  \
            FSPB_BATCH(kPlain, false, X, Y, Z);                                               \
        break;
    switch (cfg.shape) {
        FSPB_SHAPE(0, 4, 4, 4)
        FSPB_SHAPE(1, 8, 4, 2)
        FSPB_SHAPE(2, 4, 8, 2)
        FSPB_SHAPE(3, 8, 2, 4)
    }
#undef FSPB_SHAPE
#undef FSPB_BATCH
}

void launch_fill_u64(unsigned long long* p, long n, unsigned long long v, hipStream_t s) {
    if (n <= 0) return;
    int blocks = (int)std::min<long>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(fill_u64, dim3(blocks), dim3(256), 0, s, p, n, v);
}

void launch_sum_counts(const int* counts, long n, unsigned long long* partial, int n_partial,
                       unsigned long long* total, hipStream_t s) {
    hipLaunchKernelGGL(sum_counts_partial, dim3(n_partial), dim3(256), 0, s, counts, n, partial);
    hipLaunchKernelGGL(sum_counts_final, dim3(1), dim3(64), 0, s, (const unsigned long long*)partial,
                       n_partial, total);
}

}  // namespace fspb
