// pair.h -- the per-(voxel, beamlet) dose of Eqs. 2-4 with the Section 2.1
// density corrections, in FP32 VALU arithmetic for gfx950.
//
// Table layouts (built by the host, see fspb_api.hip):
//   dtab[j]          = (u1x, u1y, u2x, u2y)(t_j) * log2(e)  water steepness
//   dtab[n + j]      = slopes of the above to sample j+1
//   dtab[2n + j]     = (w1, w2, w1', w2')                   water weights + slopes
//                      (n = dt_n; three planes with a 16-byte stride: lanes
//                      at nearby depths read neighbouring 16-byte words, where
//                      a 64-byte record stride makes every lane's read start
//                      at the same offset of a 64-byte block and measured
//                      about 1.45x slower)
//   atab[r*n_A + j] = (a, b, c, e) / 4 with a = A[r][j], b = A[r+1][j] - a,
//                   c = A[r][j+1] - a, e = A[r+1][j+1] - A[r+1][j] - c: the
//                   bilinear A(j + fa, r + fr) = a + fr b + fa (c + fr e)
//                   (theta rows r, r+1; the 1/4 is the product of the
//                   factors 1/2 of both Eq. 4 profiles)
//   tT[off + j]  = (T_j, T_{j+1} - T_j)                      radiological depth
//   tTW[off + j] = (T_j, T_{j+1} - T_j, W1_j, W1_{j+1} - W1_j) depth + weight drift
//   tW2[off + j] = (W2_j, W2_{j+1} - W2_j)                    second weight drift
//                  (two planes, 16- and 8-byte strides, rather than one
//                  32-byte record)
#pragma once

#include "fspb_internal.h"

namespace fspb {

// Address-space views: table and grid pointers of a plan may be loaded from
// memory (batched launches), where the compiler cannot infer that they are
// global; the casts keep vector loads global and wave-uniform reads scalar.
// (The host pass only parses these functions; it sees plain pointers.)
#if defined(__HIP_DEVICE_COMPILE__)
#define FSPB_GLOBAL __attribute__((address_space(1)))
#define FSPB_CONST __attribute__((address_space(4)))
#define FSPB_LDS __attribute__((address_space(3)))
#else
#define FSPB_GLOBAL
#define FSPB_CONST
#define FSPB_LDS
#endif
template <class T>
__device__ __forceinline__ const FSPB_GLOBAL T* as_global(const T* p) {
    return (const FSPB_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ FSPB_GLOBAL T* as_global_rw(T* p) {
    return (FSPB_GLOBAL T*)p;
}
template <class T>
__device__ __forceinline__ const FSPB_CONST T* as_const(const T* p) {
    return (const FSPB_CONST T*)p;
}

// Element at a 32-bit byte offset from a global base: the load can use the
// scalar-base + 32-bit vector-offset form, with no 64-bit address arithmetic.
// Every table a plan owns is below 4 GiB (checked when the plan is created).
template <class T>
__device__ __forceinline__ T load_at(const FSPB_GLOBAL T* base, unsigned byte_off) {
    return *reinterpret_cast<const FSPB_GLOBAL T*>(reinterpret_cast<const FSPB_GLOBAL char*>(base) +
                                                   byte_off);
}

// Water-table readers for pair_dose: sample j of the three planes
// (steepness, slopes, weights) from global memory, or from a workgroup's LDS
// copy laid out as 48-byte records (one address, immediate offsets).
struct WaterGlobal {
    const FSPB_GLOBAL float4* p;
    int n;   // samples per plane
    __device__ __forceinline__ void get(unsigned j, float4& u0, float4& us, float4& wv) const {
        const unsigned o = j << 4;
        u0 = load_at(p, o);
        us = load_at(p + n, o);
        wv = load_at(p + 2 * n, o);
    }
};
struct WaterLds {
    const FSPB_LDS float4* p;
    __device__ __forceinline__ void get(unsigned j, float4& u0, float4& us, float4& wv) const {
        // 48 j in a 24-bit multiply (the table holds well under 2^24
        // records); indexing the pointer directly makes a 64-bit multiply-add
        const FSPB_LDS float4* r =
            (const FSPB_LDS float4*)((const FSPB_LDS char*)p + __umul24(j, 48u));
        u0 = r[0];
        us = r[1];
        wv = r[2];
    }
};

__device__ __forceinline__ float fast_exp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Eq. 4 for a beamlet of half width x0:
//   |x| >  x0:  sinh(u x0) e^{-u|x|}   = (e1 - e2) / 2
//   |x| <= x0:  1 - cosh(u x) e^{-u x0} = 1 - (e1 + e2) / 2
// with e1 = e^{-u | |x| - x0 |}, e2 = e^{-u (|x| + x0)}.  Both exponents are
// non-positive, so nothing overflows.  ul = u * log2(e); dm = | |x| - x0 |,
// dp = |x| + x0, outer = (|x| > x0).
// Returns 2 p = sg e1 + (o2 - e2) with (sg, o2) = (1, 0) outside the box and
// (-1, 2) inside (at |x| = x0 both forms agree); the factors 1/2 of both axes
// are folded into the A table.
__device__ __forceinline__ float penumbra2(float ul, float dm, float dp, float sg, float o2) {
    float e1 = fast_exp2(-ul * dm);
    float e2 = fast_exp2(-ul * dp);
    return fmaf(sg, e1, o2 - e2);
}

// The two Eq. 3 profile products, 2 p_x(u_ax) 2 p_y(u_ay) for the steepness
// pairs (u1x, u1y) and (u2x, u2y) (times log2 e), at isocentre-plane offsets
// (x, y) from the axis of a beamlet of half widths (x0, y0), given as
// (nx2, ny2) = (-2 x0, -2 y0): |x| - x0 = fma(nx2, 1/2, |x|) exactly, and the
// outer form below needs -2 u x0.  Outside the box along both axes,
// 2 p_x = e^{-u_x(|x| - x0)} (1 - e^{-2 u_x x0}), so
//   2 p_x 2 p_y = e^{-u_x(|x| - x0) - u_y(|y| - y0)} (1 - e^{-2 u_x x0}) (1 - e^{-2 u_y y0}):
// three exponentials per product instead of four.  That form is taken when
// every active lane of the wave lies outside the box along both axes (most
// pairs: the box is a beamlet wide, the ROI ten times wider); otherwise the
// general form of penumbra2.
__device__ __forceinline__ void profile_products(float x, float y, float nx2, float ny2,
                                                 float u1x, float u1y, float u2x, float u2y,
                                                 float& p1, float& p2) {
    const float ax = fabsf(x), ay = fabsf(y);
    const float ox = fmaf(nx2, 0.5f, ax), oy = fmaf(ny2, 0.5f, ay);   // |x| - x0, |y| - y0
    const bool outer = (ox > 0.0f) & (oy > 0.0f);
    if (__ballot(!outer) == 0) {              // wave-uniform branch
        // E (1 - a) (1 - b) as two fmas: t = E - a E, then t - b t
        const float e1 = fast_exp2(-fmaf(u1x, ox, u1y * oy));
        const float t1 = fmaf(-fast_exp2(u1x * nx2), e1, e1);
        p1 = fmaf(-fast_exp2(u1y * ny2), t1, t1);
        const float e2 = fast_exp2(-fmaf(u2x, ox, u2y * oy));
        const float t2 = fmaf(-fast_exp2(u2x * nx2), e2, e2);
        p2 = fmaf(-fast_exp2(u2y * ny2), t2, t2);
    } else {
        const float dmx = fabsf(ox), dpx = fmaf(nx2, -0.5f, ax);   // |x| + x0
        const float dmy = fabsf(oy), dpy = fmaf(ny2, -0.5f, ay);
        const float sgx = copysignf(1.0f, ox), o2x = 1.0f - sgx;
        const float sgy = copysignf(1.0f, oy), o2y = 1.0f - sgy;
        p1 = penumbra2(u1x, dmx, dpx, sgx, o2x) * penumbra2(u1y, dmy, dpy, sgy, o2y);
        p2 = penumbra2(u2x, dmx, dpx, sgx, o2x) * penumbra2(u2y, dmy, dpy, sgy, o2y);
    }
}

__device__ __forceinline__ float fract(float x) { return __builtin_amdgcn_fractf(x); }
__device__ __forceinline__ float clampf(float x, float lo, float hi) {
    return __builtin_amdgcn_fmed3f(x, lo, hi);
}

// Voxel centre relative to P0; identical in every kernel so that forward,
// adjoint and count take the same pair decisions.
__device__ __forceinline__ void voxel_q(const PlanConst& P, int i, int j, int k, float& qx,
                                        float& qy, float& qz) {
    qx = fmaf((float)i, P.dx, P.qx0);
    qy = fmaf((float)j, P.dy, P.qy0);
    qz = fmaf((float)k, P.dz, P.qz0);
}

// Depth below the entrance and lateral offsets of a voxel for one beamlet,
// and the pair test of Algorithm A1 step 8 (inside the ROI cylinder, t >= 0).
template <class BD>
__device__ __forceinline__ float pair_depth(const BD& d, float qx, float qy, float qz) {
    return fmaf(qx, d.d[0], fmaf(qy, d.d[1], fmaf(qz, d.d[2], d.c_t)));
}
template <class BD>
__device__ __forceinline__ bool pair_test_given_depth(const BD& d, const PlanConst& P, float qx,
                                                      float qy, float qz, float t, float& xp,
                                                      float& yp) {
    xp = fmaf(qx, d.ex[0], fmaf(qy, d.ex[1], fmaf(qz, d.ex[2], d.c_x)));
    yp = fmaf(qx, d.ey[0], fmaf(qy, d.ey[1], fmaf(qz, d.ey[2], d.c_y)));
    return (t >= 0.0f) & (fmaf(xp, xp, yp * yp) <= P.R2);
}
template <class BD>
__device__ __forceinline__ bool pair_coords(const BD& d, const PlanConst& P, float qx, float qy,
                                            float qz, float& t, float& xp, float& yp) {
    t = pair_depth(d, qx, qy, qz);
    return pair_test_given_depth(d, P, qx, qy, qz, t, xp, yp);
}

// SAD / |r_a| for a voxel at depth t below the beamlet's entrance.
template <class BD>
__device__ __forceinline__ float magnification(float t, const BD& b) {
    return b.sad * fast_rcp(t + b.s_entry);
}

// The arithmetic of Eqs. 2-4 for one pair once its table records are read:
// water parameters (u0, us, wv lerped by fd) at geometric depth t, weight
// drifts W1, W2 at that depth (Section 2.2; W1 alone when DC == kDcOneDrift,
// none for plain FSPB), the A record ae lerped by fa, magnified lateral
// offsets (x, y) and inverse square isq.
// fac = (f_u1(rho), f_u2(rho_hat), f_w1(rho_hat), f_w2(rho_hat)) of the voxel.
template <int DC, class BD>
__device__ __forceinline__ float pair_from_records(float x, float y, float isq, const BD& b,
                                                   float4 fac, const PlanConst& P, float fd,
                                                   float4 u0, float4 us, float4 wv, float W1,
                                                   float W2, float fa, float4 ae) {
    float u1x = fmaf(fd, us.x, u0.x), u1y = fmaf(fd, us.y, u0.y);
    float u2x = fmaf(fd, us.z, u0.z), u2y = fmaf(fd, us.w, u0.w);
    float w1 = fmaf(fd, wv.z, wv.x), w2 = fmaf(fd, wv.w, wv.y);

    if (DC) {
        // Section 2.1: u1 by local density, u2 and weights by smoothed
        // density, weights drift with the passing history W_c(t).
        u1x *= fac.x;
        u1y *= fac.x;
        u2x *= fac.y;
        u2y *= fac.y;
        w1 = fmaxf(fac.z * (w1 + W1), 0.0f);
        w2 = fmaxf(fac.w * (DC == kDcOneDrift ? fmaf(P.w2c, W1, w2) : w2 + W2), 0.0f);
    }

    const float A = fmaf(fa, fmaf(b.th_frac, ae.w, ae.z), fmaf(b.th_frac, ae.y, ae.x));

    // Eq. 3 with the Eq. 4 profiles
    float p1, p2;
    profile_products(x, y, b.nx2, b.ny2, u1x, u1y, u2x, u2y, p1, p2);
    float F = fmaf(w1, p1, w2 * p2);
    return F * A * isq;
}

// Unit-fluence dose D_i(r) (Eq. 2) of beamlet b at a voxel with depth t >= 0
// below the beamlet's entrance and lateral offsets (xp, yp) from its axis.
// k = SAD / |r_a| (see magnification()) is computed by the caller.
template <int DC, class BD, class WT>
__device__ __forceinline__ float pair_dose(float t, float xp, float yp, float k, const BD& b,
                                           float4 fac, const PlanConst& P, const WT& water,
                                           const FSPB_GLOBAL float4* __restrict__ atab,
                                           const FSPB_GLOBAL float2* __restrict__ tT,
                                           const FSPB_GLOBAL float4* __restrict__ tTW,
                                           const FSPB_GLOBAL float2* __restrict__ tW2) {
    // magnification to the isocentre plane and inverse square (Eq. 2)
    float x = xp * k, y = yp * k;
    float isq = k * k;   // (SAD/|r_a|)^2; the 1/4 of the two 2p factors is in A

    // Every lookup below except A's depends on t only: issue those loads
    // first so that they share one memory latency, then A's (which needs t_eq).
    // Table coordinates are clamped to the table range; the last entry of
    // each table has zero slope, so a coordinate clamped to the end reads the
    // end value.
    // water parameters at geometric depth t
    const float cd = clampf(fmaf(t, P.dt_inv, P.dt_off), 0.0f, (float)(P.dt_n - 1));
    const float fd = fract(cd);
    float4 u0, us, wv;
    water.get((unsigned)cd, u0, us, wv);

    // per-beamlet radiological depth and weight drift at depth t (Section 2.2);
    // t >= 0 (the pair test), so the sample index needs no lower clamp, and
    // voxel centres never reach the last table interval (j_last = max(K - 2, 0))
    const float c = t * P.inv_d;
    const int j = min((int)c, b.j_last);
    const float f = fract(c);
    float teq, W1 = 0.0f, W2 = 0.0f;
    if (DC) {
        const unsigned ot = (unsigned)(b.tab_off + j);
        const float4 r0 = load_at(tTW, 16u * ot);
        teq = fmaf(f, r0.y, r0.x);
        W1 = fmaf(f, r0.w, r0.z);
        if (DC == kDcTwoDrift) {
            const float2 r1 = load_at(tW2, 8u * ot);
            W2 = fmaf(f, r1.y, r1.x);
        }
    } else {
        const float2 te = load_at(tT, 8u * (unsigned)(b.tab_off + j));
        teq = fmaf(f, te.y, te.x);
    }

    // A(t_eq, theta) / 4: bilinear, theta rows fixed per beamlet
    const float ca = clampf(fmaf(teq, P.at_inv, P.at_off), 0.0f, (float)(P.at_n - 1));
    const float fa = fract(ca);
    const float4 ae = load_at(atab, 16u * ((unsigned)ca + (unsigned)b.a_off));
    return pair_from_records<DC>(x, y, isq, b, fac, P, fd, u0, us, wv, W1, W2, fa, ae);
}

// The beamlet's depth record at depth t (Section 2.2's uniform samples):
// (t_eq, its slope, W1, its slope) of sample j = floor(t / step), or
// (t_eq, slope, 0, 0) for plain FSPB.  For t >= 0 (a pair) j is the sample
// pair_dose reads; any other t gives an index inside the beamlet's own rows
// (the sample clamped to [0, j_last]), so the record can be fetched before
// the pair test has run.
template <int DC, class BD>
__device__ __forceinline__ float4 depth_record(float t, const BD& b, const PlanConst& P,
                                               const FSPB_GLOBAL float2* __restrict__ tT,
                                               const FSPB_GLOBAL float4* __restrict__ tTW) {
    const int j = min((int)fmaxf(t * P.inv_d, 0.0f), b.j_last);
    const unsigned ot = (unsigned)(b.tab_off + j);
    if (DC) return load_at(tTW, 16u * ot);
    const float2 te = load_at(tT, 8u * ot);
    return make_float4(te.x, te.y, 0.0f, 0.0f);
}

// pair_dose for DC != kDcTwoDrift in parts around other work, given the
// pair's depth record rec (see depth_record) fetched ahead of time.
// pair_depth_lerp lerps t_eq from the record at depth t; it may run on
// every lane, as the record is in bounds for any t.  pair_first_half then
// lerps W1, issues the A-table load, the one load that waits on the record,
// and forms the magnification k and the water-table coordinate cd, so that
// t is not needed afterwards.  pair_second_half reads the water parameters and
// completes the pair.  Together they compute what pair_dose computes,
// operation for operation.
template <int DC>
__device__ __forceinline__ void pair_depth_lerp(float t, float4 rec, const PlanConst& P,
                                                float& f, float& teq) {
    static_assert(DC != kDcTwoDrift, "the second drift table has a record of its own");
    f = fract(t * P.inv_d);
    teq = fmaf(f, rec.y, rec.x);
    // formed here, on every lane: the wait for the record then precedes any
    // branch on the pair test, so no path leaves its load pending
    asm volatile("" : "+v"(teq));
}
template <int DC, class BD>
__device__ __forceinline__ void pair_first_half(float t, float4 rec, float f, float teq,
                                                const BD& b, const PlanConst& P,
                                                const FSPB_GLOBAL float4* __restrict__ atab,
                                                float& W1, float& fa, float4& ae, float& k,
                                                float& cd) {
    W1 = DC ? fmaf(f, rec.w, rec.z) : 0.0f;
    // formed here, not where it is used: the record's registers are then
    // free for the next record, with no copies
    asm volatile("" : "+v"(W1));
    const float ca = clampf(fmaf(teq, P.at_inv, P.at_off), 0.0f, (float)(P.at_n - 1));
    fa = fract(ca);
    ae = load_at(atab, 16u * ((unsigned)ca + (unsigned)b.a_off));
    k = magnification(t, b);
    cd = clampf(fmaf(t, P.dt_inv, P.dt_off), 0.0f, (float)(P.dt_n - 1));
}
template <int DC, class BD, class WT>
__device__ __forceinline__ float pair_second_half(float xp, float yp, float k, float cd,
                                                  const BD& b, float4 fac, const PlanConst& P,
                                                  const WT& water, float W1, float fa, float4 ae) {
    float x = xp * k, y = yp * k;
    float isq = k * k;
    const float fd = fract(cd);
    float4 u0, us, wv;
    water.get((unsigned)cd, u0, us, wv);
    return pair_from_records<DC>(x, y, isq, b, fac, P, fd, u0, us, wv, W1, 0.0f, fa, ae);
}

// pair_dose with the exact (Siddon) depth tables: the radiological depth and
// weight drift come from the beamlet's voxel-segment records (see
// kernels.h), found by a binary search on the segment start depths -- the
// search the uniform samples of Section 2.2 avoid.  Everything else is
// pair_dose's.
template <int DC, class BD, class WT>
__device__ __forceinline__ float pair_dose_siddon(float t, float xp, float yp, float k, const BD& b,
                                                  float4 fac, const PlanConst& P, const WT& water,
                                                  const FSPB_GLOBAL float4* __restrict__ atab,
                                                  const FSPB_GLOBAL float4* __restrict__ sid) {
    float x = xp * k, y = yp * k;
    float isq = k * k;
    const float cd = clampf(fmaf(t, P.dt_inv, P.dt_off), 0.0f, (float)(P.dt_n - 1));
    const float fd = fract(cd);
    float4 u0, us, wv;
    water.get((unsigned)cd, u0, us, wv);
    const FSPB_GLOBAL float4* rec = sid + 2 * (long)b.tab_off;
    int lo = 0, hi = b.K - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rec[2 * mid].x <= t) lo = mid;
        else hi = mid - 1;
    }
    const float4 r0 = rec[2 * lo];
    const float dt = t - r0.x;
    const float teq = fmaf(dt, r0.z, r0.y);
    float W1 = 0.0f, W2 = 0.0f;
    if (DC) {
        const float4 r1 = rec[2 * lo + 1];
        W1 = fmaf(dt, r1.x, r0.w);
        W2 = fmaf(dt, r1.z, r1.y);
    }
    const float ca = clampf(fmaf(teq, P.at_inv, P.at_off), 0.0f, (float)(P.at_n - 1));
    const float fa = fract(ca);
    const float4 ae = load_at(atab, 16u * ((unsigned)ca + (unsigned)b.a_off));
    float u1x = fmaf(fd, us.x, u0.x), u1y = fmaf(fd, us.y, u0.y);
    float u2x = fmaf(fd, us.z, u0.z), u2y = fmaf(fd, us.w, u0.w);
    float w1 = fmaf(fd, wv.z, wv.x), w2 = fmaf(fd, wv.w, wv.y);
    if (DC) {
        u1x *= fac.x;
        u1y *= fac.x;
        u2x *= fac.y;
        u2y *= fac.y;
        w1 = fmaxf(fac.z * (w1 + W1), 0.0f);
        w2 = fmaxf(fac.w * (w2 + W2), 0.0f);
    }
    const float A = fmaf(fa, fmaf(b.th_frac, ae.w, ae.z), fmaf(b.th_frac, ae.y, ae.x));
    float p1, p2;
    profile_products(x, y, b.nx2, b.ny2, u1x, u1y, u2x, u2y, p1, p2);
    float F = fmaf(w1, p1, w2 * p2);
    return F * A * isq;
}

// The six Section 2.1 parameters a pair uses, in the units of the tables
// (u in 1/cm, weights dimensionless): out = (u1x, u1y, u2x, u2y, w1, w2).
// Same arithmetic as pair_dose<true>; exported as training targets of the
// learned surrogate.
template <class BD>
__device__ __forceinline__ void dc_params(float t, const BD& b, float4 fac, const PlanConst& P,
                                          const float4* __restrict__ dtab,
                                          const float4* __restrict__ tTW,
                                          const float2* __restrict__ tW2, float out[6]) {
    const float cd = clampf(fmaf(t, P.dt_inv, P.dt_off), 0.0f, (float)(P.dt_n - 1));
    const int jd = (int)cd;
    const float fd = fract(cd);
    const float4 u0 = dtab[jd], us = dtab[P.dt_n + jd], wv = dtab[2 * P.dt_n + jd];
    const float c = t * P.inv_d;
    const int j = max(min((int)c, b.K - 2), 0);
    const float f = fract(c);
    const float4 r0 = tTW[b.tab_off + j];
    const float2 r1 = tW2[b.tab_off + j];
    const float W1 = fmaf(f, r0.w, r0.z), W2 = fmaf(f, r1.y, r1.x);
    const float inv_l2e = 1.0f / kLog2e;
    out[0] = fmaf(fd, us.x, u0.x) * fac.x * inv_l2e;
    out[1] = fmaf(fd, us.y, u0.y) * fac.x * inv_l2e;
    out[2] = fmaf(fd, us.z, u0.z) * fac.y * inv_l2e;
    out[3] = fmaf(fd, us.w, u0.w) * fac.y * inv_l2e;
    out[4] = fmaxf(fac.z * (fmaf(fd, wv.z, wv.x) + W1), 0.0f);
    out[5] = fmaxf(fac.w * (fmaf(fd, wv.w, wv.y) + W2), 0.0f);
}

// Unit-fluence dose of a pair whose six parameters are given (the learned
// surrogate's prediction for the voxel and the beamlet's beam):
// ul = (u1x, u1y, u2x, u2y) * log2(e), wv = (w1, w2, ., .).  Depth, t_eq, A
// and the inverse square stay the beamlet's own (Eq. 2).  Needs the
// density-corrected tables (tTW).
template <class BD>
__device__ __forceinline__ float pair_dose_given(float t, float xp, float yp, float k, const BD& b,
                                                 float4 ul, float4 wv, const PlanConst& P,
                                                 const FSPB_GLOBAL float4* __restrict__ atab,
                                                 const FSPB_GLOBAL float4* __restrict__ tTW) {
    float x = xp * k, y = yp * k;
    float isq = k * k;
    const float c = t * P.inv_d;
    const int j = min((int)c, b.j_last);   // t >= 0 (the pair test)
    const float f = fract(c);
    const float4 r0 = load_at(tTW, 16u * (unsigned)(b.tab_off + j));
    const float teq = fmaf(f, r0.y, r0.x);
    const float ca = clampf(fmaf(teq, P.at_inv, P.at_off), 0.0f, (float)(P.at_n - 1));
    const float fa = fract(ca);
    const float4 ae = load_at(atab, 16u * ((unsigned)ca + (unsigned)b.a_off));
    const float A = fmaf(fa, fmaf(b.th_frac, ae.w, ae.z), fmaf(b.th_frac, ae.y, ae.x));
    float p1, p2;
    profile_products(x, y, b.nx2, b.ny2, ul.x, ul.y, ul.z, ul.w, p1, p2);
    float F = fmaf(wv.x, p1, wv.y * p2);
    return F * A * isq;
}

// pair_dose_given's arithmetic once the A record ae (lerped by fa) is read:
// the second part of the pipelined loop for a row the network serves (see
// pair_first_half), operation for operation.
template <class BD>
__device__ __forceinline__ float pair_given_from_A(float xp, float yp, float k, const BD& b,
                                                   float4 ul, float4 wv, float fa, float4 ae) {
    float x = xp * k, y = yp * k;
    float isq = k * k;
    const float A = fmaf(fa, fmaf(b.th_frac, ae.w, ae.z), fmaf(b.th_frac, ae.y, ae.x));
    float p1, p2;
    profile_products(x, y, b.nx2, b.ny2, ul.x, ul.y, ul.z, ul.w, p1, p2);
    float F = fmaf(wv.x, p1, wv.y * p2);
    return F * A * isq;
}

}  // namespace fspb
