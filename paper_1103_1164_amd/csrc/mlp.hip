// mlp.hip -- the learned surrogate of the Section 2.1 density correction:
// a BF16 MLP (202 -> 64 -> 64 -> 6, tanh-GELU) on the gfx950 matrix cores
// (training: forward, backward, Adam; inference fused with the gather of its
// input rows), and the kernel that writes training rows.
//
// Matrix products use v_mfma_f32_16x16x32_bf16 (BF16 operands, FP32
// accumulation).  Fragment layout of one wave for C[16x16] += A[16x32] B[32x16]:
//   A: lane l holds row l%16, k = 8*(l/16) .. +7
//   B: lane l holds column l%16, k = 8*(l/16) .. +7
//   C: lane l holds column l%16, rows 4*(l/16) .. +3
// Weights are kept as FP32 master values (the optimiser state) and as BF16
// copies in the layouts the fragments read contiguously:
//   w1t [64][224]  layer-1 weights, output-major, inputs zero-padded to 224
//   w2t [64][64]   layer-2 weights, output-major
//   w2r [64][64]   layer-2 weights, input-major (backward)
//   w3t [16][64]   layer-3 weights, output-major, outputs zero-padded to 16
//   w3r [64][32]   layer-3 weights, input-major, outputs zero-padded to 32
// Master layout (flat): W1[202][64], b1[64], W2[64][64], b2[64], W3[64][6], b3[6].
#include "mlp.h"

#include <float.h>
#include <math.h>

#include <algorithm>

#include "pair.h"
#include "wave.h"

namespace fspb {

typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;

__device__ __forceinline__ f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float gelu(float x) {
    const float c = 0.7978845608028654f;
    return 0.5f * x * (1.0f + tanhf(c * (x + 0.044715f * x * x * x)));
}
__device__ __forceinline__ float gelu_grad(float x) {
    const float c = 0.7978845608028654f;
    const float th = tanhf(c * (x + 0.044715f * x * x * x));
    return 0.5f * (1.0f + th) + 0.5f * x * (1.0f - th * th) * c * (1.0f + 3.0f * 0.044715f * x * x);
}

// fragment of 8 consecutive BF16 values at p (16-byte aligned)
__device__ __forceinline__ bf16x8 ld8(const __bf16* p) { return *reinterpret_cast<const bf16x8*>(p); }
// fragment gathered with a stride
__device__ __forceinline__ bf16x8 ld8s(const __bf16* p, int stride) {
    bf16x8 v;
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = p[j * stride];
    return v;
}

constexpr int kRows = 32;   // rows per workgroup (2 waves x 16)
constexpr int kK1 = kMlpInPad;

// ---------------------------------------------------------------------------
// Forward of one 16-row slice held by a wave; writes Z1, H1, Z2, H2 and Y
// (LDS rows r0..r0+15).  X: global BF16 [rows][224].
struct Act {
    alignas(16) float z1[kRows * kMlpHid];
    alignas(16) float z2[kRows * kMlpHid];
    alignas(16) __bf16 h1[kRows * kMlpHid];
    alignas(16) __bf16 h2[kRows * kMlpHid];
    alignas(16) float y[kRows * 16];
};

__device__ void forward_rows(const __bf16* __restrict__ X, long row_base, int n_rows,
                             const MlpWeights& W, Act& s, int r0) {
    const int lane = threadIdx.x & 63;
    const int fr = lane & 15, fk = 8 * (lane >> 4);
    const long grow = row_base + r0 + fr;
    const bool row_ok = grow < n_rows;
    // layer 1: Z1 = X W1 + b1
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int kt = 0; kt < kK1 / 32; ++kt) {
            bf16x8 a = {};
            if (row_ok) a = ld8(X + grow * kK1 + kt * 32 + fk);
            bf16x8 b = ld8(W.w1t + (nt * 16 + fr) * kK1 + kt * 32 + fk);
            acc = mfma(a, b, acc);
        }
        const int col = nt * 16 + fr;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + 4 * (lane >> 4) + j;
            const float z = acc[j] + W.b1[col];
            s.z1[r * kMlpHid + col] = z;
            s.h1[r * kMlpHid + col] = (__bf16)gelu(z);
        }
    }
    __syncthreads();
    // layer 2: Z2 = H1 W2 + b2
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            bf16x8 a = ld8(s.h1 + (r0 + fr) * kMlpHid + kt * 32 + fk);
            bf16x8 b = ld8(W.w2t + (nt * 16 + fr) * kMlpHid + kt * 32 + fk);
            acc = mfma(a, b, acc);
        }
        const int col = nt * 16 + fr;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + 4 * (lane >> 4) + j;
            const float z = acc[j] + W.b2[col];
            s.z2[r * kMlpHid + col] = z;
            s.h2[r * kMlpHid + col] = (__bf16)gelu(z);
        }
    }
    __syncthreads();
    // layer 3: Y = H2 W3 + b3 (outputs padded to 16)
    {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            bf16x8 a = ld8(s.h2 + (r0 + fr) * kMlpHid + kt * 32 + fk);
            bf16x8 b = ld8(W.w3t + fr * kMlpHid + kt * 32 + fk);
            acc = mfma(a, b, acc);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + 4 * (lane >> 4) + j;
            s.y[r * 16 + fr] = acc[j] + (fr < kMlpOut ? W.b3[fr] : 0.0f);
        }
    }
}

// ---------------------------------------------------------------------------
// Inference: Y[rows][6] (FP32) from X (BF16 [rows][224]).
__global__ __launch_bounds__(128) void mlp_forward_kernel(const __bf16* __restrict__ X, int n_rows,
                                                          MlpWeights W, float* __restrict__ Y) {
    __shared__ Act s;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long base = (long)blockIdx.x * kRows;
    forward_rows(X, base, n_rows, W, s, wid * 16);
    __syncthreads();
    for (int q = threadIdx.x; q < kRows * kMlpOut; q += blockDim.x) {
        const int r = q / kMlpOut, c = q % kMlpOut;
        if (base + r < n_rows) Y[(base + r) * kMlpOut + c] = s.y[r * 16 + c];
    }
    (void)lane;
}

// ---------------------------------------------------------------------------
// Training tile: forward, MSE loss against T (FP32 [rows][6]), backward; the
// workgroup's gradient of the mean loss over all n_total rows goes to
// grad[blockIdx.x][kMlpParams] (master layout), its loss sum to loss[blockIdx.x].
struct Bwd {
    alignas(16) __bf16 dy[kRows * 32];          // output gradient, K padded to 32
    alignas(16) float dyf[kRows * 16];
    alignas(16) __bf16 dz2[kRows * kMlpHid];
    alignas(16) float dz2f[kRows * kMlpHid];
    alignas(16) __bf16 dz1[kRows * kMlpHid];
    alignas(16) float dz1f[kRows * kMlpHid];
    float red[2];
};

__global__ __launch_bounds__(128) void mlp_train_kernel(const __bf16* __restrict__ X,
                                                        const float* __restrict__ T, int n_rows,
                                                        MlpWeights W, float* __restrict__ grad,
                                                        float* __restrict__ loss) {
    __shared__ Act s;
    __shared__ Bwd g;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int fr = lane & 15, fk = 8 * (lane >> 4);
    const long base = (long)blockIdx.x * kRows;
    const int r0 = wid * 16;
    forward_rows(X, base, n_rows, W, s, r0);
    if (threadIdx.x < 2) g.red[threadIdx.x] = 0.0f;
    __syncthreads();
    // dL/dY of mean((Y - T)^2) over n_rows x 6
    const float scale = 2.0f / ((float)n_rows * kMlpOut);
    float lsum = 0.0f;
    for (int q = threadIdx.x; q < kRows * 32; q += blockDim.x) {
        const int r = q / 32, c = q % 32;
        float d = 0.0f;
        if (c < kMlpOut && base + r < n_rows) {
            const float e = s.y[r * 16 + c] - T[(base + r) * kMlpOut + c];
            lsum += e * e;
            d = scale * e;
        }
        g.dy[q] = (__bf16)d;
        if (c < 16) g.dyf[r * 16 + c] = d;
    }
    // loss: fixed-order reduction (wave shuffle then two partials)
    for (int o = 32; o > 0; o >>= 1) lsum += __shfl_xor(lsum, o, 64);
    if (lane == 0) g.red[wid] = lsum;
    __syncthreads();
    float* gout = grad + (long)blockIdx.x * kMlpParams;
    if (threadIdx.x == 0) loss[blockIdx.x] = (g.red[0] + g.red[1]) * (0.5f * scale);   // mean share

    // dW3[in][out] = H2^T dY  (M = 64 inputs, N = 16 outputs, K = 32 rows)
    for (int mt = wid; mt < 4; mt += 2) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        bf16x8 a = ld8s(s.h2 + fk * kMlpHid + mt * 16 + fr, kMlpHid);
        bf16x8 b = ld8s(g.dy + fk * 32 + fr, 32);
        acc = mfma(a, b, acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int in = mt * 16 + 4 * (lane >> 4) + j;
            if (fr < kMlpOut) gout[kOffW3 + in * kMlpOut + fr] = acc[j];
        }
    }
    if (threadIdx.x < kMlpOut) {
        float sb = 0.0f;
        for (int r = 0; r < kRows; ++r) sb += g.dyf[r * 16 + threadIdx.x];
        gout[kOffB3 + threadIdx.x] = sb;
    }
    // dZ2 = (dY W3^T) * gelu'(Z2)  (rows x 64, K = 32 padded outputs)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        bf16x8 a = ld8(g.dy + (r0 + fr) * 32 + fk);
        bf16x8 b = ld8(W.w3r + (nt * 16 + fr) * 32 + fk);
        acc = mfma(a, b, acc);
        const int col = nt * 16 + fr;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + 4 * (lane >> 4) + j;
            const float d = acc[j] * gelu_grad(s.z2[r * kMlpHid + col]);
            g.dz2f[r * kMlpHid + col] = d;
            g.dz2[r * kMlpHid + col] = (__bf16)d;
        }
    }
    __syncthreads();
    // dW2[in][out] = H1^T dZ2 (M = N = 64, K = 32 rows); db2
    for (int t = wid; t < 16; t += 2) {
        const int mt = t >> 2, nt = t & 3;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        bf16x8 a = ld8s(s.h1 + fk * kMlpHid + mt * 16 + fr, kMlpHid);
        bf16x8 b = ld8s(g.dz2 + fk * kMlpHid + nt * 16 + fr, kMlpHid);
        acc = mfma(a, b, acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int in = mt * 16 + 4 * (lane >> 4) + j;
            gout[kOffW2 + in * kMlpHid + nt * 16 + fr] = acc[j];
        }
    }
    if (threadIdx.x < kMlpHid) {
        float sb = 0.0f;
        for (int r = 0; r < kRows; ++r) sb += g.dz2f[r * kMlpHid + threadIdx.x];
        gout[kOffB2 + threadIdx.x] = sb;
    }
    // dZ1 = (dZ2 W2^T) * gelu'(Z1)  (rows x 64, K = 64)
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            bf16x8 a = ld8(g.dz2 + (r0 + fr) * kMlpHid + kt * 32 + fk);
            bf16x8 b = ld8(W.w2r + (nt * 16 + fr) * kMlpHid + kt * 32 + fk);
            acc = mfma(a, b, acc);
        }
        const int col = nt * 16 + fr;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + 4 * (lane >> 4) + j;
            const float d = acc[j] * gelu_grad(s.z1[r * kMlpHid + col]);
            g.dz1f[r * kMlpHid + col] = d;
            g.dz1[r * kMlpHid + col] = (__bf16)d;
        }
    }
    __syncthreads();
    // dW1[in][out] = X^T dZ1 (M = 224 padded inputs, N = 64, K = 32 rows); db1
    for (int t = wid; t < (kK1 / 16) * 4; t += 2) {
        const int mt = t >> 2, nt = t & 3;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        bf16x8 a;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const long row = base + fk + j;
            a[j] = row < n_rows ? X[row * kK1 + mt * 16 + fr] : (__bf16)0.0f;
        }
        bf16x8 b = ld8s(g.dz1 + fk * kMlpHid + nt * 16 + fr, kMlpHid);
        acc = mfma(a, b, acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int in = mt * 16 + 4 * (lane >> 4) + j;
            if (in < kMlpIn) gout[kOffW1 + in * kMlpHid + nt * 16 + fr] = acc[j];
        }
    }
    if (threadIdx.x < kMlpHid) {
        float sb = 0.0f;
        for (int r = 0; r < kRows; ++r) sb += g.dz1f[r * kMlpHid + threadIdx.x];
        gout[kOffB1 + threadIdx.x] = sb;
    }
}

// ---------------------------------------------------------------------------
// Sum of the workgroup gradients (fixed order) and an Adam step on the FP32
// master weights; refreshes the BF16 copies.  step = 1 for the first update.
__device__ void write_copies(MlpWeights W, int p, float val) {
    const __bf16 v = (__bf16)val;
    if (p < kOffB1) {
        const int in = p / kMlpHid, out = p % kMlpHid;
        W.w1t_rw[out * kK1 + in] = v;
    } else if (p >= kOffW2 && p < kOffB2) {
        const int q = p - kOffW2, in = q / kMlpHid, out = q % kMlpHid;
        W.w2t_rw[out * kMlpHid + in] = v;
        W.w2r_rw[in * kMlpHid + out] = v;
    } else if (p >= kOffW3 && p < kOffB3) {
        const int q = p - kOffW3, in = q / kMlpOut, out = q % kMlpOut;
        W.w3t_rw[out * kMlpHid + in] = v;
        W.w3r_rw[in * 32 + out] = v;
    }
}

__global__ void mlp_adam_kernel(const float* __restrict__ grad, int n_parts, MlpWeights W,
                                float* __restrict__ master, float* __restrict__ m,
                                float* __restrict__ v, AdamParams ap) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    float gs = 0.0f;
    for (int q = 0; q < n_parts; ++q) gs += grad[(long)q * kMlpParams + p];
    const float mm = ap.beta1 * m[p] + (1.0f - ap.beta1) * gs;
    const float vv = ap.beta2 * v[p] + (1.0f - ap.beta2) * gs * gs;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / ap.bc1, vh = vv / ap.bc2;
    const float w = master[p] - ap.lr * mh / (sqrtf(vh) + ap.eps);
    master[p] = w;
    write_copies(W, p, w);
}

// Copies the master weights into the BF16 layouts (and zeroes the padding).
__global__ void mlp_sync_kernel(const float* __restrict__ master, MlpWeights W) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    // padding first: every padded slot of the copies is zero
    if (p < kMlpHid * kK1) {
        const int out = p / kK1, in = p % kK1;
        if (in >= kMlpIn) W.w1t_rw[p] = (__bf16)0.0f;
        (void)out;
    }
    if (p < 16 * kMlpHid && p / kMlpHid >= kMlpOut) W.w3t_rw[p] = (__bf16)0.0f;
    if (p < kMlpHid * 32 && p % 32 >= kMlpOut) W.w3r_rw[p] = (__bf16)0.0f;
    if (p < kMlpParams) write_copies(W, p, master[p]);
}

// Loss of a training launch: the per-workgroup sums in a fixed order.
__global__ void mlp_loss_sum_kernel(const float* __restrict__ parts, int n, float* __restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float acc = 0.0f;
        for (int q = 0; q < n; ++q) acc += parts[q];
        *out = acc;
    }
}

// Sum of per-workgroup gradients without an update (for gradient checks).
__global__ void mlp_grad_sum_kernel(const float* __restrict__ grad, int n_parts,
                                    float* __restrict__ out) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    float gs = 0.0f;
    for (int q = 0; q < n_parts; ++q) gs += grad[(long)q * kMlpParams + p];
    out[p] = gs;
}


// ===========================================================================
// Surrogate input rows.  A row is a (voxel, beam).  Its nearest beamlet is
// the one whose isocentre-plane centre lies nearest to the voxel's central
// projection from the source (ties round up).  The row is valid when that
// beamlet reaches the body and its pair with the voxel passes the pair test
// (inside the ROI cylinder, below the entrance).  Patch: on the ray from the
// source to the voxel centre q (unit direction u), plane k = 0..7 sits
// t (7 - k) / 7 before the voxel (t = the voxel's depth for the nearest
// beamlet), and holds a 5 x 5 lattice at 0.5 cm along e1 = the beam's x axis
// made orthogonal to u, and e2 = e1 x u.  Feature 25 k + 5 b + a is the
// trilinear density at q - t (7 - k) / 7 u + 0.5 (a - 2) e1 + 0.5 (b - 2) e2.
struct RowGeo {
    float qx, qy, qz;
    float ux, uy, uz, e1x, e1y, e1z, e2x, e2y, e2z;
    float t, theta, rho_c;
    int ib;
    long v;
    bool valid;
};

__device__ __forceinline__ RowGeo row_geometry(const DoseArgs& a, const float* __restrict__ rho,
                                               long v, int b) {
    const PlanConst& P = a.P;
    RowGeo r;
    r.v = v;
    // 32-bit index arithmetic: the surrogate's plans hold fewer than 2^28
    // voxels (checked when a surrogate call is made)
    const unsigned nx = (unsigned)P.nx, ny = (unsigned)P.ny;
    const unsigned vv = (unsigned)v, row_yz = vv / nx;
    const int i = (int)(vv - row_yz * nx), j = (int)(row_yz % ny), k = (int)(row_yz / ny);
    voxel_q(P, i, j, k, r.qx, r.qy, r.qz);
    const BeamDesc& B = a.beams[b];
    const float vx = r.qx - B.src[0], vy = r.qy - B.src[1], vz = r.qz - B.src[2];
    const float z = vx * B.cax[0] + vy * B.cax[1] + vz * B.cax[2];
    const float pa = B.sad * (vx * B.ex[0] + vy * B.ex[1] + vz * B.ex[2]) / z;
    const float pb = B.sad * (vx * B.ey[0] + vy * B.ey[1] + vz * B.ey[2]) / z;
    const int m = min(max((int)floorf((pa - B.a0) / B.wx + 0.5f), 0), B.nbx - 1);
    const int n = min(max((int)floorf((pb - B.b0) / B.wy + 0.5f), 0), B.nby - 1);
    r.ib = B.first + n * B.nbx + m;
    const BeamletDesc& d = a.bl[r.ib];
    float xp, yp;
    const bool pass = pair_coords(d, P, r.qx, r.qy, r.qz, r.t, xp, yp);
    r.valid = (z > 0.0f) && d.hit && pass;
    r.theta = d.theta;
    const float L = sqrtf(vx * vx + vy * vy + vz * vz);
    r.ux = vx / L;
    r.uy = vy / L;
    r.uz = vz / L;
    const float pr = B.ex[0] * r.ux + B.ex[1] * r.uy + B.ex[2] * r.uz;
    float ex = B.ex[0] - pr * r.ux, ey = B.ex[1] - pr * r.uy, ez = B.ex[2] - pr * r.uz;
    const float inv = 1.0f / sqrtf(ex * ex + ey * ey + ez * ez);
    r.e1x = ex * inv;
    r.e1y = ey * inv;
    r.e1z = ez * inv;
    r.e2x = r.e1y * r.uz - r.e1z * r.uy;
    r.e2y = r.e1z * r.ux - r.e1x * r.uz;
    r.e2z = r.e1x * r.uy - r.e1y * r.ux;
    r.rho_c = rho[v];
    return r;
}

// Per-feature patch coefficients, staged in LDS by the kernels that gather
// rows: feature f = 25 k + 5 b + a sits at (fraction back along the ray,
// offset along e1, offset along e2) = (-(7 - k) / 7, 0.5 (a - 2), 0.5 (b - 2)).
struct PatchCoef {
    float4 c[kPatchN];
    __device__ __forceinline__ void stage() {
        for (int f = threadIdx.x; f < kPatchN; f += blockDim.x) {
            const int k = f / 25, rem = f - 25 * k, bb = rem / 5, aa = rem - 5 * bb;
            c[f] = make_float4(-(float)(kPatchPlanes - 1 - k) / (float)(kPatchPlanes - 1),
                               kPatchPitch * (float)(aa - 2), kPatchPitch * (float)(bb - 2), 0.0f);
        }
    }
};

// Reciprocal voxel sizes of a plan (one division each, per kernel).
struct InvSpacing {
    float x, y, z;
};
__device__ __forceinline__ InvSpacing inv_spacing(const PlanConst& P) {
    return InvSpacing{1.0f / P.dx, 1.0f / P.dy, 1.0f / P.dz};
}

// Trilinear density between voxel centres, indices clamped to the grid
// (clamp-to-edge), at a point p relative to P0.  Corner offsets are 32-bit
// (the surrogate takes plans of fewer than 2^28 voxels, checked with the plan).
__device__ __forceinline__ float density_at(const FSPB_GLOBAL float* __restrict__ rho,
                                            const PlanConst& P, InvSpacing is, float px, float py,
                                            float pz) {
    const float gx = (px - P.qx0) * is.x, gy = (py - P.qy0) * is.y, gz = (pz - P.qz0) * is.z;
    const float fx0 = floorf(gx), fy0 = floorf(gy), fz0 = floorf(gz);
    const float fx = gx - fx0, fy = gy - fy0, fz = gz - fz0;
    const int ix = (int)fx0, iy = (int)fy0, iz = (int)fz0;
    const int y0 = min(max(iy, 0), P.ny - 1), y1 = min(max(iy + 1, 0), P.ny - 1);
    const int z0 = min(max(iz, 0), P.nz - 1), z1 = min(max(iz + 1, 0), P.nz - 1);
    const unsigned r00 = (unsigned)((z0 * P.ny + y0) * P.nx), r10 = (unsigned)((z0 * P.ny + y1) * P.nx);
    const unsigned r01 = (unsigned)((z1 * P.ny + y0) * P.nx), r11 = (unsigned)((z1 * P.ny + y1) * P.nx);
    const int x0 = min(max(ix, 0), P.nx - 1), x1 = min(max(ix + 1, 0), P.nx - 1);
    auto at = [&](unsigned r, int x) { return load_at(rho, 4u * (r + (unsigned)x)); };
    const float a00 = at(r00, x0), b00 = at(r00, x1), a10 = at(r10, x0), b10 = at(r10, x1);
    const float a01 = at(r01, x0), b01 = at(r01, x1), a11 = at(r11, x0), b11 = at(r11, x1);
    const float c00 = fmaf(fx, b00 - a00, a00), c10 = fmaf(fx, b10 - a10, a10);
    const float c01 = fmaf(fx, b01 - a01, a01), c11 = fmaf(fx, b11 - a11, a11);
    const float c0 = fmaf(fy, c10 - c00, c00), c1 = fmaf(fy, c11 - c01, c01);
    return fmaf(fz, c1 - c0, c0);
}

// The CT as 16-byte records, one per voxel (x, y): (rho(x, y), rho(x+1, y),
// rho(x, y+1), rho(x+1, y+1)) in plane z, neighbours clamped to the grid.
// Also clears the inference's list length, which the classify pass after it
// counts up.  32-bit indices: the surrogate's plans hold fewer than 2^28
// voxels (checked when a surrogate call is made).
__global__ __launch_bounds__(256) void make_quads(const float* __restrict__ rho, int nx, int ny,
                                                  int nz, float4* __restrict__ quad,
                                                  unsigned* __restrict__ n_live) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *n_live = 0u;
    const unsigned n = (unsigned)nx * (unsigned)ny * (unsigned)nz;
    for (unsigned v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const unsigned row = v / (unsigned)nx, x = v - row * (unsigned)nx, y = row % (unsigned)ny;
        const unsigned dx = x + 1 < (unsigned)nx ? 1u : 0u, dy = y + 1 < (unsigned)ny ? (unsigned)nx : 0u;
        quad[v] = make_float4(rho[v], rho[v + dx], rho[v + dy], rho[v + dx + dy]);
    }
}

// density_at from the quad records: two aligned 16-byte loads per sample
// (planes z0 and z1) instead of eight 4-byte ones.  Same corner values and
// the same arithmetic as density_at, so the same result bit for bit.
__device__ __forceinline__ float density_at_quad(const FSPB_GLOBAL float4* __restrict__ quad,
                                                 const PlanConst& P, InvSpacing is, float px,
                                                 float py, float pz) {
    const float gx = (px - P.qx0) * is.x, gy = (py - P.qy0) * is.y, gz = (pz - P.qz0) * is.z;
    const float fx0 = floorf(gx), fy0 = floorf(gy), fz0 = floorf(gz);
    const float fx = gx - fx0, fy = gy - fy0, fz = gz - fz0;
    const int ix = (int)fx0, iy = (int)fy0, iz = (int)fz0;
    const int x0 = min(max(ix, 0), P.nx - 1), y0 = min(max(iy, 0), P.ny - 1);
    const int z0 = min(max(iz, 0), P.nz - 1), z1 = min(max(iz + 1, 0), P.nz - 1);
    // 24-bit multiplies: ny nz and nx are below 2^24, and the byte offsets
    // 16 o fit 32 bits: fewer than 2^28 voxels (both checked with the plan)
    const unsigned o0 = __umul24(__umul24((unsigned)z0, (unsigned)P.ny) + (unsigned)y0, (unsigned)P.nx) + (unsigned)x0;
    const unsigned o1 = __umul24(__umul24((unsigned)z1, (unsigned)P.ny) + (unsigned)y0, (unsigned)P.nx) + (unsigned)x0;
    const float4 q0 = load_at(quad, 16u * o0), q1 = load_at(quad, 16u * o1);
    // below the grid in x (or y) both corners along that axis are the edge
    // voxel; above it the records already repeat the edge voxel
    const bool xl = ix < 0, yl = iy < 0;
    const float a0 = q0.x, b0 = xl ? q0.x : q0.y, c0 = yl ? q0.x : q0.z;
    const float d0 = yl ? b0 : (xl ? q0.z : q0.w);
    const float a1 = q1.x, b1 = xl ? q1.x : q1.y, c1 = yl ? q1.x : q1.z;
    const float d1 = yl ? b1 : (xl ? q1.z : q1.w);
    const float c00 = fmaf(fx, b0 - a0, a0), c10 = fmaf(fx, d0 - c0, c0);
    const float c01 = fmaf(fx, b1 - a1, a1), c11 = fmaf(fx, d1 - c1, c1);
    const float e0 = fmaf(fy, c10 - c00, c00), e1 = fmaf(fy, c11 - c01, c01);
    return fmaf(fz, e1 - e0, e0);
}

// The two density sources of gather8: the CT itself, or its quad records
// (identical values, so identical features).
struct DensityPlain {
    const FSPB_GLOBAL float* rho;
    __device__ __forceinline__ float operator()(const PlanConst& P, InvSpacing is, float px, float py,
                                                float pz) const {
        return density_at(rho, P, is, px, py, pz);
    }
};
struct DensityQuad {
    const FSPB_GLOBAL float4* quad;
    __device__ __forceinline__ float operator()(const PlanConst& P, InvSpacing is, float px, float py,
                                                float pz) const {
        return density_at_quad(quad, P, is, px, py, pz);
    }
};

// Eight scaled input features of this lane's layer-1 A fragment for k-step
// kt: lane l takes row l % 16 and features kt * 32 + 8 (l / 16) + j.  Also
// folds the lane's share of the guard statistics (min / max patch density,
// largest |rho - rho(voxel)| over the two planes next to the voxel); the
// caller combines the four lanes of a row.
template <class DS>
__device__ __forceinline__ bf16x8 gather8(const DS& density, const PlanConst& P, InvSpacing is,
                                          const PatchCoef& pc, const RowGeo& r, int kt, int lane,
                                          float& rmin, float& rmax, float& het) {
    const int f0 = kt * 32 + 8 * (lane >> 4);
    bf16x8 xk;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int f = f0 + j;
        float x = 0.0f;
        if (f < kPatchN) {
            const float4 c = pc.c[f];
            const float back = r.t * c.x;
            const float px = fmaf(c.z, r.e2x, fmaf(c.y, r.e1x, fmaf(back, r.ux, r.qx)));
            const float py = fmaf(c.z, r.e2y, fmaf(c.y, r.e1y, fmaf(back, r.uy, r.qy)));
            const float pz = fmaf(c.z, r.e2z, fmaf(c.y, r.e1z, fmaf(back, r.uz, r.qz)));
            const float rv = density(P, is, px, py, pz);
            rmin = fminf(rmin, rv);
            rmax = fmaxf(rmax, rv);
            if (f >= (kPatchPlanes - 2) * 25) het = fmaxf(het, fabsf(rv - r.rho_c));
            x = rv - 1.0f;
        } else if (f == kPatchN) {
            x = r.t * 0.1f - 1.0f;
        } else if (f == kPatchN + 1) {
            x = 10.0f * r.theta;
        }
        xk[j] = (__bf16)x;
    }
    return xk;
}

__device__ __forceinline__ void row_stats_combine(float& rmin, float& rmax, float& het) {
#pragma unroll
    for (int o = 16; o <= 32; o <<= 1) {
        rmin = fminf(rmin, __shfl_xor(rmin, o, 64));
        rmax = fmaxf(rmax, __shfl_xor(rmax, o, 64));
        het = fmaxf(het, __shfl_xor(het, o, 64));
    }
}

// ---------------------------------------------------------------------------
// Training rows: each wave takes 16 listed rows.  Invalid rows get zero
// inputs and targets.
__global__ __launch_bounds__(256) void surrogate_samples_kernel(DoseArgs a,
                                                                const float* __restrict__ rho,
                                                                const int2* __restrict__ rows,
                                                                long n, __bf16* __restrict__ X,
                                                                float* __restrict__ T,
                                                                int* __restrict__ valid) {
    __shared__ PatchCoef pc;
    pc.stage();
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const long row = ((long)blockIdx.x * (blockDim.x >> 6) + wid) * 16 + (lane & 15);
    if (row >= n) return;
    const InvSpacing is = inv_spacing(a.P);
    const int2 rv = rows[row];
    const long n_vox = (long)a.P.nx * a.P.ny * a.P.nz;
    RowGeo r;
    r.valid = false;
    // rows outside the grid or the beam list are invalid, not an error
    if (rv.x >= 0 && rv.x < n_vox && rv.y >= 0 && rv.y < a.P.n_beams)
        r = row_geometry(a, rho, rv.x, rv.y);
    float rmin = FLT_MAX, rmax = -FLT_MAX, het = 0.0f;
    const int fk = 8 * (lane >> 4);
#pragma unroll 1
    for (int kt = 0; kt < kK1 / 32; ++kt) {
        bf16x8 xk = {};
        if (r.valid) xk = gather8(DensityPlain{as_global(rho)}, a.P, is, pc, r, kt, lane, rmin, rmax, het);
        *reinterpret_cast<bf16x8*>(X + row * kK1 + kt * 32 + fk) = xk;
    }
    if (lane < 16) {
        float out[kMlpOut] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        if (r.valid) {
            const BeamletDesc& d = a.bl[r.ib];
            dc_params(r.t, d, a.fac[r.v], a.P, a.dtab, a.tTW, a.tW2, out);
        }
#pragma unroll
        for (int c = 0; c < kMlpOut; ++c) T[row * kMlpOut + c] = out[c];
        valid[row] = r.valid ? 1 : 0;
    }
}

// ---------------------------------------------------------------------------
// Inference over every (voxel, beam) row, in two passes.
//
// surrogate_classify_kernel: one thread per row (rows beam-major).  A row
// that is invalid or fails the guard's cheapest test (|rho_hat - rho| at the
// voxel) gets its fallback record at once; the others are appended to `live`
// with one atomic per block of 2,048 rows, in row order within the block.
// The blocks' order in the list is arbitrary and nothing depends on it: a
// row's result depends on that row alone (the matrix-core products sum each
// output element in a fixed order).
constexpr int kClassRows = 8;   // rows per thread per block of the classify pass

__global__ __launch_bounds__(256) void surrogate_classify_kernel(DoseArgs a,
                                                                 const float* __restrict__ rho,
                                                                 const float* __restrict__ rhohat,
                                                                 float het_max,
                                                                 float4* __restrict__ prm,
                                                                 unsigned* __restrict__ live,
                                                                 unsigned* __restrict__ n_live) {
    constexpr int kBlock = 256 * kClassRows;
    __shared__ unsigned s_bits[kBlock / 32];
    __shared__ int s_wsum[4];
    __shared__ unsigned s_base;
    const PlanConst& P = a.P;
    const long n_vox = (long)P.nx * P.ny * P.nz;
    const long n_rows = n_vox * P.n_beams;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    // a block of 2,048 consecutive rows per round, classified with coalesced
    // accesses (row q * 256 + tid); the keep bits go to an LDS bitmap, and
    // each thread then lists eight consecutive rows, so the list keeps the
    // rows' order (the gathers of a tile of 16 listed rows read neighbouring
    // voxels' patches); one atomic reserves the block's slots
    for (long blk = blockIdx.x; blk * kBlock < n_rows; blk += gridDim.x) {
#pragma unroll
        for (int q = 0; q < kClassRows; ++q) {
            const long row = blk * kBlock + q * 256 + tid;
            bool keep = false;
            if (row < n_rows) {
                // rows < 2^32 (checked when a surrogate call is made)
                const unsigned b = (unsigned)row / (unsigned)n_vox;
                const long v = (long)((unsigned)row - b * (unsigned)n_vox);
                const RowGeo r = row_geometry(a, rho, v, b);
                keep = r.valid && fabsf(rhohat[v] - r.rho_c) <= het_max;
                if (!keep) {
                    prm[2 * row] = make_float4(0.f, 0.f, 0.f, 0.f);
                    prm[2 * row + 1] = make_float4(0.f, 0.f, 1.f, 0.f);
                }
            }
            const unsigned long long m = __ballot(keep);
            if (lane == 0) {
                s_bits[(q * 256 + wid * 64) / 32] = (unsigned)m;
                s_bits[(q * 256 + wid * 64) / 32 + 1] = (unsigned)(m >> 32);
            }
        }
        __syncthreads();
        const unsigned mine = (s_bits[(tid * kClassRows) / 32] >> ((tid * kClassRows) % 32)) & 0xffu;
        const int cnt = __popc(mine);
        const int incl = wave_incl_scan_int(cnt, lane);
        if (lane == 63) s_wsum[wid] = incl;
        __syncthreads();
        int off = incl - cnt, total = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            if (w < wid) off += s_wsum[w];
            total += s_wsum[w];
        }
        if (tid == 0) s_base = total ? atomicAdd(n_live, (unsigned)total) : 0u;
        __syncthreads();
        const unsigned base = s_base;
#pragma unroll
        for (int q = 0; q < kClassRows; ++q)
            if (mine & (1u << q)) live[base + off++] = (unsigned)(blk * kBlock + tid * kClassRows + q);
        __syncthreads();   // s_bits, s_wsum and s_base are read before the next round writes them
    }
}

// surrogate_infer_kernel: the listed rows, 16 per wave (one per lane row).
// A workgroup of 8 waves keeps the BF16 weights in LDS; each lane gathers
// its own A fragments, so the inputs never touch memory.
constexpr int kW1S = kK1 + 8;       // LDS row strides (elements), padded
constexpr int kHS = kMlpHid + 8;
constexpr int kInferWaves = 8;

// One activation buffer per wave, reused layer after layer (a layer's
// inputs are all in registers before its outputs overwrite them): two
// workgroups fit a CU's LDS.
struct InferLds {
    alignas(16) __bf16 w1[kMlpHid * kW1S];
    alignas(16) __bf16 w2[kMlpHid * kHS];
    alignas(16) __bf16 w3[16 * kHS];
    float b1[kMlpHid], b2[kMlpHid], b3[16];
    alignas(16) __bf16 h[kInferWaves][16 * kHS];
    PatchCoef pc;
};
static_assert(16 * 8 * sizeof(float) <= 16 * kHS * sizeof(__bf16), "the output rows fit the buffer");

__device__ __forceinline__ void copy_rows16(__bf16* dst, int dst_stride, const __bf16* src,
                                            int src_stride, int rows, int cols) {
    const int chunks = cols / 8;
    for (int q = threadIdx.x; q < rows * chunks; q += blockDim.x) {
        const int r = q / chunks, c = (q - r * chunks) * 8;
        *reinterpret_cast<bf16x8*>(dst + r * dst_stride + c) =
            *reinterpret_cast<const bf16x8*>(src + r * src_stride + c);
    }
}

// Orders a wave's LDS writes before its later LDS reads (by other lanes of
// the same wave) without waiting for the other waves of the workgroup.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(64 * kInferWaves) __attribute__((amdgpu_waves_per_eu(4)))
void surrogate_infer_kernel(DoseArgs a,
                                                              const float* __restrict__ rho,
                                                              const float* __restrict__ rhohat,
                                                              MlpWeights W, SurrogateScale sc,
                                                              SurrogateGuard gd,
                                                              const float4* __restrict__ quad,
                                                              const unsigned* __restrict__ live,
                                                              const unsigned* __restrict__ n_live_p,
                                                              float4* __restrict__ prm) {
    __shared__ InferLds L;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int fr = lane & 15, fk = 8 * (lane >> 4);
    copy_rows16(L.w1, kW1S, W.w1t, kK1, kMlpHid, kK1);
    copy_rows16(L.w2, kHS, W.w2t, kMlpHid, kMlpHid, kMlpHid);
    copy_rows16(L.w3, kHS, W.w3t, kMlpHid, 16, kMlpHid);
    if (threadIdx.x < kMlpHid) {
        L.b1[threadIdx.x] = W.b1[threadIdx.x];
        L.b2[threadIdx.x] = W.b2[threadIdx.x];
    }
    if (threadIdx.x < 16) L.b3[threadIdx.x] = threadIdx.x < kMlpOut ? W.b3[threadIdx.x] : 0.0f;
    L.pc.stage();
    __syncthreads();

    const PlanConst& P = a.P;
    const InvSpacing is = inv_spacing(P);
    const long n_vox = (long)P.nx * P.ny * P.nz;
    const long n_live = (long)*n_live_p;
    const DensityQuad dq{as_global(quad)};
    __bf16* h = L.h[wid];
    float* yl = reinterpret_cast<float*>(h);
    // each XCD (workgroups are dealt round-robin to the 8 XCDs) walks one
    // contiguous eighth of the listed tiles: the rows it has in flight are
    // then neighbours, and the CT records their patches read stay in its L2
    const long n_tiles = (n_live + 15) / 16;
    const long per_xcd = (n_tiles + 7) / 8;
    const int xcd = blockIdx.x & 7;
    const long t_end = min((long)(xcd + 1) * per_xcd, n_tiles);
    const long wg_per_xcd = gridDim.x / 8;
    for (long tile = (long)xcd * per_xcd + (long)(blockIdx.x >> 3) * kInferWaves + wid; tile < t_end;
         tile += wg_per_xcd * kInferWaves) {
        const long li = tile * 16 + fr;
        const bool row_in = li < n_live;
        RowGeo r;
        r.valid = false;
        long v = 0;
        int b = 0;
        if (row_in) {
            const unsigned row = live[li];
            b = (int)(row / (unsigned)n_vox);
            v = (long)(row - (unsigned)b * (unsigned)n_vox);
            r = row_geometry(a, rho, v, b);
        }
        // the listed rows passed the cheap test; the two planes next to the
        // voxel (k-steps 4-6, kept as A fragments) come next, and a wave
        // whose rows all fall back then skips the rest of the gather and
        // the network
        float rmin = FLT_MAX, rmax = -FLT_MAX, het = 0.0f;
        if (r.valid) het = fabsf(rhohat[v] - r.rho_c);
        bool live_r = r.valid && het <= gd.het_max;
        constexpr int kNear = 4;            // first k-step that holds plane 6
        bf16x8 xn[kK1 / 32 - kNear];
#pragma unroll
        for (int q = 0; q < kK1 / 32 - kNear; ++q) {
            xn[q] = bf16x8{};
            if (live_r) xn[q] = gather8(dq, P, is, L.pc, r, kNear + q, lane, rmin, rmax, het);
        }
        row_stats_combine(rmin, rmax, het);
        live_r = live_r && het <= gd.het_max;
        const bool any = __ballot(live_r) != 0;
        if (any) {
            // layer 1, the remaining inputs gathered one k-step (8 features a
            // lane) at a time
            f32x4 acc[4];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
            for (int kt = 0; kt < kNear; ++kt) {
                bf16x8 xk = {};
                if (live_r) xk = gather8(dq, P, is, L.pc, r, kt, lane, rmin, rmax, het);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[nt] = mfma(xk, ld8(L.w1 + (nt * 16 + fr) * kW1S + kt * 32 + fk), acc[nt]);
            }
#pragma unroll
            for (int q = 0; q < kK1 / 32 - kNear; ++q)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    acc[nt] = mfma(xn[q], ld8(L.w1 + (nt * 16 + fr) * kW1S + (kNear + q) * 32 + fk),
                                   acc[nt]);
            row_stats_combine(rmin, rmax, het);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int col = nt * 16 + fr;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    h[(4 * (lane >> 4) + j) * kHS + col] = (__bf16)gelu(acc[nt][j] + L.b1[col]);
            }
        }
        wave_sync();
        if (any) {
            // layer 2: every fragment of h1 is read before h2 overwrites it
            bf16x8 a2[2];
#pragma unroll
            for (int kt = 0; kt < 2; ++kt) a2[kt] = ld8(h + fr * kHS + kt * 32 + fk);
            f32x4 acc[4];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kt = 0; kt < 2; ++kt)
                    acc[nt] = mfma(a2[kt], ld8(L.w2 + (nt * 16 + fr) * kHS + kt * 32 + fk), acc[nt]);
            }
            wave_sync();
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int col = nt * 16 + fr;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    h[(4 * (lane >> 4) + j) * kHS + col] = (__bf16)gelu(acc[nt][j] + L.b2[col]);
            }
        }
        wave_sync();
        if (any) {
            bf16x8 a3[2];
#pragma unroll
            for (int kt = 0; kt < 2; ++kt) a3[kt] = ld8(h + fr * kHS + kt * 32 + fk);
            f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int kt = 0; kt < 2; ++kt) acc = mfma(a3[kt], ld8(L.w3 + fr * kHS + kt * 32 + fk), acc);
            wave_sync();
            if (fr < 8) {
#pragma unroll
                for (int j = 0; j < 4; ++j) yl[(4 * (lane >> 4) + j) * 8 + fr] = acc[j] + L.b3[fr];
            }
        }
        wave_sync();
        if (lane < 16 && row_in) {
            float o[kMlpOut];
            bool fb = !live_r;
            if (live_r) {
#pragma unroll
                for (int c = 0; c < kMlpOut; ++c) {
                    o[c] = fmaf(yl[lane * 8 + c], sc.stdev[c], sc.mean[c]);
                    if (c < 4) o[c] = __expf(o[c]);     // the network predicts log u
                    fb |= !(o[c] >= gd.band_lo[c] && o[c] <= gd.band_hi[c]);
                }
                fb |= !(rmin >= gd.rho_lo && rmax <= gd.rho_hi);
            }
            float4 ul = make_float4(0.f, 0.f, 0.f, 0.f), wv = make_float4(0.f, 0.f, 1.f, 0.f);
            if (!fb) {
                ul = make_float4(o[0] * kLog2e, o[1] * kLog2e, o[2] * kLog2e, o[3] * kLog2e);
                wv = make_float4(fmaxf(o[4], 0.0f), fmaxf(o[5], 0.0f), 0.0f, 0.0f);
            }
            prm[2 * ((long)b * n_vox + v)] = ul;
            prm[2 * ((long)b * n_vox + v) + 1] = wv;
        }
        // each wave reads and writes only its own activation buffer (the
        // weights are read-only here), so waves need not wait for one
        // another: a wave's LDS accesses complete in order, and wave_sync
        // keeps the compiler from moving them across the layer boundaries
    }
}

// ---------------------------------------------------------------------------
int mlp_tiles(long n_rows) { return (int)((n_rows + kRows - 1) / kRows); }

void launch_mlp_forward(const __bf16* X, long n_rows, const MlpWeights& W, float* Y, hipStream_t s) {
    if (n_rows <= 0) return;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(mlp_tiles(n_rows)), dim3(128), 0, s, X, (int)n_rows,
                       W, Y);
}

void launch_mlp_train(const __bf16* X, const float* T, long n_rows, const MlpWeights& W,
                      float* grad, float* loss, hipStream_t s) {
    hipLaunchKernelGGL(mlp_train_kernel, dim3(mlp_tiles(n_rows)), dim3(128), 0, s, X, T, (int)n_rows,
                       W, grad, loss);
}

void launch_mlp_adam(const float* grad, int n_parts, const MlpWeights& W, float* master, float* m,
                     float* v, const AdamParams& ap, hipStream_t s) {
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, grad,
                       n_parts, W, master, m, v, ap);
}

void launch_mlp_sync(const float* master, const MlpWeights& W, hipStream_t s) {
    const int n = std::max(kMlpParams, kMlpHid * kK1);   // every parameter and every padded slot
    hipLaunchKernelGGL(mlp_sync_kernel, dim3((n + 255) / 256), dim3(256), 0, s, master, W);
}

void launch_mlp_grad_sum(const float* grad, int n_parts, float* out, hipStream_t s) {
    hipLaunchKernelGGL(mlp_grad_sum_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, grad,
                       n_parts, out);
}

void launch_surrogate_samples(const DoseArgs& a, const float* rho, const int2* rows, long n,
                              __bf16* X, float* T, int* valid, hipStream_t s) {
    if (n <= 0) return;
    const long waves = (n + 15) / 16;
    hipLaunchKernelGGL(surrogate_samples_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s,
                       a, rho, rows, n, X, T, valid);
}

void launch_surrogate_infer(const DoseArgs& a, const float* rho, const float* rhohat,
                            const MlpWeights& W, const SurrogateScale& sc,
                            const SurrogateGuard& g, float4* prm, float4* quad, unsigned* live,
                            unsigned* n_live, hipStream_t s) {
    const long n_vox = (long)a.P.nx * a.P.ny * a.P.nz;
    const long n_rows = n_vox * a.P.n_beams;
    hipLaunchKernelGGL(make_quads, dim3((unsigned)std::min<long>((n_vox + 255) / 256, 16384)), dim3(256),
                       0, s, rho, a.P.nx, a.P.ny, a.P.nz, quad, n_live);
    const unsigned cgrid = (unsigned)std::min<long>((n_rows + 2047) / 2048, 4096);
    hipLaunchKernelGGL(surrogate_classify_kernel, dim3(cgrid), dim3(256), 0, s, a, rho, rhohat,
                       g.het_max, prm, live, n_live);
    const long n_groups = ((n_rows + 15) / 16 + kInferWaves - 1) / kInferWaves;
    const unsigned grid = (unsigned)(8 * std::min<long>((n_groups + 7) / 8, 256));   // a multiple of 8
    hipLaunchKernelGGL(surrogate_infer_kernel, dim3(grid), dim3(64 * kInferWaves), 0, s, a, rho,
                       rhohat, W, sc, g, (const float4*)quad, (const unsigned*)live,
                       (const unsigned*)n_live, prm);
}

void launch_mlp_loss_sum(const float* parts, int n_parts, float* out, hipStream_t s) {
    hipLaunchKernelGGL(mlp_loss_sum_kernel, dim3(1), dim3(64), 0, s, parts, n_parts, out);
}

}  // namespace fspb
