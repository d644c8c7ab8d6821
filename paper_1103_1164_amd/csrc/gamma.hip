// gamma.hip -- the 3D gamma index of Section 2.3's evaluation (distance and
// dose-difference criteria, global to the maximum reference dose) on gfx950.
//
// gamma(r)^2 = min(cap^2, min over voxel offsets o, |o| <= cap * dd, of
//                  |o|^2 / dd^2 + (E(r + o) - R(r))^2 / dD^2)
// One thread per reference voxel, consecutive threads along x so that every
// offset's evaluated-dose loads are coalesced.  The offsets of the search
// sphere sit in LDS sorted by length: once the distance term alone reaches
// the best value found, no later offset can lower it and the search stops.
#include "gamma.h"

#include <float.h>

namespace fspb {

constexpr int kGammaBlock = 256;

__global__ __launch_bounds__(kGammaBlock) void gamma_kernel(const float* __restrict__ ref,
                                                            const float* __restrict__ ev,
                                                            const int4* __restrict__ off,
                                                            GammaArgs a,
                                                            float* __restrict__ gamma) {
    extern __shared__ int4 s_off[];   // a.n_off entries (dynamic LDS)
    for (int q = threadIdx.x; q < a.n_off; q += blockDim.x) s_off[q] = off[q];
    __syncthreads();
    const long n = (long)a.nx * a.ny * a.nz;
    const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int i = (int)(v % a.nx), j = (int)((v / a.nx) % a.ny), k = (int)(v / ((long)a.nx * a.ny));
    const float r = ref[v];
    float best = a.cap2;
    for (int q = 0; q < a.n_off; ++q) {
        const int4 o = s_off[q];
        const float d2 = __int_as_float(o.w);     // |o|^2 / dd^2
        if (d2 >= best) break;
        const int ii = i + o.x, jj = j + o.y, kk = k + o.z;
        if (ii < 0 || ii >= a.nx || jj < 0 || jj >= a.ny || kk < 0 || kk >= a.nz) continue;
        const float de = ev[((long)kk * a.ny + jj) * a.nx + ii] - r;
        best = fminf(best, fmaf(de * de, a.inv_dD2, d2));
    }
    gamma[v] = sqrtf(best);
}

// Maximum of a grid: per-block maxima, then one block over those (exact in
// any order).
__global__ __launch_bounds__(kGammaBlock) void max_partial(const float* __restrict__ x, long n,
                                                           float* __restrict__ part) {
    __shared__ float s[kGammaBlock];
    float m = -FLT_MAX;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x)
        m = fmaxf(m, x[q]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int o = kGammaBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] = fmaxf(s[threadIdx.x], s[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kGammaBlock) void max_final(const float* __restrict__ part, int n,
                                                         float* __restrict__ out) {
    __shared__ float s[kGammaBlock];
    float m = -FLT_MAX;
    for (int q = threadIdx.x; q < n; q += blockDim.x) m = fmaxf(m, part[q]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int o = kGammaBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] = fmaxf(s[threadIdx.x], s[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = s[0];
}

// Statistics: per block (fixed grid-stride order, fixed tree), then one
// thread over the blocks in order -- deterministic.
__global__ __launch_bounds__(kGammaBlock) void gamma_stats_partial(const float* __restrict__ gamma,
                                                                   const float* __restrict__ ref,
                                                                   long n, float iso,
                                                                   GammaPart* __restrict__ part) {
    __shared__ double s_sum[kGammaBlock];
    __shared__ long long s_n[kGammaBlock], s_pass[kGammaBlock];
    __shared__ float s_max[kGammaBlock];
    double sum = 0.0;
    long long cnt = 0, pass = 0;
    float mx = 0.0f;
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
        const float g = gamma[q];
        mx = fmaxf(mx, g);
        if (ref[q] >= iso) {
            sum += (double)g;
            ++cnt;
            pass += g < 1.0f ? 1 : 0;
        }
    }
    s_sum[threadIdx.x] = sum;
    s_n[threadIdx.x] = cnt;
    s_pass[threadIdx.x] = pass;
    s_max[threadIdx.x] = mx;
    __syncthreads();
    for (int o = kGammaBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            s_sum[threadIdx.x] += s_sum[threadIdx.x + o];
            s_n[threadIdx.x] += s_n[threadIdx.x + o];
            s_pass[threadIdx.x] += s_pass[threadIdx.x + o];
            s_max[threadIdx.x] = fmaxf(s_max[threadIdx.x], s_max[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        GammaPart p;
        p.sum = s_sum[0];
        p.n = s_n[0];
        p.pass = s_pass[0];
        p.max = s_max[0];
        part[blockIdx.x] = p;
    }
}

__global__ void gamma_stats_final(const GammaPart* __restrict__ part, int n,
                                  GammaPart* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    GammaPart t;
    t.sum = 0.0;
    t.n = 0;
    t.pass = 0;
    t.max = 0.0f;
    for (int q = 0; q < n; ++q) {
        t.sum += part[q].sum;
        t.n += part[q].n;
        t.pass += part[q].pass;
        t.max = fmaxf(t.max, part[q].max);
    }
    *out = t;
}

void launch_grid_max(const float* x, long n, float* part, int n_part, float* out, hipStream_t s) {
    hipLaunchKernelGGL(max_partial, dim3(n_part), dim3(kGammaBlock), 0, s, x, n, part);
    hipLaunchKernelGGL(max_final, dim3(1), dim3(kGammaBlock), 0, s, (const float*)part, n_part, out);
}

void launch_gamma(const float* ref, const float* ev, const int4* off, const GammaArgs& a,
                  float* gamma, hipStream_t s) {
    const long n = (long)a.nx * a.ny * a.nz;
    hipLaunchKernelGGL(gamma_kernel, dim3((unsigned)((n + kGammaBlock - 1) / kGammaBlock)),
                       dim3(kGammaBlock), sizeof(int4) * a.n_off, s, ref, ev, off, a, gamma);
}

void launch_gamma_stats(const float* gamma, const float* ref, long n, float iso, GammaPart* part,
                        int n_part, GammaPart* out, hipStream_t s) {
    hipLaunchKernelGGL(gamma_stats_partial, dim3(n_part), dim3(kGammaBlock), 0, s, gamma, ref, n,
                       iso, part);
    hipLaunchKernelGGL(gamma_stats_final, dim3(1), dim3(64), 0, s, (const GammaPart*)part, n_part,
                       out);
}

}  // namespace fspb
