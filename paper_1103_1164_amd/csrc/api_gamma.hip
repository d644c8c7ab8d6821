// api_gamma.hip -- host side of libfspb: the 3D gamma-index entry point of
// the C ABI (Section 2.3).
#include "api_internal.h"
#include "gamma.h"

#include <math.h>
#include <string.h>

#include <vector>

extern "C" int fspb_gamma(const float* ref, const float* eval, int nx, int ny, int nz, float dx,
                          float dy, float dz, const fspb_gamma_params* params, float* gamma,
                          fspb_gamma_stats* stats, void* stream) {
    if (!ref || !eval) return fail(FSPB_E_ARG, "gamma: NULL dose grid");
    if (nx < 1 || ny < 1 || nz < 1) return fail(FSPB_E_ARG, "gamma: grid sizes must be >= 1");
    const long long nv = (long long)nx * ny * nz;
    if (nv > (1LL << 31) - 1) return fail(FSPB_E_ARG, "gamma: grid of %lld voxels exceeds 2^31-1", nv);
    if (!finite_pos(dx) || !finite_pos(dy) || !finite_pos(dz))
        return fail(FSPB_E_ARG, "gamma: voxel spacing must be finite and > 0");
    fspb_gamma_params p{};
    if (params) p = *params;
    if (p.dist == 0) p.dist = 0.3f;
    if (p.dose_frac == 0) p.dose_frac = 0.03f;
    if (p.gamma_cap == 0) p.gamma_cap = 5.0f;
    if (p.iso_frac == 0) p.iso_frac = 0.5f;
    if (!finite_pos(p.dist) || !finite_pos(p.dose_frac) || !finite_pos(p.gamma_cap) ||
        !isfinite(p.dose_max) || !isfinite(p.iso_frac))
        return fail(FSPB_E_ARG, "gamma: criteria must be finite and > 0");
    // offsets of the search sphere, shortest first
    const double R = (double)p.gamma_cap * p.dist;
    const int mx = (int)floor(R / dx), my = (int)floor(R / dy), mz = (int)floor(R / dz);
    struct Off {
        int i, j, k;
        double d2;
    };
    std::vector<Off> offs;
    for (int k = -mz; k <= mz; ++k)
        for (int j = -my; j <= my; ++j)
            for (int i = -mx; i <= mx; ++i) {
                const double d2 = (i * (double)dx) * (i * (double)dx) + (j * (double)dy) * (j * (double)dy) +
                                  (k * (double)dz) * (k * (double)dz);
                if (d2 <= R * R) offs.push_back({i, j, k, d2});
            }
    if ((int)offs.size() > kMaxGammaOffsets)
        return fail(FSPB_E_ARG, "gamma: search sphere of %zu offsets exceeds %d (reduce the cap)",
                    offs.size(), kMaxGammaOffsets);
    std::stable_sort(offs.begin(), offs.end(), [](const Off& a, const Off& b) { return a.d2 < b.d2; });
    std::vector<int4> hoff(offs.size());
    const double inv_dd2 = 1.0 / ((double)p.dist * p.dist);
    for (size_t q = 0; q < offs.size(); ++q) {
        const float d2 = (float)(offs[q].d2 * inv_dd2);
        int bits;
        memcpy(&bits, &d2, 4);
        hoff[q] = make_int4(offs[q].i, offs[q].j, offs[q].k, bits);
    }
    int dev = 0, rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int n_part = 512;
    struct Scratch {
        int dev;
        std::vector<std::pair<void*, size_t>> b;
        ~Scratch() {
            for (auto& x : b) pool_free(dev, x.first, x.second);
        }
        int get(void** p, size_t bytes) {
            size_t cls = 0;
            int r = pool_alloc(dev, p, bytes, &cls);
            if (r == FSPB_OK) b.push_back({*p, cls});
            return r;
        }
    } S{dev, {}};
    int4* doff = nullptr;
    float* fpart = nullptr;
    float* dmax = nullptr;
    GammaPart* gpart = nullptr;
    GammaPart* gout = nullptr;
    float* g = gamma;
    if ((rc = S.get((void**)&doff, sizeof(int4) * hoff.size())) ||
        (rc = S.get((void**)&fpart, sizeof(float) * n_part)) ||
        (rc = S.get((void**)&dmax, sizeof(float))) ||
        (rc = S.get((void**)&gpart, sizeof(GammaPart) * n_part)) ||
        (rc = S.get((void**)&gout, sizeof(GammaPart))) || (!g && (rc = S.get((void**)&g, sizeof(float) * nv))))
        return rc;
    HIP_TRY(hipMemcpyAsync(doff, hoff.data(), sizeof(int4) * hoff.size(), hipMemcpyHostToDevice, s));
    float D = p.dose_max;
    if (!(D > 0.0f)) {
        launch_grid_max(ref, (long)nv, fpart, n_part, dmax, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&D, dmax, sizeof(float), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (!(D > 0.0f)) return fail(FSPB_E_ARG, "gamma: the reference dose has no positive value");
    }
    GammaArgs a;
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    const double dD = (double)p.dose_frac * D;
    a.inv_dD2 = (float)(1.0 / (dD * dD));
    a.cap2 = p.gamma_cap * p.gamma_cap;
    a.n_off = (int)hoff.size();
    launch_gamma(ref, eval, doff, a, g, s);
    HIP_TRY(hipGetLastError());
    GammaPart h{};
    if (stats) {
        launch_gamma_stats(g, ref, (long)nv, p.iso_frac * D, gpart, n_part, gout, s);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(&h, gout, sizeof(GammaPart), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));   // scratch goes back to the pool after this
    if (stats) {
        stats->gamma_max = h.max;
        stats->n_iso = h.n;
        stats->gamma_avg_iso = h.n ? h.sum / (double)h.n : 0.0;
        stats->pass_rate_iso = h.n ? (double)h.pass / (double)h.n : 0.0;
        stats->dose_max = D;
    }
    return FSPB_OK;
}

