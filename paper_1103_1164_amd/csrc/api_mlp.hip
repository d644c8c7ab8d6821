// api_mlp.hip -- host side of libfspb: the learned surrogate's entry points
// of the C ABI (network state, training steps, inference and the surrogate
// forward).
#include "api_internal.h"
#include "mlp.h"

#include <float.h>
#include <math.h>

#include <vector>

struct fspb_mlp {
    int device = 0;
    float* master = nullptr;   // FP32 parameters (flat layout of fspb.h)
    float* am = nullptr;       // Adam moments
    float* av = nullptr;
    __bf16* w1t = nullptr;     // BF16 copies in the layouts the kernels read
    __bf16* w2t = nullptr;
    __bf16* w2r = nullptr;
    __bf16* w3t = nullptr;
    __bf16* w3r = nullptr;
    float* grad_parts = nullptr;   // per-workgroup gradients of one launch
    float* loss_parts = nullptr;
    int part_tiles = 0;
    size_t grad_cls = 0, loss_cls = 0;
    long long step = 0;
    SurrogateScale sc{};
    SurrogateGuard gd{};
    std::vector<std::pair<void*, size_t>> blocks;

    int alloc(void** p, size_t bytes) {
        size_t cls = 0;
        int rc = pool_alloc(device, p, bytes, &cls);
        if (rc == FSPB_OK) blocks.push_back({*p, cls});
        return rc;
    }
    MlpWeights weights() const {
        MlpWeights W;
        W.w1t = W.w1t_rw = w1t;
        W.w2t = W.w2t_rw = w2t;
        W.w2r = W.w2r_rw = w2r;
        W.w3t = W.w3t_rw = w3t;
        W.w3r = W.w3r_rw = w3r;
        W.b1 = master + kOffB1;
        W.b2 = master + kOffB2;
        W.b3 = master + kOffB3;
        return W;
    }
    // per-workgroup scratch for a launch over n rows (grown on demand; the
    // old buffers are returned only after the device has finished with them)
    int ensure_parts(long long n) {
        const int tiles = mlp_tiles((long)n);
        if (tiles <= part_tiles) return FSPB_OK;
        HIP_TRY(hipDeviceSynchronize());
        pool_free(device, grad_parts, grad_cls);
        pool_free(device, loss_parts, loss_cls);
        grad_parts = loss_parts = nullptr;
        part_tiles = 0;
        int rc = pool_alloc(device, (void**)&grad_parts, sizeof(float) * (size_t)tiles * kMlpParams,
                            &grad_cls);
        if (rc != FSPB_OK) return rc;
        rc = pool_alloc(device, (void**)&loss_parts, sizeof(float) * (size_t)tiles, &loss_cls);
        if (rc != FSPB_OK) {
            pool_free(device, grad_parts, grad_cls);
            grad_parts = nullptr;
            return rc;
        }
        part_tiles = tiles;
        return FSPB_OK;
    }
    void release() {
        pool_free(device, grad_parts, grad_cls);
        pool_free(device, loss_parts, loss_cls);
        for (auto& b : blocks) pool_free(device, b.first, b.second);
        blocks.clear();
    }
};

namespace {

int check_rows(long long n, bool allow_zero, const char* what) {
    if (n < (allow_zero ? 0 : 1) || n > FSPB_MLP_MAX_ROWS)
        return fail(FSPB_E_ARG, "%s: row count %lld outside [%d, %d]", what, n, allow_zero ? 0 : 1,
                    FSPB_MLP_MAX_ROWS);
    return FSPB_OK;
}


int upload_state(fspb_mlp* m, const float* params, const float* am, const float* av) {
    std::vector<float> zero(kMlpParams, 0.0f);
    HIP_TRY(hipDeviceSynchronize());
    HIP_TRY(hipMemcpy(m->master, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m->am, am ? am : zero.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(m->av, av ? av : zero.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    launch_mlp_sync(m->master, m->weights(), 0);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipDeviceSynchronize());
    return FSPB_OK;
}

int check_finite(const float* v, int n, const char* what) {
    for (int q = 0; q < n; ++q)
        if (!isfinite(v[q])) return fail(FSPB_E_ARG, "%s: value %d is not finite", what, q);
    return FSPB_OK;
}

}  // namespace

extern "C" {

int fspb_mlp_create(const float* params, fspb_mlp** out) {
    if (!out) return fail(FSPB_E_ARG, "mlp_create: NULL out");
    *out = nullptr;
    if (!params) return fail(FSPB_E_ARG, "mlp_create: NULL params");
    int rc = check_finite(params, kMlpParams, "mlp_create: params");
    if (rc != FSPB_OK) return rc;
    int dev = 0;
    if ((rc = check_device(&dev)) != FSPB_OK) return rc;
    fspb_mlp* m = new (std::nothrow) fspb_mlp();
    if (!m) return fail(FSPB_E_NOMEM, "mlp_create: host allocation failed");
    m->device = dev;
    for (int c = 0; c < kMlpOut; ++c) {
        m->sc.mean[c] = 0.0f;
        m->sc.stdev[c] = 1.0f;
        m->gd.band_lo[c] = -FLT_MAX;
        m->gd.band_hi[c] = FLT_MAX;
    }
    m->gd.rho_lo = -FLT_MAX;
    m->gd.rho_hi = FLT_MAX;
    m->gd.het_max = FLT_MAX;
    const size_t fp = sizeof(float) * kMlpParams;
    if ((rc = m->alloc((void**)&m->master, fp)) != FSPB_OK ||
        (rc = m->alloc((void**)&m->am, fp)) != FSPB_OK ||
        (rc = m->alloc((void**)&m->av, fp)) != FSPB_OK ||
        (rc = m->alloc((void**)&m->w1t, sizeof(__bf16) * kW1tN)) != FSPB_OK ||
        (rc = m->alloc((void**)&m->w2t, sizeof(__bf16) * kW2N)) != FSPB_OK ||
        (rc = m->alloc((void**)&m->w2r, sizeof(__bf16) * kW2N)) != FSPB_OK ||
        (rc = m->alloc((void**)&m->w3t, sizeof(__bf16) * kW3tN)) != FSPB_OK ||
        (rc = m->alloc((void**)&m->w3r, sizeof(__bf16) * kW3rN)) != FSPB_OK ||
        (rc = upload_state(m, params, nullptr, nullptr)) != FSPB_OK) {
        m->release();
        delete m;
        return rc;
    }
    *out = m;
    log_msg(2, "network %p created on device %d", (void*)m, m->device);
    return FSPB_OK;
}

int fspb_mlp_set_scaling(fspb_mlp* m, const float* mean, const float* stdev) {
    if (!m || !mean || !stdev) return fail(FSPB_E_ARG, "mlp_set_scaling: NULL argument");
    for (int c = 0; c < kMlpOut; ++c)
        if (!isfinite(mean[c]) || !finite_pos(stdev[c]))
            return fail(FSPB_E_ARG, "mlp_set_scaling: output %d needs a finite mean and std > 0", c);
    for (int c = 0; c < kMlpOut; ++c) {
        m->sc.mean[c] = mean[c];
        m->sc.stdev[c] = stdev[c];
    }
    return FSPB_OK;
}

int fspb_mlp_set_guard(fspb_mlp* m, const fspb_surrogate_guard* g) {
    if (!m || !g) return fail(FSPB_E_ARG, "mlp_set_guard: NULL argument");
    if (std::isnan(g->rho_lo) || std::isnan(g->rho_hi) || std::isnan(g->het_max))
        return fail(FSPB_E_ARG, "mlp_set_guard: NaN bound");
    for (int c = 0; c < kMlpOut; ++c)
        if (std::isnan(g->band_lo[c]) || std::isnan(g->band_hi[c]))
            return fail(FSPB_E_ARG, "mlp_set_guard: NaN band for output %d", c);
    m->gd.rho_lo = g->rho_lo;
    m->gd.rho_hi = g->rho_hi;
    m->gd.het_max = g->het_max;
    for (int c = 0; c < kMlpOut; ++c) {
        m->gd.band_lo[c] = g->band_lo[c];
        m->gd.band_hi[c] = g->band_hi[c];
    }
    return FSPB_OK;
}

int fspb_mlp_loss_grad(fspb_mlp* m, const uint16_t* x, const float* t, long long n, float* grad,
                       float* loss, void* stream) {
    if (!m || !x || !t) return fail(FSPB_E_ARG, "mlp_loss_grad: NULL argument");
    int rc;
    if ((rc = check_rows(n, false, "mlp_loss_grad")) != FSPB_OK) return rc;
    if ((rc = check_same_device(m->device, "mlp_loss_grad")) != FSPB_OK) return rc;
    if ((rc = m->ensure_parts(n)) != FSPB_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int tiles = mlp_tiles((long)n);
    launch_mlp_train((const __bf16*)x, t, (long)n, m->weights(), m->grad_parts, m->loss_parts, s);
    HIP_TRY(hipGetLastError());
    if (grad) launch_mlp_grad_sum(m->grad_parts, tiles, grad, s);
    if (loss) launch_mlp_loss_sum(m->loss_parts, tiles, loss, s);
    HIP_TRY(hipGetLastError());
    return FSPB_OK;
}

int fspb_mlp_train_step(fspb_mlp* m, const uint16_t* x, const float* t, long long n,
                        const fspb_adam* opt, float* loss, void* stream) {
    if (!m || !x || !t || !opt) return fail(FSPB_E_ARG, "mlp_train_step: NULL argument");
    if (!finite_pos(opt->lr) || !(opt->beta1 >= 0.0f && opt->beta1 < 1.0f) ||
        !(opt->beta2 >= 0.0f && opt->beta2 < 1.0f) || !finite_pos(opt->eps))
        return fail(FSPB_E_ARG, "mlp_train_step: needs lr > 0, 0 <= beta < 1, eps > 0");
    int rc;
    if ((rc = check_rows(n, false, "mlp_train_step")) != FSPB_OK) return rc;
    if ((rc = check_same_device(m->device, "mlp_train_step")) != FSPB_OK) return rc;
    if ((rc = m->ensure_parts(n)) != FSPB_OK) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int tiles = mlp_tiles((long)n);
    const MlpWeights W = m->weights();
    launch_mlp_train((const __bf16*)x, t, (long)n, W, m->grad_parts, m->loss_parts, s);
    HIP_TRY(hipGetLastError());
    if (loss) launch_mlp_loss_sum(m->loss_parts, tiles, loss, s);
    const long long k = m->step + 1;
    AdamParams ap;
    ap.lr = opt->lr;
    ap.beta1 = opt->beta1;
    ap.beta2 = opt->beta2;
    ap.eps = opt->eps;
    ap.bc1 = (float)(1.0 - pow((double)opt->beta1, (double)k));
    ap.bc2 = (float)(1.0 - pow((double)opt->beta2, (double)k));
    launch_mlp_adam(m->grad_parts, tiles, W, m->master, m->am, m->av, ap, s);
    HIP_TRY(hipGetLastError());
    m->step = k;
    return FSPB_OK;
}

int fspb_mlp_predict(fspb_mlp* m, const uint16_t* x, long long n, float* y, void* stream) {
    if (!m) return fail(FSPB_E_ARG, "mlp_predict: NULL handle");
    int rc;
    if ((rc = check_rows(n, true, "mlp_predict")) != FSPB_OK) return rc;
    if (n == 0) return FSPB_OK;
    if (!x || !y) return fail(FSPB_E_ARG, "mlp_predict: NULL argument");
    if ((rc = check_same_device(m->device, "mlp_predict")) != FSPB_OK) return rc;
    launch_mlp_forward((const __bf16*)x, (long)n, m->weights(), y, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FSPB_OK;
}

int fspb_mlp_get_state(const fspb_mlp* m, float* params, float* adam_m, float* adam_v,
                       long long* step) {
    if (!m) return fail(FSPB_E_ARG, "mlp_get_state: NULL handle");
    HIP_TRY(hipDeviceSynchronize());
    const size_t fp = sizeof(float) * kMlpParams;
    if (params) HIP_TRY(hipMemcpy(params, m->master, fp, hipMemcpyDeviceToHost));
    if (adam_m) HIP_TRY(hipMemcpy(adam_m, m->am, fp, hipMemcpyDeviceToHost));
    if (adam_v) HIP_TRY(hipMemcpy(adam_v, m->av, fp, hipMemcpyDeviceToHost));
    if (step) *step = m->step;
    return FSPB_OK;
}

int fspb_mlp_set_state(fspb_mlp* m, const float* params, const float* adam_m,
                       const float* adam_v, long long step) {
    if (!m || !params) return fail(FSPB_E_ARG, "mlp_set_state: NULL argument");
    if (step < 0) return fail(FSPB_E_ARG, "mlp_set_state: negative step");
    int rc = check_finite(params, kMlpParams, "mlp_set_state: params");
    if (rc == FSPB_OK && adam_m) rc = check_finite(adam_m, kMlpParams, "mlp_set_state: adam_m");
    if (rc == FSPB_OK && adam_v) rc = check_finite(adam_v, kMlpParams, "mlp_set_state: adam_v");
    if (rc != FSPB_OK) return rc;
    if ((rc = check_same_device(m->device, "mlp_set_state")) != FSPB_OK) return rc;
    if ((rc = upload_state(m, params, adam_m, adam_v)) != FSPB_OK) return rc;
    m->step = step;
    return FSPB_OK;
}

void fspb_mlp_destroy(fspb_mlp* m) {
    if (!m) return;
    (void)hipDeviceSynchronize();
    m->release();
    delete m;
}

static int check_surrogate_geometry(const fspb_geometry* g, const char* what) {
    if (!g) return fail(FSPB_E_ARG, "%s: NULL geometry", what);
    if (!g->dc_created)
        return fail(FSPB_E_STATE, "%s: the geometry was created without density correction", what);
    if (g->siddon) return fail(FSPB_E_STATE, "%s: not available with exact depth tables", what);
    // row ids are 32-bit; the gathers address the CT's 16-byte records (and
    // the CT) with 32-bit byte offsets, and index its rows with 24-bit
    // multiplies
    const long long nv = (long long)g->P.nx * g->P.ny * g->P.nz;
    if (nv >= (1LL << 28) || nv * g->n_beams >= (1LL << 32) ||
        (long long)g->P.ny * g->P.nz >= (1LL << 24) || g->P.nx >= (1 << 24))
        return fail(FSPB_E_ARG, "%s: %lld voxels x %d beams exceed the surrogate's row range", what,
                    nv, g->n_beams);
    return check_same_device(g->device, what);
}

int fspb_surrogate_samples(fspb_geometry* g, const float* density, const int* rows, long long n,
                           uint16_t* x, float* t, int* valid, void* stream) {
    int rc;
    if ((rc = check_surrogate_geometry(g, "surrogate_samples")) != FSPB_OK) return rc;
    if ((rc = settle(g, (hipStream_t)stream)) != FSPB_OK) return rc;
    if (n < 0 || n > (1LL << 30)) return fail(FSPB_E_ARG, "surrogate_samples: bad row count %lld", n);
    if (n == 0) return FSPB_OK;
    if (!density || !rows || !x || !t || !valid)
        return fail(FSPB_E_ARG, "surrogate_samples: NULL argument");
    launch_surrogate_samples(g->args(), density, (const int2*)rows, (long)n, (__bf16*)x, t, valid,
                             (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FSPB_OK;
}

int fspb_surrogate_infer(fspb_geometry* g, const fspb_mlp* m, const float* density, float* prm,
                         void* stream) {
    int rc;
    if ((rc = check_surrogate_geometry(g, "surrogate_infer")) != FSPB_OK) return rc;
    if ((rc = settle(g, (hipStream_t)stream)) != FSPB_OK) return rc;
    if (!m || !density || !prm) return fail(FSPB_E_ARG, "surrogate_infer: NULL argument");
    if (m->device != g->device) return fail(FSPB_E_STATE, "surrogate_infer: handles on different devices");
    if (!g->surr_live) {
        const size_t rows = (size_t)g->P.nx * g->P.ny * g->P.nz * g->n_beams;
        if ((rc = g->alloc((void**)&g->surr_live, sizeof(unsigned) * rows)) != FSPB_OK ||
            (rc = g->alloc((void**)&g->surr_count, 256)) != FSPB_OK ||
            (rc = g->alloc((void**)&g->surr_quad,
                           sizeof(float4) * (size_t)g->P.nx * g->P.ny * g->P.nz)) != FSPB_OK)
            return rc;
    }
    launch_surrogate_infer(g->args(), density, g->rhohat, m->weights(), m->sc, m->gd,
                           (float4*)prm, g->surr_quad, g->surr_live, g->surr_count,
                           (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    log_msg(3, "surrogate_infer: geometry %p, network %p, stream %p", (void*)g, (const void*)m, stream);
    return FSPB_OK;
}

int fspb_forward_surrogate(fspb_geometry* g, const float* fluence, const float* prm, float* dose,
                           void* stream) {
    int rc;
    if ((rc = check_surrogate_geometry(g, "forward_surrogate")) != FSPB_OK) return rc;
    if ((rc = settle(g, (hipStream_t)stream)) != FSPB_OK) return rc;
    if (!fluence || !prm || !dose) return fail(FSPB_E_ARG, "forward_surrogate: NULL argument");
    launch_forward_surrogate(g->args(), g->tile, g->order, fluence, (const float4*)prm, dose,
                             (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return FSPB_OK;
}

}  // extern "C"

