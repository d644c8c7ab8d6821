/* Drives the C ABI's host-side code on a machine without a usable GPU, for
 * runs of a libfspb whose host code is built with AddressSanitizer and
 * UndefinedBehaviorSanitizer: argument validation of every rejected input,
 * the error strings, NULL handles on every entry point, and the host-only
 * queries.  Exits 0 when every call returned the expected code; prints the
 * first mismatch otherwise.  Any sanitizer report aborts the run. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "fspb.h"

static int failures = 0;
#define EXPECT(cond, what)                                         \
    do {                                                           \
        if (!(cond)) {                                             \
            fprintf(stderr, "FAIL %s (line %d): %s\n", what, __LINE__, fspb_last_error()); \
            ++failures;                                            \
        }                                                          \
    } while (0)

static float rho[6 * 5 * 4];
static float water[4] = {1.0f, 0.9f, 0.8f, 0.7f};
static float dens[4] = {0.5f, 1.0f, 1.5f, 2.0f};
static float atab[2 * 4] = {1, 1, 1, 1, 1, 1, 1, 1};

static fspb_table1d tab(float start, float step, int n, const float* v) {
    fspb_table1d t;
    t.start = start;
    t.step = step;
    t.n = n;
    t.v = v;
    return t;
}

int main(void) {
    for (int i = 0; i < 6 * 5 * 4; ++i) rho[i] = 1.0f;
    fspb_ct ct = {6, 5, 4, 0.5f, 0.5f, 0.5f, -1.25f, -1.0f, -0.75f, rho};
    fspb_beam beam = {0.3f, 0.0f, {0.0f, 0.0f, 0.0f}, 100.0f, 2, 2, 0.5f, 0.5f, 0.0f, 0.0f};
    fspb_tables t;
    memset(&t, 0, sizeof t);
    t.A = tab(0.0f, 1.0f, 4, atab);
    t.n_theta = 2;
    t.theta_step = 0.05f;
    fspb_table1d* wt[6] = {&t.u1x, &t.u1y, &t.u2x, &t.u2y, &t.w1, &t.w2};
    for (int k = 0; k < 6; ++k) *wt[k] = tab(0.0f, 1.0f, 4, water);
    fspb_table1d* dt[6] = {&t.fu1, &t.fu2, &t.fw1, &t.fw2, &t.b1, &t.b2};
    for (int k = 0; k < 6; ++k) *dt[k] = tab(0.5f, 0.5f, 4, dens);
    fspb_options o;
    memset(&o, 0, sizeof o);
    o.roi_radius = 5.0f;
    o.rho_surface = 0.5f;
    o.smooth_sigma = 0.5f;
    o.rho_min = 0.1f;
    o.rho_max = 2.0f;
    o.dc_enabled = 1;

    /* error strings */
    for (int code = 0; code >= -5; --code) EXPECT(fspb_error_string(code) && *fspb_error_string(code), "error string");
    EXPECT(strcmp(fspb_error_string(-99), "unknown error") == 0, "unknown code");

    /* a valid plan: no usable device here */
    fspb_geometry* g = (fspb_geometry*)&ct;   /* overwritten on every path */
    int rc = fspb_create_geometry(&ct, 1, &beam, &t, &o, NULL, &g);
    EXPECT(rc == FSPB_E_UNSUPPORTED || rc == FSPB_E_HIP, "valid plan without a device");
    EXPECT(g == NULL, "no handle on error");
    rc = fspb_create_geometry(&ct, 1, &beam, &t, NULL, NULL, &g);
    EXPECT(rc == FSPB_E_UNSUPPORTED || rc == FSPB_E_HIP, "default options without a device");

    /* every rejected input: FSPB_E_ARG before any device call */
#define BAD(stmt, what)                                                        \
    do {                                                                       \
        fspb_ct c2 = ct;                                                       \
        fspb_beam b2 = beam;                                                   \
        fspb_tables t2 = t;                                                    \
        fspb_options o2 = o;                                                   \
        const fspb_options* op = &o2;                                          \
        int nb = 1;                                                            \
        stmt;                                                                  \
        fspb_geometry* h = NULL;                                               \
        const int r = fspb_create_geometry(&c2, nb, &b2, &t2, op, NULL, &h);   \
        EXPECT(r == FSPB_E_ARG && h == NULL, what);                            \
        EXPECT(*fspb_last_error(), what);                                      \
    } while (0)
    BAD(c2.nx = 0, "nx = 0");
    BAD(c2.nz = -3, "nz < 0");
    BAD(c2.dy = -1.0f, "negative spacing");
    BAD(c2.dx = NAN, "NaN spacing");
    BAD(c2.oz = INFINITY, "infinite origin");
    BAD(c2.density = NULL, "NULL density");
    BAD(nb = 0, "no beams");
    BAD(b2.nbx = 0, "no beamlets");
    BAD(b2.sad = 0.0f, "zero SAD");
    BAD(b2.sad = 0.5f, "source inside the grid");
    BAD(b2.gantry = NAN, "NaN gantry");
    BAD(b2.wx = -0.5f, "negative beamlet width");
    BAD(t2.w2.n = 5, "water tables on different grids");
    BAD(t2.fu1.v = NULL, "NULL table values");
    BAD(t2.A.step = 0.0f, "zero table step");
    BAD(t2.n_theta = 0, "no theta rows");
    BAD(o2.flags = 7, "unknown flags");
    BAD((o2.rho_min = 2.0f, o2.rho_max = 0.1f), "empty density range");
    BAD(o2.dc_enabled = 3, "dc flag");
    BAD((o2.tile_shape = 4, o2.tile_waves = 8), "tile shape");
    BAD(o2.tile_waves = 3, "tile waves");
    BAD(o2.schedule = 2, "schedule");
    BAD(o2.roi_radius = -1.0f, "negative ROI radius");
    {
        fspb_geometry* h = NULL;
        EXPECT(fspb_create_geometry(NULL, 1, &beam, &t, &o, NULL, &h) == FSPB_E_ARG, "NULL ct");
        EXPECT(fspb_create_geometry(&ct, 1, NULL, &t, &o, NULL, &h) == FSPB_E_ARG, "NULL beams");
        EXPECT(fspb_create_geometry(&ct, 1, &beam, NULL, &o, NULL, &h) == FSPB_E_ARG, "NULL tables");
        EXPECT(fspb_create_geometry(&ct, 1, &beam, &t, &o, NULL, NULL) == FSPB_E_ARG, "NULL out");
    }

    /* NULL handles on every entry point */
    float f = 0.0f;
    int i0 = 0;
    unsigned long long u64 = 0;
    float* fp = &f;
    EXPECT(fspb_forward(NULL, &f, &f, NULL) == FSPB_E_ARG, "forward");
    EXPECT(fspb_adjoint(NULL, &f, &f, NULL) == FSPB_E_ARG, "adjoint");
    EXPECT(fspb_beamlet_pair_counts(NULL, &i0, NULL) == FSPB_E_ARG, "beamlet_pair_counts");
    EXPECT(fspb_count_pairs(NULL, NULL, NULL, &u64, NULL) == FSPB_E_ARG, "count_pairs");
    EXPECT(fspb_count_pairs_noalloc(NULL, NULL, &u64, NULL) == FSPB_E_ARG, "count_pairs_noalloc");
    EXPECT(fspb_set_dc(NULL, 1) == FSPB_E_ARG, "set_dc");
    fspb_info info;
    EXPECT(fspb_geometry_info(NULL, &info) == FSPB_E_ARG, "geometry_info");
    EXPECT(fspb_smoothed_density(NULL, &f, NULL) == FSPB_E_ARG, "smoothed_density");
    fspb_beamlet_info bi;
    EXPECT(fspb_beamlet(NULL, 0, &bi, NULL, NULL, NULL, 0) == FSPB_E_ARG, "beamlet");
    EXPECT(fspb_update_density(NULL, &f, NULL) == FSPB_E_ARG, "update_density");
    EXPECT(fspb_wait_ready(NULL, NULL) == FSPB_E_ARG, "wait_ready");
    EXPECT(fspb_set_tile(NULL, 0, 8, NULL) == FSPB_E_ARG, "set_tile");
    EXPECT(fspb_get_tile(NULL, &i0, &i0) == FSPB_E_ARG, "get_tile");
    EXPECT(fspb_set_schedule(NULL, 0, NULL) == FSPB_E_ARG, "set_schedule");
    EXPECT(fspb_get_schedule(NULL, &i0) == FSPB_E_ARG, "get_schedule");
    EXPECT(fspb_autotune(NULL, &f, &f, 1, NULL, NULL, 0, NULL) == FSPB_E_ARG, "autotune");
    EXPECT(fspb_set_adjoint_slab(NULL, 0) == FSPB_E_ARG, "set_adjoint_slab");
    EXPECT(fspb_get_adjoint_slab(NULL, &i0) == FSPB_E_ARG, "get_adjoint_slab");
    EXPECT(fspb_autotune_adjoint(NULL, &f, &f, 1, NULL, NULL, NULL, 0, NULL) == FSPB_E_ARG, "autotune_adjoint");
    fspb_batch* bt = NULL;
    EXPECT(fspb_batch_create(0, NULL, 0, 8, 8, 0, NULL, &bt) == FSPB_E_ARG, "batch_create");
    EXPECT(fspb_batch_forward(NULL, (const float* const*)&fp, &fp, NULL) == FSPB_E_ARG, "batch_forward");
    EXPECT(fspb_batch_replay(NULL, NULL) == FSPB_E_ARG, "batch_replay");
    long long items = 0;
    EXPECT(fspb_batch_info(NULL, &i0, &items) == FSPB_E_ARG, "batch_info");
    fspb_mlp* m = NULL;
    EXPECT(fspb_mlp_create(NULL, NULL) == FSPB_E_ARG, "mlp_create");
    EXPECT(fspb_mlp_set_scaling(NULL, &f, &f) == FSPB_E_ARG, "mlp_set_scaling");
    EXPECT(fspb_mlp_set_guard(NULL, NULL) == FSPB_E_ARG, "mlp_set_guard");
    EXPECT(fspb_surrogate_infer(NULL, m, &f, &f, NULL) == FSPB_E_ARG, "surrogate_infer");
    EXPECT(fspb_forward_surrogate(NULL, &f, &f, &f, NULL) == FSPB_E_ARG, "forward_surrogate");
    EXPECT(fspb_gamma(NULL, NULL, 1, 1, 1, 1.0f, 1.0f, 1.0f, NULL, NULL, NULL, NULL) == FSPB_E_ARG, "gamma NULL");
    EXPECT(fspb_gamma(&f, &f, 0, 1, 1, 1.0f, 1.0f, 1.0f, NULL, NULL, NULL, NULL) == FSPB_E_ARG, "gamma size");
    EXPECT(fspb_gamma(&f, &f, 1, 1, 1, -1.0f, 1.0f, 1.0f, NULL, NULL, NULL, NULL) == FSPB_E_ARG, "gamma spacing");
    fspb_destroy(NULL);
    fspb_batch_destroy(NULL);
    fspb_mlp_destroy(NULL);

    /* host-only queries */
    const int n_shapes = fspb_tile_shapes(NULL, 0);
    EXPECT(n_shapes >= 1, "tile_shapes count");
    int dims[3 * 16];
    EXPECT(fspb_tile_shapes(dims, 16) == n_shapes, "tile_shapes dims");
    for (int q = 0; q < n_shapes; ++q) EXPECT(dims[3 * q] * dims[3 * q + 1] * dims[3 * q + 2] == 64, "64 voxels a brick");
    float ratio = 0.0f;
    const int nd = fspb_drift_tables(&t, &ratio);
    EXPECT(nd == 1 || nd == 2, "drift_tables");
    EXPECT(fspb_drift_tables(NULL, &ratio) == FSPB_E_ARG, "drift_tables NULL");
    (void)fspb_release_cached_memory();

    if (failures) return 1;
    printf("ok %d shapes\n", n_shapes);
    return 0;
}
