/* Drives every entry point of the FP64 oracle on one plan read from a dump
 * file, for runs under AddressSanitizer and UndefinedBehaviorSanitizer (the
 * CPU sanitizer pass of the test suite).  Prints "ok <checksum>" and exits
 * 0 when every call returned; any sanitizer report aborts the run.
 *
 * Dump layout (little endian, written by tests/test_sanitizers_cpu.py):
 *   int32 nx, ny, nz; f64 dx, dy, dz, ox, oy, oz; f32 rho[nx ny nz]
 *   int32 n_beams; per beam: f64 gantry, couch, iso[3], sad; int32 nbx, nby;
 *                            f64 wx, wy, cx, cy
 *   13 tables (A, u1x, u1y, u2x, u2y, w1, w2, fu1, fu2, fw1, fw2, b1, b2):
 *       f64 start, step; int32 n, count; f32 v[count]
 *   int32 n_theta; f64 theta_step
 *   f64 roi_radius, rho_surface, smooth_sigma, rho_min, rho_max, sample_step;
 *   int32 dc_enabled, siddon
 *   int32 n_fluence; f32 fluence[n_fluence] */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/fspb_oracle.h"

static FILE* fp;
static void rd(void* p, size_t n) {
    if (fread(p, 1, n, fp) != n) {
        fprintf(stderr, "short dump\n");
        exit(2);
    }
}
static int rd_i32(void) { int v; rd(&v, 4); return v; }
static double rd_f64(void) { double v; rd(&v, 8); return v; }
static float* rd_f32s(long n) {
    float* v = (float*)malloc(sizeof(float) * (size_t)(n > 0 ? n : 1));
    rd(v, sizeof(float) * (size_t)n);
    return v;
}
static orc_table rd_table(float** keep) {
    orc_table t;
    t.start = rd_f64();
    t.step = rd_f64();
    t.n = rd_i32();
    const int count = rd_i32();
    *keep = rd_f32s(count);
    t.v = *keep;
    return t;
}

int main(int argc, char** argv) {
    if (argc != 2) return 2;
    fp = fopen(argv[1], "rb");
    if (!fp) return 2;
    orc_grid g;
    g.nx = rd_i32(); g.ny = rd_i32(); g.nz = rd_i32();
    g.dx = rd_f64(); g.dy = rd_f64(); g.dz = rd_f64();
    g.ox = rd_f64(); g.oy = rd_f64(); g.oz = rd_f64();
    const long nv = (long)g.nx * g.ny * g.nz;
    float* rho = rd_f32s(nv);
    g.rho = rho;
    const int nb = rd_i32();
    orc_beam* beams = (orc_beam*)calloc((size_t)nb, sizeof(orc_beam));
    for (int b = 0; b < nb; ++b) {
        beams[b].gantry = rd_f64(); beams[b].couch = rd_f64();
        for (int a = 0; a < 3; ++a) beams[b].iso[a] = rd_f64();
        beams[b].sad = rd_f64();
        beams[b].nbx = rd_i32(); beams[b].nby = rd_i32();
        beams[b].wx = rd_f64(); beams[b].wy = rd_f64();
        beams[b].cx = rd_f64(); beams[b].cy = rd_f64();
    }
    float* keep[13];
    orc_tables t;
    orc_table* slots[13] = {&t.A, &t.u1x, &t.u1y, &t.u2x, &t.u2y, &t.w1, &t.w2,
                            &t.fu1, &t.fu2, &t.fw1, &t.fw2, &t.b1, &t.b2};
    for (int k = 0; k < 13; ++k) *slots[k] = rd_table(&keep[k]);
    t.n_theta = rd_i32();
    t.theta_step = rd_f64();
    orc_options o;
    o.roi_radius = rd_f64(); o.rho_surface = rd_f64(); o.smooth_sigma = rd_f64();
    o.rho_min = rd_f64(); o.rho_max = rd_f64(); o.sample_step = rd_f64();
    o.dc_enabled = rd_i32(); o.siddon = rd_i32();
    const int nfl = rd_i32();
    float* fl = rd_f32s(nfl);
    fclose(fp);

    /* inputs the oracle must refuse */
    if (orc_create(NULL, nb, beams, &t, &o) != NULL) return 3;
    if (orc_create(&g, 0, beams, &t, &o) != NULL) return 3;

    double check = 0.0;
    for (int siddon = 0; siddon <= 1; ++siddon) {
        o.siddon = siddon;
        orc_ctx* c = orc_create(&g, nb, beams, &t, &o);
        if (!c) return 4;
        const int nbl = orc_n_beamlets(c);
        if (nbl != nfl) return 5;
        int r[3];
        orc_smooth_radius(c, r);
        double* buf = (double*)malloc(sizeof(double) * (size_t)nv);
        orc_smooth_all(c, buf);
        check += buf[nv / 2] + orc_smoothed_at(c, 0) + orc_smoothed_at(c, nv - 1);
        for (int i = 0; i < nbl; ++i) {
            double fr[16], info[10];
            orc_frame(c, i, fr);
            const int K = orc_trace(c, i, info, NULL, NULL, NULL, 0);
            if (K > 0) {
                double* T = (double*)malloc(sizeof(double) * (size_t)K);
                double* W1 = (double*)malloc(sizeof(double) * (size_t)K);
                double* W2 = (double*)malloc(sizeof(double) * (size_t)K);
                orc_trace(c, i, info, T, W1, W2, K);
                check += T[K - 1] + W1[K - 1] + W2[K - 1];
                free(T); free(W1); free(W2);
            }
            if (siddon) {
                const int Ks = orc_trace_siddon(c, i, NULL, NULL, NULL, NULL, NULL, 0);
                if (Ks > 0) {
                    double* a[5];
                    for (int q = 0; q < 5; ++q) a[q] = (double*)malloc(sizeof(double) * (size_t)Ks);
                    orc_trace_siddon(c, i, a[0], a[1], a[2], a[3], a[4], Ks);
                    check += a[1][Ks - 1];
                    for (int q = 0; q < 5; ++q) free(a[q]);
                }
            }
            float pc[12];
            orc_pair_consts(c, i, pc);
            check += pc[3];
        }
        /* dose, adjoint and counts over the whole grid / every beamlet */
        double* amb = (double*)malloc(sizeof(double) * (size_t)nv);
        long long* pairs = (long long*)malloc(sizeof(long long) * (size_t)nv);
        orc_dose(c, fl, nv, NULL, buf, amb, pairs);
        check += buf[nv / 3] + (double)pairs[nv / 3];
        long vox[3] = {0, nv / 2, nv - 1};
        orc_dose(c, fl, 3, vox, buf, amb, pairs);
        float* w = (float*)malloc(sizeof(float) * (size_t)nv);
        for (long v = 0; v < nv; ++v) w[v] = (float)((v % 7) * 0.125);
        double* gr = (double*)malloc(sizeof(double) * (size_t)nbl);
        double* gamb = (double*)malloc(sizeof(double) * (size_t)nbl);
        if (!siddon) {
            orc_adjoint(c, w, nbl, NULL, gr, gamb);
            check += gr[nbl / 2];
            int list[2] = {0, nbl - 1};
            orc_adjoint(c, w, 2, list, gr, gamb);
        }
        int* cnt = (int*)malloc(sizeof(int) * (size_t)nv);
        orc_pair_counts(c, nv, NULL, cnt);
        long long* bc = (long long*)malloc(sizeof(long long) * (size_t)nbl);
        orc_beamlet_pair_counts(c, nbl, NULL, bc);
        check += (double)cnt[nv / 2] + (double)bc[0];
        for (int i = 0; i < nbl; i += 7) {
            int flags = 0;
            check += orc_pair(c, nv / 2, i, &flags);
        }
        /* the surrogate support functions */
        if (!siddon && o.dc_enabled) {
            const double p_out[3] = {1e3, -1e3, 0.5};
            check += orc_density_at(c, p_out);
            for (long v = 0; v < nv; v += nv / 17 + 1) {
                for (int b = 0; b < nb; ++b) {
                    double tie = 0.0, feat[202], prm[6];
                    int ambf = 0, flags = 0;
                    const int i = orc_nearest_beamlet(c, v, b, &tie);
                    const int ok = orc_surrogate_row(c, v, b, feat, &ambf);
                    if (i >= 0 && orc_params(c, v, i, prm)) {
                        check += orc_pair_given(c, v, i, prm, &flags);
                    }
                    if (ok >= 0) check += feat[201];
                }
            }
        }
        if (!siddon) {
            /* every row falls back: the method's own parameters */
            double* prm = (double*)calloc((size_t)3 * nb * 7, sizeof(double));
            for (int q = 0; q < 3 * nb; ++q) prm[7 * q + 6] = 1.0;
            orc_dose_given(c, fl, 3, vox, prm, buf, amb);
            check += buf[1];
            free(prm);
        }
        free(buf); free(amb); free(pairs); free(w); free(gr); free(gamb); free(cnt); free(bc);
        orc_destroy(c);
    }
    for (int k = 0; k < 13; ++k) free(keep[k]);
    free(rho); free(beams); free(fl);
    printf("ok %.17g\n", check);
    return 0;
}
