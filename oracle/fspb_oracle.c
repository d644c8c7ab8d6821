/*
 * fspb_oracle.c -- plain FP64 CPU oracle of DC-FSPB.
 *
 * TEST INFRASTRUCTURE ONLY (see fspb_oracle.h).  Slow on purpose: every step
 * follows the paper's definitions in their own order, with no blocking,
 * fusion or reordering, so that it can be read against the paper.
 *
 * Readings of points the paper leaves open are marked "reading:".
 */
#include "fspb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double src[3], d[3], ex[3], ey[3];
    double theta, x0, y0, sad;
    int beam;
} frame_t;

typedef struct {
    double src[3], cax[3], ex[3], ey[3];
    double sad, a0, b0, wx, wy;
    int nbx, nby, first;
} beam_t;

typedef struct {
    int hit;
    double s_in, s_out, s_entry, s_exit, amb_rho, step;
    int k_entry, n_samples, K;
    double *T, *W1, *W2;
    /* Siddon tables (siddon mode): segment starts and integrals */
    int Ks;
    double *st, *sT, *sW1, *sW2, *srho, *sb1, *sb2;
} trace_t;

/* The pair test's single-precision constants of one beamlet (see
 * pair_counted): t = q.a + c over the voxel centre q relative to the grid
 * centre, for the depth (t), and the two lateral offsets (x, y). */
typedef struct {
    float t[4], x[4], y[4];
} pair32_t;

struct orc_ctx {
    orc_grid g;
    orc_tables tab;
    orc_options opt;
    int n_beams, n_beamlets;
    frame_t* fr;
    trace_t* tr;
    beam_t* bm;
    pair32_t* p32;     /* per beamlet */
    float q0[3], d32[3], R2f;   /* voxel (0,0,0) relative to the grid centre, spacing, R^2 */
    int rad[3];
    double* wts;      /* normalised 3D smoothing weights, [2rz+1][2ry+1][2rx+1] */
};

static void build_pair32(orc_ctx* c);

/* ------------------------------------------------------------------ */
/* small vector helpers                                                 */
static double dot3(const double* a, const double* b) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }
static void normalize3(double* a) {
    double n = sqrt(dot3(a, a));
    a[0] /= n; a[1] /= n; a[2] /= n;
}
static void cross3(const double* a, const double* b, double* c) {
    c[0] = a[1]*b[2] - a[2]*b[1];
    c[1] = a[2]*b[0] - a[0]*b[2];
    c[2] = a[0]*b[1] - a[1]*b[0];
}
static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
static double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Linear interpolation in a uniformly sampled table, coordinate clamped to
 * the table range (reading: lookups outside a table hold its end value). */
static double lerp_table(const orc_table* t, double x) {
    if (t->n == 1) return t->v[0];
    double c = clampd((x - t->start) / t->step, 0.0, (double)(t->n - 1));
    int i = (int)floor(c);
    if (i > t->n - 2) i = t->n - 2;
    double f = c - i;
    return (1.0 - f) * t->v[i] + f * t->v[i + 1];
}

/* Same for a table held in doubles (per-beamlet depth tables). */
static double lerp_array(const double* v, int n, double c) {
    if (n == 1) return v[0];
    c = clampd(c, 0.0, (double)(n - 1));
    int i = (int)floor(c);
    if (i > n - 2) i = n - 2;
    double f = c - i;
    return (1.0 - f) * v[i] + f * v[i + 1];
}

/* Bilinear A(t_eq, theta): rows are theta, columns radiological depth. */
static double lookup_A(const orc_tables* tb, double teq, double theta) {
    int nt = tb->A.n, nth = tb->n_theta;
    double cr = clampd(theta / tb->theta_step, 0.0, (double)(nth - 1));
    int r = (int)floor(cr);
    if (r > nth - 2) r = nth - 2;
    if (r < 0) r = 0;
    double fr = (nth == 1) ? 0.0 : cr - r;
    orc_table row0 = tb->A, row1 = tb->A;
    row0.v = tb->A.v + (size_t)r * nt;
    row1.v = tb->A.v + (size_t)(nth == 1 ? r : r + 1) * nt;
    double a0 = lerp_table(&row0, teq), a1 = lerp_table(&row1, teq);
    return (1.0 - fr) * a0 + fr * a1;
}

/* ------------------------------------------------------------------ */
/* Eq. 4: penumbra profile of a beamlet of half-width x0 (reading: x0 is the
 * half width, so adjacent beamlets at pitch 2 x0 tile the field). */
double orc_p(double x, double u, double x0) {
    if (x < -x0) return sinh(u * x0) * exp(u * x);
    if (x > x0)  return sinh(u * x0) * exp(-u * x);
    return 1.0 - cosh(u * x) * exp(-u * x0);
}

/* ------------------------------------------------------------------ */
/* Algorithm A1 step 3 and the Eq. 2 geometry: source, beamlet direction,
 * off-axis angle theta, and the beamlet's own lateral axes.
 * Conventions: gantry rotates about z; at gantry 0 the source is at
 * iso - SAD*(0,1,0).  The couch rotates the beam about the y axis.
 * reading: the lateral axes of a beamlet are the beam's x axis made
 * orthogonal to the beamlet direction, and y = x cross direction. */
static void rot_couch(double psi, const double* a, double* b) {
    double c = cos(psi), s = sin(psi);
    b[0] = c * a[0] + s * a[2];
    b[1] = a[1];
    b[2] = -s * a[0] + c * a[2];
}

static void build_frames(orc_ctx* c, const orc_beam* beams) {
    int i = 0;
    for (int b = 0; b < c->n_beams; ++b) {
        const orc_beam* bm = &beams[b];
        double phi = bm->gantry;
        double c0[3] = {-sin(phi), cos(phi), 0.0}, ex0[3] = {cos(phi), sin(phi), 0.0},
               ey0[3] = {0.0, 0.0, 1.0};
        double cax[3], ex[3], ey[3];
        rot_couch(bm->couch, c0, cax);
        rot_couch(bm->couch, ex0, ex);
        rot_couch(bm->couch, ey0, ey);
        double src[3];
        for (int k = 0; k < 3; ++k) src[k] = bm->iso[k] - bm->sad * cax[k];
        beam_t* B = &c->bm[b];
        memcpy(B->src, src, sizeof src);
        memcpy(B->cax, cax, sizeof cax);
        memcpy(B->ex, ex, sizeof ex);
        memcpy(B->ey, ey, sizeof ey);
        B->sad = bm->sad;
        B->wx = bm->wx;
        B->wy = bm->wy;
        B->a0 = -0.5 * (bm->nbx - 1) * bm->wx + bm->cx;
        B->b0 = -0.5 * (bm->nby - 1) * bm->wy + bm->cy;
        B->nbx = bm->nbx;
        B->nby = bm->nby;
        B->first = i;
        for (int n = 0; n < bm->nby; ++n) {
            for (int m = 0; m < bm->nbx; ++m, ++i) {
                frame_t* f = &c->fr[i];
                double a = (m - 0.5 * (bm->nbx - 1)) * bm->wx + bm->cx;
                double bb = (n - 0.5 * (bm->nby - 1)) * bm->wy + bm->cy;
                double d[3];
                for (int k = 0; k < 3; ++k) d[k] = bm->sad * cax[k] + a * ex[k] + bb * ey[k];
                normalize3(d);
                double exi[3], eyi[3];
                double pr = dot3(ex, d);
                for (int k = 0; k < 3; ++k) exi[k] = ex[k] - pr * d[k];
                normalize3(exi);
                cross3(exi, d, eyi);
                memcpy(f->src, src, sizeof src);
                memcpy(f->d, d, sizeof d);
                memcpy(f->ex, exi, sizeof exi);
                memcpy(f->ey, eyi, sizeof eyi);
                f->theta = atan(sqrt(a * a + bb * bb) / bm->sad);
                f->x0 = 0.5 * bm->wx;
                f->y0 = 0.5 * bm->wy;
                f->sad = bm->sad;
                f->beam = b;
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Density at a point: trilinear between voxel centres, indices clamped to
 * the grid (clamp-to-edge outside the outermost centres). */
static double rho_at_voxel(const orc_grid* g, int i, int j, int k) {
    return g->rho[((size_t)k * g->ny + j) * g->nx + i];
}

static double trilinear(const orc_grid* g, const double* p) {
    double gx = (p[0] - g->ox) / g->dx, gy = (p[1] - g->oy) / g->dy, gz = (p[2] - g->oz) / g->dz;
    int ix = (int)floor(gx), iy = (int)floor(gy), iz = (int)floor(gz);
    double fx = gx - ix, fy = gy - iy, fz = gz - iz;
    double acc = 0.0;
    for (int c = 0; c < 8; ++c) {
        int ox = c & 1, oy = (c >> 1) & 1, oz = (c >> 2) & 1;
        double w = (ox ? fx : 1.0 - fx) * (oy ? fy : 1.0 - fy) * (oz ? fz : 1.0 - fz);
        acc += w * rho_at_voxel(g, clampi(ix + ox, 0, g->nx - 1), clampi(iy + oy, 0, g->ny - 1),
                                clampi(iz + oz, 0, g->nz - 1));
    }
    return acc;
}

/* ------------------------------------------------------------------ */
/* Algorithm A1 steps 4-6 with the uniform sampling of Section 2.2.
 * The beamlet axis r_s + s d is clipped to the grid box; samples sit at
 * s_k = s_in + k d with d = sample step (default half the smallest voxel).
 * reading: the body surface (entrance point) is the first sample whose
 *   density reaches rho_surface; the exit is the last such sample.
 * reading: mu/mu_water is taken as the relative density, and the integrals
 *   t_eq = int rho dt' and omega_corr_c = int b_c(rho) dt' are trapezoid sums
 *   over the samples starting at the entrance.
 * reading: the tables run from the entrance until they cover the deepest
 *   point of the grid box along the axis plus one sample, so every voxel
 *   centre's depth interpolates between two samples; samples beyond the box
 *   see the clamp-to-edge density. */
static void trace_beamlet(orc_ctx* c, int i) {
    const orc_grid* g = &c->g;
    frame_t* f = &c->fr[i];
    trace_t* t = &c->tr[i];
    memset(t, 0, sizeof *t);
    double lo[3] = {g->ox - 0.5 * g->dx, g->oy - 0.5 * g->dy, g->oz - 0.5 * g->dz};
    double hi[3] = {g->ox + (g->nx - 0.5) * g->dx, g->oy + (g->ny - 0.5) * g->dy,
                    g->oz + (g->nz - 0.5) * g->dz};
    double s_in = -1e300, s_out = 1e300;
    for (int a = 0; a < 3; ++a) {
        if (f->d[a] == 0.0) {
            if (f->src[a] < lo[a] || f->src[a] > hi[a]) return;  /* misses the box */
            continue;
        }
        double t1 = (lo[a] - f->src[a]) / f->d[a], t2 = (hi[a] - f->src[a]) / f->d[a];
        double tmin = t1 < t2 ? t1 : t2, tmax = t1 < t2 ? t2 : t1;
        if (tmin > s_in) s_in = tmin;
        if (tmax < s_out) s_out = tmax;
    }
    if (s_in < 0.0) s_in = 0.0;
    if (!(s_in < s_out)) return;
    double s_cover = -1e300;
    for (int k = 0; k < 8; ++k) {
        double p[3] = {(k & 1) ? hi[0] : lo[0], (k & 2) ? hi[1] : lo[1], (k & 4) ? hi[2] : lo[2]};
        double v[3] = {p[0] - f->src[0], p[1] - f->src[1], p[2] - f->src[2]};
        double s = dot3(v, f->d);
        if (s > s_cover) s_cover = s;
    }
    double d = c->opt.sample_step;
    int N = (int)floor((s_cover - s_in) / d) + 2;
    double* rho = (double*)malloc(sizeof(double) * N);
    for (int k = 0; k < N; ++k) {
        double s = s_in + k * d;
        double p[3] = {f->src[0] + s * f->d[0], f->src[1] + s * f->d[1], f->src[2] + s * f->d[2]};
        rho[k] = trilinear(g, p);
    }
    int ke = -1, kx = -1;
    double amb = 1e300;
    for (int k = 0; k < N; ++k) {
        double m = fabs(rho[k] - c->opt.rho_surface);
        if (ke < 0 && m < amb) amb = m;
        if (rho[k] >= c->opt.rho_surface) {
            if (ke < 0) ke = k;
            kx = k;
        }
    }
    t->s_in = s_in;
    t->s_out = s_out;
    t->step = d;
    t->n_samples = N;
    t->amb_rho = amb;
    if (ke < 0) { free(rho); return; }
    t->hit = 1;
    t->k_entry = ke;
    t->s_entry = s_in + ke * d;
    t->s_exit = s_in + kx * d;
    int K = N - ke;
    t->K = K;
    t->T = (double*)malloc(sizeof(double) * K);
    t->W1 = (double*)malloc(sizeof(double) * K);
    t->W2 = (double*)malloc(sizeof(double) * K);
    t->T[0] = t->W1[0] = t->W2[0] = 0.0;
    for (int j = 1; j < K; ++j) {
        double ra = rho[ke + j - 1], rb = rho[ke + j];
        double rca = clampd(ra, c->opt.rho_min, c->opt.rho_max);
        double rcb = clampd(rb, c->opt.rho_min, c->opt.rho_max);
        t->T[j] = t->T[j - 1] + d * 0.5 * (ra + rb);
        t->W1[j] = t->W1[j - 1] + d * 0.5 * (lerp_table(&c->tab.b1, rca) + lerp_table(&c->tab.b1, rcb));
        t->W2[j] = t->W2[j - 1] + d * 0.5 * (lerp_table(&c->tab.b2, rca) + lerp_table(&c->tab.b2, rcb));
    }
    free(rho);
}

/* ------------------------------------------------------------------ */
/* Siddon's exact radiological path (the alternative Section 2.2 sets
 * aside): the density is constant inside each voxel, the axis is cut at
 * every voxel-boundary plane it crosses inside the grid box, and each
 * segment contributes density x length.  The crossing depths are sorted and
 * each segment's voxel is the one holding its midpoint.
 * reading: the entrance is the start of the first segment whose voxel
 *   density reaches rho_surface; past the box exit the last segment's
 *   density continues (the analogue of clamp-to-edge). */
static int cmp_double(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

static void trace_siddon(orc_ctx* c, int i) {
    const orc_grid* g = &c->g;
    const frame_t* f = &c->fr[i];
    trace_t* t = &c->tr[i];
    t->Ks = 0;
    t->hit = 0;
    double lo[3] = {g->ox - 0.5 * g->dx, g->oy - 0.5 * g->dy, g->oz - 0.5 * g->dz};
    double del[3] = {g->dx, g->dy, g->dz};
    int n[3] = {g->nx, g->ny, g->nz};
    double s_in = t->s_in, s_out = t->s_out;
    if (!(s_in < s_out)) return;
    int cap = 2 + n[0] + n[1] + n[2] + 3;
    double* cut = (double*)malloc(sizeof(double) * cap);
    int nc = 0;
    cut[nc++] = s_in;
    for (int a = 0; a < 3; ++a) {
        if (f->d[a] == 0.0) continue;
        for (int m = 0; m <= n[a]; ++m) {
            double s = (lo[a] + m * del[a] - f->src[a]) / f->d[a];
            if (s > s_in && s < s_out) cut[nc++] = s;
        }
    }
    cut[nc++] = s_out;
    qsort(cut, nc, sizeof(double), cmp_double);
    /* segments with their voxel density */
    double* seg_s = (double*)malloc(sizeof(double) * nc);
    double* seg_r = (double*)malloc(sizeof(double) * nc);
    int ns = 0;
    for (int k = 0; k + 1 < nc; ++k) {
        if (!(cut[k + 1] > cut[k])) continue;            /* zero-length: an edge or corner */
        double mid = 0.5 * (cut[k] + cut[k + 1]);
        int idx[3];
        for (int a = 0; a < 3; ++a)
            idx[a] = clampi((int)floor((f->src[a] + mid * f->d[a] - lo[a]) / del[a]), 0, n[a] - 1);
        seg_s[ns] = cut[k];
        seg_r[ns] = rho_at_voxel(g, idx[0], idx[1], idx[2]);
        ++ns;
    }
    int e = -1;
    for (int k = 0; k < ns && e < 0; ++k)
        if (seg_r[k] >= c->opt.rho_surface) e = k;
    if (e >= 0) {
        int K = ns - e;
        t->hit = 1;
        t->s_entry = seg_s[e];
        t->Ks = K;
        t->st = (double*)malloc(sizeof(double) * K);
        t->sT = (double*)malloc(sizeof(double) * K);
        t->sW1 = (double*)malloc(sizeof(double) * K);
        t->sW2 = (double*)malloc(sizeof(double) * K);
        t->srho = (double*)malloc(sizeof(double) * K);
        t->sb1 = (double*)malloc(sizeof(double) * K);
        t->sb2 = (double*)malloc(sizeof(double) * K);
        double T = 0.0, W1 = 0.0, W2 = 0.0;
        for (int k = 0; k < K; ++k) {
            double r = seg_r[e + k], rc = clampd(r, c->opt.rho_min, c->opt.rho_max);
            t->st[k] = seg_s[e + k] - t->s_entry;
            t->sT[k] = T;
            t->sW1[k] = W1;
            t->sW2[k] = W2;
            t->srho[k] = r;
            t->sb1[k] = lerp_table(&c->tab.b1, rc);
            t->sb2[k] = lerp_table(&c->tab.b2, rc);
            double len = (k + 1 < K ? seg_s[e + k + 1] : s_out) - seg_s[e + k];
            T += r * len;
            W1 += t->sb1[k] * len;
            W2 += t->sb2[k] * len;
        }
    }
    free(cut);
    free(seg_s);
    free(seg_r);
}

/* Integral at depth t >= 0 from Siddon segment tables: the last segment
 * starting at or before t, then linear inside it. */
static double siddon_at(const double* st, const double* v, const double* slope, int K, double t) {
    int lo = 0, hi = K - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (st[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return v[lo] + slope[lo] * (t - st[lo]);
}

int orc_trace_siddon(const orc_ctx* c, int i, double* t, double* T, double* W1, double* W2,
                     double* rho, int maxK) {
    const trace_t* tr = &c->tr[i];
    int n = tr->Ks < maxK ? tr->Ks : maxK;
    for (int k = 0; k < n; ++k) {
        if (t) t[k] = tr->st[k];
        if (T) T[k] = tr->sT[k];
        if (W1) W1[k] = tr->sW1[k];
        if (W2) W2[k] = tr->sW2[k];
        if (rho) rho[k] = tr->srho[k];
    }
    return tr->Ks;
}

/* ------------------------------------------------------------------ */
/* Algorithm A1 step 1: smoothed density = density convolved with a 3D
 * Gaussian.  reading: width smooth_sigma, truncated to a cube of
 * ceil(3 sigma / delta) voxels per axis, weights normalised to sum 1,
 * clamp-to-edge beyond the grid. */
static void build_weights(orc_ctx* c) {
    double del[3] = {c->g.dx, c->g.dy, c->g.dz};
    double s = c->opt.smooth_sigma;
    for (int a = 0; a < 3; ++a) c->rad[a] = s > 0.0 ? (int)ceil(3.0 * s / del[a] - 1e-6) : 0;
    int nx = 2 * c->rad[0] + 1, ny = 2 * c->rad[1] + 1, nz = 2 * c->rad[2] + 1;
    c->wts = (double*)malloc(sizeof(double) * nx * ny * nz);
    double sum = 0.0;
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                double x = (i - c->rad[0]) * del[0], y = (j - c->rad[1]) * del[1],
                       z = (k - c->rad[2]) * del[2];
                double w = s > 0.0 ? exp(-(x * x + y * y + z * z) / (2.0 * s * s)) : 1.0;
                c->wts[((size_t)k * ny + j) * nx + i] = w;
                sum += w;
            }
    for (int q = 0; q < nx * ny * nz; ++q) c->wts[q] /= sum;
}

double orc_smoothed_at(const orc_ctx* c, long vox) {
    const orc_grid* g = &c->g;
    int i = (int)(vox % g->nx), j = (int)((vox / g->nx) % g->ny), k = (int)(vox / ((long)g->nx * g->ny));
    int rx = c->rad[0], ry = c->rad[1], rz = c->rad[2];
    int nx = 2 * rx + 1, ny = 2 * ry + 1;
    double acc = 0.0;
    for (int dk = -rz; dk <= rz; ++dk)
        for (int dj = -ry; dj <= ry; ++dj)
            for (int di = -rx; di <= rx; ++di) {
                double w = c->wts[((size_t)(dk + rz) * ny + (dj + ry)) * nx + (di + rx)];
                acc += w * rho_at_voxel(g, clampi(i + di, 0, g->nx - 1), clampi(j + dj, 0, g->ny - 1),
                                        clampi(k + dk, 0, g->nz - 1));
            }
    return acc;
}

void orc_smooth_all(const orc_ctx* c, double* out) {
    long n = (long)c->g.nx * c->g.ny * c->g.nz;
#pragma omp parallel for schedule(dynamic, 256)
    for (long v = 0; v < n; ++v) out[v] = orc_smoothed_at(c, v);
}

void orc_smooth_radius(const orc_ctx* c, int r[3]) { r[0] = c->rad[0]; r[1] = c->rad[1]; r[2] = c->rad[2]; }

/* ------------------------------------------------------------------ */
orc_ctx* orc_create(const orc_grid* g, int n_beams, const orc_beam* beams,
                    const orc_tables* tab, const orc_options* opt) {
    if (!g || !beams || !tab || !opt || n_beams <= 0 || g->nx <= 0 || g->ny <= 0 || g->nz <= 0)
        return NULL;
    orc_ctx* c = (orc_ctx*)calloc(1, sizeof *c);
    c->g = *g;
    c->tab = *tab;
    c->opt = *opt;
    if (c->opt.sample_step <= 0.0) {
        double m = g->dx < g->dy ? g->dx : g->dy;
        if (g->dz < m) m = g->dz;
        c->opt.sample_step = 0.5 * m;   /* Section 2.2: d = min(delta)/2 */
    }
    c->n_beams = n_beams;
    for (int b = 0; b < n_beams; ++b) c->n_beamlets += beams[b].nbx * beams[b].nby;
    c->fr = (frame_t*)calloc(c->n_beamlets, sizeof(frame_t));
    c->tr = (trace_t*)calloc(c->n_beamlets, sizeof(trace_t));
    c->bm = (beam_t*)calloc(n_beams, sizeof(beam_t));
    build_frames(c, beams);
#pragma omp parallel for schedule(dynamic, 1)
    for (int i = 0; i < c->n_beamlets; ++i) {
        trace_beamlet(c, i);
        if (c->opt.siddon) trace_siddon(c, i);
    }
    build_weights(c);
    build_pair32(c);
    return c;
}

void orc_destroy(orc_ctx* c) {
    if (!c) return;
    for (int i = 0; i < c->n_beamlets; ++i) {
        free(c->tr[i].T);
        free(c->tr[i].W1);
        free(c->tr[i].W2);
        free(c->tr[i].st);
        free(c->tr[i].sT);
        free(c->tr[i].sW1);
        free(c->tr[i].sW2);
        free(c->tr[i].srho);
        free(c->tr[i].sb1);
        free(c->tr[i].sb2);
    }
    free(c->tr);
    free(c->fr);
    free(c->bm);
    free(c->p32);
    free(c->wts);
    free(c);
}

int orc_n_beamlets(const orc_ctx* c) { return c->n_beamlets; }

void orc_frame(const orc_ctx* c, int i, double out[16]) {
    const frame_t* f = &c->fr[i];
    for (int k = 0; k < 3; ++k) {
        out[k] = f->src[k];
        out[3 + k] = f->d[k];
        out[6 + k] = f->ex[k];
        out[9 + k] = f->ey[k];
    }
    out[12] = f->theta;
    out[13] = f->x0;
    out[14] = f->y0;
    out[15] = f->sad;
}

int orc_trace(const orc_ctx* c, int i, double info[10], double* T, double* W1, double* W2, int maxK) {
    const trace_t* t = &c->tr[i];
    info[0] = t->hit;
    info[1] = t->s_in;
    info[2] = t->s_out;
    info[3] = t->s_entry;
    info[4] = t->k_entry;
    info[5] = t->K;
    info[6] = t->s_exit;
    info[7] = t->amb_rho;
    info[8] = t->step;
    info[9] = t->n_samples;
    int n = t->K < maxK ? t->K : maxK;
    for (int j = 0; j < n; ++j) {
        if (T) T[j] = t->T[j];
        if (W1) W1[j] = t->W1[j];
        if (W2) W2[j] = t->W2[j];
    }
    return t->K;
}

static void voxel_center(const orc_grid* g, long vox, double* r) {
    int i = (int)(vox % g->nx), j = (int)((vox / g->nx) % g->ny), k = (int)(vox / ((long)g->nx * g->ny));
    r[0] = g->ox + i * g->dx;
    r[1] = g->oy + j * g->dy;
    r[2] = g->oz + k * g->dz;
}

/* ------------------------------------------------------------------ */
/* The pair test of Algorithm A1 step 8: the voxel lies inside the ROI
 * cylinder (distance from the beamlet axis at most R, inclusive) and below
 * the entrance (t >= 0).  Its outcome is discrete, so near the cylinder
 * surface and the entrance plane the precision of the arithmetic decides it.
 * reading: the test is taken in single precision, the precision of the
 * method's GPU implementation, by this recipe.  With P0 the grid centre
 * (o + (n - 1) delta / 2, in double), the voxel centre relative to P0 is
 * q_a = fma(index_a, (float)delta_a, (float)(o_a - P0_a)); each beamlet
 * holds, rounded to single precision from double, its direction d, lateral
 * axes ex, ey and the offsets c_t = (P0 - r_s).d - s_entry,
 * c_x = (P0 - r_s).ex, c_y = (P0 - r_s).ey; then
 *   t  = fma(q_x, d_x, fma(q_y, d_y, fma(q_z, d_z, c_t)))   (xp, yp alike)
 * and the pair counts iff t >= 0 and fma(xp, xp, yp * yp) <= R * R (all
 * single precision, fma rounded once).  Everything else about the pair is
 * computed in double. */
static void build_pair32(orc_ctx* c) {
    const orc_grid* g = &c->g;
    const int n[3] = {g->nx, g->ny, g->nz};
    const double o[3] = {g->ox, g->oy, g->oz}, del[3] = {g->dx, g->dy, g->dz};
    double P0[3];
    for (int a = 0; a < 3; ++a) {
        P0[a] = o[a] + 0.5 * (n[a] - 1) * del[a];
        c->q0[a] = (float)(o[a] - P0[a]);
        c->d32[a] = (float)del[a];
    }
    const float Rf = (float)c->opt.roi_radius;
    c->R2f = Rf * Rf;
    c->p32 = (pair32_t*)calloc(c->n_beamlets, sizeof(pair32_t));
    for (int i = 0; i < c->n_beamlets; ++i) {
        const frame_t* f = &c->fr[i];
        double v0[3] = {P0[0] - f->src[0], P0[1] - f->src[1], P0[2] - f->src[2]};
        pair32_t* p = &c->p32[i];
        for (int a = 0; a < 3; ++a) {
            p->t[a] = (float)f->d[a];
            p->x[a] = (float)f->ex[a];
            p->y[a] = (float)f->ey[a];
        }
        p->t[3] = (float)(dot3(v0, f->d) - c->tr[i].s_entry);
        p->x[3] = (float)dot3(v0, f->ex);
        p->y[3] = (float)dot3(v0, f->ey);
    }
}

static int pair_counted(const orc_ctx* c, long vox, int i) {
    const orc_grid* g = &c->g;
    const int idx[3] = {(int)(vox % g->nx), (int)((vox / g->nx) % g->ny),
                        (int)(vox / ((long)g->nx * g->ny))};
    float q[3];
    for (int a = 0; a < 3; ++a) q[a] = fmaf((float)idx[a], c->d32[a], c->q0[a]);
    const pair32_t* p = &c->p32[i];
    const float t = fmaf(q[0], p->t[0], fmaf(q[1], p->t[1], fmaf(q[2], p->t[2], p->t[3])));
    const float xp = fmaf(q[0], p->x[0], fmaf(q[1], p->x[1], fmaf(q[2], p->x[2], p->x[3])));
    const float yp = fmaf(q[0], p->y[0], fmaf(q[1], p->y[1], fmaf(q[2], p->y[2], p->y[3])));
    const float yy = yp * yp;
    return t >= 0.0f && fmaf(xp, xp, yy) <= c->R2f;
}

/* Eqs. 2-4 for one (voxel, beamlet) pair, Algorithm A1 steps 8-12.
 * x and y are the lateral offsets of the voxel from the beamlet axis scaled
 * to the isocentre plane by SAD/|r_a| (reading), |r_a| is the distance along
 * the beamlet direction, t = |r_a| - s_entry is the depth below the surface.
 * rho_c and rhohat_c are the voxel's density and smoothed density clamped to
 * the commissioned range (reading).  flags: bit 0 = the pair counts. */
static double pair_value(const orc_ctx* c, long vox, int i, double rho_c, double rhohat_c,
                         int* flags, const double* given, double* params) {
    const frame_t* f = &c->fr[i];
    const trace_t* t = &c->tr[i];
    const orc_tables* tb = &c->tab;
    *flags = 0;
    if (!t->hit) return 0.0;
    if (!pair_counted(c, vox, i)) return 0.0;
    double r[3];
    voxel_center(&c->g, vox, r);
    double v[3] = {r[0] - f->src[0], r[1] - f->src[1], r[2] - f->src[2]};
    double s = dot3(v, f->d);
    double xp = dot3(v, f->ex), yp = dot3(v, f->ey);
    double depth = s - t->s_entry;
    if (s <= 0.0) return 0.0;
    *flags = 1;

    double mag = f->sad / s;
    double x = xp * mag, y = yp * mag;
    double isq = mag * mag;
    double ci = depth / t->step;
    const int sid = c->opt.siddon;
    double teq = sid ? siddon_at(t->st, t->sT, t->srho, t->Ks, depth) : lerp_array(t->T, t->K, ci);
    double A = lookup_A(tb, teq, f->theta);
    double u1x = lerp_table(&tb->u1x, depth), u1y = lerp_table(&tb->u1y, depth);
    double u2x = lerp_table(&tb->u2x, depth), u2y = lerp_table(&tb->u2y, depth);
    double w1 = lerp_table(&tb->w1, depth), w2 = lerp_table(&tb->w2, depth);
    if (c->opt.dc_enabled) {
        /* Section 2.1 density corrections (Algorithm A1 step 11). */
        double fu1 = lerp_table(&tb->fu1, rho_c), fu2 = lerp_table(&tb->fu2, rhohat_c);
        double fw1 = lerp_table(&tb->fw1, rhohat_c), fw2 = lerp_table(&tb->fw2, rhohat_c);
        u1x *= fu1;
        u1y *= fu1;
        u2x *= fu2;
        u2y *= fu2;
        w1 = fw1 * (w1 + (sid ? siddon_at(t->st, t->sW1, t->sb1, t->Ks, depth)
                              : lerp_array(t->W1, t->K, ci)));
        w2 = fw2 * (w2 + (sid ? siddon_at(t->st, t->sW2, t->sb2, t->Ks, depth)
                              : lerp_array(t->W2, t->K, ci)));
        if (w1 < 0.0) w1 = 0.0;   /* reading: weights cannot go negative */
        if (w2 < 0.0) w2 = 0.0;
    }
    if (given) {
        /* surrogate: the six parameters come from outside (per voxel and
         * beam); depth, t_eq, A and the inverse square stay per beamlet */
        u1x = given[0];
        u1y = given[1];
        u2x = given[2];
        u2y = given[3];
        w1 = given[4];
        w2 = given[5];
    }
    if (params) {
        params[0] = u1x;
        params[1] = u1y;
        params[2] = u2x;
        params[3] = u2y;
        params[4] = w1;
        params[5] = w2;
    }
    double F = w1 * orc_p(x, u1x, f->x0) * orc_p(y, u1y, f->y0)
             + w2 * orc_p(x, u2x, f->x0) * orc_p(y, u2y, f->y0);
    return F * A * isq;
}


static void voxel_densities(const orc_ctx* c, long vox, const double* rhohat_all, double* rc, double* rhc) {
    double rho = c->g.rho[vox];
    *rc = clampd(rho, c->opt.rho_min, c->opt.rho_max);
    *rhc = 1.0;
    if (c->opt.dc_enabled) {
        double rh = rhohat_all ? rhohat_all[vox] : orc_smoothed_at(c, vox);
        *rhc = clampd(rh, c->opt.rho_min, c->opt.rho_max);
    }
}

void orc_pair_consts(const orc_ctx* c, int i, float out[12]) {
    const pair32_t* p = &c->p32[i];
    for (int a = 0; a < 4; ++a) {
        out[a] = p->t[a];
        out[4 + a] = p->x[a];
        out[8 + a] = p->y[a];
    }
}

double orc_pair(const orc_ctx* c, long vox, int i, int* flags) {
    double r[3], rc, rhc;
    int fl;
    voxel_center(&c->g, vox, r);
    voxel_densities(c, vox, NULL, &rc, &rhc);
    double v = pair_value(c, vox, i, rc, rhc, &fl, NULL, NULL);
    if (flags) *flags = fl;
    return v;
}

/* Eq. 1: D(r) = sum_i f_i D_i(r), beamlets in their fixed (beam-major) order. */
void orc_dose(const orc_ctx* c, const float* fluence, long n, const long* vox,
              double* dose, double* amb, long long* pairs) {
#pragma omp parallel for schedule(dynamic, 64)
    for (long q = 0; q < n; ++q) {
        long v = vox ? vox[q] : q;
        double r[3], rc, rhc;
        voxel_center(&c->g, v, r);
        voxel_densities(c, v, NULL, &rc, &rhc);
        double acc = 0.0, a = 0.0;
        long long np = 0;
        for (int i = 0; i < c->n_beamlets; ++i) {
            if (fluence[i] == 0.0f) continue;
            int fl;
            double d = pair_value(c, v, i, rc, rhc, &fl, NULL, NULL);
            if (fl & 1) {
                acc += fluence[i] * d;
                ++np;
            }
            if (fl & 2) a += fabs(fluence[i] * d);
        }
        dose[q] = acc;
        if (amb) amb[q] = a;
        if (pairs) pairs[q] = np;
    }
}

/* Transpose of Eq. 1: g_i = sum_r w(r) D_i(r), voxels in index order. */
void orc_adjoint(const orc_ctx* c, const float* w, int n, const int* list, double* g, double* amb) {
    long nv = (long)c->g.nx * c->g.ny * c->g.nz;
    double* rh = NULL;
    if (c->opt.dc_enabled) {
        /* smoothed density wherever one of the listed beamlets reaches */
        rh = (double*)malloc(sizeof(double) * nv);
#pragma omp parallel for schedule(dynamic, 256)
        for (long v = 0; v < nv; ++v) {
            double r[3];
            voxel_center(&c->g, v, r);
            int need = 0;
            for (int q = 0; q < n && !need; ++q) {
                int fl;
                int i = list ? list[q] : q;
                pair_value(c, v, i, 1.0, 1.0, &fl, NULL, NULL);
                need = fl != 0;
            }
            rh[v] = need ? orc_smoothed_at(c, v) : 1.0;
        }
    }
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = 0; q < n; ++q) {
        int i = list ? list[q] : q;
        double acc = 0.0, a = 0.0;
        for (long v = 0; v < nv; ++v) {
            if (w[v] == 0.0f) continue;
            double r[3], rc, rhc;
            int fl;
            voxel_center(&c->g, v, r);
            voxel_densities(c, v, rh, &rc, &rhc);
            double d = pair_value(c, v, i, rc, rhc, &fl, NULL, NULL);
            if (fl & 1) acc += w[v] * d;
            if (fl & 2) a += fabs(w[v] * d);
        }
        g[q] = acc;
        if (amb) amb[q] = a;
    }
    free(rh);
}

void orc_pair_counts(const orc_ctx* c, long n, const long* vox, int* counts) {
#pragma omp parallel for schedule(dynamic, 64)
    for (long q = 0; q < n; ++q) {
        long v = vox ? vox[q] : q;
        double r[3];
        voxel_center(&c->g, v, r);
        int cnt = 0;
        for (int i = 0; i < c->n_beamlets; ++i) {
            int fl;
            pair_value(c, v, i, 1.0, 1.0, &fl, NULL, NULL);
            if (fl & 1) ++cnt;
        }
        counts[q] = cnt;
    }
}

/* Per beamlet: the number of voxels it is paired with (Algorithm A1 step 8,
 * the same pair test as orc_pair_counts, summed over voxels instead). */
void orc_beamlet_pair_counts(const orc_ctx* c, int n, const int* beamlets, long long* counts) {
    const long nv = (long)c->g.nx * c->g.ny * c->g.nz;
#pragma omp parallel for schedule(dynamic, 1)
    for (int q = 0; q < n; ++q) {
        const int i = beamlets ? beamlets[q] : q;
        long long cnt = 0;
        for (long v = 0; v < nv; ++v) {
            int fl;
            pair_value(c, v, i, 1.0, 1.0, &fl, NULL, NULL);
            if (fl & 1) ++cnt;
        }
        counts[q] = cnt;
    }
}

/* ------------------------------------------------------------------ */
/* Learned-surrogate support.  The surrogate is an extension beside the
 * method (not in the paper): for a (voxel, beam) row it predicts the six
 * Section 2.1 parameters (u1x, u1y, u2x, u2y, w1, w2) from a density patch.
 * The functions below define its inputs and training targets, and the dose
 * it produces, so that the tests can check the GPU's. */

double orc_density_at(const orc_ctx* c, const double p[3]) { return trilinear(&c->g, p); }

int orc_params(const orc_ctx* c, long vox, int i, double out[6]) {
    double r[3], rc, rhc;
    int fl;
    voxel_center(&c->g, vox, r);
    voxel_densities(c, vox, NULL, &rc, &rhc);
    for (int k = 0; k < 6; ++k) out[k] = 0.0;
    pair_value(c, vox, i, rc, rhc, &fl, NULL, out);
    return fl;
}

double orc_pair_given(const orc_ctx* c, long vox, int i, const double prm[6], int* flags) {
    double r[3];
    int fl;
    voxel_center(&c->g, vox, r);
    double v = pair_value(c, vox, i, 1.0, 1.0, &fl, prm, NULL);
    if (flags) *flags = fl;
    return v;
}

/* The beamlet of `beam` whose isocentre-plane centre lies nearest to the
 * voxel's central projection from the source (ties round up); -1 if the
 * voxel is not in front of the source.  *tie gets the distance of either
 * rounding decision from its tie, in beamlet widths. */
int orc_nearest_beamlet(const orc_ctx* c, long vox, int beam, double* tie) {
    const beam_t* B = &c->bm[beam];
    double r[3];
    voxel_center(&c->g, vox, r);
    double v[3] = {r[0] - B->src[0], r[1] - B->src[1], r[2] - B->src[2]};
    double z = dot3(v, B->cax);
    if (tie) *tie = 1.0;
    if (!(z > 0.0)) return -1;
    double a = B->sad * dot3(v, B->ex) / z, b = B->sad * dot3(v, B->ey) / z;
    double ga = (a - B->a0) / B->wx, gb = (b - B->b0) / B->wy;
    int m = clampi((int)floor(ga + 0.5), 0, B->nbx - 1);
    int n = clampi((int)floor(gb + 0.5), 0, B->nby - 1);
    if (tie) {
        double ta = fabs(ga - floor(ga) - 0.5), tb = fabs(gb - floor(gb) - 0.5);
        *tie = ta < tb ? ta : tb;
    }
    return B->first + n * B->nbx + m;
}

/* One surrogate input row for (voxel, beam).  The nearest beamlet i must
 * hit the body and its pair with the voxel must be counted (inside the ROI,
 * below the entrance); otherwise the row is invalid and -1 is returned.
 * Patch: along the ray from the source S to the voxel centre r (length L,
 * unit direction u), 8 planes at distances L - t (7 - k) / 7, k = 0..7,
 * from the depth of the entrance (t = the voxel's depth for beamlet i) to
 * the voxel; in each plane a 5 x 5 lattice at 0.5 cm along e1 and e2,
 * where e1 is the beam's lateral x axis made orthogonal to u and
 * e2 = e1 x u.  feat[25 k + 5 b + a] = trilinear density at
 * S + s_k u + 0.5 (a - 2) e1 + 0.5 (b - 2) e2;  feat[200] = t,
 * feat[201] = theta_i.  *amb gets 1 when the pair test of beamlet i lies
 * within the ambiguity tolerance of its boundary. */
int orc_surrogate_row(const orc_ctx* c, long vox, int beam, double feat[202], int* amb) {
    double tie;
    if (amb) *amb = 0;
    int i = orc_nearest_beamlet(c, vox, beam, &tie);
    if (i < 0) return -1;
    double prm[6];
    int fl = orc_params(c, vox, i, prm);
    if (amb) *amb = (fl & 2) ? 1 : 0;
    if (!(fl & 1)) return -1;
    const frame_t* f = &c->fr[i];
    const trace_t* tr = &c->tr[i];
    const beam_t* B = &c->bm[beam];
    double r[3];
    voxel_center(&c->g, vox, r);
    double v[3] = {r[0] - f->src[0], r[1] - f->src[1], r[2] - f->src[2]};
    double t = dot3(v, f->d) - tr->s_entry;
    double L = sqrt(dot3(v, v));
    double u[3] = {v[0] / L, v[1] / L, v[2] / L};
    double e1[3], e2[3];
    double pr = dot3(B->ex, u);
    for (int k = 0; k < 3; ++k) e1[k] = B->ex[k] - pr * u[k];
    normalize3(e1);
    cross3(e1, u, e2);
    for (int k = 0; k < 8; ++k) {
        double s = L - t * (7 - k) / 7.0;
        for (int b = 0; b < 5; ++b)
            for (int a = 0; a < 5; ++a) {
                double p[3];
                for (int q = 0; q < 3; ++q)
                    p[q] = f->src[q] + s * u[q] + 0.5 * (a - 2) * e1[q] + 0.5 * (b - 2) * e2[q];
                feat[25 * k + 5 * b + a] = trilinear(&c->g, p);
            }
    }
    feat[200] = t;
    feat[201] = f->theta;
    return i;
}

/* Dose with the surrogate's parameters: D(r) = sum_i f_i D_i(r) where each
 * pair takes the six parameters of its (voxel, beam) row,
 * prm[(q * n_beams + b) * 7 + 0..5], unless the row's fallback flag
 * prm[... + 6] is non-zero, in which case the pair is evaluated by the
 * method itself.  amb as for orc_dose. */
void orc_dose_given(const orc_ctx* c, const float* fluence, long n, const long* vox,
                    const double* prm, double* dose, double* amb) {
#pragma omp parallel for schedule(dynamic, 16)
    for (long q = 0; q < n; ++q) {
        long v = vox ? vox[q] : q;
        double r[3], rc, rhc;
        voxel_center(&c->g, v, r);
        voxel_densities(c, v, NULL, &rc, &rhc);
        double acc = 0.0, a = 0.0;
        for (int i = 0; i < c->n_beamlets; ++i) {
            if (fluence[i] == 0.0f) continue;
            const double* row = prm + (q * c->n_beams + c->fr[i].beam) * 7;
            int fl;
            double d = row[6] != 0.0 ? pair_value(c, v, i, rc, rhc, &fl, NULL, NULL)
                                     : pair_value(c, v, i, rc, rhc, &fl, row, NULL);
            if (fl & 1) acc += fluence[i] * d;
            if (fl & 2) a += fabs(fluence[i] * d);
        }
        dose[q] = acc;
        if (amb) amb[q] = a;
    }
}
