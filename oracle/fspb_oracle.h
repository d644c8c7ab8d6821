/*
 * fspb_oracle.h -- plain FP64 CPU oracle of the finite-size pencil beam dose
 * method with 3D density correction (DC-FSPB).
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the GPU library.  It
 * is not part of the product path: only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it.  It shares no code, header,
 * table or constant with the GPU library.
 *
 * What it computes (Gu et al., "GPU-based finite-size pencil beam algorithm
 * with 3D-density correction"):
 *   smoothed density      Section 2.1 and Algorithm A1 step 1
 *   beamlet frame, theta  Eq. 2 definitions and Algorithm A1 step 3
 *   ray trace, tables     Algorithm A1 steps 4-6, uniform sampling of Sec. 2.2
 *   pair dose D_i(r)      Eqs. 2-4 and the density corrections of Sec. 2.1,
 *                         inside the 5 cm ROI cylinder of Algorithm A1
 *   dose superposition    Eq. 1
 *   adjoint g = D^T w     (transpose of Eq. 1; not in the paper)
 *
 * Every value is computed in double precision, brute force over every voxel
 * and every beamlet, in a fixed summation order -- except the pair test (is
 * the voxel inside the beamlet's ROI cylinder and below its entrance?),
 * whose discrete outcome is taken in single precision by a fixed recipe (see
 * orc_pair_consts).  Parity status of each function is listed at its
 * declaration.
 */
#ifndef FSPB_ORACLE_H
#define FSPB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double start, step;   /* value i sits at start + i*step */
    int n;
    const float* v;       /* host array, read only */
} orc_table;

typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;    /* cm */
    double ox, oy, oz;    /* centre of voxel (0,0,0), cm */
    const float* rho;     /* [nz][ny][nx], g/cm^3 relative to water */
} orc_grid;

typedef struct {
    double gantry, couch; /* rad */
    double iso[3];        /* cm */
    double sad;           /* cm */
    int nbx, nby;
    double wx, wy;        /* beamlet full width at the isocentre plane */
    double cx, cy;        /* beamlet grid centre offset at the isocentre plane */
} orc_beam;

typedef struct {
    orc_table A;          /* row-major [n_theta][A.n] over radiological depth */
    int n_theta;
    double theta_step;    /* theta rows start at 0 */
    orc_table u1x, u1y, u2x, u2y, w1, w2;   /* vs geometric depth t */
    orc_table fu1, fu2, fw1, fw2, b1, b2;   /* vs density */
} orc_tables;

typedef struct {
    double roi_radius, rho_surface, smooth_sigma, rho_min, rho_max, sample_step;
    int dc_enabled;
    int siddon;           /* 1: exact radiological path (Siddon) instead of the
                             uniform samples of Section 2.2, see orc_trace_siddon */
} orc_options;


typedef struct orc_ctx orc_ctx;

/* Builds frames and ray-trace tables for every beamlet.  Copies nothing: the
 * grid and tables must outlive the context.  Returns NULL on bad input. */
orc_ctx* orc_create(const orc_grid* g, int n_beams, const orc_beam* beams,
                    const orc_tables* tab, const orc_options* opt);
void orc_destroy(orc_ctx* c);
int  orc_n_beamlets(const orc_ctx* c);

/* Eq. 4 penumbra profile p(x, u, x0).  Pinned by quadrature of a box of
 * half-width x0 against the Laplace density (u/2) exp(-u|x|). */
double orc_p(double x, double u, double x0);

/* Beamlet frame: out[0..2] source, [3..5] direction, [6..8] lateral x axis,
 * [9..11] lateral y axis, [12] theta, [13] x0, [14] y0, [15] SAD. */
void orc_frame(const orc_ctx* c, int i, double out[16]);

/* Ray-trace results of beamlet i.  info[0] hit (1/0), [1] s_in, [2] s_out,
 * [3] s_entry, [4] k_entry, [5] K (table length), [6] s_exit,
 * [7] min |rho_k - rho_surface| over samples up to the entry (ambiguity
 * margin of the entry decision), [8] sample step d, [9] n_samples.
 * Copies min(K, maxK) table entries to T, W1, W2 when they are non-NULL.
 * Returns K. */
int orc_trace(const orc_ctx* c, int i, double info[10], double* T,
              double* W1, double* W2, int maxK);

/* Siddon tables of beamlet i (when the context was built with siddon = 1).
 * The density is constant inside each voxel; the axis is cut at every voxel
 * boundary between the grid-box entry and exit.  Segment m covers depths
 * [t[m], t[m+1]) below the entrance (the last one runs on past the box) in
 * a voxel of density rho[m]; T[m], W1[m], W2[m] are the integrals of rho and
 * b_c(clamped rho) from the entrance to t[m].  The entrance is the start of
 * the first segment whose voxel density reaches rho_surface.  Copies
 * min(K, maxK) entries to the non-NULL arrays; returns K (0 if the beamlet
 * misses the body). */
int orc_trace_siddon(const orc_ctx* c, int i, double* t, double* T, double* W1, double* W2,
                     double* rho, int maxK);
/* Smoothed density at one voxel (direct, non-separable 3D sum). */
double orc_smoothed_at(const orc_ctx* c, long vox);
/* Smoothed density of the whole grid into out[n_vox]. */
void orc_smooth_all(const orc_ctx* c, double* out);
/* Truncation radius (voxels) of the smoothing kernel along each axis. */
void orc_smooth_radius(const orc_ctx* c, int r[3]);

/* The pair test (Algorithm A1 step 8: inside the ROI cylinder, below the
 * entrance) decides a discrete outcome, so it is taken in single precision,
 * the precision of the method's GPU implementation, by a fixed recipe (see
 * pair_counted in the source); the pair's dose is computed in double.  The
 * recipe's per-beamlet constants: out[0..3] = (d, c_t), out[4..7] = (ex, c_x),
 * out[8..11] = (ey, c_y), each rounded to single precision. */
void orc_pair_consts(const orc_ctx* c, int i, float out[12]);

/* Unit-fluence dose of beamlet i at voxel vox (Eq. 2).  flags (if non-NULL)
 * gets bit 0 = pair counted (beamlet hits, in ROI and t >= 0).  Returns 0 for
 * a pair that does not count. */
double orc_pair(const orc_ctx* c, long vox, int i, int* flags);

/* Dose (Eq. 1) at n voxels listed in vox (or every voxel when vox is NULL, in
 * which case n must equal the grid size).  pairs[k] gets the number of
 * counted pairs with f_i != 0.  amb[k] is an allowance for pairs that two
 * implementations of the method may count differently: 0, since the pair test
 * follows the single-precision recipe above.  amb and pairs may be NULL. */
void orc_dose(const orc_ctx* c, const float* fluence, long n, const long* vox,
              double* dose, double* amb, long long* pairs);

/* Adjoint g_i = sum_r w(r) D_i(r) for the n beamlets listed (all beamlets
 * when list is NULL and n equals the beamlet count); amb as for orc_dose.
 * amb may be NULL. */
void orc_adjoint(const orc_ctx* c, const float* w, int n, const int* list,
                 double* g, double* amb);

/* Number of counted pairs (all beamlets, regardless of fluence) per listed
 * voxel; vox may be NULL for the whole grid. */
void orc_pair_counts(const orc_ctx* c, long n, const long* vox, int* counts);
/* Voxels paired with each listed beamlet (all when beamlets is NULL). */
void orc_beamlet_pair_counts(const orc_ctx* c, int n, const int* beamlets, long long* counts);


/* ---- Learned-surrogate support (an extension beside the method, not in
 * the paper).  A row is a (voxel, beam); its six parameters are
 * (u1x, u1y, u2x, u2y, w1, w2) in the units of the tables. ---- */

/* Trilinear density at a point (clamp-to-edge), as the ray trace samples it.
 * Pinned: reproduces voxel values at centres and linear fields exactly. */
double orc_density_at(const orc_ctx* c, const double p[3]);
/* The six parameters the pair (vox, i) uses: with density correction on,
 * after Section 2.1; otherwise the water values.  Returns the orc_pair flags
 * (the parameters are meaningful when bit 0 is set).  Pinned: water values
 * in water, closed forms in a uniform medium. */
int orc_params(const orc_ctx* c, long vox, int i, double out[6]);
/* Pair dose with the six parameters given (Eqs. 2-4; depth, t_eq, A and the
 * inverse square of beamlet i).  Pinned: equals orc_pair when given
 * orc_params of the same pair. */
double orc_pair_given(const orc_ctx* c, long vox, int i, const double prm[6], int* flags);
/* Nearest beamlet of a beam to a voxel by central projection onto the
 * isocentre plane (ties round up), or -1.  *tie (may be NULL) gets the
 * smaller distance of the two rounding decisions from a tie, in beamlet
 * widths.  Pinned: a voxel on a beamlet's axis selects that beamlet. */
int orc_nearest_beamlet(const orc_ctx* c, long vox, int beam, double* tie);
/* Surrogate input row (200 patch densities, depth, theta) of (voxel, beam),
 * definition at the function.  Returns the nearest beamlet, or -1 when the
 * row is invalid.  *amb (may be NULL) gets 0 (the pair test follows the
 * single-precision recipe, so no row is ambiguous).  Pinned: linear density fields give the analytic patch. */
int orc_surrogate_row(const orc_ctx* c, long vox, int beam, double feat[202], int* amb);
/* Dose with per-(voxel, beam) parameters prm[n][n_beams][7] (six parameters
 * and a fallback flag: non-zero means the method's own parameters).
 * Pinned: all-fallback equals orc_dose; rows set to orc_params of the
 * nearest beamlet give orc_dose in a uniform medium. */
void orc_dose_given(const orc_ctx* c, const float* fluence, long n, const long* vox,
                    const double* prm, double* dose, double* amb);

#ifdef __cplusplus
}
#endif
#endif
