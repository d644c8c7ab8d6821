/*
 * fspb.h -- C ABI of the MI355X (gfx950) finite-size pencil beam dose engine
 * with 3D density correction (DC-FSPB).
 *
 * The method (Gu, Jelen, Li, Jia, Jiang, "GPU-based finite-size pencil beam
 * algorithm with 3D-density correction for radiotherapy dose calculation"):
 *   D(r)   = sum_i f_i D_i(r)                                          (Eq. 1)
 *   D_i(r) = F(x, y, omega, u_x, u_y, x0, y0) A(t_eq, theta) (SAD/|r_a|)^2 (Eq. 2)
 *   F      = sum_{c=1,2} omega_c p(x, u_cx, x0) p(y, u_cy, y0)         (Eq. 3)
 *   p      = the exponential penumbra profile of Eq. 4
 * with the lateral/weight density corrections of Section 2.1, evaluated for
 * every (voxel, beamlet) pair inside a 5 cm cylinder around the beamlet axis
 * (Algorithm A1), using per-beamlet radiological-depth and weight-drift
 * tables sampled uniformly along the axis (Section 2.2).
 *
 * Conventions
 *   Units: cm, radians, g/cm^3 relative to water; dose in arbitrary units
 *   (fluence x table units).
 *   Voxel grids: float32, [nz][ny][nx] with x fastest; voxel (i,j,k) has its
 *   centre at (ox + i dx, oy + j dy, oz + k dz).
 *   Beams: gantry rotates about z; at gantry 0 the source sits at
 *   iso - SAD*(0,1,0) so the beam travels +y; the couch angle rotates the
 *   beam about y.  Beamlet (n, m) of a beam (row n along the beam's y axis,
 *   column m along its x axis) is centred at
 *   ((m-(nbx-1)/2) wx + cx, (n-(nby-1)/2) wy + cy) in the isocentre plane.
 *   Fluence order: beam-major, then row n, then column m.
 *   "stream" arguments are hipStream_t values passed as void* (NULL = the
 *   null stream).
 *
 * Memory ownership
 *   Pointers marked "device" must point to device memory of the current HIP
 *   device; pointers marked "host" to host memory.  The library never frees
 *   caller memory.  A geometry handle owns its own device buffers.
 *
 * Errors
 *   Every int-returning entry point returns FSPB_OK (0) or a negative code;
 *   fspb_last_error() gives a description of the last failure on the calling
 *   thread.  On error, output arguments are left untouched (and *out is set
 *   to NULL for fspb_create_geometry).
 *
 * Concurrency
 *   A handle may be used from one stream at a time.  Distinct handles are
 *   independent.
 */
#ifndef FSPB_H
#define FSPB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSPB_OK             0
#define FSPB_E_ARG         -1   /* invalid argument or inconsistent sizes */
#define FSPB_E_HIP         -2   /* a HIP runtime call failed */
#define FSPB_E_NOMEM       -3   /* device or host allocation failed */
#define FSPB_E_STATE       -4   /* operation not valid for this handle */
#define FSPB_E_UNSUPPORTED -5   /* no usable gfx950 device */

typedef struct fspb_geometry fspb_geometry;

/* CT density grid (Algorithm A2 step 1 input).  density: device, read only,
 * n = nx*ny*nz floats; only read during fspb_create_geometry. */
typedef struct {
    int nx, ny, nz;
    float dx, dy, dz;
    float ox, oy, oz;
    const float* density;
} fspb_ct;

/* One beam: gantry/couch angles, isocentre, source-axis distance (Eq. 2) and
 * its beamlet grid.  wx, wy are the beamlet full widths at the isocentre
 * plane; the half widths are the x0, y0 of Eq. 4. */
typedef struct {
    float gantry, couch;
    float iso[3];
    float sad;
    int nbx, nby;
    float wx, wy;
    float cx, cy;
} fspb_beam;

/* Uniformly sampled table: v[i] (host) is the value at start + i*step.
 * Lookups interpolate linearly and hold the end values outside the range. */
typedef struct {
    float start, step;
    int n;
    const float* v;
} fspb_table1d;

/* Commissioned model parameters (Section 2.1).
 *   A        2-D table [n_theta][A.n]: row r is A(t_eq, r*theta_step) over
 *            radiological depth on A's grid; looked up bilinearly.
 *   u1x..w2  water parameters vs geometric depth t; all six must share one
 *            grid (start, step, n).
 *   fu1,fu2  penumbra widening factors vs density: u1 = fu1(rho) u1^w,
 *            u2 = fu2(rho_hat) u2^w.
 *   fw1,fw2  weight factors vs smoothed density.
 *   b1,b2    weight drift per cm vs density:
 *            omega_c = fw_c(rho_hat) (omega_c^w(t) + int_0^t b_c(rho) dt').
 * All host pointers; copied during fspb_create_geometry. */
typedef struct {
    fspb_table1d A;
    int n_theta;
    float theta_step;
    fspb_table1d u1x, u1y, u2x, u2y, w1, w2;
    fspb_table1d fu1, fu2, fw1, fw2, b1, b2;
} fspb_tables;

/* Options.  Zero float fields take the defaults in brackets.  The integer
 * fields are used as given, so a zero-initialised struct selects plain FSPB
 * (dc_enabled = 0), the default tile and the brick-major schedule, while
 * opts = NULL in fspb_create_geometry selects every default with the density
 * correction on (dc_enabled = 1). */
typedef struct {
    float roi_radius;    /* ROI cylinder radius [5 cm] (Algorithm A1 footnote) */
    float rho_surface;   /* body-surface density threshold [0.5] */
    float smooth_sigma;  /* Gaussian width of the smoothed density [0.5 cm] */
    float rho_min;       /* commissioned density range [0.1] */
    float rho_max;       /*                            [2.0] */
    float sample_step;   /* ray sampling step [min(dx,dy,dz)/2] (Section 2.2) */
    int dc_enabled;      /* 1: 3D density correction, 0: plain FSPB (A1 without step 11);
                            no bracketed default: 0 here means plain FSPB */
    int flags;           /* 0, or FSPB_FLAG_SIDDON */
    /* forward tile built at creation (see fspb_set_tile): tile_waves = 0
     * takes the default (brick shape 0, 8 waves per workgroup); otherwise
     * 1, 2, 4 or 8 waves per workgroup with brick shape tile_shape
     * (0 .. fspb_tile_shapes() - 1).  Equivalent to fspb_set_tile right
     * after creation, without building the default schedule first. */
    int tile_shape;
    int tile_waves;
    /* forward work schedule built at creation (see fspb_set_schedule):
     * 0 = bricks longest-first, 1 = per-beam items */
    int schedule;
} fspb_options;

/* fspb_options.flags: build exact radiological-depth tables (Siddon's
 * path through voxel-constant density, the alternative Section 2.2 sets
 * aside) instead of the uniform samples.  Each voxel segment past the
 * entrance is a record; the entrance is the start of the first segment whose
 * voxel density reaches rho_surface; the forward searches the records per
 * pair.  Such a geometry supports fspb_forward, fspb_count_pairs,
 * fspb_update_density, the tiling calls and the inspection calls (without
 * the sampled tables); the adjoint, batches and the surrogate return
 * FSPB_E_STATE. */
#define FSPB_FLAG_SIDDON 1

typedef struct {
    int n_beams, n_beamlets;
    int nx, ny, nz;
    long long n_vox;
    int k_stride;          /* samples reserved per beamlet depth table */
    int k_max;             /* longest depth table actually used */
    int n_hit;             /* beamlets whose axis enters the body */
    int n_entry_ambiguous; /* beamlets whose entrance sample lies within 1e-9 of rho_surface */
    int smooth_radius[3];  /* Gaussian truncation radius in voxels */
    float sample_step;
    int dc_enabled;
    long long device_bytes;
    /* weight-drift tables a density-corrected pair reads: 1 when the
     * commissioned b2 equals drift_ratio * b1 at every sample of one density
     * grid (Section 2.1's single b: drift_ratio = 1), so that the second
     * drift is drift_ratio * W1; 2 otherwise (a table per component) */
    int drift_tables;
    float drift_ratio;
} fspb_info;

/* Per-beamlet geometry and tables, for inspection and tests. */
typedef struct {
    int hit;               /* 1 if the axis enters the body */
    int k_entry;           /* entrance sample index from the grid-box entry */
    int n_samples;         /* samples from the box entry to the end of the table */
    int K;                 /* depth-table length (samples from the entrance) */
    double s_in;           /* box entry distance from the source */
    double s_entry;        /* entrance distance from the source */
    double theta;          /* angle to the beam's central axis */
    double src[3], dir[3], ex[3], ey[3];
    double entry_margin;   /* min |rho_k - rho_surface| over samples up to the entrance */
    /* The single-precision constants of the pair test (Algorithm A1 step 8)
     * as the dose kernels read them: with q the voxel centre relative to the
     * grid centre P0 = o + (n - 1) delta / 2, each q_a = fma(index_a,
     * delta_a, o_a - P0_a) in single precision,
     *   t  = fma(q_x, pair_t[0], fma(q_y, pair_t[1], fma(q_z, pair_t[2], pair_t[3])))
     * is the depth below the entrance and xp, yp (pair_x, pair_y alike) the
     * lateral offsets from the axis; the pair counts iff t >= 0 and
     * fma(xp, xp, yp * yp) <= R * R, all in single precision.  pair_t[0..2]
     * is dir rounded to single precision, pair_t[3] = (P0 - src).dir -
     * s_entry rounded from double; pair_x, pair_y likewise with ex, ey. */
    float pair_t[4], pair_x[4], pair_y[4];
} fspb_beamlet_info;

/* Builds the per-plan geometry on the device (Algorithm A2 steps 2-5):
 * smoothed density and per-voxel correction factors (DC only), beamlet
 * frames and angles, entrance points, and radiological-depth and
 * weight-drift tables.  The handle takes its own device copy of the CT and
 * returns once that copy is complete, so the caller may free or overwrite
 * ct->density afterwards; the geometry kernels may still be running on
 * stream.  Later calls on the same stream are ordered after them; a call on
 * another stream makes that stream wait for them on the device (on the host
 * while the stream captures a graph), and a call that reads results on the
 * host waits for them on the host.
 *   ct      host struct; ct->density device.
 *   beams   host array [n_beams].
 *   tables  host struct with host arrays (copied).
 *   opts    host struct, or NULL for the defaults with the density
 *           correction on (a zero-initialised struct turns it off).
 *   out     receives the handle (NULL on error).
 * Errors: FSPB_E_ARG for empty or inconsistent inputs (non-positive sizes,
 * source inside the grid box, depth tables on different grids, nonzero
 * flags), FSPB_E_NOMEM, FSPB_E_HIP, FSPB_E_UNSUPPORTED. */
int fspb_create_geometry(const fspb_ct* ct, int n_beams, const fspb_beam* beams,
                         const fspb_tables* tables, const fspb_options* opts,
                         void* stream, fspb_geometry** out);

/* Dose superposition (Eq. 1 over Eqs. 2-4, Algorithm A2 step 6).
 *   fluence  device [n_beamlets]; beamlets with f_i == 0 are skipped.
 *   dose     device [n_vox], overwritten (every voxel is written once).
 * Asynchronous on stream.  Uses the density correction iff it is enabled on
 * the handle (see fspb_set_dc). */
int fspb_forward(fspb_geometry* g, const float* fluence, float* dose, void* stream);

/* Adjoint of fspb_forward (Eq. 1 transposed): grad_i = sum_r voxel_weight(r)
 * D_i(r) for every beamlet, including those with zero fluence.  For
 * L = sum w (D - D0)^2 pass voxel_weight = 2 w (D - D0) to get dL/df.
 * Deterministic: each beamlet's sum is taken over fixed parts of the grid and
 * the parts are added in a fixed order, whatever the scheduling.
 *   voxel_weight  device [n_vox].
 *   grad          device [n_beamlets], overwritten.
 * Asynchronous on stream.  Uses per-handle scratch memory: adjoint and
 * beamlet_pair_counts calls on one handle that overlap in time (on different
 * streams without ordering) race.  FSPB_E_STATE with exact depth tables. */
int fspb_adjoint(fspb_geometry* g, const float* voxel_weight, float* grad, void* stream);

/* Number of voxels paired with each beamlet (the pairs of Algorithm A1 step
 * 8: inside the ROI cylinder, depth t >= 0, beamlets that enter the body),
 * found by the beamlet-major traversal fspb_adjoint uses.  Their sum equals
 * fspb_count_pairs' total with fluence NULL.
 *   counts  device int [n_beamlets], overwritten.
 * Asynchronous on stream; the same per-handle scratch as fspb_adjoint. */
int fspb_beamlet_pair_counts(fspb_geometry* g, int* counts, void* stream);

/* Number of evaluated pairs: voxel-beamlet pairs inside the ROI with t >= 0
 * for beamlets that enter the body; with fluence non-NULL, only beamlets with
 * f_i != 0 (the pairs fspb_forward evaluates).
 *   fluence  device [n_beamlets] or NULL.
 *   counts   device int [n_vox] or NULL; per-voxel counts.
 *   total    host; receives the sum.  The call synchronises the stream. */
int fspb_count_pairs(fspb_geometry* g, const float* fluence, int* counts,
                     unsigned long long* total, void* stream);

/* fspb_count_pairs for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same count of the pairs fspb_forward evaluates (or of all pairs with
 * fluence NULL), written to a device word, with no allocation, no host
 * synchronisation and no memset, so the call can be captured in a graph.
 *   fluence  device [n_beamlets] or NULL.
 *   total    device unsigned long long; receives the sum (asynchronously).
 * Its scratch is a static array of 4 MiB + 2 KiB on each device the library
 * runs on (held until the process ends): per-brick counts for at most
 * 1,048,576 bricks of the handle's tile shape (about 64 million voxels), then
 * the partial sums.  A larger plan returns FSPB_E_ARG.  Every call on one
 * device shares that device's array, so calls whose work overlaps on the
 * device (on different streams without ordering between them) race; calls
 * ordered on one stream do not.  The handle's device must be the current
 * device (else FSPB_E_ARG).  Asynchronous on stream. */
int fspb_count_pairs_noalloc(fspb_geometry* g, const float* fluence, unsigned long long* total,
                             void* stream);

/* Switches the forward/adjoint between the density-corrected model (1) and
 * plain FSPB (0).  Enabling DC on a handle created with dc_enabled = 0
 * returns FSPB_E_STATE. */
int fspb_set_dc(fspb_geometry* g, int enabled);

/* Plan summary (host struct). */
int fspb_geometry_info(const fspb_geometry* g, fspb_info* info);

/* Weight-drift tables a density-corrected pair reads with these commissioned
 * tables (host call; needs no device).  Returns 1 when b2 equals
 * ratio * b1 at every sample of one density grid (Section 2.1 integrates a
 * single b: ratio 1), so that the second drift is ratio * W1; 2 otherwise
 * (ratio 0).  ratio (host) may be NULL.  FSPB_E_ARG when t, or the b1 or b2
 * values, are NULL or a table has no samples.  fspb_geometry_info reports
 * the same for a handle (drift_tables, drift_ratio). */
int fspb_drift_tables(const fspb_tables* t, float* ratio);

/* Copies the smoothed density (device [n_vox]) of a DC handle. */
int fspb_smoothed_density(const fspb_geometry* g, float* out, void* stream);

/* Copies beamlet i's geometry (host struct) and up to max_k entries of its
 * depth tables T (radiological depth), W1, W2 (weight drift) into host
 * arrays (each may be NULL).  Synchronous. */
int fspb_beamlet(const fspb_geometry* g, int i, fspb_beamlet_info* info,
                 float* T, float* W1, float* W2, int max_k);

/* Re-runs the density-dependent part of fspb_create_geometry (smoothed
 * density and correction factors, entrance points and depth tables) for a new
 * CT of the same grid, beams and tables -- e.g. the next fraction of an
 * adaptive session.  Asynchronous on stream with no allocation and no host
 * synchronisation, so it can be captured in a HIP graph; density (device,
 * [n_vox]) must stay valid until the work has run.  The brick schedule of the
 * forward kernel is kept from the previous density. */
int fspb_update_density(fspb_geometry* g, const float* density, void* stream);

/* Makes stream wait, on the device, for the handle's creation work (a no-op
 * on the creation stream or once that work is known to be done).  For
 * callers that create plans on one stream and use them on another and want
 * their own work on that stream -- or a timing event -- ordered after the
 * geometry; the library's own calls order themselves.  Asynchronous. */
int fspb_wait_ready(fspb_geometry* g, void* stream);

/* ---- forward-kernel tiling and autotuning -------------------------------
 * The forward kernel assigns one 64-voxel brick to each wavefront.  Brick
 * shapes (voxels along x, y, z) are listed by fspb_tile_shapes; a tile
 * configuration is a shape index and 1, 2, 4 or 8 waves per workgroup.  With
 * 8, each workgroup stages the water (depth) table in LDS when it fits in
 * 64 KB, i.e. up to 1365 depth samples (else that launch uses 4 waves and
 * reads the table from global memory).  A new handle starts with shape 0,
 * 4 x 4 x 4 voxels, and 8 waves, or with the tile given in
 * fspb_options.tile_shape / tile_waves.  For a given brick shape results do not
 * depend on the configuration (each voxel sums its pairs in the same order,
 * from the same table values); another shape may change a pair's rounding,
 * as each wave picks one of two exact forms of the Eq. 4 profile product,
 * so doses then agree to a few FP32 ulps. */
typedef struct {
    int shape;            /* shape index */
    int dims[3];          /* brick voxels along x, y, z */
    int waves_per_block;
    float ms;             /* median forward time */
    int per_beam;         /* forward schedule (fspb_set_schedule) */
} fspb_tune_result;

/* Number of brick shapes; writes dims[3*q .. 3*q+2] for q < max_shapes when
 * dims is non-NULL (host). */
int fspb_tile_shapes(int* dims, int max_shapes);

/* Selects the tile configuration of a handle (recomputes its brick schedule
 * on the stream when the shape changes; calls on other streams then wait for
 * that work on the device, as after fspb_create_geometry). */
int fspb_set_tile(fspb_geometry* g, int shape, int waves_per_block, void* stream);
int fspb_get_tile(const fspb_geometry* g, int* shape, int* waves_per_block);

/* Selects the forward's work schedule (Algorithm A2 kernel 5).
 *   per_beam = 0  (default) a wavefront takes a whole brick and sums every
 *                 beam's pairs; bricks run longest-first.
 *   per_beam = 1  a wavefront takes a (brick, beam) item and writes that
 *                 beam's partial dose to a plane [n_beams][n_vox] the handle
 *                 owns (allocated on first use: 4 n_beams n_vox bytes); a
 *                 second pass adds the planes in beam order.  The items are
 *                 sorted by beam and by depth along the beam's central axis,
 *                 and the sorted list is cut into 16 segments of about equal
 *                 estimated work, XCD x running segments x and x + 8, so each
 *                 XCD sweeps one beam's slabs at a time and the depth-table
 *                 lines its bricks share stay in its L2.  With 8 waves per
 *                 workgroup (water table in LDS) the workgroups are
 *                 persistent and take their XCD's items one at a time from a
 *                 counter the handle owns.  For a given brick shape the dose
 *                 is bitwise that of per_beam = 0.
 * Builds the schedule on the stream (calls on other streams then wait for it
 * on the device).  FSPB_E_STATE with exact depth tables (FSPB_FLAG_SIDDON).
 * fspb_autotune covers both schedules. */
int fspb_set_schedule(fspb_geometry* g, int per_beam, void* stream);
int fspb_get_schedule(const fspb_geometry* g, int* per_beam);

/* Times every tile configuration on this plan (reps timed forwards each,
 * median) and keeps the fastest.  fluence: device [n_beamlets];
 * dose_scratch: device [n_vox], overwritten.  results (host, up to
 * max_results entries) and n_results may be NULL.  Synchronous. */
int fspb_autotune(fspb_geometry* g, const float* fluence, float* dose_scratch, int reps,
                  void* stream, fspb_tune_result* results, int max_results, int* n_results);

/* The adjoint's work unit is (beamlet, slab of `planes` grid planes k); each
 * XCD takes its beamlets' units slab by slab, so thinner slabs keep more of
 * the voxel data the units share in the XCDs' L2, thicker ones pay the
 * per-unit set-up fewer times.  planes = 0 restores the default (the planes
 * holding about 5 MiB of voxel weights and factors); otherwise
 * ceil(nz / 64) <= planes <= nz, else FSPB_E_ARG.  The adjoint's per-slab
 * partial sums are added in slab order, so its result depends on the
 * thickness in the last bits only (and is deterministic for each).  Host
 * state only: affects calls enqueued afterwards. */
int fspb_set_adjoint_slab(fspb_geometry* g, int planes);
int fspb_get_adjoint_slab(const fspb_geometry* g, int* planes);

/* Times fspb_adjoint (reps timed calls each, median) with the default slab
 * thickness, half and two and four times it, and the whole grid, and keeps
 * the fastest.  voxel_weight: device [n_vox]; grad_scratch: device
 * [n_beamlets], overwritten.  planes / ms (host, up to max_results entries)
 * and n_results may be NULL.  Synchronous.  FSPB_E_STATE with exact depth
 * tables (no adjoint). */
int fspb_autotune_adjoint(fspb_geometry* g, const float* voxel_weight, float* grad_scratch,
                          int reps, void* stream, int* planes, float* ms, int max_results,
                          int* n_results);

/* ---- batches: many plans in one persistent launch -----------------------
 * A batch schedules every brick of up to 64 plans (sharing the
 * density-correction mode) over waves_per_cu x (number of CUs) persistent
 * wavefronts.  The static schedule assigns bricks longest-first to the least
 * loaded wavefront, so no atomics are needed.  Each wavefront records the wall
 * clock after its last brick of every plan; fspb_batch_latencies turns those
 * into per-plan completion times.  The geometries must outlive the batch. */
typedef struct fspb_batch fspb_batch;

#define FSPB_SCHEDULE_THROUGHPUT 0  /* one longest-first list over all plans */
#define FSPB_SCHEDULE_LATENCY    1  /* plans by increasing work, bricks longest-first */

/* geoms: host array [n] of handles.  shape / waves_per_block: tile
 * configuration of the persistent kernel (plans are re-scheduled for that
 * shape); with 8 waves per workgroup the water table is staged in LDS when
 * every plan uses the same commissioned tables and it fits (as for
 * fspb_set_tile), else the launch uses 4 waves per workgroup.  policy:
 * FSPB_SCHEDULE_THROUGHPUT minimises the whole launch;
 * FSPB_SCHEDULE_LATENCY lets small plans complete first.  Synchronises the
 * stream. */
int fspb_batch_create(int n, fspb_geometry* const* geoms, int shape, int waves_per_block,
                      int waves_per_cu, int policy, void* stream, fspb_batch** out);

/* One persistent launch: dose[p] (device [n_vox of plan p]) = forward of
 * fluence[p] (device [n_beamlets of plan p]); both arrays are host arrays of
 * n device pointers.  Asynchronous. */
int fspb_batch_forward(fspb_batch* b, const float* const* fluence, float* const* dose, void* stream);

/* Captures into a HIP graph owned by the batch: for each plan
 * fspb_update_density(density[p]) when density is non-NULL (host array of n
 * device pointers), then the batch forward.  stream must not be the null
 * stream.  Replace any earlier capture. */
int fspb_batch_capture(fspb_batch* b, const float* const* fluence, float* const* dose,
                       const float* const* density, void* stream);

/* Launches the captured graph on stream. */
int fspb_batch_replay(fspb_batch* b, void* stream);

/* After the last batch forward or replay on stream (the call synchronises
 * it): plan_ms[p] (host, [n] or NULL) = time from the earliest wavefront start
 * to plan p's last brick; total_ms = the whole launch.  Device wall clock. */
int fspb_batch_latencies(const fspb_batch* b, double* plan_ms, double* total_ms, void* stream);

/* Number of persistent wavefronts and scheduled bricks. */
int fspb_batch_info(const fspb_batch* b, int* n_waves, long long* n_items);

/* Frees the batch (not its geometries).  NULL-safe. */
void fspb_batch_destroy(fspb_batch* b);

/* ------------------------------------------------------------------------
 * Learned surrogate of the density correction (an extension beside the
 * method; it changes nothing above).  A small MLP predicts the six Section
 * 2.1 parameters (u1x, u1y, u2x, u2y, w1, w2) of a (voxel, beam) row from a
 * density patch; the dose then uses that prediction for every beamlet of the
 * beam at the voxel, while depth, t_eq, A and the inverse square stay per
 * beamlet.  Rows whose guard fires fall back to the corrected parameters.
 *
 * Network: 202 inputs -> 64 -> 64 -> 6, tanh-approximated GELU, BF16 weights
 * and activations with FP32 accumulation on the matrix cores, FP32 master
 * weights, Adam.  Parameters, flat FP32 (FSPB_MLP_PARAMS values), row-major:
 *   W1 [202][64], b1 [64], W2 [64][64], b2 [64], W3 [64][6], b3 [6]
 * with y = W3^T gelu(W2^T gelu(W1^T x + b1) + b2) + b3.
 *
 * Input row (FSPB_MLP_IN values, stored BF16 in rows of FSPB_MLP_IN_PAD with
 * zero padding): the nearest beamlet of the beam is the one whose
 * isocentre-plane centre lies nearest to the voxel's central projection from
 * the source (ties round up); the row is valid when that beamlet reaches the
 * body and its pair with the voxel passes the pair test.  On the ray from
 * the source to the voxel centre (direction u), plane k = 0..7 lies
 * t (7 - k) / 7 before the voxel, t being the voxel's depth for the nearest
 * beamlet; each plane holds a 5 x 5 lattice at 0.5 cm along e1 (the beam's
 * x axis made orthogonal to u) and e2 = e1 x u.  Input 25 k + 5 b + a is the
 * trilinear density at lattice point (a, b) minus 1; input 200 is
 * t / 10 cm - 1 and input 201 is 10 theta of the nearest beamlet.
 * Targets are the corrected parameters of the nearest beamlet at the voxel
 * (u in 1/cm).  The network's outputs are z = (log u1x, log u1y, log u2x,
 * log u2y, w1, w2) standardised: z = y std + mean.
 * ------------------------------------------------------------------------ */
#define FSPB_MLP_IN 202
#define FSPB_MLP_IN_PAD 224
#define FSPB_MLP_HIDDEN 64
#define FSPB_MLP_OUT 6
#define FSPB_MLP_PARAMS 17542
#define FSPB_MLP_MAX_ROWS (1 << 22)   /* rows per training or gradient call */

typedef struct fspb_mlp fspb_mlp;

typedef struct {
    float lr, beta1, beta2, eps;
} fspb_adam;

/* Guard: a row falls back when a patch density leaves [rho_lo, rho_hi],
 * when the larger of max |rho - rho(voxel)| over the two planes next to the
 * voxel and |rho_hat(voxel) - rho(voxel)| (rho_hat: the smoothed density of
 * Section 2.1) exceeds het_max, or when a predicted parameter (u1x, u1y,
 * u2x, u2y, w1, w2) leaves [band_lo[c], band_hi[c]]. */
typedef struct {
    float rho_lo, rho_hi, het_max;
    float band_lo[6], band_hi[6];
} fspb_surrogate_guard;

/* Creates a network on the current device from params (host, FSPB_MLP_PARAMS
 * values); Adam moments start at zero, step at 0, scaling at mean 0 / std 1,
 * and the guard open (nothing falls back but invalid rows). */
int fspb_mlp_create(const float* params, fspb_mlp** out);

/* Standardisation of the network's outputs z (host, 6 values each;
 * std > 0). */
int fspb_mlp_set_scaling(fspb_mlp* m, const float* mean, const float* stdev);

/* Fallback guard (host struct, copied). */
int fspb_mlp_set_guard(fspb_mlp* m, const fspb_surrogate_guard* guard);

/* Mean-square loss over n rows (1 <= n <= FSPB_MLP_MAX_ROWS) of x (device,
 * BF16 bit patterns [n][224]) against standardised targets t (device, FP32
 * [n][6]), and its gradient with respect to the parameters (device, FP32
 * [FSPB_MLP_PARAMS], flat layout above).  loss (device, 1 float) and grad
 * may each be NULL.  The network is unchanged. */
int fspb_mlp_loss_grad(fspb_mlp* m, const uint16_t* x, const float* t, long long n, float* grad,
                       float* loss, void* stream);

/* One Adam step on the loss of the n rows (as fspb_mlp_loss_grad); loss
 * (device, may be NULL) receives the loss before the step.  Deterministic:
 * equal states and inputs give bitwise equal results. */
int fspb_mlp_train_step(fspb_mlp* m, const uint16_t* x, const float* t, long long n,
                        const fspb_adam* opt, float* loss, void* stream);

/* Network outputs (standardised units) y (device, FP32 [n][6]) of n >= 0
 * rows x (device, BF16 [n][224]). */
int fspb_mlp_predict(fspb_mlp* m, const uint16_t* x, long long n, float* y, void* stream);

/* Checkpoint: parameters, Adam moments (host, FSPB_MLP_PARAMS each; any may
 * be NULL) and the step count.  get synchronises the device; set replaces
 * the state (a NULL moment array is set to zero). */
int fspb_mlp_get_state(const fspb_mlp* m, float* params, float* adam_m, float* adam_v,
                       long long* step);
int fspb_mlp_set_state(fspb_mlp* m, const float* params, const float* adam_m,
                       const float* adam_v, long long step);

/* Frees the network.  NULL-safe; waits for queued device work. */
void fspb_mlp_destroy(fspb_mlp* m);

/* Training rows for the n (voxel, beam) pairs in rows (device, int32
 * [n][2]) of a geometry created with density correction on; density is the
 * CT the geometry was built from (device, [nz][ny][nx]).  Writes x (device,
 * BF16 [n][224]), t (device, FP32 [n][6], the corrected parameters of the
 * nearest beamlet, unstandardised) and valid (device, int32 [n], 1 if the
 * row is valid; invalid rows get zeros). */
int fspb_surrogate_samples(fspb_geometry* g, const float* density, const int* rows, long long n,
                           uint16_t* x, float* t, int* valid, void* stream);

/* Inference for every (voxel, beam) row: prm (device, FP32
 * [n_beams][n_vox][8]) gets (u1x, u1y, u2x, u2y) * log2(e), w1, w2, the
 * fallback flag (1 or 0) and 0.  Needs a density-corrected geometry with
 * n_vox < 2^28 (the CT's 16-byte records below are addressed with 32-bit
 * byte offsets) and n_vox * n_beams < 2^32 (else FSPB_E_ARG).  A first pass
 * writes the fallback rows (invalid, or |rho_hat - rho| at the voxel above
 * the guard's het_max) and lists the others; the gather and the network
 * then run on the listed rows only, reading the CT through 16-byte records
 * of each voxel's 2x2 (x, y) neighbourhood built at the start of the call.
 * The list and the records live in per-handle memory ((4 n_beams + 16)
 * n_vox bytes, allocated on the first call): calls on one handle that
 * overlap in time race.  Requires ny nz and nx below 2^24. */
int fspb_surrogate_infer(fspb_geometry* g, const fspb_mlp* m, const float* density, float* prm,
                         void* stream);

/* Eq. 1 with the surrogate's rows prm (as written by fspb_surrogate_infer):
 * a pair whose row's fallback flag is 0 uses the row's parameters, any other
 * pair the corrected ones.  dose as for fspb_forward. */
int fspb_forward_surrogate(fspb_geometry* g, const float* fluence, const float* prm, float* dose,
                           void* stream);

/* ------------------------------------------------------------------------
 * 3D gamma index (the evaluation of Section 2.3: distance-to-agreement and
 * dose-difference criteria, the dose criterion global to the maximum
 * reference dose).  For every voxel r of the reference grid
 *   gamma(r)^2 = min(cap^2, min over voxel offsets o with |o| <= cap * dist
 *                of |o|^2 / dist^2 + (E(r + o) - R(r))^2 / (dose_frac D)^2)
 * with |o| the physical length of the offset (anisotropic voxels allowed),
 * offsets leaving the grid skipped, and D = dose_max (or max R).  Statistics:
 * the maximum gamma over the grid, and the mean gamma and the fraction with
 * gamma < 1 over voxels with R >= iso_frac D.
 * ------------------------------------------------------------------------ */
typedef struct {
    float dist;        /* distance criterion, cm (0: 0.3) */
    float dose_frac;   /* dose criterion as a fraction of D (0: 0.03) */
    float gamma_cap;   /* search radius cap * dist; gamma is at most cap (0: 5) */
    float dose_max;    /* D; <= 0: the maximum of the reference */
    float iso_frac;    /* statistics region R >= iso_frac D (0: 0.5) */
} fspb_gamma_params;

typedef struct {
    double gamma_max;      /* over the whole grid */
    double gamma_avg_iso;  /* mean over the statistics region */
    double pass_rate_iso;  /* fraction of the region with gamma < 1 */
    double dose_max;       /* D used */
    long long n_iso;       /* voxels in the region */
} fspb_gamma_stats;

/* ref, eval: device [nz][ny][nx] on the same grid (spacing dx, dy, dz cm).
 * gamma: device [nz][ny][nx] output or NULL; stats: host output or NULL;
 * params: host struct or NULL for the defaults.  Synchronises the stream.
 * Errors: FSPB_E_ARG for bad sizes or criteria, or a search sphere of more
 * than 4096 voxel offsets. */
int fspb_gamma(const float* ref, const float* eval, int nx, int ny, int nz, float dx, float dy,
               float dz, const fspb_gamma_params* params, float* gamma, fspb_gamma_stats* stats,
               void* stream);

/* Frees the handle.  NULL-safe.  Its device buffers return to the library's
 * per-device cache (reused by later fspb_create_geometry calls) once the work
 * queued with the handle has finished.  If that work went to at most four
 * streams, the call does not wait for it (it waits only when more than two
 * such releases are pending); if the handle was used on more streams or
 * inside a graph capture, it waits for the whole device first. */
void fspb_destroy(fspb_geometry* g);

/* Returns every cached device buffer to the HIP runtime.  Buffers of live
 * handles are not affected. */
int fspb_release_cached_memory(void);

/* Static description of an error code. */
const char* fspb_error_string(int code);

/* Description of the last error on the calling thread ("" if none). */
const char* fspb_last_error(void);

/* Diagnostic messages on stderr, one line each, prefixed "[fspb] ":
 *   0  none (the default)
 *   1  every error an entry point returns, with its description
 *   2  also plan-level events: geometry creation and release, tile and
 *      schedule choices, autotuner results, batch and network creation,
 *      device memory taken from or returned to the HIP runtime
 *   3  also each forward, adjoint, surrogate inference and batch replay
 *      queued (handle, stream)
 * The initial level is read once from the environment variable
 * FSPB_LOG_LEVEL (an integer; anything else means 0).  Sets the level for
 * the whole process and returns the previous one; a level outside 0..3 is
 * clamped. */
int fspb_set_log_level(int level);

#ifdef __cplusplus
}
#endif
#endif /* FSPB_H */
