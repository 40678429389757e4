/*
 * mpgeo.h — C ABI of the MI355X (gfx950) mixed-precision Gaussian log-likelihood library.
 *
 * The library evaluates, for n locations s_1..s_n in R^2 and data Z (Section IV-A),
 *   Sigma_ab = C(||s_a - s_b||; theta)                          Matérn, eq. (1)
 *   Sigma = L L^T   (tile Cholesky, mixed precision)            Section VI, Algorithm 1
 *   y = L^-1 Z,  logdet = 2 sum log L_ii,  quad = y^T y
 *   loglik = -n/2 log(2 pi) - logdet/2 - quad/2                 eq. (2)
 * and, optionally, simple-kriging predictions at new sites from the same factor.
 *
 * Precision map (Algorithm 1, with its "diag_thick" = band64 + 1): the matrix is split
 * into tiles of tile x tile entries; tile (i, j), i >= j, is stored and updated in FP64
 * when i - j <= band64 and in FP32 otherwise.  An operation runs in the precision of the
 * tile it writes: FP64 inputs of an FP32 operation are rounded to nearest-even, FP32
 * inputs of an FP64 operation are promoted exactly.  Diagonal tiles (and so the
 * log-determinant) are always FP64.  The forward solve accumulates in FP64.
 * Optional third tier (more precision layers, the paper's future work in Section IX):
 * with band32 = c >= 0 and lowp = 1 (FP16) or 2 (BF16), tiles with i - j > band64 + c stay
 * FP32-stored but their trailing updates take 16-bit operands.  Tile row i has one power of
 * two s_i = 2^max(e_i - 14, -60), e_i = ceil(log2 sqrt(max Sigma_rr)) over its rows (every
 * |L_rk| <= sqrt(Sigma_rr)); each finished panel tile is rounded to nearest-even once into a
 * 16-bit copy Q_ik = L_ik / s_i of the factor, and a far tile is updated as
 * A_ij <- -s_i s_j (-A_ij / (s_i s_j) + sum_k Q_ik Q_jk^T) on the matrix cores, accumulating in
 * FP32 from -A_ij / (s_i s_j), panels in ascending k (a far tile takes its earlier panels in
 * one pass about two steps before it is solved; the result does not depend on how the
 * panels are grouped into passes).
 *
 * Conventions for every entry point:
 *  - Return value: an mpgeo_status code; MPGEO_OK (0) on success.
 *  - Ownership: the caller owns every pointer it passes and keeps it valid for the call;
 *    the library owns the device memory inside contexts and datasets and frees it on
 *    destroy.  Pointer arguments are host memory unless MPGEO_INPUT_DEVICE is set in the
 *    flags of the call (or of the dataset), in which case they are device pointers on
 *    the context's device (for example torch's tensor.data_ptr()).
 *  - Layout: locations are n x 2 row-major float64 (x, y), or (longitude, latitude) in
 *    degrees with MPGEO_DIST_GCD; vectors are float64.
 *  - Ordering: all calls are ordered on the context's HIP stream and are synchronous at
 *    return (results filled in); inside a factorization the library fans work out to
 *    streams of its own, which start after and join back into the context's stream.  A
 *    context is used by one host thread at a time.
 *  - Errors: on a non-OK return the outputs are undefined except mpgeo_result.info.
 *    MPGEO_E_ARG: n < 1, tile < 1 or > 512, band64 < -1, band32 < -1, band0 < -1, lowp outside 0..2,
 *    band32 >= 0 without a lowp format or lowp without band32 >= 0, a non-finite or
 *    non-positive theta component, a null pointer that is not nullable, a non-finite
 *    location, datum, kriging site or normal draw (host inputs are checked on the host,
 *    device inputs by a reduction on the device before any other work; Section IV-A's data
 *    are real-valued measurements at points of the plane or the sphere).
 *    MPGEO_E_NOT_SPD: a non-positive (or NaN) pivot; info = its 0-based global column in
 *    the (Morton-ordered) matrix.  MPGEO_E_NOMEM: device allocation failed, or the tiles a
 *    plan needs (mpgeo_footprint_bytes) exceed the context's HBM budget.
 *    MPGEO_E_DEVICE: a HIP runtime error.  MPGEO_E_UNSUPPORTED: a feature not built.
 */
#ifndef MPGEO_H
#define MPGEO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MPGEO_OK = 0,
    MPGEO_E_ARG = 1,
    MPGEO_E_NOT_SPD = 2,
    MPGEO_E_NOMEM = 3,
    MPGEO_E_DEVICE = 4,
    MPGEO_E_UNSUPPORTED = 5,
    MPGEO_E_TOO_LARGE = 6   /* a problem's work buffers exceed the fixed array of
                               mpgeo_batch_loglik_noalloc */
} mpgeo_status;

/* Flags (mpgeo_plan.flags and dataset flags). */
#define MPGEO_ORDER_MORTON 1u   /* reorder locations (and Z) by Z-order key before tiling */
#define MPGEO_INPUT_DEVICE 2u   /* pointer arguments are device pointers */
#define MPGEO_TIMING       4u   /* record HIP events per kernel launch (see mpgeo_ctx_kernel_stats) */
/* Profile likelihood in (theta2, theta3) (Section IV-C: for fixed range and smoothness the
 * variance maximising eq. (2) is theta1 = Z^T Sigma~^-1 Z / n, Sigma~ the correlation matrix,
 * i.e. eq. (1) at theta1 = 1).  With this flag theta.sigma2 is ignored (it must still be
 * finite and positive), the tiles hold
 * Sigma~, mpgeo_result.logdet = log|Sigma~|, .quad = q~ = Z^T Sigma~^-1 Z, and
 *   .loglik = -n/2 log(2 pi) - n/2 - n/2 log(q~ / n) - logdet/2,
 * which equals eq. (2) at theta = (q~/n, theta2, theta3).  The printed profile equation has
 * its trailing terms garbled; this is the form the substitution gives.  The variance
 * estimate is q~/n.  Kriging after such an evaluation uses theta1 = q~/n. */
#define MPGEO_PROFILE      8u
/* Great-circle distance (Section IV-B: for large regions): locations are (longitude,
 * latitude) in degrees and r in eq. (1) is the great-circle distance in km on a sphere of
 * radius 6371 km (the mean Earth radius), by the haversine formula
 *   a = sin^2(dlat/2) + cos(lat1) cos(lat2) sin^2(dlon/2),  r = 2 R asin(sqrt(min(a, 1))).
 * The Z-order key is then taken of ((lon + 180)/360, (lat + 90)/180).  A dataset flag (and
 * a one-shot plan flag); kriging sites use the same convention. */
#define MPGEO_DIST_GCD    16u
/* Batched evaluation (mpgeo_batch_loglik) as one persistent kernel over a device task queue
 * instead of per-problem launch sequences: every problem is cut into 128 x 128 tiles, FP64
 * within band64 tiles of the diagonal and FP32 beyond (Algorithm 1's map, each problem its own
 * band with MPGEO_TUNE_BAND), and factored left-looking, one task per lower tile (covariance
 * block in the tile's precision, the products with its earlier panels in that precision, then
 * the diagonal Cholesky fused with the forward solve, or the panel solve through the diagonal
 * inverse), workgroups taking tasks in dependency order from an atomic counter and waiting on
 * per-tile done flags.  For small problems, whose launch sequences leave the device idle.
 * Needs a two-tier plan (band64 >= -1, band32 = -1, lowp = 0, band0 = -1, dist64 = 0), tile
 * 128 or 0 (then 128), and n <= 16384 per problem; otherwise MPGEO_E_UNSUPPORTED.  Results agree
 * with mpgeo_loglik to rounding (the products are summed in another order), not bit for bit. */
#define MPGEO_BATCH_QUEUE 32u
/* Escalation on loss of positive definiteness.  With too much of the matrix in reduced
 * precision the factorization can meet a non-positive pivot even though Sigma itself is
 * positive definite (Section VIII-D-1 reports this for single precision near the diagonal,
 * which stops the MLE).  With this flag an evaluation that fails so is repeated with every
 * reduced band widened, b -> 2b + 1 for band64, band32 and band0, a band that reaches the
 * last tile row becoming "all" (-1: every tile FP64 and nothing dropped, and then no third
 * tier); a map drawn from distances goes straight to all-FP64.  The repetition stops at the
 * first success or after the all-FP64 plan.  mpgeo_result.escalations counts the repetitions
 * and .band64 / .band32 / .band0 give the bands of the reported result.  Honoured by
 * mpgeo_loglik, mpgeo_dataset_loglik, mpgeo_dataset_mle (every evaluation of the search),
 * mpgeo_dataset_simulate, mpgeo_factor_dense, and the persistent-queue batch
 * (mpgeo_batch_loglik with MPGEO_BATCH_QUEUE, mpgeo_batch_loglik_noalloc), where the problems
 * that failed run again in a launch of their own at the widened FP64 band; the batched lanes and
 * the serving loop return MPGEO_E_UNSUPPORTED with it. */
#define MPGEO_ESCALATE    64u
/* Band tuning for batched evaluation (mpgeo_batch_loglik; the choice of the precision map that
 * Section VIII-C-1 makes by hand for each size).  plan.band64 is then ignored: for each class
 * of problems (half-octave of n, smoothness to a quarter, half-octave of the range: the last
 * two set Sigma's conditioning; tile, path) the first two problems of the class are evaluated
 * all-FP64 and with FP64 bands 0, 1, 2, 4, 8 tiles (FP32 beyond), and the narrowest band at
 * which both factor and stay within 1e-7 of their all-FP64 log-likelihood is used for the
 * whole class (all-FP64 when none is).  The 1e-7 is relative to the size of the terms that
 * eq. (2) sums, S = (n log 2 pi + |log|Sigma|| + z^T Sigma^-1 z) / 2 (of the profiled form with
 * MPGEO_PROFILE), not to l, which passes through zero where they cancel.  To keep l within
 * 1e-5 of itself, a problem whose result at the class's band has |l| < 3 e S / 1e-5 (e: the
 * larger error of the two probes, at least 1e-9) is evaluated again all-FP64
 * (mpgeo_result.escalations counts it, band64 is then -1).  The choice depends only on the
 * probes' deterministic results and is kept in the context for later batches;
 * mpgeo_result.band64 reports the band each problem was computed at.  With plan.tile = 0 the
 * tile is tuned first, on the all-FP64 plan.  Works with and without MPGEO_BATCH_QUEUE; other
 * entry points ignore the flag. */
#define MPGEO_TUNE_BAND  128u
/* Reserved for graph replay of the factorization (the launch sequence of one evaluation
 * captured into a HIP graph and replayed per theta, for problems whose time is dominated by
 * launching small kernels).  Switched off: every entry point returns MPGEO_E_UNSUPPORTED when
 * it is set. */
#define MPGEO_GRAPH      256u

/* theta of eq. (1): sigma2 = theta1 (variance), beta = theta2 (range), nu = theta3
 * (smoothness); all must be finite and > 0. */
typedef struct {
    double sigma2;
    double beta;
    double nu;
} mpgeo_theta;

/* Tiling and precision plan.
 *  tile:   tile size nb (1..512); the matrix has p = ceil(n / nb) tile rows.
 *  band64: b >= 0: tile (i, j) is FP64 iff i - j <= b; -1: every tile FP64.
 *  band32: c >= 0: FP32 operands for band64 < i - j <= band64 + c, 16-bit operands beyond;
 *          -1: FP32 from band64 + 1 to the edge of the matrix (two tiers).
 *  lowp:   0 with band32 = -1; 1 (FP16) or 2 (BF16) with band32 >= 0.
 *  flags:  MPGEO_ORDER_MORTON | MPGEO_INPUT_DEVICE | MPGEO_TIMING | MPGEO_PROFILE |
 *          MPGEO_DIST_GCD | MPGEO_BATCH_QUEUE, MPGEO_TUNE_BAND (mpgeo_batch_loglik only) |
 *          MPGEO_ESCALATE.
 *  band0:  z >= 0: tiles with i - j > z are dropped (taken as zero, never stored, generated or
 *          updated: the diagonal-super-tile approximation the paper compares against, which
 *          factors the block-banded matrix exactly because the Cholesky factor of a matrix of
 *          tile bandwidth z has no fill-in beyond z); the other bands are capped at z.
 *          -1: no tile is dropped.
 *  dist64: > 0: the precision map is drawn from distances instead of tile offsets: tile (i, j)
 *          is FP64 when the bounding boxes of its two blocks of (ordered) sites come within
 *          dist64 of each other (diagonal tiles always), FP32 otherwise, or, with dist32 > 0 and
 *          a lowp format, FP32 within dist32 and 16-bit operands beyond.  band64 and band32
 *          are then ignored; band0 must be -1; Euclidean sites only; needs a dataset (not
 *          mpgeo_factor_dense).  0: the tile-offset bands above.
 *  dist32: see dist64; 0 unless dist64 > 0 with a lowp format (then dist32 >= dist64). */
typedef struct {
    int32_t tile;
    int32_t band64;
    int32_t band32;
    int32_t lowp;
    uint32_t flags;
    int32_t band0;
    double dist64;
    double dist32;
} mpgeo_plan;

/* Result of one evaluation.  loglik, logdet (natural log of det Sigma) and quad
 * (Z^T Sigma^-1 Z) are those of eq. (2).  info: -1, or the failing global column when
 * the status is MPGEO_E_NOT_SPD.  Times are seconds measured with HIP events on the
 * context stream: covariance generation, factorisation (including the fused forward
 * solve), final reduction, and the whole call. */
typedef struct {
    double loglik;
    double logdet;
    double quad;
    int64_t info;
    double t_covgen;
    double t_factor;
    double t_solve;
    double t_total;
    int32_t band64;        /* bands of the plan the result was computed with: the plan's own, */
    int32_t band32;        /* or the widened ones after MPGEO_ESCALATE */
    int32_t band0;
    int32_t escalations;   /* repetitions with wider bands (MPGEO_ESCALATE) or all-FP64 (MPGEO_TUNE_BAND) */
} mpgeo_result;

/* Per-kernel-class launch statistics accumulated while MPGEO_TIMING is set. */
typedef struct {
    char name[32];
    int64_t launches;
    double seconds;     /* sum of HIP-event durations of those launches */
    double flops;       /* algorithmic flops of those launches */
    double bytes;       /* algorithmic bytes (read + written) of those launches */
} mpgeo_kernel_stat;

typedef struct mpgeo_ctx mpgeo_ctx;
typedef struct mpgeo_dataset mpgeo_dataset;

/* Create a context on HIP device `device`, ordering all work on `hip_stream`
 * (a hipStream_t; NULL: the library creates its own stream).  hbm_budget_bytes > 0 caps the
 * tile memory of any one evaluation in this context: a call whose plan needs more lower-triangle
 * tile bytes than that (mpgeo_footprint_bytes, the 16-bit factor copy included) returns
 * MPGEO_E_NOMEM before allocating; batched calls size their groups within it.  0: no cap
 * beyond the device's memory.  *out receives the handle. */
int mpgeo_ctx_create(mpgeo_ctx **out, int device, void *hip_stream, size_t hbm_budget_bytes);

/* Free a context and its cached device memory.  NULL is accepted. */
int mpgeo_ctx_destroy(mpgeo_ctx *ctx);

/* Kernel statistics since the last reset: writes up to `max` entries to `out` and the
 * number of kernel classes to *count.  Reset clears them. */
int mpgeo_ctx_kernel_stats(mpgeo_ctx *ctx, mpgeo_kernel_stat *out, int max, int *count);
int mpgeo_ctx_reset_stats(mpgeo_ctx *ctx);

/* One-shot log-likelihood, eq. (2): orders the n locations (MPGEO_ORDER_MORTON), builds
 * the Matérn tiles, factors them with the plan's precision map, solves, and reduces.
 * locs: n x 2, z: n (host, or device with MPGEO_INPUT_DEVICE); not modified.  Device
 * workspace is cached in the context and reused by later calls of the same size. */
int mpgeo_loglik(mpgeo_ctx *ctx, int64_t n, const double *locs, const double *z,
                 mpgeo_theta theta, mpgeo_plan plan, mpgeo_result *out);

/* Resident dataset: copies locations and z to the device once, Morton-orders them when
 * flags has MPGEO_ORDER_MORTON, and keeps tile memory across evaluations (the
 * maximum-likelihood loop of Section IV-C changes only theta). */
int mpgeo_dataset_create(mpgeo_ctx *ctx, int64_t n, const double *locs, const double *z,
                         uint32_t flags, mpgeo_dataset **out);
int mpgeo_dataset_destroy(mpgeo_dataset *ds);

/* eq. (2) at theta for the resident dataset (or the profile likelihood with
 * MPGEO_PROFILE).  plan.flags may add MPGEO_TIMING and MPGEO_PROFILE; its ordering and
 * input flags are ignored (fixed at dataset creation). */
int mpgeo_dataset_loglik(mpgeo_dataset *ds, mpgeo_theta theta, mpgeo_plan plan,
                         mpgeo_result *out);

/* Simple-kriging prediction (Section VIII-D) at m new sites from the factor of the last
 * successful mpgeo_dataset_loglik call: pred = Sigma(new, S) Sigma^-1 Z, and, when var is
 * not NULL, var = theta1 - Sigma(new, S) Sigma^-1 Sigma(S, new).  new_locs: m x 2;
 * pred, var: m entries in the order of new_locs; host or device like the dataset.
 * MPGEO_E_ARG if no factor is available. */
int mpgeo_dataset_krige(mpgeo_dataset *ds, int64_t m, const double *new_locs,
                        double *pred, double *var);

/* Inspection (tests): copy to HOST memory
 *  perm:   n int64, the ordering used (ordered position -> caller index);
 *  matrix: the n x n lower triangle (column-major, ld >= n) of the tiles as they are now:
 *          after mpgeo_dataset_covariance the tier-rounded Sigma, after a loglik the
 *          factor L; FP32 tiles promoted; the strict upper triangle is left untouched;
 *  y:      the forward-solve vector L^-1 Z (n entries, ordered). */
int mpgeo_dataset_perm(mpgeo_dataset *ds, int64_t *perm);
int mpgeo_dataset_covariance(mpgeo_dataset *ds, mpgeo_theta theta, mpgeo_plan plan);
int mpgeo_dataset_matrix(mpgeo_dataset *ds, double *out, int64_t ld);
int mpgeo_dataset_solution(mpgeo_dataset *ds, double *y);

/* Synthetic data (Section VIII-B.1: measurements drawn from a parameter vector theta_0):
 * factors Sigma(theta) of the dataset's locations with the plan and writes
 * z = P^T L P eps, a draw of the zero-mean Gaussian field with covariance Sigma(theta),
 * where P is the dataset's ordering.  eps (n standard normal values) and z_out are in
 * the caller's order, host or device like the dataset.  The dataset's own data vector is
 * not changed; the factor stays resident as after a loglik call.  MPGEO_E_ARG with
 * MPGEO_PROFILE (a draw needs the variance). */
int mpgeo_dataset_simulate(mpgeo_dataset *ds, mpgeo_theta theta, mpgeo_plan plan,
                           const double *eps, double *z_out);

/* Sampled entries of the stored lower triangle (tests at sizes where a dense copy does
 * not fit): out[q] = M[max(r, c)][min(r, c)] for r = rows[q], c = cols[q] (0-based indices
 * in the ordered matrix), where M is the tier-rounded Sigma after mpgeo_dataset_covariance
 * or the factor L after a loglik (pass r >= c for L).  rows, cols, out: count entries in
 * HOST memory.  MPGEO_E_ARG for an index outside [0, n). */
int mpgeo_dataset_entries(mpgeo_dataset *ds, int64_t count, const int64_t *rows,
                          const int64_t *cols, double *out);

/* Maximum-likelihood estimate of theta (Section IV-C: maximise eq. (2)) with a
 * Nelder-Mead simplex on u = log(theta): reflection 1, expansion 2, contraction 1/2,
 * shrink 1/2, initial steps of 0.1 in each log-parameter from `start`; theta is clamped
 * to [0.01, 10] x [0.001, 2] x [0.1, 3]; a point whose matrix is not positive definite
 * scores -infinity.  Stops when the simplex spans less than xtol (log units, max-norm),
 * when ftol > 0 and its log-likelihoods differ by less than ftol * |best|, or after
 * max_evals evaluations.  Writes the best theta, its log-likelihood, and the evaluation and
 * iteration counts (any output pointer may be NULL).  With MPGEO_PROFILE in plan.flags the
 * simplex is two-dimensional, over (log theta2, log theta3) of the profile likelihood
 * (start.sigma2 is ignored), and theta_hat.sigma2 = q~/n at the best point. */
int mpgeo_dataset_mle(mpgeo_dataset *ds, mpgeo_theta start, mpgeo_plan plan, double xtol,
                      double ftol, int32_t max_evals, mpgeo_theta *theta_hat,
                      double *loglik_hat, int32_t *evals, int32_t *iters);

/* mpgeo_dataset_mle that also records the search's trajectory, the sequence of parameter
 * vectors an optimiser asks a likelihood service for (Section VIII-D-2: each fit is many
 * evaluations of eq. (2)): trace[e] (max_evals entries, host memory, not NULL) receives the
 * e-th evaluated theta and trace_loglik[e] (nullable) its log-likelihood, -infinity where the
 * matrix was not positive definite; *evals of them are written.  Same search, same result. */
int mpgeo_dataset_mle_trace(mpgeo_dataset *ds, mpgeo_theta start, mpgeo_plan plan, double xtol,
                            double ftol, int32_t max_evals, mpgeo_theta *theta_hat,
                            double *loglik_hat, int32_t *evals, int32_t *iters,
                            mpgeo_theta *trace, double *trace_loglik);

/* Algorithm 1 on a caller-given symmetric positive-definite matrix: A is n x n,
 * column-major with leading dimension lda >= n, only its lower triangle is read; z
 * (n entries) is optional (NULL: quad = 0 and loglik uses quad = 0).  No reordering.
 * Fills logdet, quad and loglik as for eq. (2) (with MPGEO_PROFILE: A is taken as Sigma~ and
 * loglik is the profile form, which needs z). */
int mpgeo_factor_dense(mpgeo_ctx *ctx, int64_t n, const double *a, int64_t lda,
                       const double *z, mpgeo_plan plan, mpgeo_result *out);

/* One problem of a batch: its own n sites (n x 2, host memory), data z (n, host) and theta. */
typedef struct {
    int64_t n;
    const double *locs;
    const double *z;
    mpgeo_theta theta;
} mpgeo_instance;

/* Batched evaluation of eq. (2) for `count` independent problems (many small and medium
 * likelihoods, e.g. one per region or per candidate model, Section VIII).  Every instance is
 * Morton-ordered, tiled and factored with the plan's precision map, exactly as
 * mpgeo_loglik would; the evaluations are spread over private lanes of the context (each its
 * own pair of streams and workspace; MPGEO_BATCH_LANES, default 4) and enqueued without host
 * synchronisation, largest first.  plan.tile = 0 selects the tile size per instance by an
 * autotuner: for each half-octave of n (and precision plan) the first instance is timed (the
 * faster of two runs) with a tile covering it and with 128, 256, 384, 512 below n, and the
 * largest tile within 5% of the fastest is kept in the context for later batches.  The bands
 * of a mixed plan count tiles, so its results follow the tile chosen, which the timing decides:
 * pass a tile, or MPGEO_TUNE_BAND (whose band is probed for the tuned tile and keeps l within
 * its bar), where results must not depend on timing.  out[i] receives loglik, logdet, quad and info (times are 0); tiles, if
 * not NULL, the tile size used.  Inputs are host memory (MPGEO_INPUT_DEVICE and MPGEO_TIMING
 * are rejected).  With MPGEO_BATCH_QUEUE the batch runs as one persistent kernel instead
 * (see the flag); a wait in it that exceeds about two seconds aborts the kernel and returns
 * MPGEO_E_DEVICE.  Returns MPGEO_E_NOT_SPD if any instance failed (see out[i].info). */
int mpgeo_batch_loglik(mpgeo_ctx *ctx, int64_t count, const mpgeo_instance *inst, mpgeo_plan plan,
                       mpgeo_result *out, int32_t *tiles);

/* For callers that cannot allocate device memory (code that must not call hipMalloc or hipFree:
 * tight serving loops, harnesses that forbid allocation).  The persistent-queue batch of
 * mpgeo_batch_loglik (as with MPGEO_BATCH_QUEUE, which may be set or not: all-FP64 or
 * FP64-band/FP32 plans at tile 128 or 0, host inputs) with every work buffer -- packed inputs,
 * tiles, diagonal inverses, vectors, task list, done flags, results -- carved from one fixed
 * device array of MPGEO_NOALLOC_SCRATCH_BYTES (320 MiB) per GPU, which each GPU the library runs
 * on holds from its first context until the process ends.  The call makes no device allocation
 * and frees nothing; it copies the inputs in and the results out through the context's stream
 * and returns when they are on the host.  Problems are packed into groups that fit in the array,
 * one ordering launch and one queue launch per group; a problem that alone does not fit returns
 * MPGEO_E_TOO_LARGE before any work (all-FP64: up to n = 8,960 sites, 70 tile rows; FP64 band 2
 * with FP32 beyond: up to about n = 12,100), and MPGEO_TUNE_BAND returns MPGEO_E_UNSUPPORTED (its probe
 * evaluations would allocate).  Results are those of mpgeo_batch_loglik with MPGEO_BATCH_QUEUE
 * (same kernels, same arithmetic), out[i] as there.  Every call on one GPU shares that GPU's
 * array, which keeps the previous call's contents: calls that overlap on one GPU (from two
 * contexts or two host threads) race, and the caller must serialise them. */
#define MPGEO_NOALLOC_SCRATCH_BYTES (320ull << 20)
int mpgeo_batch_loglik_noalloc(mpgeo_ctx *ctx, int64_t count, const mpgeo_instance *inst,
                               mpgeo_plan plan, mpgeo_result *out);

/* Serving loop for many likelihood requests (the inner loop of many maximum-likelihood fits,
 * Section VIII-D-2): datasets are registered once (host copies kept); requests (dataset, theta)
 * are submitted with arrival times in seconds; mpgeo_server_run replays them in real time from
 * its start: a request is ready at its arrival, and a dispatcher gives the oldest ready
 * request whose dataset is idle to a free lane (lanes as in mpgeo_batch_loglik) without waiting
 * for other requests.  A dataset's tiles stay resident on the device between its requests;
 * a dataset is admitted when its tile footprint (mpgeo_footprint_bytes) fits in
 * hbm_budget_bytes next to the resident ones, evicting idle datasets least recently used first.
 * Results match mpgeo_dataset_loglik of the same dataset and theta (same kernels).  A server
 * belongs to one context; run is synchronous and clears the submitted requests. */
typedef struct mpgeo_server mpgeo_server;
typedef struct {
    double loglik, logdet, quad;
    int64_t info;        /* -1, or the failing column (MPGEO_E_NOT_SPD is then returned) */
    double arrival_s;    /* as submitted */
    double start_s;      /* dispatched to a lane, seconds since the run began */
    double finish_s;     /* completion observed by the dispatcher */
} mpgeo_served;
int mpgeo_server_create(mpgeo_ctx *ctx, uint64_t hbm_budget_bytes, int32_t lanes, mpgeo_server **out);
/* MPGEO_E_NOMEM if the dataset could never fit in the budget. */
int mpgeo_server_add_dataset(mpgeo_server *srv, int64_t n, const double *locs, const double *z,
                             mpgeo_plan plan, int32_t *id);
int mpgeo_server_submit(mpgeo_server *srv, int32_t dataset, mpgeo_theta theta, double arrival_s,
                        int64_t *ticket);
/* A kriging request (the prediction experiment, Section VIII-D): the factor of (dataset, theta)
 * as for mpgeo_server_submit (its loglik, logdet and quad are reported alike), then simple
 * kriging from it on the same lane: predictions at m >= 1 new sites (m x 2, host memory, copied
 * at submission) into pred (m doubles, host) and, when var is not NULL (m <= 65535), the
 * prediction variances into var.  The outputs are written when mpgeo_server_run returns and
 * must stay valid until then.  Results equal mpgeo_dataset_krige after mpgeo_dataset_loglik of
 * the same dataset and theta. */
int mpgeo_server_submit_krige(mpgeo_server *srv, int32_t dataset, mpgeo_theta theta, int64_t m,
                              const double *new_locs, double *pred, double *var, double arrival_s,
                              int64_t *ticket);
/* out: one entry per submitted request, in submission (ticket) order. */
int mpgeo_server_run(mpgeo_server *srv, mpgeo_served *out);
int mpgeo_server_destroy(mpgeo_server *srv);

/* HBM bytes of the lower-triangle tiles for n and plan, plus, with a 16-bit tier, the 16-bit
 * copy of the factor that its left-looking updates read (2 bytes per entry of every lower
 * tile); admission control.  For a map drawn from distances, which needs the sites, the
 * all-FP64 bound. */
size_t mpgeo_footprint_bytes(int64_t n, mpgeo_plan plan);

/* The precision map of Algorithm 1 for n and plan, computed on the host (no device call):
 * effective bands, tile counts per tier and the algorithmic flops of each tier (the trailing
 * SYRK/GEMM updates counted by the tier of the tile they write, the panel TRSMs by the tier of
 * the panel tile, POTRF as rows^3/3 per diagonal tile).  MPGEO_E_ARG for an invalid plan. */
typedef struct {
    int64_t p;                 /* tile rows, ceil(n / tile) */
    int32_t nbp;               /* physical tile size (tile rounded up to 32) */
    int32_t band64;            /* effective: FP64 iff i - j <= band64 */
    int32_t edge;              /* effective: 16-bit update operands iff i - j > edge */
    int32_t band0;             /* effective: dropped iff i - j > band0 */
    int32_t lowp;              /* effective 16-bit format (0 when no tile is in that tier) */
    int32_t reserved;
    int64_t tiles[4];          /* FP64, FP32, FP32 with 16-bit operands, dropped */
    double update_flops[3];    /* FP64, FP32, 16-bit tier */
    double trsm_flops[2];      /* FP64, FP32 */
    double potrf_flops;
    uint64_t footprint_bytes;  /* as mpgeo_footprint_bytes */
} mpgeo_tier_summary;
int mpgeo_plan_tiers(int64_t n, mpgeo_plan plan, mpgeo_tier_summary *out);

/* Static text for a status code. */
const char *mpgeo_status_string(int status);

#ifdef __cplusplus
}
#endif

#endif /* MPGEO_H */
