// Internal declarations shared by the HIP sources of libmpgeo (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstddef>

namespace mpgeo {

// Physical tiles are padded to a multiple of kTileQuantum rows/columns; the padding
// rows and columns hold an identity block (unit diagonal, zero elsewhere) and a zero
// right-hand side.  Because those rows are decoupled from the rest, the Cholesky
// factor, log-determinant and quadratic form of the padded matrix equal those of the
// true matrix exactly.
constexpr int kTileQuantum = 32;
constexpr int kMaxTile = 512;

struct TileIJ {
    int32_t i;
    int32_t j;
};

// Index of lower tile (i, j), i >= j, in row-major packed lower-triangular order.
__host__ __device__ inline int64_t tri_index(int64_t i, int64_t j) {
    return i * (i + 1) / 2 + j;
}

// Where the tiles live: one pool per precision; off[tri_index(i, j)] is the element
// offset of tile (i, j) inside the pool of its precision (FP64 iff i - j <= band, or, for a
// precision map drawn from distances, iff fp64tab[tri_index(i, j)] is non-zero).
struct TileMap {
    const int64_t *off;
    double *pool64;
    float *pool32;
    int band;   // FP64 iff i - j <= band (band >= p - 1 means every tile is FP64)
    int nbp;    // physical tile size (multiple of kTileQuantum)
    int nb;     // logical tile size
    int p;      // tiles per side
    int64_t n;  // logical matrix order
    const signed char *fp64tab = nullptr;   // per-tile FP64 flag (distance map), or nullptr
};

__host__ __device__ inline bool tile_is_fp64(const TileMap &m, int i, int j) {
    return m.fp64tab ? m.fp64tab[tri_index(i, j)] != 0 : (i - j) <= m.band;
}

// ---- launchers (host functions; every kernel is enqueued on `stream`) -------------

// Matérn covariance of eq. (1) for every lower tile, written in the tile's precision.
struct MaternParams {
    double sigma2, beta, nu;
    double pref;   // sigma2 / (2^(nu-1) Gamma(nu))
    int nl;        // nu = mu + nl with mu in [-1/2, 1/2)
    double mu;
    int mode;      // 0 general nu, 1: nu = 1/2, 2: nu = 3/2, 3: nu = 5/2
    int gcd;       // 0: Euclidean distance; 1: great-circle distance of (lon, lat) in degrees
};

// Sphere radius of the great-circle distance (mean Earth radius, km).
constexpr double kEarthRadiusKm = 6371.0;
MaternParams make_matern_params(double sigma2, double beta, double nu);

void launch_covgen(const TileMap &map, const double *locs, const TileIJ *tiles,
                   int64_t ntiles, const MaternParams &mp, hipStream_t stream);

// Caller matrix (device, column-major, ld) -> tiles in their precision (identity padding).
void launch_import_dense(const TileMap &map, const double *a, int64_t lda,
                         const TileIJ *tiles, int64_t ntiles, hipStream_t stream);

// Tiles -> dense lower triangle (device, column-major, ld), FP32 promoted.
void launch_export_dense(const TileMap &map, double *out, int64_t ld, const TileIJ *tiles,
                         int64_t ntiles, hipStream_t stream);

// Sampled entries of the stored lower triangle (host-side indices copied in by the caller).
void launch_entries(const TileMap &map, int64_t count, const int64_t *rows, const int64_t *cols,
                    double *out, hipStream_t stream);

// count words of value (a kernel, not a memset node, so that the call may sit in a captured
// graph).
void launch_fill_u64(unsigned long long *p, unsigned long long value, int64_t count, hipStream_t stream);

// Logical vector (n) -> physical padded vector (p * nbp), zero in padding rows.
void launch_pad_vector(const double *src, double *dst, int64_t n, int nb, int nbp, int p,
                       hipStream_t stream);
void launch_unpad_vector(const double *src, double *dst, int64_t n, int nb, int nbp,
                         hipStream_t stream);

// Input check: *flag (zeroed by the caller) is set to 1 when an entry of the rows x cols
// column-major array a (leading dimension ld) is not finite; with lower, only entries on or
// below the diagonal are looked at.
void launch_find_nonfinite(const double *a, int64_t rows, int64_t cols, int64_t ld, bool lower,
                           int *flag, hipStream_t stream);

// Z-order keys, sort, and gather of locations and data.
void launch_morton_order(const double *locs_in, const double *z_in, int64_t n, bool lonlat,
                         uint64_t *keys, int64_t n2, double *locs_out, double *z_out,
                         int64_t *perm_out, hipStream_t stream);

// FP64 factorisation of diagonal tile k in place, its inverse (FP64 and FP32 copies),
// the forward-solve block y_k = L_kk^-1 r_k, and the step's log-det / quad parts.
struct PotrfArgs {
    double *a;         // tile (k, k), nbp x nbp column-major
    double *linv;      // out: L_kk^-1, nbp x nbp
    float *linv32;     // out: FP32 copy of L_kk^-1
    const double *r;   // residual block r_k (nbp)
    double *y;         // out: y_k (nbp)
    double *logdet_part;
    double *quad_part;
    unsigned long long *info;   // atomic min of the failing global column
    int64_t col_base;  // global logical column of the tile's first column
    int nb;            // logical tile size (columns >= nb are padding)
    int nbp;
    int ld = 0;        // leading dimension of a, linv, linv32 (0: nbp)
};
void launch_potrf(const PotrfArgs &a, hipStream_t stream);

// Panel TRSM of step k through the explicit inverse: X_i = A_ik L_kk^-T for
// i in [i_begin, i_begin + count), or, when `list` is not null, for the tiles
// list[0 .. count-1] (their .i; a precision map drawn from distances); writes the staging
// panels P64[i], P32[i].
void launch_trsm(const TileMap &map, int k, int i_begin, int count, bool fp64,
                 const double *linv, const float *linv32, double *p64, float *p32,
                 hipStream_t stream, bool narrow = false, const TileIJ *list = nullptr);

// Trailing update of step k: A_ij -= P_i P_j^T over list[0, count) (tiles all of one
// precision), with P the staging panel of that precision.
void launch_update(const TileMap &map, const TileIJ *list, int64_t count, bool fp64,
                   const double *p64, const float *p32, hipStream_t stream,
                   bool narrow = false);

// Third tier: the power of two s_i of each tile row i from the diagonal tiles of Sigma (to be
// called before the factorization overwrites them), into rscale[0 .. p).
void launch_row_scale(const TileMap &map, float *rscale, hipStream_t stream);
// Third tier: quantise panel tiles (i, k), i in [first, first + count), of the FP32 staging
// panel (tile i at p32 + i * nbp^2) to 16-bit (lowp 1: FP16, 2: BF16) as L_ik / s_i, row-major,
// into the 16-bit factor copy q at slot tri_index(i, k).
void launch_quantize(const TileMap &map, int k, int first, int count, const float *p32,
                     const float *rscale, void *q, int lowp, hipStream_t stream);
// Third tier: A_ij <- -s_i s_j (-A_ij / (s_i s_j) + sum_k Q_ik Q_jk^T) over list[0, count)
// (FP32-stored tiles), for panels k in [max(k0, i - zband), kend), ascending, from the 16-bit
// factor copy; k0 is kstart[t] for entry t when kstart is given, else kbeg.
void launch_update_lowp(const TileMap &map, const TileIJ *list, int64_t count, int kbeg, int kend,
                        int zband, const void *q, const float *rscale, int lowp, hipStream_t stream,
                        const int32_t *kstart = nullptr);
// Output tiles the many-panel 16-bit update runs at once on `cus` compute units (one wave of
// workgroups), 0 when unknown.
int lowp_wave_tiles(int nbp, int lowp, int cus);

// Panel step of the fused forward solve: r_i -= P64_i y_k for i = k+1 .. k+count, and copy
// the finished panel tile (i, k) from staging into its storage precision.
void launch_panel_solve(const TileMap &map, int k, int count, const double *p64, const double *yk,
                        double *r, hipStream_t stream);

// z = L eps over the tiles (physical padded vectors), lower triangle of diagonal tiles only.
void launch_trmv(const TileMap &map, const double *eps, double *z, hipStream_t stream);
// dst[perm[a]] = src[a] (to_caller) or dst[a] = src[perm[a]] (!to_caller), a < n.
void launch_permute(const double *src, double *dst, const int64_t *perm, int64_t n, bool to_caller,
                    hipStream_t stream);

// Reduction of the per-step parts into {loglik, logdet, quad} (device double[3]).
void launch_finalize(const double *logdet_part, const double *quad_part, int p, int64_t n,
                     bool profile, double *result, hipStream_t stream);

// Backward solve w = L^-T y over the tiles (uses the stored diagonal inverses).
void launch_backward_solve(const TileMap &map, const double *linv_all, const double *y,
                           double *t, double *w, hipStream_t stream);

// Kriging: pred_j = sum_a C(||s0_j - s_a||) w_a (physical padded w), j < m.
void launch_krige_predict(const double *locs, int64_t n, int nb, int nbp,
                          const double *new_locs, int64_t m, const double *w,
                          const MaternParams &mp, double *pred, hipStream_t stream);

// Cross-covariance columns for the kriging variance: c[(a phys) + j * ldc] = C(s0_j, s_a).
void launch_cross_cov(const double *locs, int64_t n, int nb, int nbp, int p,
                      const double *new_locs, int64_t m, const MaternParams &mp, double *c,
                      int64_t ldc, hipStream_t stream);

// Forward solve of many right-hand sides and their column norms:
// var_j = scale * (sigma2 - |L^-1 c_j|^2).
void launch_forward_multi(const TileMap &map, const double *linv_all, double *c, int64_t ldc,
                          int64_t m, double *tmp, hipStream_t stream);
void launch_column_var(const double *c, int64_t ldc, int64_t rows, int64_t m, double sigma2,
                       double scale, double *var, hipStream_t stream);

// ---- batched evaluation as one persistent kernel over a device task queue -------------------
constexpr int kQueueTile = 128;        // tile size of the queue path
constexpr int kQueueMaxN = 16384;      // largest problem (its sort runs in one workgroup's LDS)

// Tiles of a queued problem are packed in row-major lower order, a tile (i, j) with
// i - j <= band in FP64 (2 kQueueTile^2 four-byte units), the others in FP32 (kQueueTile^2
// units).  Offset of tile (i, j) in four-byte units: FP64 tiles before it (rows r < i hold
// min(r, band) + 1 each; row i those with j' >= i - band) count twice.
__host__ __device__ inline int64_t queue_fp64_before(int64_t i, int64_t j, int64_t band) {
    const int64_t rows = (i <= band + 1) ? i * (i + 1) / 2
                                         : (band + 1) * (band + 2) / 2 + (i - band - 1) * (band + 1);
    const int64_t first = i - band > 0 ? i - band : 0;
    return rows + (j > first ? j - first : 0);
}
__host__ __device__ inline int64_t queue_tile_units(int64_t i, int64_t j, int64_t band) {
    const int64_t te = (int64_t)kQueueTile * kQueueTile;
    return (tri_index(i, j) + queue_fp64_before(i, j, band)) * te;
}

// One problem of a queued batch; all offsets are in elements of the shared buffers.
struct BatchInst {
    int64_t n;
    int64_t in0;     // first site / datum in the packed inputs and ordered sites (sites 2 in0)
    int64_t tile0;   // tile (i, j) at tile0 + queue_tile_units(i, j, band) four-byte units
    int64_t linv0;   // L_jj^-1 at linv0 + j
    int64_t vec0;    // padded vectors z, r, y: element e at vec0 + e (p * kQueueTile long)
    int64_t flag0;   // done flag of tile (i, j) at flag0 + tri_index(i, j)
    int64_t part0;   // logdet parts at part0 + j, quadratic-form parts at part0 + p + j
    int32_t p;
    int32_t band;    // tile (i, j) is FP64 iff i - j <= band (band >= p - 1: every tile)
    MaternParams mp;
};
struct BatchTask {
    int32_t inst, i, j, pad_;
};
struct QueueArgs {
    const BatchTask *tasks;
    int64_t ntasks;
    const BatchInst *insts;
    const double *locs;        // ordered sites
    const double *z;           // ordered, padded data
    float *tiles;              // four-byte units (see queue_tile_units)
    double *linv, *r, *y, *parts;
    int *flags;                // zero on entry
    unsigned *head;            // zero on entry
    int *abort_flag;           // zero on entry; non-zero on exit: a wait timed out
    unsigned long long *info;  // per problem: all ones on entry, else the failing column
    double *result;            // per problem: loglik, logdet, quad
    int profile;
    int spin_limit;            // sleeps of ~0.25 us per wait before giving up
};
// Sites and data of every problem Morton-ordered (order) into locs / zpad; max_n <= kQueueMaxN.
void launch_batch_order(const BatchInst *insts, int64_t count, int max_n, const double *locs_in,
                        const double *z_in, double *locs, double *zpad, bool order, bool lonlat,
                        hipStream_t stream);
void launch_batch_queue(const QueueArgs &args, int workgroups, hipStream_t stream);
// p[0 .. count) = value (clearing flags and counters without a memset node)
void launch_fill_u32(uint32_t *p, uint32_t value, size_t count, hipStream_t stream);

}  // namespace mpgeo
