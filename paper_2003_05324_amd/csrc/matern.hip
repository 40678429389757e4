// Matérn covariance tiles (eq. (1), Section IV-B) and kriging cross-covariances.  The
// covariance and distance evaluation is in matern_dev.h.
#include "matern_dev.h"

#include <cmath>

namespace mpgeo {

MaternParams make_matern_params(double sigma2, double beta, double nu) {
    MaternParams mp{};
    mp.sigma2 = sigma2;
    mp.beta = beta;
    mp.nu = nu;
    mp.pref = sigma2 / (std::pow(2.0, nu - 1.0) * std::tgamma(nu));
    mp.nl = (int)std::floor(nu + 0.5);
    mp.mu = nu - mp.nl;
    mp.mode = (nu == 0.5) ? 1 : (nu == 1.5) ? 2 : (nu == 2.5) ? 3 : 0;
    return mp;
}

namespace {

constexpr int kCovCols = 32;   // tile columns per workgroup
constexpr int kCovThreads = 256;

// Physical row r of tile row i -> logical global index, or -1 for a padding row.
__device__ inline int64_t logical_row(int i, int r, int nb, int64_t n) {
    if (r >= nb) return -1;
    const int64_t g = (int64_t)i * nb + r;
    return g < n ? g : -1;
}

template <typename Source>
__global__ __launch_bounds__(kCovThreads) void fill_tiles_kernel(TileMap map, const TileIJ *tiles,
                                                                   Source src) {
    const TileIJ t = tiles[blockIdx.x];
    const int nbp = map.nbp;
    const int c0 = blockIdx.y * kCovCols;
    const bool f64 = tile_is_fp64(map, t.i, t.j);
    const int64_t off = map.off[tri_index(t.i, t.j)];
    __shared__ int64_t gcol[kCovCols];
    if (threadIdx.x < kCovCols) gcol[threadIdx.x] = logical_row(t.j, c0 + threadIdx.x, map.nb, map.n);
    src.prepare_cols(t, c0, gcol);
    __syncthreads();
    for (int r = threadIdx.x; r < nbp; r += kCovThreads) {
        const int64_t gr = logical_row(t.i, r, map.nb, map.n);
        src.prepare_row(gr);
        for (int cc = 0; cc < kCovCols; ++cc) {
            const int c = c0 + cc;
            double v;
            if (gr < 0 || gcol[cc] < 0) v = (t.i == t.j && r == c) ? 1.0 : 0.0;
            else v = src.value(gr, cc, gcol[cc]);
            const int64_t e = off + r + (int64_t)c * nbp;
            if (f64) map.pool64[e] = v;
            else map.pool32[e] = (float)v;   // round to nearest even
        }
    }
}

struct MaternSource {
    const double *locs;
    MaternParams mp;
    double xr, yr, cr;          // row site: x, y (great-circle: lon in degrees, lat in radians, cos lat)
    double *sx, *sy, *sc;       // shared column sites, same convention
    const MaternTable *tab;     // smoothness-only factors of K_mu (read for general smoothness only)
    __device__ void prepare_cols(const TileIJ &, int, const int64_t *gcol) {
        __shared__ double cx[kCovCols], cy[kCovCols], ccs[kCovCols];
        __shared__ MaternTable mtab;
        sx = cx;
        sy = cy;
        sc = ccs;
        tab = &mtab;
        if (mp.mode == 0 && mp.mu != -0.5) matern_table_build(mp.mu, mtab);
        if (threadIdx.x < kCovCols) {
            const int64_t g = gcol[threadIdx.x];
            const double x = g >= 0 ? locs[2 * g] : 0.0;
            const double y = g >= 0 ? locs[2 * g + 1] : 0.0;
            cx[threadIdx.x] = x;
            cy[threadIdx.x] = mp.gcd ? y * kDegToRad : y;
            ccs[threadIdx.x] = mp.gcd ? cos(y * kDegToRad) : 0.0;
        }
    }
    __device__ void prepare_row(int64_t gr) {
        if (gr >= 0) {
            xr = locs[2 * gr];
            yr = locs[2 * gr + 1];
            if (mp.gcd) {
                yr *= kDegToRad;
                cr = cos(yr);
            }
        }
    }
    __device__ double value(int64_t gr, int cc, int64_t gc) const {
        if (gr == gc) return mp.sigma2;
        if (mp.gcd) return matern_cov_tab(haversine(sx[cc] - xr, yr, cr, sy[cc], sc[cc]), mp, *tab);
        const double dx = xr - sx[cc];
        const double dy = yr - sy[cc];
        return matern_cov_tab(sqrt(dx * dx + dy * dy), mp, *tab);
    }
};

struct DenseSource {
    const double *a;
    int64_t lda;
    __device__ void prepare_cols(const TileIJ &, int, const int64_t *) {}
    __device__ void prepare_row(int64_t) {}
    __device__ double value(int64_t gr, int, int64_t gc) const {
        // only the lower triangle of the caller's matrix is read
        return gr >= gc ? a[gr + gc * lda] : a[gc + gr * lda];
    }
};

__global__ __launch_bounds__(kCovThreads) void export_tiles_kernel(TileMap map, const TileIJ *tiles,
                                                                     double *out, int64_t ld) {
    const TileIJ t = tiles[blockIdx.x];
    const int nbp = map.nbp;
    const int c0 = blockIdx.y * kCovCols;
    const bool f64 = tile_is_fp64(map, t.i, t.j);
    const int64_t off = map.off[tri_index(t.i, t.j)];
    for (int r = threadIdx.x; r < nbp; r += kCovThreads) {
        const int64_t gr = logical_row(t.i, r, map.nb, map.n);
        if (gr < 0) continue;
        for (int cc = 0; cc < kCovCols; ++cc) {
            const int c = c0 + cc;
            const int64_t gc = logical_row(t.j, c, map.nb, map.n);
            if (gc < 0 || gc > gr) continue;
            const int64_t e = off + r + (int64_t)c * nbp;
            out[gr + gc * ld] = f64 ? map.pool64[e] : (double)map.pool32[e];
        }
    }
}

__global__ void entries_kernel(TileMap map, int64_t count, const int64_t *rows,
                               const int64_t *cols, double *out) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count) return;
    int64_t r = rows[q], c = cols[q];
    if (r < c) {
        const int64_t t = r;
        r = c;
        c = t;
    }
    const int i = (int)(r / map.nb), j = (int)(c / map.nb);
    const int64_t e = map.off[tri_index(i, j)] + (r - (int64_t)i * map.nb) +
                      (c - (int64_t)j * map.nb) * map.nbp;
    out[q] = tile_is_fp64(map, i, j) ? map.pool64[e] : (double)map.pool32[e];
}

__global__ void pad_vector_kernel(const double *src, double *dst, int64_t n, int nb, int nbp,
                                  int64_t total) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int64_t i = e / nbp;
    const int r = (int)(e - i * nbp);
    const int64_t g = i * nb + r;
    dst[e] = (r < nb && g < n) ? src[g] : 0.0;
}

__global__ void unpad_vector_kernel(const double *src, double *dst, int64_t n, int nb, int nbp) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const int64_t i = g / nb;
    const int64_t r = g - i * nb;
    dst[g] = src[i * nbp + r];
}

constexpr int kKrigeThreads = 256;
constexpr int kKrigeChunk = 256;

// pred_j = sum_a C(||s0_j - s_a||) w_a; one thread per prediction site, locations
// streamed through LDS in chunks.
__global__ __launch_bounds__(kKrigeThreads) void krige_predict_kernel(
    const double *locs, int64_t n, int nb, int nbp, const double *new_locs, int64_t m,
    const double *w, MaternParams mp, double *pred) {
    __shared__ double sx[kKrigeChunk], sy[kKrigeChunk], sw[kKrigeChunk];
    const int64_t j = (int64_t)blockIdx.x * kKrigeThreads + threadIdx.x;
    const double x0 = j < m ? new_locs[2 * j] : 0.0;
    const double y0 = j < m ? new_locs[2 * j + 1] : 0.0;
    double acc = 0.0;
    for (int64_t a0 = 0; a0 < n; a0 += kKrigeChunk) {
        const int64_t a = a0 + threadIdx.x;
        if (a < n) {
            sx[threadIdx.x] = locs[2 * a];
            sy[threadIdx.x] = locs[2 * a + 1];
            const int64_t ti = a / nb;
            sw[threadIdx.x] = w[ti * nbp + (a - ti * nb)];
        }
        __syncthreads();
        const int cnt = (int)((n - a0) < kKrigeChunk ? (n - a0) : kKrigeChunk);
        for (int q = 0; q < cnt; ++q) acc += matern_cov(site_distance(x0, y0, sx[q], sy[q], mp.gcd), mp) * sw[q];
        __syncthreads();
    }
    if (j < m) pred[j] = acc;
}

// c[(physical row of a) + j * ldc] = C(||s0_j - s_a||); padding rows are zero.
__global__ void cross_cov_kernel(const double *locs, int64_t n, int nb, int nbp, int64_t rows,
                                 const double *new_locs, int64_t m, MaternParams mp, double *c,
                                 int64_t ldc) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (e >= rows || j >= m) return;
    const int64_t ti = e / nbp;
    const int r = (int)(e - ti * nbp);
    const int64_t a = ti * nb + r;
    double v = 0.0;
    if (r < nb && a < n)
        v = matern_cov(site_distance(new_locs[2 * j], new_locs[2 * j + 1], locs[2 * a], locs[2 * a + 1], mp.gcd), mp);
    c[e + j * ldc] = v;
}

}  // namespace

void launch_covgen(const TileMap &map, const double *locs, const TileIJ *tiles, int64_t ntiles,
                   const MaternParams &mp, hipStream_t stream) {
    if (ntiles == 0) return;
    MaternSource src{locs, mp, 0.0, 0.0, 0.0, nullptr, nullptr, nullptr};
    dim3 grid((unsigned)ntiles, map.nbp / kCovCols);
    hipLaunchKernelGGL(fill_tiles_kernel<MaternSource>, grid, dim3(kCovThreads), 0, stream, map,
                       tiles, src);
}

void launch_import_dense(const TileMap &map, const double *a, int64_t lda, const TileIJ *tiles,
                         int64_t ntiles, hipStream_t stream) {
    if (ntiles == 0) return;
    DenseSource src{a, lda};
    dim3 grid((unsigned)ntiles, map.nbp / kCovCols);
    hipLaunchKernelGGL(fill_tiles_kernel<DenseSource>, grid, dim3(kCovThreads), 0, stream, map,
                       tiles, src);
}

void launch_export_dense(const TileMap &map, double *out, int64_t ld, const TileIJ *tiles,
                         int64_t ntiles, hipStream_t stream) {
    if (ntiles == 0) return;
    dim3 grid((unsigned)ntiles, map.nbp / kCovCols);
    hipLaunchKernelGGL(export_tiles_kernel, grid, dim3(kCovThreads), 0, stream, map, tiles, out,
                       ld);
}

void launch_entries(const TileMap &map, int64_t count, const int64_t *rows, const int64_t *cols,
                    double *out, hipStream_t stream) {
    if (count <= 0) return;
    hipLaunchKernelGGL(entries_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream, map,
                       count, rows, cols, out);
}

void launch_pad_vector(const double *src, double *dst, int64_t n, int nb, int nbp, int p,
                       hipStream_t stream) {
    const int64_t total = (int64_t)p * nbp;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    hipLaunchKernelGGL(pad_vector_kernel, dim3(blocks), dim3(256), 0, stream, src, dst, n, nb,
                       nbp, total);
}

namespace {
__global__ void fill_u64_kernel(unsigned long long *p, unsigned long long value, int64_t count) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) p[e] = value;
}
}  // namespace

void launch_fill_u64(unsigned long long *p, unsigned long long value, int64_t count, hipStream_t stream) {
    if (count <= 0) return;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream, p, value,
                       count);
}

void launch_unpad_vector(const double *src, double *dst, int64_t n, int nb, int nbp,
                         hipStream_t stream) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(unpad_vector_kernel, dim3(blocks), dim3(256), 0, stream, src, dst, n, nb,
                       nbp);
}

void launch_krige_predict(const double *locs, int64_t n, int nb, int nbp, const double *new_locs,
                          int64_t m, const double *w, const MaternParams &mp, double *pred,
                          hipStream_t stream) {
    if (m == 0) return;
    const unsigned blocks = (unsigned)((m + kKrigeThreads - 1) / kKrigeThreads);
    hipLaunchKernelGGL(krige_predict_kernel, dim3(blocks), dim3(kKrigeThreads), 0, stream, locs,
                       n, nb, nbp, new_locs, m, w, mp, pred);
}

void launch_cross_cov(const double *locs, int64_t n, int nb, int nbp, int p,
                      const double *new_locs, int64_t m, const MaternParams &mp, double *c,
                      int64_t ldc, hipStream_t stream) {
    if (m == 0) return;
    const int64_t rows = (int64_t)p * nbp;
    dim3 grid((unsigned)((rows + 255) / 256), (unsigned)m);
    hipLaunchKernelGGL(cross_cov_kernel, grid, dim3(256), 0, stream, locs, n, nb, nbp, rows,
                       new_locs, m, mp, c, ldc);
}

}  // namespace mpgeo
