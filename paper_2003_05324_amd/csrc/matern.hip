// Matérn covariance tiles (eq. (1), Section IV-B) and kriging cross-covariances.
//
// K_nu for general smoothness: nu = mu + nl with mu in [-1/2, 1/2).  K_mu and K_mu+1
// come from Temme's series (J. Comput. Phys. 19, 1975) for x <= 2 and, for x > 2, from
// the ratios of the minimal solution u_k = U(mu + 1/2 + k, 2 mu + 1, 2x) of Kummer's
// contiguous recurrence, computed by backward (Miller) recurrence and normalised with
// Temme's identity sum_k (1/2+mu)_k (1/2-mu)_k / k! u_k = (2x)^(-mu-1/2) (the approach of
// Temme 1975 and Thompson & Barnett 1987).  Forward recurrence in the order then reaches
// nu.  Half-integer smoothness 1/2, 3/2, 5/2 uses the elementary closed forms.
#include "common.h"
#include "rgamma_coeffs.h"

#include <cmath>

namespace mpgeo {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Gamma1(mu) = (1/Gamma(1-mu) - 1/Gamma(1+mu)) / (2 mu) and
// Gamma2(mu) = (1/Gamma(1-mu) + 1/Gamma(1+mu)) / 2 from the power series of 1/Gamma(1+x).
__device__ inline void temme_gammas(double mu, double &g1, double &g2) {
    const double m2 = mu * mu;
    double odd = 0.0, even = 0.0;
#pragma unroll
    for (int j = MPGEO_RGAMMA_NCOEF - 1; j >= 0; --j) {
        if (j & 1) odd = odd * m2 + kRGammaCoef[j];
        else even = even * m2 + kRGammaCoef[j];
    }
    g1 = -odd;
    g2 = even;
}

// K_mu(x), K_mu+1(x) for |mu| <= 1/2 and 0 < x <= 2 (Temme's series).
__device__ void bessel_k_small(double mu, double x, double &k0, double &k1) {
    double g1, g2;
    temme_gammas(mu, g1, g2);
    const double gp = 1.0 / (g2 - mu * g1);   // Gamma(1 + mu)
    const double gm = 1.0 / (g2 + mu * g1);   // Gamma(1 - mu)
    const double lg = log(2.0 / x);
    const double sig = mu * lg;
    const double fact = (mu == 0.0) ? 1.0 : (kPi * mu) / sinpi(mu);
    const double fact2 = (sig == 0.0) ? 1.0 : sinh(sig) / sig;
    double f = fact * (cosh(sig) * g1 + fact2 * lg * g2);
    const double e = exp(sig);                // (2/x)^mu
    double p = 0.5 * e * gp;
    double q = 0.5 / e * gm;
    double c = 1.0;
    const double d = 0.25 * x * x;
    double s0 = f, s1 = p;
    const double m2 = mu * mu;
    for (int k = 1; k < 64; ++k) {
        const double dk = (double)k;
        f = (dk * f + p + q) / (dk * dk - m2);
        c *= d / dk;
        p /= (dk - mu);
        q /= (dk + mu);
        const double h = p - dk * f;
        const double t0 = c * f, t1 = c * h;
        s0 += t0;
        s1 += t1;
        if (fabs(t0) < 1e-17 * fabs(s0) && fabs(t1) < 1e-17 * fabs(s1)) break;
    }
    k0 = s0;
    k1 = s1 * 2.0 / x;
}

// e^x K_mu(x), e^x K_mu+1(x) for |mu| < 1/2 and x > 2.
__device__ void bessel_k_large_scaled(double mu, double x, double &k0s, double &k1s) {
    const double m2 = mu * mu;
    int kmax = 20 + (int)(130.0 / x);
    if (kmax > 90) kmax = 90;
    // C_k = (1/2 + mu)_k (1/2 - mu)_k / k!  at k = kmax
    double ck = 1.0;
    for (int t = 1; t <= kmax; ++t) {
        const double h = t - 0.5;
        ck *= (h * h - m2) / t;
    }
    double up1 = 0.0, u = 1.0;   // u_{k+1}, u_k (unnormalised), starting at k = kmax
    double s = ck * u;
    for (int k = kmax; k >= 1; --k) {
        const double kh = k + 0.5;
        const double um1 = 2.0 * (k + x) * u - (kh * kh - m2) * up1;
        up1 = u;
        u = um1;
        const double hm = k - 0.5;
        ck *= k / (hm * hm - m2);   // C_{k-1}
        s += ck * u;
    }
    k0s = sqrt(kPi / (2.0 * x)) / (s / u);
    k1s = k0s / x * (x + mu + 0.5 + (m2 - 0.25) * up1 / u);
}

}  // namespace

// C(r; theta) of eq. (1); C(0) = sigma2 (the r -> 0 limit).
__device__ inline double matern_cov(double r, const MaternParams &mp) {
    if (r == 0.0) return mp.sigma2;
    const double x = r / mp.beta;
    switch (mp.mode) {
        case 1: return mp.sigma2 * exp(-x);
        case 2: return mp.sigma2 * (1.0 + x) * exp(-x);
        case 3: return mp.sigma2 * (1.0 + x + x * x * (1.0 / 3.0)) * exp(-x);
        default: break;
    }
    if (x > 745.0) return 0.0;
    const double mu = mp.mu;
    double k0, k1;
    bool scaled;
    if (mu == -0.5) {          // K_{-1/2} = K_{1/2} = sqrt(pi/2x) e^-x, K_{1/2}(1 + 1/x) next
        k0 = sqrt(kPi / (2.0 * x));
        k1 = k0 * (1.0 + 1.0 / x);
        scaled = true;
    } else if (x <= 2.0) {
        bessel_k_small(mu, x, k0, k1);
        scaled = false;
    } else {
        bessel_k_large_scaled(mu, x, k0, k1);
        scaled = true;
    }
    for (int i = 1; i <= mp.nl; ++i) {
        const double k2 = (2.0 * (mu + i) / x) * k1 + k0;
        k0 = k1;
        k1 = k2;
    }
    if (scaled) return mp.pref * exp(mp.nu * log(x) - x) * k0;
    return mp.pref * pow(x, mp.nu) * k0;
}

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

constexpr double kDegToRad = 3.14159265358979323846 / 180.0;

// Great-circle distance by the haversine formula, from latitudes in radians (with their
// cosines) and the longitude difference in degrees:
//   a = sin^2(dlat / 2) + cos(lat1) cos(lat2) sin^2(dlon / 2),  d = 2 R asin(sqrt(min(a, 1))).
__device__ inline double haversine(double dlon_deg, double lat1, double cos1, double lat2, double cos2) {
    const double sp = sin(0.5 * (lat2 - lat1));
    const double sl = sin(0.5 * (dlon_deg * kDegToRad));
    double a = sp * sp + (cos1 * cos2) * (sl * sl);
    a = a < 1.0 ? a : 1.0;
    return 2.0 * kEarthRadiusKm * asin(sqrt(a));
}

// Distance between two sites: Euclidean, or great-circle for (lon, lat) in degrees.
__device__ inline double site_distance(double x1, double y1, double x2, double y2, int gcd) {
    if (gcd) {
        const double p1 = y1 * kDegToRad, p2 = y2 * kDegToRad;
        return haversine(x2 - x1, p1, cos(p1), p2, cos(p2));
    }
    const double dx = x1 - x2, dy = y1 - y2;
    return sqrt(dx * dx + dy * dy);
}

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
    __device__ void prepare_cols(const TileIJ &, int, const int64_t *gcol) {
        __shared__ double cx[kCovCols], cy[kCovCols], ccs[kCovCols];
        sx = cx;
        sy = cy;
        sc = ccs;
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
        if (mp.gcd) return matern_cov(haversine(sx[cc] - xr, yr, cr, sy[cc], sc[cc]), mp);
        const double dx = xr - sx[cc];
        const double dy = yr - sy[cc];
        return matern_cov(sqrt(dx * dx + dy * dy), mp);
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
