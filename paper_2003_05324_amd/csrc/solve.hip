// Triangular solves and reductions around the factorisation (eq. (2), kriging).
//
// Forward solve y = L^-1 Z is fused into the right-looking factorisation: after the
// panel of step k is solved, r_i -= L_ik y_k for every i > k (this file), and the next
// diagonal step forms y_k+1 = L_k+1,k+1^-1 r_k+1.  Sums run in FP64 in a fixed order.
#include "common.h"

namespace mpgeo {

namespace {

constexpr double kLog2Pi = 1.8378770664093454836;

// r_i -= P64_i y_k, and the finished panel tile (i, k) is copied from staging into its storage
// precision.  A workgroup takes 64 rows of one tile; each of its four waves walks a quarter of
// the columns (one coalesced 64-row read per column) with four running sums, and the sums are
// added in a fixed order, so the result does not depend on scheduling.
__global__ __launch_bounds__(256) void panel_solve_kernel(TileMap map, int k, const double *p64,
                                                          const double *yk, double *r) {
    __shared__ double ys[kMaxTile];
    __shared__ double part[4][64];
    const int nbp = map.nbp;
    const int i = k + 1 + blockIdx.x;
    const int rl = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int row = blockIdx.y * 64 + rl;
    for (int c = threadIdx.x; c < nbp; c += 256) ys[c] = yk[c];
    __syncthreads();
    const int quarter = nbp / 4;   // a multiple of 8 (nbp is a multiple of 32)
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    if (row < nbp) {
        const double *P = p64 + (int64_t)i * nbp * nbp;
        const bool f64 = tile_is_fp64(map, i, k);
        const int64_t off = map.off[tri_index(i, k)];
        for (int c = g * quarter; c < (g + 1) * quarter; c += 4) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t e = row + (int64_t)(c + u) * nbp;
                const double v = P[e];
                s[u] += v * ys[c + u];
                if (f64) map.pool64[off + e] = v;
                else map.pool32[off + e] = (float)v;   // exact: v is an FP32 value promoted
            }
        }
    }
    part[g][rl] = (s[0] + s[1]) + (s[2] + s[3]);
    __syncthreads();
    if (g == 0 && row < nbp)
        r[(int64_t)i * nbp + row] -= (part[0][rl] + part[1][rl]) + (part[2][rl] + part[3][rl]);
}

// eq. (2) from the per-tile parts; with `profile` the tiles held the correlation matrix and
// eq. (2) is taken at its maximising variance q~/n (the profile likelihood).
__global__ void finalize_kernel(const double *logdet_part, const double *quad_part, int p,
                                int64_t n, int profile, double *result) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double logdet = 0.0, quad = 0.0;
    for (int k = 0; k < p; ++k) {
        logdet += logdet_part[k];
        quad += quad_part[k];
    }
    const double dn = (double)n;
    if (profile)
        result[0] = -0.5 * dn * (kLog2Pi + 1.0) - 0.5 * dn * log(quad / dn) - 0.5 * logdet;
    else
        result[0] = -0.5 * dn * kLog2Pi - 0.5 * logdet - 0.5 * quad;
    result[1] = logdet;
    result[2] = quad;
}

// w_k = L_kk^-T t_k (thread per column c of L_kk^-1: w[c] = sum_{r >= c} Linv[r][c] t[r]).
__global__ __launch_bounds__(256) void back_diag_kernel(const double *linv, const double *t,
                                                        double *w, int nbp) {
    __shared__ double ts[kMaxTile];
    for (int c = threadIdx.x; c < nbp; c += 256) ts[c] = t[c];
    __syncthreads();
    for (int c = threadIdx.x; c < nbp; c += 256) {
        const double *col = linv + (int64_t)c * nbp;
        double s = 0.0;
        for (int r = c; r < nbp; ++r) s += col[r] * ts[r];
        w[c] = s;
    }
}

// t_j -= L_kj^T w_k for j < k: one workgroup per tile (k, j); thread per column c.
__global__ __launch_bounds__(256) void back_row_kernel(TileMap map, int k, const double *wk,
                                                       double *t) {
    __shared__ double ws[kMaxTile];
    const int nbp = map.nbp;
    const int j = blockIdx.x;
    for (int r = threadIdx.x; r < nbp; r += 256) ws[r] = wk[r];
    __syncthreads();
    const bool f64 = tile_is_fp64(map, k, j);
    const int64_t off = map.off[tri_index(k, j)];
    for (int c = threadIdx.x; c < nbp; c += 256) {
        double s = 0.0;
        if (f64) {
            const double *col = map.pool64 + off + (int64_t)c * nbp;
            for (int r = 0; r < nbp; ++r) s += col[r] * ws[r];
        } else {
            const float *col = map.pool32 + off + (int64_t)c * nbp;
            for (int r = 0; r < nbp; ++r) s += (double)col[r] * ws[r];
        }
        t[(int64_t)j * nbp + c] -= s;
    }
}

// Many right-hand sides: X_k = Linv_kk C_k (C_k: nbp x m block rows of C, in place via tmp).
__global__ __launch_bounds__(256) void multi_diag_kernel(const double *linv, double *c, int64_t ldc,
                                                         int64_t m, int nbp, double *tmp) {
    const int64_t j = blockIdx.y;
    const int row = blockIdx.x * 256 + threadIdx.x;
    if (row >= nbp || j >= m) return;
    double s = 0.0;
    for (int q = 0; q <= row; ++q) s += linv[row + (int64_t)q * nbp] * c[q + j * ldc];
    tmp[row + j * nbp] = s;
}
__global__ __launch_bounds__(256) void multi_copy_kernel(const double *tmp, double *c, int64_t ldc,
                                                         int64_t m, int nbp) {
    const int64_t j = blockIdx.y;
    const int row = blockIdx.x * 256 + threadIdx.x;
    if (row >= nbp || j >= m) return;
    c[row + j * ldc] = tmp[row + j * nbp];
}
// C_i -= L_ik X_k for i > k (one workgroup per (tile i, row block, rhs)).
__global__ __launch_bounds__(256) void multi_update_kernel(TileMap map, int k, const double *xk,
                                                           double *c, int64_t ldc, int64_t m) {
    const int nbp = map.nbp;
    const int i = k + 1 + blockIdx.x / ((nbp + 255) / 256);
    const int row = (blockIdx.x % ((nbp + 255) / 256)) * 256 + threadIdx.x;
    const int64_t j = blockIdx.y;
    if (row >= nbp || j >= m) return;
    const bool f64 = tile_is_fp64(map, i, k);
    const int64_t off = map.off[tri_index(i, k)];
    const double *x = xk + j * ldc;
    double s = 0.0;
    for (int q = 0; q < nbp; ++q) {
        const int64_t e = off + row + (int64_t)q * nbp;
        const double lv = f64 ? map.pool64[e] : (double)map.pool32[e];
        s += lv * x[q];
    }
    c[(int64_t)i * nbp + row + j * ldc] -= s;
}

// var_j = scale * (sigma2 - |c_j|^2)
__global__ void column_var_kernel(const double *c, int64_t ldc, int64_t rows, int64_t m,
                                  double sigma2, double scale, double *var) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    double s = 0.0;
    for (int64_t r = 0; r < rows; ++r) {
        const double v = c[r + j * ldc];
        s += v * v;
    }
    var[j] = scale * (sigma2 - s);
}

// z_i = sum_{j <= i} L_ij eps_j: one workgroup per (tile row i, 256-row block).
__global__ __launch_bounds__(256) void trmv_kernel(TileMap map, const double *eps, double *z) {
    __shared__ double es[kMaxTile];
    const int nbp = map.nbp;
    const int i = blockIdx.x;
    const int row = blockIdx.y * 256 + threadIdx.x;
    double s = 0.0;
    for (int j = 0; j <= i; ++j) {
        __syncthreads();
        for (int c = threadIdx.x; c < nbp; c += 256) es[c] = eps[(int64_t)j * nbp + c];
        __syncthreads();
        if (row >= nbp) continue;
        const bool f64 = tile_is_fp64(map, i, j);
        const int64_t off = map.off[tri_index(i, j)];
        const int cend = (j == i) ? row + 1 : nbp;   // only the lower triangle of L_ii
        for (int c = 0; c < cend; ++c) {
            const int64_t e = off + row + (int64_t)c * nbp;
            const double lv = f64 ? map.pool64[e] : (double)map.pool32[e];
            s += lv * es[c];
        }
    }
    if (row < nbp) z[(int64_t)i * nbp + row] = s;
}

__global__ void permute_kernel(const double *src, double *dst, const int64_t *perm, int64_t n,
                               bool to_caller) {
    const int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= n) return;
    if (to_caller) dst[perm[a]] = src[a];
    else dst[a] = src[perm[a]];
}

}  // namespace

void launch_trmv(const TileMap &map, const double *eps, double *z, hipStream_t stream) {
    dim3 grid((unsigned)map.p, (unsigned)((map.nbp + 255) / 256));
    hipLaunchKernelGGL(trmv_kernel, grid, dim3(256), 0, stream, map, eps, z);
}

void launch_permute(const double *src, double *dst, const int64_t *perm, int64_t n, bool to_caller,
                    hipStream_t stream) {
    hipLaunchKernelGGL(permute_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, src,
                       dst, perm, n, to_caller);
}

void launch_panel_solve(const TileMap &map, int k, int count, const double *p64, const double *yk,
                        double *r, hipStream_t stream) {
    if (count <= 0) return;
    dim3 grid((unsigned)count, (unsigned)((map.nbp + 63) / 64));
    hipLaunchKernelGGL(panel_solve_kernel, grid, dim3(256), 0, stream, map, k, p64, yk, r);
}

void launch_finalize(const double *logdet_part, const double *quad_part, int p, int64_t n,
                     bool profile, double *result, hipStream_t stream) {
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(64), 0, stream, logdet_part, quad_part, p, n,
                       profile ? 1 : 0, result);
}

// t (physical, p*nbp) holds y on entry and is consumed; w (physical) receives L^-T y.
void launch_backward_solve(const TileMap &map, const double *linv_all, const double *y, double *t,
                           double *w, hipStream_t stream) {
    const int nbp = map.nbp;
    const size_t bytes = (size_t)map.p * nbp * sizeof(double);
    (void)hipMemcpyAsync(t, y, bytes, hipMemcpyDeviceToDevice, stream);
    for (int k = map.p - 1; k >= 0; --k) {
        hipLaunchKernelGGL(back_diag_kernel, dim3(1), dim3(256), 0, stream,
                           linv_all + (int64_t)k * nbp * nbp, t + (int64_t)k * nbp,
                           w + (int64_t)k * nbp, nbp);
        if (k > 0)
            hipLaunchKernelGGL(back_row_kernel, dim3((unsigned)k), dim3(256), 0, stream, map, k,
                               w + (int64_t)k * nbp, t);
    }
}

void launch_forward_multi(const TileMap &map, const double *linv_all, double *c, int64_t ldc,
                          int64_t m, double *tmp, hipStream_t stream) {
    const int nbp = map.nbp;
    const unsigned rb = (unsigned)((nbp + 255) / 256);
    for (int k = 0; k < map.p; ++k) {
        double *ck = c + (int64_t)k * nbp;
        hipLaunchKernelGGL(multi_diag_kernel, dim3(rb, (unsigned)m), dim3(256), 0, stream,
                           linv_all + (int64_t)k * nbp * nbp, ck, ldc, m, nbp, tmp);
        hipLaunchKernelGGL(multi_copy_kernel, dim3(rb, (unsigned)m), dim3(256), 0, stream, tmp, ck,
                           ldc, m, nbp);
        if (k + 1 < map.p)
            hipLaunchKernelGGL(multi_update_kernel, dim3((unsigned)((map.p - k - 1) * rb), (unsigned)m),
                               dim3(256), 0, stream, map, k, ck, c, ldc, m);
    }
}

void launch_column_var(const double *c, int64_t ldc, int64_t rows, int64_t m, double sigma2,
                       double scale, double *var, hipStream_t stream) {
    if (m == 0) return;
    hipLaunchKernelGGL(column_var_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream, c,
                       ldc, rows, m, sigma2, scale, var);
}

}  // namespace mpgeo
