// FP64 Cholesky of one diagonal tile (dpotrf of Algorithm 1) fused with its inverse,
// the forward-solve block and the log-determinant / quadratic-form parts of eq. (2).
//
// One workgroup factors the nbp x nbp tile in 32-column blocks, right-looking, and
// applies the same eliminations to an identity matrix B, so that on exit the tile holds
// L (lower, positive diagonal) and B holds L^-1.  Per block c:
//   1. the 32 x 32 diagonal block D is factored in LDS and inverted (Dinv);
//   2. every column t < 32(c+1) of B gets its block rows c multiplied by Dinv, and every
//      tile row t >= 32(c+1) of the panel is solved against D^T (x Dinv^T); the results
//      form one 32-vector V[t] per index t;
//   3. for rows i >= 32(c+1) and columns j <= i:  M_ij -= V[i] . V[j], where M is B for
//      j < 32(c+1) and the tile otherwise.
// Then y = L^-1 r, quad = y^T y and logdet = 2 sum log L_ii are formed.
#include "common.h"

#include <climits>

namespace mpgeo {

namespace {

constexpr int kPotrfThreads = 512;
constexpr int kBlk = 32;
constexpr int kMicro = 8;
constexpr int kVs = kBlk + 1;   // LDS row stride of V (odd: spreads rows over banks)

__global__ __launch_bounds__(kPotrfThreads) void potrf_tile_kernel(PotrfArgs args) {
    __shared__ double V[kMaxTile * kVs];        // V[t * kVs + l]
    __shared__ double D[kBlk][kBlk + 1];
    __shared__ double Dinv[kBlk][kBlk + 1];
    __shared__ double red[kPotrfThreads / 64];
    __shared__ int fail_col;

    const int nbp = args.nbp;
    const int tid = threadIdx.x;
    double *A = args.a;
    double *B = args.linv;
    if (tid == 0) fail_col = INT_MAX;
    for (int64_t e = tid; e < (int64_t)nbp * nbp; e += kPotrfThreads) {
        const int r = (int)(e % nbp), c = (int)(e / nbp);
        B[e] = (r == c) ? 1.0 : 0.0;
    }
    double logdet = 0.0;
    __syncthreads();

    const int nblk = nbp / kBlk;
    for (int cblk = 0; cblk < nblk; ++cblk) {
        const int cb = cblk * kBlk;
        // ---- 1. diagonal block -------------------------------------------------------
        for (int e = tid; e < kBlk * kBlk; e += kPotrfThreads) {
            const int i = e % kBlk, j = e / kBlk;
            D[i][j] = (i >= j) ? A[(cb + i) + (int64_t)(cb + j) * nbp] : 0.0;
        }
        __syncthreads();
        for (int j = 0; j < kBlk; ++j) {
            if (tid == 0) {
                double d = D[j][j];
                if (!(d > 0.0)) {          // non-positive or NaN pivot
                    if (fail_col == INT_MAX) fail_col = cb + j;
                    d = 1.0;
                }
                D[j][j] = sqrt(d);
            }
            __syncthreads();
            if (tid > j && tid < kBlk) D[tid][j] /= D[j][j];
            __syncthreads();
            for (int e = tid; e < kBlk * kBlk; e += kPotrfThreads) {
                const int i = e % kBlk, l = e / kBlk;
                if (l > j && i >= l) D[i][l] -= D[i][j] * D[l][j];
            }
            __syncthreads();
        }
        if (tid < kBlk) {               // column tid of Dinv by forward substitution
            const int j = tid;
            for (int i = 0; i < j; ++i) Dinv[i][j] = 0.0;
            Dinv[j][j] = 1.0 / D[j][j];
            for (int i = j + 1; i < kBlk; ++i) {
                double s = 0.0;
                for (int t = j; t < i; ++t) s += D[i][t] * Dinv[t][j];
                Dinv[i][j] = -s / D[i][i];
            }
            logdet += 2.0 * log(D[j][j]);
        }
        for (int e = tid; e < kBlk * kBlk; e += kPotrfThreads) {
            const int i = e % kBlk, j = e / kBlk;
            if (i >= j) A[(cb + i) + (int64_t)(cb + j) * nbp] = D[i][j];
        }
        __syncthreads();
        // ---- 2. V vectors: B block rows (t < cb + 32) and panel rows (t >= cb + 32) ----
        const int split = cb + kBlk;
        for (int t = tid; t < nbp; t += kPotrfThreads) {
            double x[kBlk];
            if (t < split) {
#pragma unroll
                for (int l = 0; l < kBlk; ++l) x[l] = B[(cb + l) + (int64_t)t * nbp];
#pragma unroll
                for (int l = 0; l < kBlk; ++l) {
                    double s = 0.0;
#pragma unroll
                    for (int q = 0; q <= l; ++q) s += Dinv[l][q] * x[q];
                    V[t * kVs + l] = s;
                }
#pragma unroll
                for (int l = 0; l < kBlk; ++l) B[(cb + l) + (int64_t)t * nbp] = V[t * kVs + l];
            } else {
#pragma unroll
                for (int l = 0; l < kBlk; ++l) x[l] = A[t + (int64_t)(cb + l) * nbp];
#pragma unroll
                for (int l = 0; l < kBlk; ++l) {
                    double s = 0.0;
#pragma unroll
                    for (int q = 0; q <= l; ++q) s += x[q] * Dinv[l][q];
                    V[t * kVs + l] = s;
                }
#pragma unroll
                for (int l = 0; l < kBlk; ++l) A[t + (int64_t)(cb + l) * nbp] = V[t * kVs + l];
            }
        }
        __syncthreads();
        // ---- 3. trailing update on 8 x 8 micro tiles ------------------------------------
        const int rows = nbp - split;
        if (rows > 0) {
            const int nrb = rows / kMicro;
            const int a0 = split / kMicro;   // column blocks left of the first row block
            // row block rb (rows split + 8 rb ...) has a0 + rb + 1 column blocks
            const int total = nrb * a0 + nrb * (nrb + 1) / 2;
            for (int w = tid; w < total; w += kPotrfThreads) {
                // invert w -> (rb, cbk): cumulative count before rb is rb*a0 + rb(rb+1)/2
                int rb = (int)((-(2.0 * a0 + 1.0) + sqrt((2.0 * a0 + 1.0) * (2.0 * a0 + 1.0) + 8.0 * w)) * 0.5);
                if (rb < 0) rb = 0;
                while (rb > 0 && rb * a0 + rb * (rb + 1) / 2 > w) --rb;
                while ((rb + 1) * a0 + (rb + 1) * (rb + 2) / 2 <= w) ++rb;
                const int cbk = w - (rb * a0 + rb * (rb + 1) / 2);
                const int i0 = split + rb * kMicro;
                const int j0 = cbk * kMicro;
                double acc[kMicro][kMicro];
#pragma unroll
                for (int u = 0; u < kMicro; ++u)
#pragma unroll
                    for (int v = 0; v < kMicro; ++v) acc[u][v] = 0.0;
                for (int l = 0; l < kBlk; ++l) {
                    double av[kMicro], bv[kMicro];
#pragma unroll
                    for (int u = 0; u < kMicro; ++u) av[u] = V[(i0 + u) * kVs + l];
#pragma unroll
                    for (int v = 0; v < kMicro; ++v) bv[v] = V[(j0 + v) * kVs + l];
#pragma unroll
                    for (int u = 0; u < kMicro; ++u)
#pragma unroll
                        for (int v = 0; v < kMicro; ++v) acc[u][v] += av[u] * bv[v];
                }
                double *M = (j0 < split) ? B : A;
#pragma unroll
                for (int v = 0; v < kMicro; ++v) {
                    const int j = j0 + v;
#pragma unroll
                    for (int u = 0; u < kMicro; ++u) {
                        const int i = i0 + u;
                        if (j <= i) M[i + (int64_t)j * nbp] -= acc[u][v];
                    }
                }
            }
        }
        __syncthreads();
    }

    // ---- FP32 copy of the inverse, forward-solve block, reductions ---------------------
    for (int64_t e = tid; e < (int64_t)nbp * nbp; e += kPotrfThreads) args.linv32[e] = (float)B[e];
    double *rs = V;   // reuse LDS for r_k
    for (int t = tid; t < nbp; t += kPotrfThreads) rs[t] = args.r[t];
    __syncthreads();
    double quad = 0.0;
    for (int i = tid; i < nbp; i += kPotrfThreads) {
        double s = 0.0;
        for (int j = 0; j <= i; ++j) s += B[i + (int64_t)j * nbp] * rs[j];
        args.y[i] = s;
        quad += s * s;
    }
    // block reductions (fixed order -> deterministic)
    double vals[2] = {logdet, quad};
    double out[2];
    for (int q = 0; q < 2; ++q) {
        double v = vals[q];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        __syncthreads();
        if ((tid & 63) == 0) red[tid >> 6] = v;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < kPotrfThreads / 64; ++w) s += red[w];
            out[q] = s;
        }
    }
    if (tid == 0) {
        *args.logdet_part = out[0];
        *args.quad_part = out[1];
        if (fail_col != INT_MAX && fail_col < args.nb)
            atomicMin(args.info, (unsigned long long)(args.col_base + fail_col));
    }
}

}  // namespace

void launch_potrf(const PotrfArgs &a, hipStream_t stream) {
    hipLaunchKernelGGL(potrf_tile_kernel, dim3(1), dim3(kPotrfThreads), 0, stream, a);
}

}  // namespace mpgeo
