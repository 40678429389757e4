// FP64 Cholesky of one diagonal tile (dpotrf of Algorithm 1) fused with its inverse,
// the forward-solve block and the log-determinant / quadratic-form parts of eq. (2).
//
// One workgroup factors the nbp x nbp tile A in 32-column blocks, right-looking, and
// applies the same eliminations to an identity matrix B, so that on exit A holds L (lower,
// positive diagonal) and B holds L^-1.  Per block c (columns cb .. cb+31, split = cb + 32):
//   1. one wave factors the 32 x 32 diagonal block D in LDS and inverts it (Dinv);
//   2. the block rows c of B are multiplied by Dinv (rows of L^-1 for this block), and the
//      panel rows t >= split of A are solved against D^T (rows of L) — both in place, on
//      the matrix cores;
//   3. for rows i >= split and columns j <= i:  M_ij -= sum_l V_il V_jl, with M = B and
//      V_j = (new B block rows)(:, j) for j < split, M = A and V_j = L(j, block c) otherwise.
//      This rank-32 update runs on v_mfma_f64_16x16x4_f64 over 16 x 16 blocks, with the
//      operands read from the tile (L2-resident) rather than staged in LDS, so the kernel
//      needs little LDS and can share a compute unit with the trailing-update kernels.
// Then y = L^-1 r, quad = y^T y and logdet = 2 sum log L_ii are formed.
#include "common.h"

#include <climits>

namespace mpgeo {

namespace {

constexpr int kPotrfThreads = 1024;
constexpr int kWaves = kPotrfThreads / 64;
constexpr int kBlk = 32;

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kPotrfThreads) void potrf_tile_kernel(PotrfArgs args) {
    __shared__ double D[kBlk][kBlk + 1];
    __shared__ double Dinv[kBlk][kBlk + 1];
    __shared__ double rs[kMaxTile];
    __shared__ double red[2][kWaves];
    __shared__ int fail_col;

    const int nbp = args.nbp;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    double *A = args.a;
    double *B = args.linv;
    if (tid == 0) fail_col = INT_MAX;
    for (int64_t e = tid; e < (int64_t)nbp * nbp; e += kPotrfThreads) {
        const int r = (int)(e % nbp), c = (int)(e / nbp);
        B[e] = (r == c) ? 1.0 : 0.0;
    }
    double logdet = 0.0;
    __syncthreads();

    for (int cb = 0; cb < nbp; cb += kBlk) {
        const int split = cb + kBlk;
        // ---- 1. diagonal block, one wave ---------------------------------------------
        if (wave == 0) {
            for (int e = lane; e < kBlk * kBlk; e += 64) {
                const int i = e % kBlk, j = e / kBlk;
                D[i][j] = (i >= j) ? A[(cb + i) + (int64_t)(cb + j) * nbp] : 0.0;
            }
            wave_sync();
            for (int j = 0; j < kBlk; ++j) {
                double d = D[j][j];
                if (!(d > 0.0)) {                       // non-positive or NaN pivot
                    if (lane == 0 && fail_col == INT_MAX) fail_col = cb + j;
                    d = 1.0;
                }
                const double piv = sqrt(d);
                wave_sync();
                if (lane == 0) D[j][j] = piv;
                if (lane > j && lane < kBlk) D[lane][j] /= piv;
                wave_sync();
                for (int e = lane; e < kBlk * kBlk; e += 64) {
                    const int i = e % kBlk, l = e / kBlk;
                    if (l > j && i >= l) D[i][l] -= D[i][j] * D[l][j];
                }
                wave_sync();
            }
            if (lane < kBlk) {                          // column `lane` of Dinv
                const int j = lane;
                for (int i = 0; i < j; ++i) Dinv[i][j] = 0.0;
                Dinv[j][j] = 1.0 / D[j][j];
                for (int i = j + 1; i < kBlk; ++i) {
                    double s = 0.0;
                    for (int t = j; t < i; ++t) s += D[i][t] * Dinv[t][j];
                    Dinv[i][j] = -s / D[i][i];
                }
                logdet += 2.0 * log(D[j][j]);
            }
            wave_sync();
            for (int e = lane; e < kBlk * kBlk; e += 64) {
                const int i = e % kBlk, j = e / kBlk;
                if (i >= j) A[(cb + i) + (int64_t)(cb + j) * nbp] = D[i][j];
            }
        }
        __syncthreads();
        // ---- 2. block rows of B (columns t < split) and panel rows of A (t >= split) ------
        // For 16 indices t at a time: out[t][l] = sum_q X[t][q] Dinv[l][q], where X[t][q] is
        // B[cb + q][t] (t < split) or A[t][cb + q] (t >= split); two 16 x 16 MFMA blocks
        // (l in 0..15 and 16..31), result register q of lane (16 g + r) = out[t0 + r][l0 + g + 4q].
        {
            const int lr = lane & 15, lg = lane >> 4;
            for (int t0 = wave * 16; t0 < nbp; t0 += kWaves * 16) {
                const bool isB = t0 < split;   // split is a multiple of 16
                f64x4 o0 = {0.0, 0.0, 0.0, 0.0}, o1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < kBlk / 4; ++s) {
                    const int k = 4 * s + lg;
                    const double xv = isB ? B[(cb + k) + (int64_t)(t0 + lr) * nbp]
                                          : A[(t0 + lr) + (int64_t)(cb + k) * nbp];
                    o0 = __builtin_amdgcn_mfma_f64_16x16x4f64(Dinv[lr][k], xv, o0, 0, 0, 0);
                    o1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Dinv[16 + lr][k], xv, o1, 0, 0, 0);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int t = t0 + lr;
                    const int l0 = lg + 4 * q, l1 = 16 + lg + 4 * q;
                    if (isB) {
                        B[(cb + l0) + (int64_t)t * nbp] = o0[q];
                        B[(cb + l1) + (int64_t)t * nbp] = o1[q];
                    } else {
                        A[t + (int64_t)(cb + l0) * nbp] = o0[q];
                        A[t + (int64_t)(cb + l1) * nbp] = o1[q];
                    }
                }
            }
        }
        __syncthreads();
        // ---- 3. rank-32 update of rows >= split on 16 x 16 MFMA blocks ----------------
        const int rows = nbp - split;
        if (rows > 0) {
            const int nrb = rows / 16;
            const int a0 = split / 16;          // 16-column blocks of B left of row block 0
            const int total = nrb * a0 + nrb * (nrb + 1) / 2;
            const int lr = lane & 15, lg = lane >> 4;
            for (int w = wave; w < total; w += kWaves) {
                int rb = (int)((-(2.0 * a0 + 1.0) + sqrt((2.0 * a0 + 1.0) * (2.0 * a0 + 1.0) + 8.0 * w)) * 0.5);
                if (rb < 0) rb = 0;
                while (rb > 0 && rb * a0 + rb * (rb + 1) / 2 > w) --rb;
                while ((rb + 1) * a0 + (rb + 1) * (rb + 2) / 2 <= w) ++rb;
                const int cbk = w - (rb * a0 + rb * (rb + 1) / 2);
                const int i0 = split + rb * 16;
                const int j0 = cbk * 16;
                const bool inB = j0 < split;
                double *M = inB ? B : A;
                // result register q of lane (16 g + r) is M[i0 + r][j0 + g + 4q]
                f64x4 acc;
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] = M[(i0 + lr) + (int64_t)(j0 + lg + 4 * q) * nbp];
#pragma unroll
                for (int s = 0; s < kBlk / 4; ++s) {
                    const int k = cb + 4 * s + lg;
                    const double rv = A[(i0 + lr) + (int64_t)k * nbp];
                    const double qv = inB ? B[k + (int64_t)(j0 + lr) * nbp] : A[(j0 + lr) + (int64_t)k * nbp];
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-qv, rv, acc, 0, 0, 0);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = i0 + lr, j = j0 + lg + 4 * q;
                    if (inB || j <= i) M[i + (int64_t)j * nbp] = acc[q];
                }
            }
        }
        __syncthreads();
    }

    // ---- FP32 copy of the inverse, forward-solve block, reductions ---------------------
    for (int64_t e = tid; e < (int64_t)nbp * nbp; e += kPotrfThreads) args.linv32[e] = (float)B[e];
    for (int t = tid; t < nbp; t += kPotrfThreads) rs[t] = args.r[t];
    __syncthreads();
    double quad = 0.0;
    for (int i = tid; i < nbp; i += kPotrfThreads) {
        double s = 0.0;
        for (int j = 0; j <= i; ++j) s += B[i + (int64_t)j * nbp] * rs[j];
        args.y[i] = s;
        quad += s * s;
    }
    // block reductions in a fixed order (deterministic)
    for (int off = 32; off > 0; off >>= 1) {
        logdet += __shfl_down(logdet, off, 64);
        quad += __shfl_down(quad, off, 64);
    }
    if (lane == 0) {
        red[0][wave] = logdet;
        red[1][wave] = quad;
    }
    __syncthreads();
    if (tid == 0) {
        double sl = 0.0, sq = 0.0;
        for (int w = 0; w < kWaves; ++w) {
            sl += red[0][w];
            sq += red[1][w];
        }
        *args.logdet_part = sl;
        *args.quad_part = sq;
        if (fail_col != INT_MAX && fail_col < args.nb)
            atomicMin(args.info, (unsigned long long)(args.col_base + fail_col));
    }
}

}  // namespace

void launch_potrf(const PotrfArgs &a, hipStream_t stream) {
    hipLaunchKernelGGL(potrf_tile_kernel, dim3(1), dim3(kPotrfThreads), 0, stream, a);
}

}  // namespace mpgeo
