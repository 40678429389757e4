// Device body of the FP64 diagonal-tile Cholesky (dpotrf of Algorithm 1) fused with the tile's
// inverse, the forward-solve block and the log-determinant / quadratic-form parts of eq. (2),
// executed by one workgroup of kPotrfThreads threads.  Used by the one-tile kernel of the
// step-ordered factorization and by the persistent batched kernel.
//
// The workgroup factors the nbp x nbp tile A in 32-column blocks, right-looking, and builds
// B = L^-1 block row by block row, so that on exit A holds L (lower, positive diagonal) and
// B holds L^-1 (upper part zero).  Per block c (columns cb .. cb+31, split = cb + 32):
//   1. the 32 x 32 diagonal block D is staged in LDS and factored by one wave;
//   2. forward substitution with D, one thread per index t: for t < split the block rows c
//      of L^-1 (right-hand side B[cb + q][t], or the identity inside the diagonal block),
//      for t >= split the panel rows of L (right-hand side A[t][cb + q], solved against
//      D^T).  These block rows of B are final, so their FP32 copy is written here too
//      (when one is asked for); B's entries above the diagonal blocks are zeroed once, at the
//      start;
//   3. for rows i >= split and columns j <= i:  M_ij -= sum_l V_il V_jl, with M = B and
//      V_j = (new B block rows)(:, j) for j < split, M = A and V_j = L(j, block c) otherwise.
//      This rank-32 update runs on v_mfma_f64_16x16x4_f64, each wave taking 32 x 32 regions,
//      with the operands read from the tile (L2-resident) rather than staged in LDS, so the
//      kernel needs little LDS and can share a compute unit with the trailing-update kernels.
// Then y = L^-1 r, quad = y^T y and logdet = 2 sum log L_ii are formed.
#pragma once
#include "common.h"

#include <climits>

namespace mpgeo {

namespace {

constexpr int kBlk = 32;

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

// value of v in lane l (l uniform), through the scalar registers
__device__ inline double readlane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// diagonal block and the reciprocals of its diagonal (LDS); rows padded so that the staging
// writes (one column per pass) spread over the banks and row reads stay 16-byte aligned
__shared__ double D[kBlk][kBlk + 2];
__shared__ double rdiag[kBlk];

__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Diagonal 32 x 32 block (in D) factored in place by one wave.  Lane i holds row i in
// registers; for column j the pivot and the entries L(l, j) of the other rows are read
// across lanes (readlane) and each lane applies the rank-1 update to its own row.
__device__ inline double factor_diag_block(int lane, int cb, int *fail_col) {
    // Opaque copy of the lane index: the per-column lane masks below are then formed where
    // they are used instead of being hoisted out of the caller's loop.
    asm volatile("" : "+v"(lane));
    const int row = lane & (kBlk - 1);
    double d[kBlk];
#pragma unroll
    for (int l = 0; l < kBlk; ++l) d[l] = D[row][l];
    double diag = 1.0;
    int bad = INT_MAX;
#pragma unroll
    for (int j = 0; j < kBlk; ++j) {
        double pj = readlane(d[j], j);
        if (!(pj > 0.0)) {                              // non-positive or NaN pivot
            bad = min(bad, j);
            pj = 1.0;
        }
        const double piv = sqrt(pj);
        const double lij = (row == j) ? piv : d[j] / piv;
        d[j] = lij;
        if (row == j) diag = piv;
#pragma unroll
        for (int l = j + 1; l < kBlk; ++l) d[l] -= lij * readlane(lij, l);
    }
    if (lane == 0 && bad != INT_MAX && *fail_col == INT_MAX) *fail_col = cb + bad;
    double ld = 0.0;
    if (lane < kBlk) {
#pragma unroll
        for (int l = 0; l < kBlk; ++l) D[lane][l] = (l <= lane) ? d[l] : 0.0;
        rdiag[lane] = 1.0 / diag;
        ld = 2.0 * log(diag);
    }
    return ld;
}

template <int kPotrfThreads>
__device__ void potrf_tile_body(const PotrfArgs &args) {
    constexpr int kWaves = kPotrfThreads / 64;
    __shared__ double rs[kMaxTile];
    __shared__ double red[2][kWaves];
    __shared__ int fail_col;

    const int nbp = args.nbp;
    const int ld = args.ld > 0 ? args.ld : nbp;   // leading dimension of A, B and B32
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    double *A = args.a;
    double *B = args.linv;
    float *B32 = args.linv32;
    if (tid == 0) fail_col = INT_MAX;
    double logdet = 0.0;
    // the strictly upper part of B (and B32) outside the diagonal blocks is zero: written once
    // here, column by column, rather than by the panel rows of every block
    for (int j = kBlk; j < nbp; ++j) {
        const int top = j / kBlk * kBlk;   // rows 0 .. top-1 lie above column j's diagonal block
        for (int i = tid; i < top; i += kPotrfThreads) {
            B[i + (int64_t)j * ld] = 0.0;
            if (B32) B32[i + (int64_t)j * ld] = 0.0f;
        }
    }
    __syncthreads();

    for (int cb = 0; cb < nbp; cb += kBlk) {
        const int split = cb + kBlk;
        // ---- 1. diagonal block: staged in LDS by all threads, factored by one wave ------
        for (int e = tid; e < kBlk * kBlk; e += kPotrfThreads) {
            const int r = e & (kBlk - 1), c = e / kBlk;
            D[r][c] = (r >= c) ? A[(cb + r) + (int64_t)(cb + c) * ld] : 0.0;
        }
        __syncthreads();
        if (wave == 0) logdet += factor_diag_block(lane, cb, &fail_col);
        __syncthreads();
        // L block back to the tile (the diagonal block is not touched by steps 2 and 3)
        for (int e = tid; e < kBlk * kBlk; e += kPotrfThreads) {
            const int r = e & (kBlk - 1), c = e / kBlk;
            if (r >= c) A[(cb + r) + (int64_t)(cb + c) * ld] = D[r][c];
        }
        // ---- 2. block rows of B (columns t < split) and panel rows of A (t >= split) ------
        // Thread t solves D y = x: x[q] = B[cb + q][t] for t < cb, the unit vector e_(t - cb)
        // inside the diagonal block, A[t][cb + q] for t >= split.  The compiler barrier per
        // column keeps the broadcast reads of D from being issued all at once.
        // (a thread's 32 entries of B are contiguous in column t: read and written 16 bytes at a
        // time; cb and ld are multiples of 32, so the vectors are aligned)
        for (int t = tid; t < nbp; t += kPotrfThreads) {
            const bool isB = t < split;
            double y[kBlk];
            if (t < cb) {
                const d2v *src = reinterpret_cast<const d2v *>(B + cb + (int64_t)t * ld);
#pragma unroll
                for (int q = 0; q < kBlk / 2; ++q) {
                    const d2v v = src[q];
                    y[2 * q] = v.x;
                    y[2 * q + 1] = v.y;
                }
            } else if (isB) {
#pragma unroll
                for (int q = 0; q < kBlk; ++q) y[q] = (q == t - cb) ? 1.0 : 0.0;
            } else {
#pragma unroll
                for (int q = 0; q < kBlk; ++q) y[q] = A[t + (int64_t)(cb + q) * ld];
            }
#pragma unroll
            for (int l = 0; l < kBlk; ++l) {
                double s0 = y[l], s1 = 0.0;
#pragma unroll
                for (int q = 0; q + 1 < l; q += 2) {
                    s0 -= D[l][q] * y[q];
                    s1 -= D[l][q + 1] * y[q + 1];
                }
                if (l & 1) s0 -= D[l][l - 1] * y[l - 1];
                y[l] = (s0 + s1) * rdiag[l];
                asm volatile("" ::: "memory");
            }
            if (isB) {
                d2v *dst = reinterpret_cast<d2v *>(B + cb + (int64_t)t * ld);
#pragma unroll
                for (int l = 0; l < kBlk / 2; ++l) dst[l] = (d2v){y[2 * l], y[2 * l + 1]};
                if (B32) {
                    f4v *dst32 = reinterpret_cast<f4v *>(B32 + cb + (int64_t)t * ld);
#pragma unroll
                    for (int l = 0; l < kBlk / 4; ++l)
                        dst32[l] = (f4v){(float)y[4 * l], (float)y[4 * l + 1], (float)y[4 * l + 2], (float)y[4 * l + 3]};
                }
            } else {
#pragma unroll
                for (int l = 0; l < kBlk; ++l) A[t + (int64_t)(cb + l) * ld] = y[l];
            }
        }
        __syncthreads();
        // ---- 3. rank-32 update of rows >= split, 32 x 32 regions per wave item ----------
        // Regions are numbered row strip by row strip (strip rb has a2 + rb + 1 of them, the
        // last one on the diagonal, where the block above it is skipped) and dealt to the
        // waves round-robin.  The products are accumulated from zero and subtracted once.
        // B below the diagonal block (columns cb .. split-1) has not been written yet: its
        // entries are those of the identity there, i.e. zero.
        const int rows = nbp - split;
        if (rows > 0) {
            const int nr2 = rows / 32;
            const int a2 = split / 32;
            const int lr = lane & 15, lg = lane >> 4;
            int rb = 0, cbk = wave;
            while (rb < nr2 && cbk >= a2 + rb + 1) cbk -= a2 + ++rb;
            while (rb < nr2) {
                const int i0 = split + rb * 32, j0 = cbk * 32;
                const bool inB = j0 < split;
                const bool diag = j0 == i0;
                const bool fresh = inB && j0 >= cb;
                double *M = inB ? B : A;
                double rv[2][kBlk / 4], qv[2][kBlk / 4], cv[2][2][4];
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int st = 0; st < kBlk / 4; ++st) {
                        const int k = cb + 4 * st + lg;
                        rv[h][st] = A[(i0 + 16 * h + lr) + (int64_t)k * ld];
                        qv[h][st] = inB ? B[k + (int64_t)(j0 + 16 * h + lr) * ld]
                                        : A[(j0 + 16 * h + lr) + (int64_t)k * ld];
                    }
#pragma unroll
                for (int hi = 0; hi < 2; ++hi)
#pragma unroll
                    for (int hj = 0; hj < 2; ++hj)
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            cv[hi][hj][q] = ((diag && hj > hi) || fresh) ? 0.0
                                : M[(i0 + 16 * hi + lr) + (int64_t)(j0 + 16 * hj + lg + 4 * q) * ld];
                f64x4 acc[2][2];
#pragma unroll
                for (int hi = 0; hi < 2; ++hi)
#pragma unroll
                    for (int hj = 0; hj < 2; ++hj) acc[hi][hj] = (f64x4){0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int st = 0; st < kBlk / 4; ++st)
#pragma unroll
                    for (int hi = 0; hi < 2; ++hi)
#pragma unroll
                        for (int hj = 0; hj < 2; ++hj)
                            if (!(diag && hj > hi))
                                acc[hi][hj] = __builtin_amdgcn_mfma_f64_16x16x4f64(qv[hj][st], rv[hi][st], acc[hi][hj], 0, 0, 0);
#pragma unroll
                for (int hi = 0; hi < 2; ++hi)
#pragma unroll
                    for (int hj = 0; hj < 2; ++hj) {
                        if (diag && hj > hi) continue;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int i = i0 + 16 * hi + lr, j = j0 + 16 * hj + lg + 4 * q;
                            if (!diag || j <= i) M[i + (int64_t)j * ld] = cv[hi][hj][q] - acc[hi][hj][q];
                        }
                    }
                cbk += kWaves;
                while (rb < nr2 && cbk >= a2 + rb + 1) cbk -= a2 + ++rb;
            }
        }
        __syncthreads();
    }

    // ---- forward-solve block, reductions (a block of a larger tile has no right-hand side) ----
    double quad = 0.0;
    if (args.r) {
        for (int t = tid; t < nbp; t += kPotrfThreads) rs[t] = args.r[t];
        __syncthreads();
        for (int i = tid; i < nbp; i += kPotrfThreads) {
            // the row of L^-1 read eight entries ahead of the (in-order) accumulation
            double s = 0.0;
            int j = 0;
            for (; j + 8 <= i + 1; j += 8) {
                double b[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) b[u] = B[i + (int64_t)(j + u) * ld];
#pragma unroll
                for (int u = 0; u < 8; ++u) s += b[u] * rs[j + u];
            }
            for (; j <= i; ++j) s += B[i + (int64_t)j * ld] * rs[j];
            args.y[i] = s;
            quad += s * s;
        }
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
        if (args.logdet_part) *args.logdet_part = sl;
        if (args.quad_part) *args.quad_part = sq;
        if (fail_col != INT_MAX && fail_col < args.nb)
            atomicMin(args.info, (unsigned long long)(args.col_base + fail_col));
    }
}

}  // namespace

}  // namespace mpgeo
