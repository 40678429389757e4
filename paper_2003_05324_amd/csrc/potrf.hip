// FP64 Cholesky of one diagonal tile (dpotrf of Algorithm 1) fused with its inverse, the
// forward-solve block and the log-determinant / quadratic-form parts of eq. (2), on the
// critical path of the step-ordered factorization.  The single-workgroup body is in
// potrf_dev.h.
//
// Tiles of 256 or 512 columns are factored blocked instead, 128 columns at a time (the plan is
// in potrf_plan.h), so that most of the work spreads over many compute units; the products run
// on v_mfma_f64_16x16x4_f64 with operands read from the tile (L2-resident), like the
// single-workgroup body.
#include "potrf_dev.h"
#include "potrf_plan.h"

#include <algorithm>

namespace mpgeo {

namespace {

template <int kPotrfThreads>
__global__ __launch_bounds__(kPotrfThreads) void potrf_tile_kernel(PotrfArgs args) {
    potrf_tile_body<kPotrfThreads>(args);
}

constexpr int kSubThreads = 256;  // 4 waves, each a 32 x 32 quadrant of a 64 x 64 output block
constexpr int kMaxJobs = kPotrfMaxJobs;

// One job of a launch, a PotrfJob with its buffers resolved to pointers (c32: the FP32 copy
// of the result, or null).
struct SubJob {
    double *c;
    const double *a, *b;
    float *c32;
    int m, n, k;
    int transb, lower;
    double alpha, beta;
};
struct SubArgs {
    SubJob job[kMaxJobs];
    int first[kMaxJobs + 1];   // first 64 x 64 output block of each job
    int njobs;
    int ld;
};

__global__ __launch_bounds__(kSubThreads) void subblock_kernel(SubArgs g) {
    int jb = 0;
    while (jb + 1 < g.njobs && (int)blockIdx.x >= g.first[jb + 1]) ++jb;
    const SubJob &J = g.job[jb];
    const int local = (int)blockIdx.x - g.first[jb];
    const int mb = J.m / 64;
    const int r0 = (local % mb) * 64, c0 = (local / mb) * 64;
    const int ld = g.ld;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = r0 + (wave & 1) * 32, wc = c0 + (wave >> 1) * 32;
    const int lr = lane & 15, lg = lane >> 4;
    if (J.lower && wc >= wr + 32) return;   // this wave's quadrant lies above the diagonal
    if (J.a == nullptr || J.k == 0) {       // zero or copy
        for (int e = lane; e < 32 * 32; e += 64) {
            const int i = wr + (e & 31), j = wc + (e >> 5);
            if (J.lower && j > i) continue;
            const double v = J.a ? J.a[i + (int64_t)j * ld] : 0.0;
            J.c[i + (int64_t)j * ld] = v;
            if (J.c32) J.c32[i + (int64_t)j * ld] = (float)v;
        }
        return;
    }
    f64x4 acc[2][2];
#pragma unroll
    for (int hi = 0; hi < 2; ++hi)
#pragma unroll
        for (int hj = 0; hj < 2; ++hj) acc[hi][hj] = (f64x4){0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < J.k; k0 += 16) {
        double rv[2][4], qv[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const int k = k0 + 4 * st + lg;
                const int row = wr + 16 * h + lr, col = wc + 16 * h + lr;
                rv[h][st] = J.a[row + (int64_t)k * ld];
                qv[h][st] = J.transb ? J.b[col + (int64_t)k * ld] : J.b[k + (int64_t)col * ld];
            }
#pragma unroll
        for (int st = 0; st < 4; ++st)
#pragma unroll
            for (int hi = 0; hi < 2; ++hi)
#pragma unroll
                for (int hj = 0; hj < 2; ++hj)
                    acc[hi][hj] = __builtin_amdgcn_mfma_f64_16x16x4f64(qv[hj][st], rv[hi][st], acc[hi][hj], 0, 0, 0);
    }
    // result register q of lane (16 g + r): row r, column g + 4 q of the 16 x 16 block
#pragma unroll
    for (int hi = 0; hi < 2; ++hi)
#pragma unroll
        for (int hj = 0; hj < 2; ++hj)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int i = wr + 16 * hi + lr, j = wc + 16 * hj + lg + 4 * q;
                if (J.lower && j > i) continue;
                double *pc = J.c + i + (int64_t)j * ld;
                const double v = (J.beta == 0.0 ? 0.0 : J.beta * *pc) + J.alpha * acc[hi][hj][q];
                *pc = v;
                if (J.c32) J.c32[i + (int64_t)j * ld] = (float)v;
            }
}

// y = L^-1 r, y^T y and 2 sum log L_ii of the whole tile, after the blocked factorization.
constexpr int kFinishThreads = 1024;
__global__ __launch_bounds__(kFinishThreads) void potrf_finish_kernel(PotrfArgs args) {
    __shared__ double rs[kMaxTile];
    __shared__ double red[2][kFinishThreads / 64];
    const int nbp = args.nbp, ld = nbp;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int t = tid; t < nbp; t += kFinishThreads) rs[t] = args.r[t];
    __syncthreads();
    double quad = 0.0, logdet = 0.0;
    for (int i = tid; i < nbp; i += kFinishThreads) {
        double s = 0.0;
        for (int j = 0; j <= i; ++j) s += args.linv[i + (int64_t)j * ld] * rs[j];
        args.y[i] = s;
        quad += s * s;
        logdet += 2.0 * log(args.a[i + (int64_t)i * ld]);
    }
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
        for (int w = 0; w < kFinishThreads / 64; ++w) {
            sl += red[0][w];
            sq += red[1][w];
        }
        *args.logdet_part = sl;
        *args.quad_part = sq;
    }
}

void launch_potrf_blocked(const PotrfArgs &a, hipStream_t stream) {
    const int nbp = a.nbp;
    auto ptr = [&](int buf, int64_t off) -> double * {
        return buf == kBufA ? a.a + off : buf == kBufB ? a.linv + off : nullptr;
    };
    for (const PotrfStep &st : potrf_blocked_plan(nbp, a.linv32 != nullptr)) {
        if (st.diag >= 0) {   // one 128 x 128 diagonal block: L_kk in place, L_kk^-1 into the inverse
            const int kb = st.diag;
            const int64_t off = (int64_t)kb * kPotrfBlock * (nbp + 1);
            PotrfArgs d{};
            d.a = a.a + off;
            d.linv = a.linv + off;
            d.linv32 = nullptr;
            d.r = nullptr;
            d.y = nullptr;
            d.logdet_part = nullptr;
            d.quad_part = nullptr;
            d.info = a.info;
            d.col_base = a.col_base + (int64_t)kb * kPotrfBlock;
            d.nb = std::max(0, std::min(kPotrfBlock, a.nb - kb * kPotrfBlock));
            d.nbp = kPotrfBlock;
            d.ld = nbp;
            hipLaunchKernelGGL((potrf_tile_kernel<256>), dim3(1), dim3(256), 0, stream, d);
            continue;
        }
        SubArgs g{};
        g.ld = nbp;
        int blocks = 0;
        for (const PotrfJob &j : st.jobs) {   // at most kMaxJobs (the plan splits larger steps)
            g.job[g.njobs] = SubJob{ptr(j.c_buf, j.c_off), ptr(j.a_buf, j.a_off), ptr(j.b_buf, j.b_off),
                                    j.to32 ? a.linv32 + j.c_off : nullptr, j.m, j.n, j.k,
                                    j.transb ? 1 : 0, j.lower ? 1 : 0, j.alpha, j.beta};
            g.first[g.njobs] = blocks;
            blocks += (j.m / 64) * (j.n / 64);
            ++g.njobs;
            g.first[g.njobs] = blocks;
        }
        hipLaunchKernelGGL(subblock_kernel, dim3((unsigned)blocks), dim3(kSubThreads), 0, stream, g);
    }
    hipLaunchKernelGGL(potrf_finish_kernel, dim3(1), dim3(kFinishThreads), 0, stream, a);
}

}  // namespace

template <int T>
void launch_potrf_threads(const PotrfArgs &a, hipStream_t stream) {
    hipLaunchKernelGGL((potrf_tile_kernel<T>), dim3(1), dim3(T), 0, stream, a);
}

void launch_potrf(const PotrfArgs &a, hipStream_t stream) {
    if ((a.nbp == 256 || a.nbp == 512) && (a.ld == 0 || a.ld == a.nbp)) launch_potrf_blocked(a, stream);
    else launch_potrf_threads<512>(a, stream);
}

}  // namespace mpgeo
