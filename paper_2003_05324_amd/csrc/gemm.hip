// Tile products of the mixed-precision Cholesky (Algorithm 1) on the matrix cores.
//
// Both the trailing update (dsyrk/dgemm/sgemm: A_ij -= A_ik A_jk^T) and the panel
// solve (dtrsm/strsm, done as X = A_ik L_kk^-T with the explicit inverse) are
// C[rows, cols] (+)= sum_t R[row, t] Q[col, t] over square nbp x nbp column-major tiles,
// where R supplies the rows of the output and Q its columns.
//
// A workgroup of 256 threads (4 waves, 2 x 2) computes an MT x MT block of one output
// tile; each wave owns an (MT/2) x (MT/2) sub-block made of 16 x 16 MFMA blocks
// (v_mfma_f64_16x16x4_f64 for FP64 tiles, v_mfma_f32_16x16x4_f32 for FP32 tiles).
// K is walked in chunks of KC columns staged through LDS as [t][row] (rows contiguous,
// like the tiles), double-buffered, with the next chunk prefetched into registers while
// the current one feeds the MFMAs.  In MFMA terms the A operand is Q (its "m" index is
// the output column) and the B operand is R ("n" = output row), so each lane of the
// 16 x 16 result holds 4 output columns of one row, and a store instruction writes 16
// consecutive rows of 4 columns.  (The f32 and f64 instructions order those 4 columns
// differently across lanes and registers; see Mfma<T>::m_index.)
#include "common.h"

namespace mpgeo {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<float> {
    using acc_t = f32x4;
    static constexpr int kKC = 16;
    __device__ static acc_t mac(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // result register q of lane (16 * g + j) holds D[m][j] with m = 4 g + q
    __device__ static int m_index(int g, int q) { return 4 * g + q; }
};
template <> struct Mfma<double> {
    using acc_t = f64x4;
    static constexpr int kKC = 16;
    __device__ static acc_t mac(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // result register q of lane (16 * g + j) holds D[m][j] with m = g + 4 q
    __device__ static int m_index(int g, int q) { return g + 4 * q; }
};

constexpr int kThreads = 256;
constexpr int kXcds = 8;

enum Epilogue { kUpdate = 0, kTrsm = 1 };

struct GemmArgs {
    TileMap map;
    int64_t ntiles;       // output tiles in this launch
    const TileIJ *list;   // update: output tiles (i, j)
    int k;                // step (trsm: panel column; output rows i = i_begin + tile)
    int i_begin;
    const void *panel;    // update: staging panel of the kernel's precision (tile i at i*nbp^2)
    const void *linv;     // trsm: L_kk^-1 in the kernel's precision
    double *p64;          // trsm outputs
    float *p32;
};

template <typename T, int MT, int EPI>
__global__ __launch_bounds__(kThreads) void tile_gemm_kernel(GemmArgs g) {
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    constexpr int KC = M::kKC;
    constexpr int WT = MT / 2;          // wave sub-block
    constexpr int NB16 = WT / 16;       // 16 x 16 blocks per wave side
    constexpr int LDS_LD = MT + 16;     // padded LDS row (spreads the 4 k-rows over banks)
    constexpr int VEC = 16 / sizeof(T); // elements per 16-byte load
    constexpr int NVEC = KC * MT / VEC; // 16-byte vectors per operand chunk
    constexpr int VPT = (NVEC + kThreads - 1) / kThreads;
    typedef T vec_t __attribute__((ext_vector_type(VEC)));

    __shared__ T lds[2][2][KC * LDS_LD];   // [buffer][operand: 0 = Q, 1 = R]

    const int nbp = g.map.nbp;
    const int per_side = nbp / MT;
    const int per_tile = per_side * per_side;
    // Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  Map
    // them so that all macro blocks of one output tile run on the same XCD: its row and
    // column panel slices are then re-read from that XCD's L2.
    const int xcd = blockIdx.x % kXcds;
    const int local = blockIdx.x / kXcds;
    const int macro = local % per_tile;
    const int tile = (local / per_tile) * kXcds + xcd;
    if (tile >= g.ntiles) return;
    const int mr = macro % per_side;   // row block
    const int mc = macro / per_side;   // column block

    const T *R;
    const T *Q;
    int ti, tj;
    if (EPI == kUpdate) {
        const TileIJ t = g.list[tile];
        ti = t.i;
        tj = t.j;
        if (ti == tj && mc > mr) return;   // strictly upper part of a diagonal tile
        const T *panel = static_cast<const T *>(g.panel);
        R = panel + (int64_t)ti * nbp * nbp;
        Q = panel + (int64_t)tj * nbp * nbp;
    } else {
        ti = g.i_begin + tile;
        tj = g.k;
        const int64_t off = g.map.off[tri_index(ti, tj)];
        R = (sizeof(T) == 8) ? reinterpret_cast<const T *>(g.map.pool64 + off)
                             : reinterpret_cast<const T *>(g.map.pool32 + off);
        Q = static_cast<const T *>(g.linv);
    }
    const int row0 = mr * MT;
    const int col0 = mc * MT;
    R += row0;
    Q += col0;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave & 1;    // wave row half
    const int wc = wave >> 1;   // wave column half

    const int lrow = lane & 15;      // position inside a 16-block
    const int lk = lane >> 4;        // k within the 4-step

    // FP64 update: the accumulators start from the C block itself (its loads overlap the
    // first chunk's) and take -R Q^T; the epilogue is then a plain store.  FP32 update: the
    // product is accumulated from zero and subtracted from C once at the end, so partial sums
    // are rounded at the scale of the product rather than of C (as a BLAS sgemm with beta = 1
    // would).  TRSM starts from 0.
    constexpr bool kPreload = (EPI == kUpdate) && (sizeof(T) == 8);
    T *C = nullptr;
    if (EPI == kUpdate) {
        const int64_t off = g.map.off[tri_index(ti, tj)];
        C = (sizeof(T) == 8) ? reinterpret_cast<T *>(g.map.pool64 + off)
                             : reinterpret_cast<T *>(g.map.pool32 + off);
    }
    acc_t acc[NB16][NB16];      // [col block][row block]
#pragma unroll
    for (int a = 0; a < NB16; ++a)
#pragma unroll
        for (int b = 0; b < NB16; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (kPreload) {
                    const int row = row0 + wr * WT + b * 16 + lrow;
                    const int col = col0 + wc * WT + a * 16 + M::m_index(lk, q);
                    acc[a][b][q] = C[row + (int64_t)col * nbp];
                } else {
                    acc[a][b][q] = 0;
                }
            }

    vec_t regQ[VPT], regR[VPT];
    auto load_chunk = [&](int k0) {
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const int idx = v * kThreads + tid;
            if (idx < NVEC) {
                const int t = idx / (MT / VEC);
                const int rv = idx % (MT / VEC);
                const int64_t e = (int64_t)(k0 + t) * nbp + rv * VEC;
                regQ[v] = *reinterpret_cast<const vec_t *>(Q + e);
                regR[v] = *reinterpret_cast<const vec_t *>(R + e);
            }
        }
    };
    auto store_chunk = [&](int buf) {
#pragma unroll
        for (int v = 0; v < VPT; ++v) {
            const int idx = v * kThreads + tid;
            if (idx < NVEC) {
                const int t = idx / (MT / VEC);
                const int rv = idx % (MT / VEC);
                *reinterpret_cast<vec_t *>(&lds[buf][0][t * LDS_LD + rv * VEC]) = regQ[v];
                *reinterpret_cast<vec_t *>(&lds[buf][1][t * LDS_LD + rv * VEC]) = regR[v];
            }
        }
    };

    // TRSM: Q = L_kk^-1 is lower triangular (Q[col][t] = 0 for t > col), so K stops after
    // this block's last column
    const int nchunks = (EPI == kTrsm) ? (col0 + MT) / KC : nbp / KC;
    load_chunk(0);
    store_chunk(0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunks) load_chunk((c + 1) * KC);
        const T *sq = lds[buf][0];
        const T *sr = lds[buf][1];
#pragma unroll
        for (int s = 0; s < KC / 4; ++s) {
            const int t = 4 * s + lk;
            T qa[NB16], rb[NB16];
#pragma unroll
            for (int a = 0; a < NB16; ++a) {
                qa[a] = sq[t * LDS_LD + wc * WT + a * 16 + lrow];
                if (EPI == kUpdate) qa[a] = -qa[a];
            }
#pragma unroll
            for (int b = 0; b < NB16; ++b) rb[b] = sr[t * LDS_LD + wr * WT + b * 16 + lrow];
#pragma unroll
            for (int a = 0; a < NB16; ++a)
#pragma unroll
                for (int b = 0; b < NB16; ++b) acc[a][b] = M::mac(qa[a], rb[b], acc[a][b]);
        }
        if (c + 1 < nchunks) store_chunk(buf ^ 1);
        __syncthreads();
    }

    // acc[a][b][q] holds output (row = b-block row lrow, col = a-block col m_index(lk, q))
    if (EPI == kUpdate) {
#pragma unroll
        for (int a = 0; a < NB16; ++a)
#pragma unroll
            for (int b = 0; b < NB16; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = row0 + wr * WT + b * 16 + lrow;
                    const int col = col0 + wc * WT + a * 16 + M::m_index(lk, q);
                    T *pc = C + row + (int64_t)col * nbp;
                    if (kPreload) *pc = acc[a][b][q];
                    else *pc = *pc + acc[a][b][q];
                }
    } else {
        double *o64 = g.p64 + (int64_t)ti * nbp * nbp;
        float *o32 = g.p32 + (int64_t)ti * nbp * nbp;
#pragma unroll
        for (int a = 0; a < NB16; ++a)
#pragma unroll
            for (int b = 0; b < NB16; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = row0 + wr * WT + b * 16 + lrow;
                    const int col = col0 + wc * WT + a * 16 + M::m_index(lk, q);
                    const int64_t e = row + (int64_t)col * nbp;
                    const T v = acc[a][b][q];
                    o64[e] = (double)v;
                    o32[e] = (float)v;   // FP64 result rounded to nearest even / FP32 kept
                }
    }
}

template <typename T, int EPI>
void launch_gemm(const GemmArgs &g, int64_t ntiles, bool diag_skip_free, hipStream_t stream) {
    (void)diag_skip_free;
    const int nbp = g.map.nbp;
    if (ntiles <= 0) return;
    GemmArgs ga = g;
    ga.ntiles = ntiles;
    const int64_t slots = (ntiles + kXcds - 1) / kXcds * kXcds;   // whole tiles per XCD
    if (nbp % 128 == 0) {
        const int64_t blocks = slots * (nbp / 128) * (nbp / 128);
        hipLaunchKernelGGL((tile_gemm_kernel<T, 128, EPI>), dim3((unsigned)blocks), dim3(kThreads), 0,
                           stream, ga);
    } else if (nbp % 64 == 0) {
        const int64_t blocks = slots * (nbp / 64) * (nbp / 64);
        hipLaunchKernelGGL((tile_gemm_kernel<T, 64, EPI>), dim3((unsigned)blocks), dim3(kThreads), 0,
                           stream, ga);
    } else {
        const int64_t blocks = slots * (nbp / 32) * (nbp / 32);
        hipLaunchKernelGGL((tile_gemm_kernel<T, 32, EPI>), dim3((unsigned)blocks), dim3(kThreads), 0,
                           stream, ga);
    }
}

}  // namespace

void launch_trsm(const TileMap &map, int k, int i_begin, int count, bool fp64, const double *linv,
                 const float *linv32, double *p64, float *p32, hipStream_t stream) {
    if (count <= 0) return;
    GemmArgs g{};
    g.map = map;
    g.k = k;
    g.i_begin = i_begin;
    g.p64 = p64;
    g.p32 = p32;
    if (fp64) {
        g.linv = linv;
        launch_gemm<double, kTrsm>(g, count, false, stream);
    } else {
        g.linv = linv32;
        launch_gemm<float, kTrsm>(g, count, false, stream);
    }
}

void launch_update(const TileMap &map, const TileIJ *list, int64_t count, bool fp64,
                   const double *p64, const float *p32, hipStream_t stream) {
    if (count <= 0) return;
    GemmArgs g{};
    g.map = map;
    g.list = list;
    if (fp64) {
        g.panel = p64;
        launch_gemm<double, kUpdate>(g, count, false, stream);
    } else {
        g.panel = p32;
        launch_gemm<float, kUpdate>(g, count, false, stream);
    }
}

}  // namespace mpgeo
