// Tile products of the mixed-precision Cholesky (Algorithm 1) on the matrix cores.
//
// Both the trailing update (dsyrk/dgemm/sgemm: A_ij -= A_ik A_jk^T) and the panel
// solve (dtrsm/strsm, done as X = A_ik L_kk^-T with the explicit inverse) are
// C[rows, cols] (+)= sum_t R[row, t] Q[col, t] over square nbp x nbp column-major tiles,
// where R supplies the rows of the output and Q its columns.
//
// A workgroup of 64 * WM * WN threads computes a BM x BN block of one output tile; wave
// (wr, wc) owns a (BM/WM) x (BN/WN) sub-block made of 16 x 16 MFMA blocks
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
    __device__ static acc_t mac(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // result register q of lane (16 * g + j) holds D[m][j] with m = 4 g + q
    __device__ static int m_index(int g, int q) { return 4 * g + q; }
};
template <> struct Mfma<double> {
    using acc_t = f64x4;
    __device__ static acc_t mac(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // result register q of lane (16 * g + j) holds D[m][j] with m = g + 4 q
    __device__ static int m_index(int g, int q) { return g + 4 * q; }
};

constexpr int kXcds = 8;

enum Epilogue { kUpdate = 0, kTrsm = 1 };

struct GemmArgs {
    TileMap map;
    int64_t ntiles;       // output tiles in this launch
    const TileIJ *list;   // update: output tiles (i, j); trsm: panel tiles (i, k), or null for a range
    int k;                // step (trsm: panel column; output rows i = i_begin + tile)
    int i_begin;
    const void *panel;    // update: staging panel of the kernel's precision (tile i at i*nbp^2)
    const void *linv;     // trsm: L_kk^-1 in the kernel's precision
    double *p64;          // trsm outputs
    float *p32;
};

// Block shape: BM output rows x BN output columns per workgroup, WM x WN waves, K chunk KC.
template <int BM_, int BN_, int WM_, int WN_, int KC_> struct Shape {
    static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, KC = KC_;
    static constexpr int kThreads = 64 * WM * WN;
};

template <typename T, typename S, int EPI>
__global__ __launch_bounds__(S::kThreads) void tile_gemm_kernel(GemmArgs g) {
    using M = Mfma<T>;
    using acc_t = typename M::acc_t;
    constexpr int BM = S::BM, BN = S::BN, KC = S::KC, NT = S::kThreads;
    constexpr int NBR = BM / S::WM / 16;   // 16-row blocks per wave
    constexpr int NBC = BN / S::WN / 16;   // 16-column blocks per wave
    constexpr int LDQ = BN + 16;           // padded LDS rows (spread the 4 k-rows over banks)
    constexpr int LDR = BM + 16;
    constexpr int VEC = 16 / sizeof(T);    // elements per 16-byte load
    constexpr int NVQ = KC * BN / VEC;     // 16-byte vectors per chunk of Q
    constexpr int NVR = KC * BM / VEC;
    constexpr int VPQ = (NVQ + NT - 1) / NT;
    constexpr int VPR = (NVR + NT - 1) / NT;
    typedef T vec_t __attribute__((ext_vector_type(VEC)));

    __shared__ T ldsq[2][KC * LDQ];
    __shared__ T ldsr[2][KC * LDR];

    const int nbp = g.map.nbp;
    const int rows_per = nbp / BM, cols_per = nbp / BN;
    const int per_tile = rows_per * cols_per;
    // Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2).  Map
    // them so that all blocks of one output tile run on the same XCD: its row and column
    // panel slices are then re-read from that XCD's L2.
    const int xcd = blockIdx.x % kXcds;
    const int local = blockIdx.x / kXcds;
    const int macro = local % per_tile;
    const int tile = (local / per_tile) * kXcds + xcd;
    if (tile >= g.ntiles) return;
    const int mr = macro % rows_per;   // row block
    const int mc = macro / rows_per;   // column block
    const int row0 = mr * BM;
    const int col0 = mc * BN;

    const T *R;
    const T *Q;
    int ti, tj;
    if (EPI == kUpdate) {
        const TileIJ t = g.list[tile];
        ti = t.i;
        tj = t.j;
        if (ti == tj && col0 >= row0 + BM) return;   // strictly upper part of a diagonal tile
        const T *panel = static_cast<const T *>(g.panel);
        R = panel + (int64_t)ti * nbp * nbp;
        Q = panel + (int64_t)tj * nbp * nbp;
    } else {
        ti = g.list ? g.list[tile].i : g.i_begin + tile;
        tj = g.k;
        const int64_t off = g.map.off[tri_index(ti, tj)];
        R = (sizeof(T) == 8) ? reinterpret_cast<const T *>(g.map.pool64 + off)
                             : reinterpret_cast<const T *>(g.map.pool32 + off);
        Q = static_cast<const T *>(g.linv);
    }
    R += row0;
    Q += col0;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave % S::WM;
    const int wc = wave / S::WM;
    const int wrow = wr * (BM / S::WM);
    const int wcol = wc * (BN / S::WN);
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
    acc_t acc[NBC][NBR];      // [column block][row block]
#pragma unroll
    for (int a = 0; a < NBC; ++a)
#pragma unroll
        for (int b = 0; b < NBR; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (kPreload) {
                    const int row = row0 + wrow + b * 16 + lrow;
                    const int col = col0 + wcol + a * 16 + M::m_index(lk, q);
                    acc[a][b][q] = C[row + (int64_t)col * nbp];
                } else {
                    acc[a][b][q] = 0;
                }
            }

    vec_t regQ[VPQ], regR[VPR];
    auto load_chunk = [&](int k0) {
#pragma unroll
        for (int v = 0; v < VPQ; ++v) {
            const int idx = v * NT + tid;
            if (NVQ % NT == 0 || idx < NVQ) {
                const int t = idx / (BN / VEC), rv = idx % (BN / VEC);
                regQ[v] = *reinterpret_cast<const vec_t *>(Q + (int64_t)(k0 + t) * nbp + rv * VEC);
            }
        }
#pragma unroll
        for (int v = 0; v < VPR; ++v) {
            const int idx = v * NT + tid;
            if (NVR % NT == 0 || idx < NVR) {
                const int t = idx / (BM / VEC), rv = idx % (BM / VEC);
                regR[v] = *reinterpret_cast<const vec_t *>(R + (int64_t)(k0 + t) * nbp + rv * VEC);
            }
        }
    };
    auto store_chunk = [&](int buf) {
#pragma unroll
        for (int v = 0; v < VPQ; ++v) {
            const int idx = v * NT + tid;
            if (NVQ % NT == 0 || idx < NVQ) {
                const int t = idx / (BN / VEC), rv = idx % (BN / VEC);
                *reinterpret_cast<vec_t *>(&ldsq[buf][t * LDQ + rv * VEC]) = regQ[v];
            }
        }
#pragma unroll
        for (int v = 0; v < VPR; ++v) {
            const int idx = v * NT + tid;
            if (NVR % NT == 0 || idx < NVR) {
                const int t = idx / (BM / VEC), rv = idx % (BM / VEC);
                *reinterpret_cast<vec_t *>(&ldsr[buf][t * LDR + rv * VEC]) = regR[v];
            }
        }
    };

    // TRSM: Q = L_kk^-1 is lower triangular (Q[col][t] = 0 for t > col), so K stops after
    // this block's last column
    const int nchunks = (EPI == kTrsm) ? (col0 + BN) / KC : nbp / KC;
    load_chunk(0);
    store_chunk(0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunks) load_chunk((c + 1) * KC);
        const T *sq = ldsq[buf];
        const T *sr = ldsr[buf];
#pragma unroll
        for (int s = 0; s < KC / 4; ++s) {
            const int t = 4 * s + lk;
            T qa[NBC], rb[NBR];
#pragma unroll
            for (int a = 0; a < NBC; ++a) {
                qa[a] = sq[t * LDQ + wcol + a * 16 + lrow];
                if (EPI == kUpdate) qa[a] = -qa[a];
            }
#pragma unroll
            for (int b = 0; b < NBR; ++b) rb[b] = sr[t * LDR + wrow + b * 16 + lrow];
#pragma unroll
            for (int a = 0; a < NBC; ++a)
#pragma unroll
                for (int b = 0; b < NBR; ++b) acc[a][b] = M::mac(qa[a], rb[b], acc[a][b]);
        }
        if (c + 1 < nchunks) store_chunk(buf ^ 1);
        __syncthreads();
    }

    // acc[a][b][q] holds output (row = b-block row lrow, col = a-block col m_index(lk, q))
    if (EPI == kUpdate) {
#pragma unroll
        for (int a = 0; a < NBC; ++a)
#pragma unroll
            for (int b = 0; b < NBR; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = row0 + wrow + b * 16 + lrow;
                    const int col = col0 + wcol + a * 16 + M::m_index(lk, q);
                    T *pc = C + row + (int64_t)col * nbp;
                    if (kPreload) *pc = acc[a][b][q];
                    else *pc = *pc + acc[a][b][q];
                }
    } else {
        double *o64 = g.p64 + (int64_t)ti * nbp * nbp;
        float *o32 = g.p32 + (int64_t)ti * nbp * nbp;
#pragma unroll
        for (int a = 0; a < NBC; ++a)
#pragma unroll
            for (int b = 0; b < NBR; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = row0 + wrow + b * 16 + lrow;
                    const int col = col0 + wcol + a * 16 + M::m_index(lk, q);
                    const int64_t e = row + (int64_t)col * nbp;
                    const T v = acc[a][b][q];
                    o64[e] = (double)v;
                    o32[e] = (float)v;   // FP64 result rounded to nearest even / FP32 kept
                }
    }
}

template <typename T, typename S, int EPI>
void launch_shape(const GemmArgs &g, int64_t ntiles, hipStream_t stream) {
    GemmArgs ga = g;
    ga.ntiles = ntiles;
    const int nbp = g.map.nbp;
    const int64_t slots = (ntiles + kXcds - 1) / kXcds * kXcds;   // whole tiles per XCD
    const int64_t blocks = slots * (nbp / S::BM) * (nbp / S::BN);
    hipLaunchKernelGGL((tile_gemm_kernel<T, S, EPI>), dim3((unsigned)blocks), dim3(S::kThreads), 0,
                       stream, ga);
}

// Production shapes: 128 x 128 blocks of 8 waves (64 x 32 each) when the tile allows, else 64
// or 32; K chunks of 16 columns.  `narrow` (the few-tile FP64 launches of the critical path,
// which run beside the wide trailing updates): 64 x 64 blocks with K chunks of 8, 20 KB of LDS
// instead of 72 KB, so a workgroup fits where one of the concurrent update workgroups ends.
// Measured in the n ~ 1e5 evaluations: FP32 updates 123 TFLOP/s with 8 waves of 64 x 32 (8
// waves of 32 x 64: 119.6; 4 waves of 64 x 64, accumulators in AGPRs at 3 waves per SIMD: 114;
// 256 x 128 or 256 x 256 blocks, or K chunks of 32 or 8: 93-106); the all-FP64 evaluation 5.32 s
// against 5.54 s with 4 waves.  The panel TRSMs keep 4 waves of 64 x 64: with 8 waves they ran
// 3.8x faster on the lookahead stream but took compute units from the 16-bit pass beside them
// (three-tier evaluation 1.00 against 1.06 evaluations/s).  FP64 band lists (a third
// of them diagonal tiles) run faster on 64 x 64 blocks of 4 waves (56.5 TFLOP/s measured alone
// on the step-0 lists against 51.7 with 128 x 128: the diagonal tiles' skipped upper blocks
// waste less).
constexpr int64_t kShortFp64List = 1024;
template <typename T, int EPI>
void launch_gemm(const GemmArgs &g, int64_t ntiles, hipStream_t stream, bool narrow = false) {
    const int nbp = g.map.nbp;
    if (ntiles <= 0) return;
    if (narrow && nbp % 64 == 0) launch_shape<T, Shape<64, 64, 2, 2, 8>, EPI>(g, ntiles, stream);
    else if (EPI == kUpdate && sizeof(T) == 8 && nbp % 64 == 0 && ntiles <= kShortFp64List)
        launch_shape<T, Shape<64, 64, 2, 2, 16>, EPI>(g, ntiles, stream);
    else if (nbp % 128 == 0 && EPI == kTrsm) launch_shape<T, Shape<128, 128, 2, 2, 16>, EPI>(g, ntiles, stream);
    else if (nbp % 128 == 0) launch_shape<T, Shape<128, 128, 2, 4, 16>, EPI>(g, ntiles, stream);
    else if (nbp % 64 == 0) launch_shape<T, Shape<64, 64, 2, 2, 16>, EPI>(g, ntiles, stream);
    else launch_shape<T, Shape<32, 32, 2, 2, 16>, EPI>(g, ntiles, stream);
}

}  // namespace

void launch_trsm(const TileMap &map, int k, int i_begin, int count, bool fp64, const double *linv,
                 const float *linv32, double *p64, float *p32, hipStream_t stream, bool narrow,
                 const TileIJ *list) {
    if (count <= 0) return;
    GemmArgs g{};
    g.map = map;
    g.k = k;
    g.i_begin = i_begin;
    g.list = list;
    g.p64 = p64;
    g.p32 = p32;
    if (fp64) {
        g.linv = linv;
        launch_gemm<double, kTrsm>(g, count, stream, narrow);
    } else {
        g.linv = linv32;
        launch_gemm<float, kTrsm>(g, count, stream);
    }
}

void launch_update(const TileMap &map, const TileIJ *list, int64_t count, bool fp64,
                   const double *p64, const float *p32, hipStream_t stream, bool narrow) {
    if (count <= 0) return;
    GemmArgs g{};
    g.map = map;
    g.list = list;
    if (fp64) {
        g.panel = p64;
        launch_gemm<double, kUpdate>(g, count, stream, narrow);
    } else {
        g.panel = p32;
        launch_gemm<float, kUpdate>(g, count, stream);
    }
}

}  // namespace mpgeo
