// Third precision tier: trailing updates of the farthest tiles with FP16 or BF16 operands on
// the matrix cores (the paper's future work, Section IX: more than two precision layers).
//
// Tiles with i - j > band64 + band32 keep FP32 storage and FP32 accumulation; only the
// operands of their update A_ij -= sum_k L_ik L_jk^T drop to a 16-bit format.
//
// Scaling.  Row r of the factor satisfies sum_k L_rk^2 = Sigma_rr, so |L_rk| <= sqrt(Sigma_rr).
// Tile row i takes one power of two from the diagonal of Sigma before the factorization,
//   s_i = 2^max(e_i - 14, -60),   e_i = ceil(log2 sqrt(max_{r in row block i} Sigma_rr)),
// so every 16-bit operand Q_ik = round_to_nearest_even(L_ik / s_i) lies below 2^14 in magnitude
// (FP16 holds up to 65504) and entries down to 2^-28 of the row's bound stay normal FP16
// numbers.  After the panel of step k is solved, each panel tile is quantised once into a
// 16-bit copy of the factor that lives for the whole factorization (tile (i, k) at slot
// tri_index(i, k), row-major, K contiguous).
//
// Update.  A far tile takes its panels in one left-looking pass:
//   A_ij <- -s_i s_j (-A_ij / (s_i s_j) + sum_k Q_ik Q_jk^T),
// with the FP32 accumulator of each element starting at -A_ij / (s_i s_j) (exact: a power of
// two) and v_mfma_f32_16x16x32_{f16,bf16} adding Q_ik Q_jk^T to it 32 products at a time,
// panels in ascending k; the final product by -s_i s_j is exact again.  Each element therefore
// sees one fixed sequence of FP32 roundings, set by the panels it takes and not by how they
// are split between launches or which of the two kernels below runs them.
#include "common.h"

namespace mpgeo {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 b8 __attribute__((ext_vector_type(8)));

template <typename T> struct Lowp;
template <> struct Lowp<_Float16> {
    using vec8 = h8;
    __device__ static f32x4 mac(vec8 a, vec8 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
    }
};
template <> struct Lowp<__bf16> {
    using vec8 = b8;
    __device__ static f32x4 mac(vec8 a, vec8 b, f32x4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
};

constexpr int kXcds = 8;
constexpr int kQThreads = 256;

// Power of two of each tile row from the diagonal tiles of Sigma (before factorization):
// s_i = 2^max(e_i - 14, -60) with e_i = ceil(log2 sqrt(max Sigma_rr)) over the row block's
// rows; s_i = 1 when that maximum is not positive (the factorization then fails anyway).
__global__ __launch_bounds__(64) void row_scale_kernel(TileMap map, float *rscale) {
    const int i = blockIdx.x;
    const int rows = (int)min((int64_t)map.nb, map.n - (int64_t)i * map.nb);
    const double *d = map.pool64 + map.off[tri_index(i, i)];
    double mx = 0.0;
    for (int r = threadIdx.x; r < rows; r += 64) mx = fmax(mx, d[r + (int64_t)r * map.nbp]);
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
    if (threadIdx.x == 0) {
        int es = 0;
        if (mx > 0.0) {
            int ex = 0;
            const double fr = frexp(sqrt(mx), &ex);   // sqrt(mx) = fr * 2^ex, fr in [0.5, 1)
            if (fr == 0.5) ex -= 1;                    // an exact power of two is its own bound
            es = max(ex - 14, -60);
        }
        rscale[i] = ldexpf(1.0f, es);
    }
}

// One workgroup per QB x QB block of panel tile (i, k): divide by the row's power of two
// (exact), round to the 16-bit format (nearest even) and store transposed (row-major, K
// contiguous) at slot tri_index(i, k).
template <typename T, int QB>
__global__ __launch_bounds__(kQThreads) void quantize_kernel(const float *p32, const float *rscale,
                                                             T *q, int k, int first, int nbp) {
    __shared__ float blk[QB][QB + 1];
    const int per_side = nbp / QB;
    const int i = first + blockIdx.x / (per_side * per_side);
    const int b = blockIdx.x % (per_side * per_side);
    const int r0 = (b % per_side) * QB, t0 = (b / per_side) * QB;
    const float inv = 1.0f / rscale[i];   // a power of two
    const int64_t slot = tri_index(i, k);
    const float *src = p32 + (int64_t)i * nbp * nbp;
    T *dst = q + slot * nbp * nbp;
    for (int e = threadIdx.x; e < QB * QB; e += kQThreads) {
        const int rr = e % QB, tt = e / QB;
        blk[rr][tt] = src[(r0 + rr) + (int64_t)(t0 + tt) * nbp] * inv;   // exact
    }
    __syncthreads();
    for (int e = threadIdx.x; e < QB * QB; e += kQThreads) {
        const int tt = e % QB, rr = e / QB;
        dst[(int64_t)(r0 + rr) * nbp + t0 + tt] = (T)blk[rr][tt];   // round to nearest even
    }
}

struct LowpArgs {
    TileMap map;
    int64_t ntiles;
    const TileIJ *list;
    const void *q;        // 16-bit factor copy: tile (i, k) at tri_index(i, k) * nbp^2, row-major
    const float *rscale;  // power of two of each tile row
    int kbeg, kend;       // target (i, j) takes panels k in [max(k0, i - zband), kend)
    int zband;            // tiles (i, k) with i - k > zband are dropped (zero)
    const int32_t *kstart;   // per list entry: its k0 (null: k0 = kbeg for every entry)
};

// BM x BN output block, WM x WN waves, K chunk KC, DEPTH chunks of operands in flight;
// PAD: 16-bit elements of padding per LDS row (spreads the rows over the banks).
template <int BM_, int BN_, int WM_, int WN_, int KC_, int DEPTH_ = 1, int PAD_ = 8>
struct LShape {
    static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, KC = KC_, DEPTH = DEPTH_, PAD = PAD_;
    static constexpr int kThreads = 64 * WM * WN;
};

// One BM x BN block of target tile (i, j):
//   C <- -s_i s_j (-C / (s_i s_j) + sum over panels k of sum_t Q_ik[row][t] Q_jk[col][t]).
// The block's accumulators are held in registers for the whole K loop (their load latency
// hides behind the first chunks); operands are staged global -> registers -> LDS.
template <typename T, typename S>
__global__ __launch_bounds__(S::kThreads) void lowp_update_kernel(LowpArgs g) {
    using L = Lowp<T>;
    using vec8 = typename L::vec8;
    constexpr int BM = S::BM, BN = S::BN, KC = S::KC, NT = S::kThreads;
    constexpr int NBR = BM / S::WM / 16;
    constexpr int NBC = BN / S::WN / 16;
    constexpr int LD = KC + S::PAD;        // padded LDS row
    constexpr int VPR_ROW = KC / 8;        // 16-byte vectors per row of a chunk
    constexpr int NVQ = BN * VPR_ROW, NVR = BM * VPR_ROW;
    constexpr int VPQ = (NVQ + NT - 1) / NT, VPR = (NVR + NT - 1) / NT;

    __shared__ __attribute__((aligned(16))) T ldsq[2][BN * LD];
    __shared__ __attribute__((aligned(16))) T ldsr[2][BM * LD];

    const int nbp = g.map.nbp;
    const int rows_per = nbp / BM, cols_per = nbp / BN;
    const int per_tile = rows_per * cols_per;
    const int xcd = blockIdx.x % kXcds;
    const int local = blockIdx.x / kXcds;
    const int macro = local % per_tile;
    const int tile = (local / per_tile) * kXcds + xcd;
    if (tile >= g.ntiles) return;
    const int row0 = (macro % rows_per) * BM;
    const int col0 = (macro / rows_per) * BN;
    const TileIJ tij = g.list[tile];
    const int kfirst = max(g.kstart ? g.kstart[tile] : g.kbeg, tij.i - g.zband);
    if (kfirst >= g.kend) return;
    const int cpp = nbp / KC;                           // chunks per panel
    const int nchunks = (g.kend - kfirst) * cpp;
    const int64_t te = (int64_t)nbp * nbp;
    const T *qbase = static_cast<const T *>(g.q);
    // panel k's operands: tile (i, k) = tile (i, 0) + k
    const T *R0 = qbase + tri_index(tij.i, kfirst) * te + (int64_t)row0 * nbp;
    const T *Q0 = qbase + tri_index(tij.j, kfirst) * te + (int64_t)col0 * nbp;
    const float f = g.rscale[tij.i] * g.rscale[tij.j];   // a power of two (at least 2^-120)
    const float ninv_f = -1.0f / f;
    float *C = g.map.pool32 + g.map.off[tri_index(tij.i, tij.j)];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wrow = (wave % S::WM) * (BM / S::WM);
    const int wcol = (wave / S::WM) * (BN / S::WN);
    const int lr = lane & 15, lg = lane >> 4;

    f32x4 acc[NBC][NBR];
#pragma unroll
    for (int a = 0; a < NBC; ++a)
#pragma unroll
        for (int b = 0; b < NBR; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc[a][b][q] = C[(row0 + wrow + b * 16 + lr) + (int64_t)(col0 + wcol + a * 16 + 4 * lg + q) * nbp] * ninv_f;

    // Operand chunks stream global -> registers -> LDS.  Chunk x waits in register set
    // x % DEPTH; DEPTH chunks are in flight while the chunk in LDS feeds the matrix cores
    // (the 16-bit MFMAs consume a chunk far faster than memory returns one).
    constexpr int D = S::DEPTH;
    vec8 rq[D][VPQ], rr[D][VPR];
    auto load_chunk = [&](vec8 (&sq)[VPQ], vec8 (&sr)[VPR], int c) {
        const int64_t off = (int64_t)(c / cpp) * te + (c % cpp) * KC;
#pragma unroll
        for (int v = 0; v < VPQ; ++v) {
            const int idx = v * NT + tid;
            if (NVQ % NT == 0 || idx < NVQ) {
                const int row = idx / VPR_ROW, col = idx % VPR_ROW;
                sq[v] = *reinterpret_cast<const vec8 *>(Q0 + off + (int64_t)row * nbp + col * 8);
            }
        }
#pragma unroll
        for (int v = 0; v < VPR; ++v) {
            const int idx = v * NT + tid;
            if (NVR % NT == 0 || idx < NVR) {
                const int row = idx / VPR_ROW, col = idx % VPR_ROW;
                sr[v] = *reinterpret_cast<const vec8 *>(R0 + off + (int64_t)row * nbp + col * 8);
            }
        }
    };
    auto store_chunk = [&](const vec8 (&sq)[VPQ], const vec8 (&sr)[VPR], int buf) {
#pragma unroll
        for (int v = 0; v < VPQ; ++v) {
            const int idx = v * NT + tid;
            if (NVQ % NT == 0 || idx < NVQ) {
                const int row = idx / VPR_ROW, col = idx % VPR_ROW;
                *reinterpret_cast<vec8 *>(&ldsq[buf][row * LD + col * 8]) = sq[v];
            }
        }
#pragma unroll
        for (int v = 0; v < VPR; ++v) {
            const int idx = v * NT + tid;
            if (NVR % NT == 0 || idx < NVR) {
                const int row = idx / VPR_ROW, col = idx % VPR_ROW;
                *reinterpret_cast<vec8 *>(&ldsr[buf][row * LD + col * 8]) = sr[v];
            }
        }
    };
    auto compute = [&](int buf) {
#pragma unroll
        for (int s = 0; s < KC / 32; ++s) {
            const int k = 32 * s + 8 * lg;     // this lane's 8 consecutive k
            vec8 qa[NBC], rb[NBR];
#pragma unroll
            for (int a = 0; a < NBC; ++a)
                qa[a] = *reinterpret_cast<const vec8 *>(&ldsq[buf][(wcol + a * 16 + lr) * LD + k]);
#pragma unroll
            for (int b = 0; b < NBR; ++b)
                rb[b] = *reinterpret_cast<const vec8 *>(&ldsr[buf][(wrow + b * 16 + lr) * LD + k]);
#pragma unroll
            for (int a = 0; a < NBC; ++a)
#pragma unroll
                for (int b = 0; b < NBR; ++b) acc[a][b] = L::mac(qa[a], rb[b], acc[a][b]);
        }
    };

#pragma unroll
    for (int j = 0; j < D; ++j)
        if (j < nchunks) load_chunk(rq[j], rr[j], j);
    store_chunk(rq[0], rr[0], 0);
    if (D < nchunks) load_chunk(rq[0], rr[0], D);
    __syncthreads();
    for (int c0 = 0; c0 < nchunks; c0 += D) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int c = c0 + j;
            if (c < nchunks) {
                compute(c & 1);
                const int nxt = (j + 1) % D;   // register set of chunk c + 1
                if (c + 1 < nchunks) store_chunk(rq[nxt], rr[nxt], (c + 1) & 1);
                if (c + 1 + D < nchunks) load_chunk(rq[nxt], rr[nxt], c + 1 + D);
                __syncthreads();
            }
        }
    }
    // result register q of lane (16 g + r): row lr of the b block, column 4 g + q of the a block
#pragma unroll
    for (int a = 0; a < NBC; ++a)
#pragma unroll
        for (int b = 0; b < NBR; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = row0 + wrow + b * 16 + lr;
                const int col = col0 + wcol + a * 16 + 4 * lg + q;
                C[row + (int64_t)col * nbp] = -(acc[a][b][q] * f);
            }
}

// The same block update with the operand chunks copied global -> LDS directly
// (global_load_lds_dwordx4: each lane's 16 bytes land at a wave-uniform LDS offset + 16 * lane),
// two chunks of K = 64 in LDS, no registers staging the operands.  One wave instruction fills
// 8 rows of 64 elements; row r keeps its 16-byte vector v at slot v ^ (r & 7), which keeps the
// fragment reads free of bank conflicts without padding.  Chunk c + 1 is in flight while chunk c
// feeds the matrix cores.
extern __shared__ __attribute__((aligned(16))) char lowp_dyn_lds[];

// 16 bytes from global src to LDS byte offset lds_off + 16 * lane (lds_off wave-uniform).  The
// builtin exists only for the device; the host pass sees an empty body.
__device__ inline void lds_copy16(const void *src, int lds_off) {
#if __HIP_DEVICE_COMPILE__
    __builtin_amdgcn_global_load_lds(src, lowp_dyn_lds + lds_off, 16, 0, 0);
#endif
}

template <int BM_, int BN_, int WM_, int WN_>
struct DShape {
    static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, KC = 64;
    static constexpr int kThreads = 64 * WM * WN;
    static constexpr size_t kLds = (size_t)2 * (BM + BN) * KC * 2;   // two chunks, bytes
};

template <typename T, typename S>
__global__ __launch_bounds__(S::kThreads) void lowp_direct_kernel(LowpArgs g) {
    using L = Lowp<T>;
    using vec8 = typename L::vec8;
    constexpr int BM = S::BM, BN = S::BN, KC = S::KC, NW = S::WM * S::WN;
    constexpr int NBR = BM / S::WM / 16;
    constexpr int NBC = BN / S::WN / 16;
    constexpr int ROWB = KC * 2;                       // bytes per LDS row
    constexpr int RB = BM * ROWB, QB = BN * ROWB;      // bytes per chunk and operand
    constexpr int GROUPS = (BM + BN) / 8;              // wave instructions per chunk
    static_assert(GROUPS % NW == 0, "row groups must split evenly over the waves");
    constexpr int GPW = GROUPS / NW;

    const int nbp = g.map.nbp;
    const int rows_per = nbp / BM, cols_per = nbp / BN;
    const int per_tile = rows_per * cols_per;
    const int xcd = blockIdx.x % kXcds;
    const int local = blockIdx.x / kXcds;
    const int macro = local % per_tile;
    const int tile = (local / per_tile) * kXcds + xcd;
    if (tile >= g.ntiles) return;
    const int row0 = (macro % rows_per) * BM;
    const int col0 = (macro / rows_per) * BN;
    const TileIJ tij = g.list[tile];
    const int kfirst = max(g.kstart ? g.kstart[tile] : g.kbeg, tij.i - g.zband);
    if (kfirst >= g.kend) return;
    const int cpp = nbp / KC;
    const int nchunks = (g.kend - kfirst) * cpp;
    const int64_t te = (int64_t)nbp * nbp;
    const T *qbase = static_cast<const T *>(g.q);
    const T *R0 = qbase + tri_index(tij.i, kfirst) * te + (int64_t)row0 * nbp;
    const T *Q0 = qbase + tri_index(tij.j, kfirst) * te + (int64_t)col0 * nbp;
    const float f = g.rscale[tij.i] * g.rscale[tij.j];
    const float ninv_f = -1.0f / f;
    float *C = g.map.pool32 + g.map.off[tri_index(tij.i, tij.j)];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wrow = (wave % S::WM) * (BM / S::WM);
    const int wcol = (wave / S::WM) * (BN / S::WN);
    const int lr = lane & 15, lg = lane >> 4;

    f32x4 acc[NBC][NBR];
#pragma unroll
    for (int a = 0; a < NBC; ++a)
#pragma unroll
        for (int b = 0; b < NBR; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc[a][b][q] = C[(row0 + wrow + b * 16 + lr) + (int64_t)(col0 + wcol + a * 16 + 4 * lg + q) * nbp] * ninv_f;

    // this lane's source within a group of 8 rows: row lane / 8, vector (lane & 7) ^ (lane / 8)
    const int lrow = lane >> 3, lvec = (lane & 7) ^ (lane >> 3);
    auto issue = [&](int c, int buf) {
        const int64_t off = (int64_t)(c / cpp) * te + (c % cpp) * KC + lvec * 8;
#pragma unroll
        for (int m = 0; m < GPW; ++m) {
            const int grp = wave + NW * m;   // wave-uniform
            const bool isr = grp < BM / 8;
            const int r = (isr ? grp : grp - BM / 8) * 8 + lrow;
            const T *src = (isr ? R0 : Q0) + off + (int64_t)r * nbp;
            const int dst = buf * (RB + QB) + (isr ? 0 : RB) + (isr ? grp : grp - BM / 8) * 8 * ROWB;
            lds_copy16(src, dst);
        }
    };
    auto compute = [&](int buf) {
        const char *chunk = lowp_dyn_lds + buf * (RB + QB);
#pragma unroll
        for (int s = 0; s < KC / 32; ++s) {
            const int v = 4 * s + lg;               // this lane's 16-byte vector of the row
            const int sw = (v ^ (lr & 7)) * 16;     // its slot (rows of a fragment share r & 7 = lr & 7)
            vec8 qa[NBC], rb[NBR];
#pragma unroll
            for (int a = 0; a < NBC; ++a)
                qa[a] = *reinterpret_cast<const vec8 *>(chunk + RB + (wcol + a * 16 + lr) * ROWB + sw);
#pragma unroll
            for (int b = 0; b < NBR; ++b)
                rb[b] = *reinterpret_cast<const vec8 *>(chunk + (wrow + b * 16 + lr) * ROWB + sw);
#pragma unroll
            for (int a = 0; a < NBC; ++a)
#pragma unroll
                for (int b = 0; b < NBR; ++b) acc[a][b] = L::mac(qa[a], rb[b], acc[a][b]);
        }
    };

    issue(0, 0);
    for (int c = 0; c < nchunks; ++c) {
        __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's copies of chunk c landed
        __syncthreads();                       // everyone's, and everyone is done with chunk c-1
        if (c + 1 < nchunks) issue(c + 1, (c + 1) & 1);
        compute(c & 1);
    }
#pragma unroll
    for (int a = 0; a < NBC; ++a)
#pragma unroll
        for (int b = 0; b < NBR; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = row0 + wrow + b * 16 + lr;
                const int col = col0 + wcol + a * 16 + 4 * lg + q;
                C[row + (int64_t)col * nbp] = -(acc[a][b][q] * f);
            }
}

template <typename T, typename S>
void launch_direct_shape(const LowpArgs &g, int64_t ntiles, hipStream_t stream) {
    LowpArgs ga = g;
    ga.ntiles = ntiles;
    const int nbp = g.map.nbp;
    const int64_t slots = (ntiles + kXcds - 1) / kXcds * kXcds;
    const int64_t blocks = slots * (nbp / S::BM) * (nbp / S::BN);
    hipLaunchKernelGGL((lowp_direct_kernel<T, S>), dim3((unsigned)blocks), dim3(S::kThreads), S::kLds,
                       stream, ga);
}

template <typename T, typename S>
void launch_lowp_shape(const LowpArgs &g, int64_t ntiles, hipStream_t stream) {
    LowpArgs ga = g;
    ga.ntiles = ntiles;
    const int nbp = g.map.nbp;
    const int64_t slots = (ntiles + kXcds - 1) / kXcds * kXcds;
    const int64_t blocks = slots * (nbp / S::BM) * (nbp / S::BN);
    hipLaunchKernelGGL((lowp_update_kernel<T, S>), dim3((unsigned)blocks), dim3(S::kThreads), 0, stream,
                       ga);
}

// many panels (the left-looking pass): 256 x 256 blocks when the tile allows, else 128 x 128
template <typename T, int BM> struct ManyPanel;
template <typename T> struct ManyPanel<T, 256> { using S = DShape<256, 256, 4, 4>; };
template <typename T> struct ManyPanel<T, 128> { using S = LShape<128, 128, 2, 2, 32, 1, 16>; };

template <typename T>
void launch_lowp(const LowpArgs &g, int64_t ntiles, hipStream_t stream) {
    const int nbp = g.map.nbp;
    const bool many = g.kstart != nullptr || g.kend - g.kbeg > 1;
    if (many && nbp % 256 == 0) {
        // many panels (the left-looking pass, long K): 256 x 256 blocks of 16 waves with 64 x 64
        // each, K chunks of 64 copied straight into LDS (measured alone on n ~ 1e5 columns:
        // 820-980 TFLOP/s; staged through registers: 770-905; 256 x 128 blocks: 705-770)
        launch_direct_shape<T, typename ManyPanel<T, 256>::S>(g, ntiles, stream);
    } else if (many && nbp % 128 == 0) {
        launch_lowp_shape<T, typename ManyPanel<T, 128>::S>(g, ntiles, stream);
    } else if (nbp % 128 == 0) {
        // one panel (the lookahead column, K = nbp): 128 x 64 blocks, K chunks of 64 with two in
        // flight, LDS rows padded by 16 elements (no bank conflicts)
        launch_lowp_shape<T, LShape<128, 64, 2, 2, 64, 2, 16>>(g, ntiles, stream);
    } else if (nbp % 64 == 0) {
        launch_lowp_shape<T, LShape<64, 64, 2, 2, 64, 2, 16>>(g, ntiles, stream);
    } else {
        launch_lowp_shape<T, LShape<32, 32, 2, 2, 32, 1>>(g, ntiles, stream);
    }
}

}  // namespace

void launch_row_scale(const TileMap &map, float *rscale, hipStream_t stream) {
    hipLaunchKernelGGL(row_scale_kernel, dim3((unsigned)map.p), dim3(64), 0, stream, map, rscale);
}

void launch_quantize(const TileMap &map, int k, int first, int count, const float *p32,
                     const float *rscale, void *q, int lowp, hipStream_t stream) {
    if (count <= 0) return;
    const int qb = (map.nbp % 64 == 0) ? 64 : 32;   // transpose block (nbp is a multiple of 32)
    const int per_side = map.nbp / qb;
    const unsigned blocks = (unsigned)((int64_t)count * per_side * per_side);
#define MPGEO_QUANT(T, QB)                                                                          \
    hipLaunchKernelGGL((quantize_kernel<T, QB>), dim3(blocks), dim3(kQThreads), 0, stream, p32, rscale, \
                       static_cast<T *>(q), k, first, map.nbp)
    if (lowp == 1) {
        if (qb == 64) MPGEO_QUANT(_Float16, 64);
        else MPGEO_QUANT(_Float16, 32);
    } else {
        if (qb == 64) MPGEO_QUANT(__bf16, 64);
        else MPGEO_QUANT(__bf16, 32);
    }
#undef MPGEO_QUANT
}

void launch_update_lowp(const TileMap &map, const TileIJ *list, int64_t count, int kbeg, int kend,
                        int zband, const void *q, const float *rscale, int lowp, hipStream_t stream,
                        const int32_t *kstart) {
    if (count <= 0 || (!kstart && kend <= kbeg)) return;
    LowpArgs g{};
    g.map = map;
    g.list = list;
    g.q = q;
    g.rscale = rscale;
    g.kbeg = kbeg;
    g.kend = kend;
    g.zband = zband;
    g.kstart = kstart;
    if (lowp == 1) launch_lowp<_Float16>(g, count, stream);
    else launch_lowp<__bf16>(g, count, stream);
}

namespace {
template <typename T, int BM> int wave_tiles_of(int nbp, int cus) {
    using S = typename ManyPanel<T, BM>::S;
    int per_cu = 0;
    hipError_t e;
    if constexpr (BM == 256)
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, lowp_direct_kernel<T, S>, S::kThreads, S::kLds);
    else
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, lowp_update_kernel<T, S>, S::kThreads, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const int per_tile = (nbp / S::BM) * (nbp / S::BN);
    return per_cu > 0 ? cus * per_cu / per_tile : 0;
}
}  // namespace

int lowp_wave_tiles(int nbp, int lowp, int cus) {
    if (cus <= 0 || lowp < 1 || lowp > 2) return 0;
    if (nbp % 256 == 0)
        return lowp == 1 ? wave_tiles_of<_Float16, 256>(nbp, cus) : wave_tiles_of<__bf16, 256>(nbp, cus);
    if (nbp % 128 == 0)
        return lowp == 1 ? wave_tiles_of<_Float16, 128>(nbp, cus) : wave_tiles_of<__bf16, 128>(nbp, cus);
    return 0;
}

}  // namespace mpgeo
