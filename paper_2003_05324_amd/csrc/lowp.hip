// Third precision tier: trailing updates of the farthest tiles with FP16 or BF16 operands on
// the matrix cores (the paper's future work, Section IX: more than two precision layers).
//
// Tiles with i - j > band64 + band32 keep FP32 storage and FP32 accumulation; only the
// operands of their update A_ij -= L_ik L_jk^T drop to a 16-bit format.  After the panel of
// step k is solved, every panel tile L_ik is quantised once:
//   s_i = 2^ceil(log2 max|L_ik|)   (a power of two, so the scaling is exact),
//   Q_i = round_to_nearest_even(L_ik / s_i)   in FP16 or BF16,
// stored row-major (K contiguous) for 16-byte operand loads.  The update is then
//   A_ij -= (s_i s_j) * (Q_i Q_j^T)   with v_mfma_f32_16x16x32_{f16,bf16} accumulating in FP32.
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

// One workgroup per 64 x 64 block of a panel tile: scale by the tile's power of two
// s = 2^e with 2^(e-1) < max|x| <= 2^e (s = 1 for an all-zero tile), round to the 16-bit
// format (nearest even) and store transposed (row-major, K contiguous).
template <typename T, int QB>
__global__ __launch_bounds__(kQThreads) void quantize_kernel(const float *p32, const unsigned *absmax,
                                                             T *q, float *scale, int first, int nbp) {
    __shared__ float blk[QB][QB + 1];
    const int per_side = nbp / QB;
    const int i = first + blockIdx.x / (per_side * per_side);
    const int b = blockIdx.x % (per_side * per_side);
    const int r0 = (b % per_side) * QB, t0 = (b / per_side) * QB;
    const float mx = __uint_as_float(absmax[i]);
    int ex = 0;
    if (mx > 0.0f) {
        const float fr = frexpf(mx, &ex);   // mx = fr * 2^ex, fr in [0.5, 1)
        if (fr == 0.5f) ex -= 1;            // an exact power of two maps to 1
    }
    const float inv = ldexpf(1.0f, -ex);
    if (b == 0 && threadIdx.x == 0) scale[i] = ldexpf(1.0f, ex);
    const float *src = p32 + (int64_t)i * nbp * nbp;
    T *dst = q + (int64_t)i * nbp * nbp;
    for (int e = threadIdx.x; e < QB * QB; e += kQThreads) {
        const int rr = e % QB, tt = e / QB;
        blk[rr][tt] = src[(r0 + rr) + (int64_t)(t0 + tt) * nbp] * inv;   // exact (power of two)
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
    const void *q;        // quantised panel, tile i at i * nbp^2, row-major
    const float *scale;   // per panel tile
};

// BM x BN output block, WM x WN waves, K chunk KC, DEPTH chunks of operands in flight;
// CPRE: load the C block into registers before the K loop (its latency hides behind it);
// PAD: 16-bit elements of padding per LDS row (spreads the rows over the banks).
template <int BM_, int BN_, int WM_, int WN_, int KC_, int DEPTH_ = 1, int CPRE_ = 0, int PAD_ = 8>
struct LShape {
    static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, KC = KC_, DEPTH = DEPTH_, PAD = PAD_;
    static constexpr bool CPRE = CPRE_ != 0;
    static constexpr int kThreads = 64 * WM * WN;
};

// C[rows, cols] -= s_i s_j * sum_t Q_i[row][t] Q_j[col][t] on one BM x BN block of a tile.
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
    const T *qbase = static_cast<const T *>(g.q);
    const T *R = qbase + (int64_t)tij.i * nbp * nbp + (int64_t)row0 * nbp;
    const T *Q = qbase + (int64_t)tij.j * nbp * nbp + (int64_t)col0 * nbp;
    const float factor = -g.scale[tij.i] * g.scale[tij.j];
    float *C = g.map.pool32 + g.map.off[tri_index(tij.i, tij.j)];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wrow = (wave % S::WM) * (BM / S::WM);
    const int wcol = (wave / S::WM) * (BN / S::WN);
    const int lr = lane & 15, lg = lane >> 4;

    f32x4 acc[NBC][NBR];
    f32x4 cpre[S::CPRE ? NBC : 1][S::CPRE ? NBR : 1];
#pragma unroll
    for (int a = 0; a < NBC; ++a)
#pragma unroll
        for (int b = 0; b < NBR; ++b) {
            acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
            if (S::CPRE)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    cpre[a][b][q] = C[(row0 + wrow + b * 16 + lr) + (int64_t)(col0 + wcol + a * 16 + 4 * lg + q) * nbp];
        }

    // Operand chunks stream global -> registers -> LDS.  Chunk x waits in register set
    // x % DEPTH; DEPTH chunks are in flight while the chunk in LDS feeds the matrix cores
    // (the 16-bit MFMAs consume a chunk far faster than memory returns one).
    constexpr int D = S::DEPTH;
    vec8 rq[D][VPQ], rr[D][VPR];
    auto load_chunk = [&](vec8 (&sq)[VPQ], vec8 (&sr)[VPR], int k0) {
#pragma unroll
        for (int v = 0; v < VPQ; ++v) {
            const int idx = v * NT + tid;
            if (NVQ % NT == 0 || idx < NVQ) {
                const int row = idx / VPR_ROW, cv = idx % VPR_ROW;
                sq[v] = *reinterpret_cast<const vec8 *>(Q + (int64_t)row * nbp + k0 + cv * 8);
            }
        }
#pragma unroll
        for (int v = 0; v < VPR; ++v) {
            const int idx = v * NT + tid;
            if (NVR % NT == 0 || idx < NVR) {
                const int row = idx / VPR_ROW, cv = idx % VPR_ROW;
                sr[v] = *reinterpret_cast<const vec8 *>(R + (int64_t)row * nbp + k0 + cv * 8);
            }
        }
    };
    auto store_chunk = [&](const vec8 (&sq)[VPQ], const vec8 (&sr)[VPR], int buf) {
#pragma unroll
        for (int v = 0; v < VPQ; ++v) {
            const int idx = v * NT + tid;
            if (NVQ % NT == 0 || idx < NVQ) {
                const int row = idx / VPR_ROW, cv = idx % VPR_ROW;
                *reinterpret_cast<vec8 *>(&ldsq[buf][row * LD + cv * 8]) = sq[v];
            }
        }
#pragma unroll
        for (int v = 0; v < VPR; ++v) {
            const int idx = v * NT + tid;
            if (NVR % NT == 0 || idx < NVR) {
                const int row = idx / VPR_ROW, cv = idx % VPR_ROW;
                *reinterpret_cast<vec8 *>(&ldsr[buf][row * LD + cv * 8]) = sr[v];
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

    const int nchunks = nbp / KC;
#pragma unroll
    for (int j = 0; j < D; ++j)
        if (j < nchunks) load_chunk(rq[j], rr[j], j * KC);
    store_chunk(rq[0], rr[0], 0);
    if (D < nchunks) load_chunk(rq[0], rr[0], D * KC);
    __syncthreads();
    for (int c0 = 0; c0 < nchunks; c0 += D) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const int c = c0 + j;
            if (c < nchunks) {
                compute(c & 1);
                const int nxt = (j + 1) % D;   // register set of chunk c + 1
                if (c + 1 < nchunks) store_chunk(rq[nxt], rr[nxt], (c + 1) & 1);
                if (c + 1 + D < nchunks) load_chunk(rq[nxt], rr[nxt], (c + 1 + D) * KC);
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
                float *pc = C + row + (int64_t)col * nbp;
                const float c0v = S::CPRE ? cpre[S::CPRE ? a : 0][S::CPRE ? b : 0][q] : *pc;
                *pc = c0v + factor * acc[a][b][q];
            }
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

template <typename T>
void launch_lowp(const LowpArgs &g, int64_t ntiles, hipStream_t stream) {
    const int nbp = g.map.nbp;
    // 128 x 64 blocks, K chunks of 64 with two in flight, C loaded up front, LDS rows padded by
    // 16 elements (no bank conflicts): measured best on the n ~ 1e5 step-0 list (402 TFLOP/s;
    // K chunks of 32: 373, and padding 8 showed 5 conflict cycles per LDS instruction)
    if (nbp % 128 == 0) launch_lowp_shape<T, LShape<128, 64, 2, 2, 64, 2, 1, 16>>(g, ntiles, stream);
    else if (nbp % 64 == 0) launch_lowp_shape<T, LShape<64, 64, 2, 2, 64, 2, 1, 16>>(g, ntiles, stream);
    else launch_lowp_shape<T, LShape<32, 32, 2, 2, 32, 1, 0>>(g, ntiles, stream);
}

}  // namespace

void launch_quantize(const TileMap &map, int first, int count, const float *p32, const unsigned *absmax,
                     void *q, float *scale, int lowp, hipStream_t stream) {
    if (count <= 0) return;
    const int qb = (map.nbp % 64 == 0) ? 64 : 32;   // transpose block (nbp is a multiple of 32)
    const int per_side = map.nbp / qb;
    const unsigned blocks = (unsigned)((int64_t)count * per_side * per_side);
#define MPGEO_QUANT(T, QB)                                                                          \
    hipLaunchKernelGGL((quantize_kernel<T, QB>), dim3(blocks), dim3(kQThreads), 0, stream, p32, absmax, \
                       static_cast<T *>(q), scale, first, map.nbp)
    if (lowp == 1) {
        if (qb == 64) MPGEO_QUANT(_Float16, 64);
        else MPGEO_QUANT(_Float16, 32);
    } else {
        if (qb == 64) MPGEO_QUANT(__bf16, 64);
        else MPGEO_QUANT(__bf16, 32);
    }
#undef MPGEO_QUANT
}

void launch_update_lowp(const TileMap &map, const TileIJ *list, int64_t count, const void *q,
                        const float *scale, int lowp, hipStream_t stream) {
    if (count <= 0) return;
    LowpArgs g{};
    g.map = map;
    g.list = list;
    g.q = q;
    g.scale = scale;
    if (lowp == 1) launch_lowp<_Float16>(g, count, stream);
    else launch_lowp<__bf16>(g, count, stream);
}

}  // namespace mpgeo
