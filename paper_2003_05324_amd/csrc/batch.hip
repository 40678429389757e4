// Batched evaluation of eq. (2) for many independent problems as one persistent kernel over a
// device task queue (many small likelihoods, Section VIII; the tile size question of
// Section V-C at the scale of a batch).
//
// Each problem is cut into 128 x 128 tiles, FP64 within `band` tiles of the diagonal and FP32
// beyond (the precision map of Algorithm 1; an operation runs in the precision of the tile it
// writes, FP32 tiles promoted exactly into FP64 products, FP64 tiles rounded to nearest even
// into FP32 products), and factored left-looking, one task per lower tile (Algorithm 1's
// operations regrouped by output tile):
//   T(i, j):  A_ij <- C(s_i, s_j; theta)                    (eq. (1), generated in place)
//             A_ij <- A_ij - sum_{k<j} L_ik L_jk^T          (the dsyrk / dgemm / sgemm updates;
//                                                            FP32 tiles accumulate the product
//                                                            from zero and subtract it once)
//             i == j:  r_j = z_j - sum_{k<j} L_jk y_k, then dpotrf of A_jj fused with L_jj^-1,
//                      y_j = L_jj^-1 r_j and the logdet / quadratic-form parts;
//                      the last diagonal tile also reduces the parts to ell(theta);
//             i >  j:  L_ij = A_ij L_jj^-T                  (dtrsm / strsm through the explicit
//                                                            inverse, rounded for the FP32 tier)
// T(i, j) needs T(i, k) and T(j, k) for k < j, and T(j, j) when i > j.  The tasks of all
// problems sit in one array in an order where every task comes after the tasks it needs
// (column by column; in a column the diagonal tiles of all problems first).  Workgroups take
// tasks in that order from an atomic counter and wait for what a task needs on per-tile done
// flags (device-scope release / acquire), so the oldest unfinished task never waits and the
// queue always drains.  A wait is bounded: past the limit the workgroup raises an abort flag,
// every workgroup then skips its remaining tasks, and the host reports a device error.
#include "matern_dev.h"
#include "morton_dev.h"
#include "potrf_dev.h"

#include <algorithm>

namespace mpgeo {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kQThreads = 256;          // 4 waves, each a 64 x 64 quarter of the tile
constexpr int kQTile = kQueueTile;      // 128
constexpr int kQKc = 16;                // K chunk staged through LDS
constexpr int kQLd = kQTile + 16;       // padded LDS row
constexpr int kOrderThreads = 1024;
constexpr double kQLog2Pi = 1.8378770664093454836;

// Done flag of a task: wait (one thread) until set, the abort flag is raised, or the limit.
__device__ bool wait_done(const int *flag, int *abort_flag, int limit) {
    for (int s = 0;; ++s) {
        if (__hip_atomic_load(flag, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0) return true;
        if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return false;
        if (s >= limit) {
            __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(8);
    }
}

// One workgroup per problem: Morton keys of its sites, bitonic sort in LDS (keys
// (key << 32) | index, so ties keep input order), then the ordered sites and the ordered,
// zero-padded data vector.  order == 0 keeps the input order.
__global__ __launch_bounds__(kOrderThreads) void batch_order_kernel(const BatchInst *insts,
                                                                    const double *locs_in,
                                                                    const double *z_in, double *locs,
                                                                    double *zpad, int order, int lonlat) {
    extern __shared__ uint64_t okeys[];
    const BatchInst in = insts[blockIdx.x];
    const int n = (int)in.n;
    int n2 = 2;
    while (n2 < n) n2 *= 2;
    const int tid = threadIdx.x;
    const double *src_l = locs_in + 2 * in.in0;
    for (int e = tid; e < n2; e += kOrderThreads) {
        uint64_t key = ~0ull;
        if (e < n) {
            const uint32_t k = order ? morton_key(src_l[2 * e], src_l[2 * e + 1], lonlat) : 0u;
            key = ((uint64_t)k << 32) | (uint64_t)e;
        }
        okeys[e] = key;
    }
    __syncthreads();
    for (int size = 2; size <= n2; size *= 2)
        for (int stride = size / 2; stride > 0; stride /= 2) {
            for (int t = tid; t < n2 / 2; t += kOrderThreads) {
                const int lo = (t / stride) * (2 * stride) + (t % stride);
                const int hi = lo + stride;
                const bool ascending = (lo & size) == 0;
                const uint64_t a = okeys[lo], b = okeys[hi];
                if ((a > b) == ascending) {
                    okeys[lo] = b;
                    okeys[hi] = a;
                }
            }
            __syncthreads();
        }
    const int pad = in.p * kQTile;
    for (int e = tid; e < pad; e += kOrderThreads) {
        if (e < n) {
            const int src = (int)(okeys[e] & 0xFFFFFFFFull);
            locs[2 * (in.in0 + e)] = src_l[2 * src];
            locs[2 * (in.in0 + e) + 1] = src_l[2 * src + 1];
            zpad[in.vec0 + e] = z_in[in.in0 + src];
        } else {
            zpad[in.vec0 + e] = 0.0;
        }
    }
}

// Operand tile of one pair of a tile product: column-major 128 x 128, FP64 or FP32.
struct QSrc {
    const void *p;
    bool f64;
};

// acc (+)= sum over pairs q < npairs of R_q Q_q^T (R_q = src_r(q) supplies the output rows,
// Q_q = src_q(q) the columns), in FP64: with MIXED, FP32 operand tiles are promoted exactly
// (without, every operand is an FP64 tile).  The Q operand is negated when neg.  K runs through
// LDS in chunks of kQKc, double-buffered, the next chunk prefetched into registers.  Ends with a
// barrier (the LDS may be reused).
template <bool MIXED, class SR, class SQ>
__device__ void queue_gemm(f64x4 (&acc)[4][4], SR src_r, SQ src_q, int npairs, bool neg,
                           double (*ldsq)[kQKc * kQLd], double (*ldsr)[kQKc * kQLd]) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    typedef float f2 __attribute__((ext_vector_type(2)));
    constexpr int cpp = kQTile / kQKc;                    // chunks per pair
    constexpr int NV = kQKc * kQTile / 2;                 // 2-element vectors per chunk and operand
    constexpr int VP = NV / kQThreads;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wrow = (wave & 1) * 64, wcol = (wave >> 1) * 64;
    const int lr = lane & 15, lg = lane >> 4;
    const int nchunks = npairs * cpp;
    d2 rq[VP], rr[VP];
    auto fetch = [&](const QSrc &src, int64_t e) -> d2 {
        if (!MIXED || src.f64) return *reinterpret_cast<const d2 *>(static_cast<const double *>(src.p) + e);
        const f2 v = *reinterpret_cast<const f2 *>(static_cast<const float *>(src.p) + e);
        return (d2){(double)v.x, (double)v.y};   // exact
    };
    auto load = [&](int c) {
        const QSrc sq = src_q(c / cpp), sr = src_r(c / cpp);
        const int64_t off = (int64_t)((c % cpp) * kQKc) * kQTile;
#pragma unroll
        for (int v = 0; v < VP; ++v) {
            const int idx = v * kQThreads + tid;
            const int t = idx / (kQTile / 2), cv = idx % (kQTile / 2);
            rq[v] = fetch(sq, off + (int64_t)t * kQTile + 2 * cv);
            rr[v] = fetch(sr, off + (int64_t)t * kQTile + 2 * cv);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int v = 0; v < VP; ++v) {
            const int idx = v * kQThreads + tid;
            const int t = idx / (kQTile / 2), cv = idx % (kQTile / 2);
            *reinterpret_cast<d2 *>(&ldsq[buf][t * kQLd + 2 * cv]) = rq[v];
            *reinterpret_cast<d2 *>(&ldsr[buf][t * kQLd + 2 * cv]) = rr[v];
        }
    };
    if (nchunks > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunks) load(c + 1);
#pragma unroll
        for (int s = 0; s < kQKc / 4; ++s) {
            const int t = 4 * s + lg;
            double qa[4], rb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                qa[a] = ldsq[buf][t * kQLd + wcol + a * 16 + lr];
                if (neg) qa[a] = -qa[a];
            }
#pragma unroll
            for (int b = 0; b < 4; ++b) rb[b] = ldsr[buf][t * kQLd + wrow + b * 16 + lr];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[a], rb[b], acc[a][b], 0, 0, 0);
        }
        if (c + 1 < nchunks) store(buf ^ 1);
        __syncthreads();
    }
}

// The same product in FP32 for the FP32 tier (v_mfma_f32_16x16x4_f32): FP64 operand tiles
// are rounded to FP32 (nearest even) as they are staged, and K runs in chunks of kQKc32
// through the same LDS.  acc (+)= sum R_q Q_q^T.
constexpr int kQKc32 = 2 * kQKc;
template <class SR, class SQ>
__device__ void queue_gemm32(f32x4 (&acc)[4][4], SR src_r, SQ src_q, int npairs, float (*ldsq)[kQKc32 * kQLd],
                             float (*ldsr)[kQKc32 * kQLd]) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr int cpp = kQTile / kQKc32;
    constexpr int NV = kQKc32 * kQTile / 4;               // 4-element vectors per chunk and operand
    constexpr int VP = NV / kQThreads;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wrow = (wave & 1) * 64, wcol = (wave >> 1) * 64;
    const int lr = lane & 15, lg = lane >> 4;
    const int nchunks = npairs * cpp;
    f4 rq[VP], rr[VP];
    auto fetch = [&](const QSrc &src, int64_t e) -> f4 {
        if (!src.f64) return *reinterpret_cast<const f4 *>(static_cast<const float *>(src.p) + e);
        const double *d = static_cast<const double *>(src.p) + e;
        const d2 lo = *reinterpret_cast<const d2 *>(d), hi = *reinterpret_cast<const d2 *>(d + 2);
        return (f4){(float)lo.x, (float)lo.y, (float)hi.x, (float)hi.y};   // round to nearest even
    };
    auto load = [&](int c) {
        const QSrc sq = src_q(c / cpp), sr = src_r(c / cpp);
        const int64_t off = (int64_t)((c % cpp) * kQKc32) * kQTile;
#pragma unroll
        for (int v = 0; v < VP; ++v) {
            const int idx = v * kQThreads + tid;
            const int t = idx / (kQTile / 4), cv = idx % (kQTile / 4);
            rq[v] = fetch(sq, off + (int64_t)t * kQTile + 4 * cv);
            rr[v] = fetch(sr, off + (int64_t)t * kQTile + 4 * cv);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int v = 0; v < VP; ++v) {
            const int idx = v * kQThreads + tid;
            const int t = idx / (kQTile / 4), cv = idx % (kQTile / 4);
            *reinterpret_cast<f4 *>(&ldsq[buf][t * kQLd + 4 * cv]) = rq[v];
            *reinterpret_cast<f4 *>(&ldsr[buf][t * kQLd + 4 * cv]) = rr[v];
        }
    };
    if (nchunks > 0) {
        load(0);
        store(0);
    }
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
        const int buf = c & 1;
        if (c + 1 < nchunks) load(c + 1);
#pragma unroll
        for (int s = 0; s < kQKc32 / 4; ++s) {
            const int t = 4 * s + lg;
            float qa[4], rb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) qa[a] = ldsq[buf][t * kQLd + wcol + a * 16 + lr];
#pragma unroll
            for (int b = 0; b < 4; ++b) rb[b] = ldsr[buf][t * kQLd + wrow + b * 16 + lr];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(qa[a], rb[b], acc[a][b], 0, 0, 0);
        }
        if (c + 1 < nchunks) store(buf ^ 1);
        __syncthreads();
    }
}

// acc register q of lane (16 g + r) in block (a, b): row wrow + 16 b + r, column
// wcol + 16 a + g + 4 q (the f64 MFMA's layout)
__device__ inline void acc_store(const f64x4 (&acc)[4][4], double *T) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wrow = (wave & 1) * 64, wcol = (wave >> 1) * 64;
    const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                T[(wrow + b * 16 + lr) + (int64_t)(wcol + a * 16 + lg + 4 * q) * kQTile] = acc[a][b][q];
}

// FP32 results (the f32 MFMA's layout: column wcol + 16 a + 4 g + q): T = base - acc when
// subtract (base read from T itself), else T = acc.
__device__ inline void acc32_store(const f32x4 (&acc)[4][4], float *T, bool subtract) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wrow = (wave & 1) * 64, wcol = (wave >> 1) * 64;
    const int lr = lane & 15, lg = lane >> 4;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float *e = T + (wrow + b * 16 + lr) + (int64_t)(wcol + a * 16 + 4 * lg + q) * kQTile;
                *e = subtract ? *e - acc[a][b][q] : acc[a][b][q];
            }
}

// The diagonal-tile factorization and the covariance generation run out of line: their
// registers are not live together with the accumulators of the tile products.
__device__ __attribute__((noinline)) void queue_potrf(PotrfArgs pa) { potrf_tile_body<kQThreads>(pa); }

// Covariance block of tile (i, j), eq. (1) evaluated in FP64 and stored in the tile's
// precision (FP32 tiles rounded to nearest even).
template <typename T>
__device__ __attribute__((noinline)) void queue_covariance(T *tile, const double *locs, int64_t n, int i, int j,
                                                           MaternParams mp) {
    for (int e = threadIdx.x; e < kQTile * kQTile; e += kQThreads) {
        const int row = e % kQTile, col = e / kQTile;
        const int64_t gr = (int64_t)i * kQTile + row, gc = (int64_t)j * kQTile + col;
        double v;
        if (gr >= n || gc >= n) {
            v = (i == j && row == col) ? 1.0 : 0.0;   // identity padding
        } else if (gr == gc) {
            v = mp.sigma2;
        } else {
            const double xr = locs[2 * gr], yr = locs[2 * gr + 1];
            const double xc = locs[2 * gc], yc = locs[2 * gc + 1];
            double r;
            if (mp.gcd) {
                const double pr = yr * kDegToRad, pc = yc * kDegToRad;
                r = haversine(xc - xr, pr, cos(pr), pc, cos(pc));
            } else {
                const double dx = xr - xc, dy = yr - yc;
                r = sqrt(dx * dx + dy * dy);
            }
            v = matern_cov(r, mp);
        }
        tile[e] = (T)v;
    }
}

// A_ij -= sum_{k<j} L_ik L_jk^T on the FP64 tile Tij (accumulators started from the tile).
// MIXED: some operand tiles are FP32 (promoted exactly).
template <bool MIXED>
__device__ inline void queue_update64(double *Tij, float *tiles, int band, int i, int j,
                                      double (*ldsq)[kQKc * kQLd], double (*ldsr)[kQKc * kQLd]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wrow = (wave & 1) * 64, wcol = (wave >> 1) * 64;
    const int lr = lane & 15, lg = lane >> 4;
    auto tile_src = [&](int a, int b) { return QSrc{tiles + queue_tile_units(a, b, band), a - b <= band}; };
    f64x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                acc[a][b][q] = Tij[(wrow + b * 16 + lr) + (int64_t)(wcol + a * 16 + lg + 4 * q) * kQTile];
    queue_gemm<MIXED>(acc, [&](int k) { return tile_src(i, k); }, [&](int k) { return tile_src(j, k); }, j, true,
                      ldsq, ldsr);
    acc_store(acc, Tij);
}
__device__ __attribute__((noinline)) void queue_update64_mixed(double *Tij, float *tiles, int band, int i, int j,
                                                               double (*ldsq)[kQKc * kQLd],
                                                               double (*ldsr)[kQKc * kQLd]) {
    queue_update64<true>(Tij, tiles, band, i, j, ldsq, ldsr);
}

// A task of the FP32 tier: covariance rounded to FP32, A_ij -= sum_k L_ik L_jk^T in FP32 (the
// product accumulated from zero and subtracted once), then L_ij = A_ij L_jj^-T in FP32 with the
// rounded diagonal inverse.  Out of line: its accumulators are not live with the FP64 path's.
__device__ __attribute__((noinline)) void queue_task32(float *tiles, int band, int i, int j, const double *linv_jj,
                                                       const double *locs, int64_t n, MaternParams mp,
                                                       float (*ldsq32)[kQKc32 * kQLd],
                                                       float (*ldsr32)[kQKc32 * kQLd]) {
    auto tile_src = [&](int a, int b) { return QSrc{tiles + queue_tile_units(a, b, band), a - b <= band}; };
    float *Tij = tiles + queue_tile_units(i, j, band);
    queue_covariance<float>(Tij, locs, n, i, j, mp);
    __syncthreads();
    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
    queue_gemm32(acc, [&](int k) { return tile_src(i, k); }, [&](int k) { return tile_src(j, k); }, j, ldsq32,
                 ldsr32);
    acc32_store(acc, Tij, true);
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
    queue_gemm32(acc, [&](int) { return QSrc{Tij, false}; }, [&](int) { return QSrc{linv_jj, true}; }, 1, ldsq32,
                 ldsr32);
    acc32_store(acc, Tij, false);
}

__global__ __launch_bounds__(kQThreads) void batch_queue_kernel(QueueArgs g) {
    __shared__ double ldsq[2][kQKc * kQLd];
    __shared__ double ldsr[2][kQKc * kQLd];
    __shared__ int s_task, s_skip, s_ok;
    // the FP32 products stage their chunks in the same LDS
    static_assert(sizeof(float) * kQKc32 == sizeof(double) * kQKc, "FP32 chunks reuse the FP64 buffers");
    float (*ldsq32)[kQKc32 * kQLd] = reinterpret_cast<float (*)[kQKc32 * kQLd]>(ldsq);
    float (*ldsr32)[kQKc32 * kQLd] = reinterpret_cast<float (*)[kQKc32 * kQLd]>(ldsr);
    constexpr int64_t te = (int64_t)kQTile * kQTile;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wrow = (wave & 1) * 64, wcol = (wave >> 1) * 64;
    const int lr = lane & 15, lg = lane >> 4;

    for (;;) {
        // one thread takes the next task and reads the abort flag; the workgroup follows it
        if (tid == 0) {
            s_task = (int)atomicAdd(g.head, 1u);
            s_skip = __hip_atomic_load(g.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        const int task = s_task, skip = s_skip;
        __syncthreads();
        if (task >= g.ntasks) break;
        if (skip) continue;   // drain the queue after an abort
        const BatchTask tk = g.tasks[task];
        const BatchInst &in = g.insts[tk.inst];
        const int i = tk.i, j = tk.j;
        const int band = in.band;
        int *flags = g.flags + in.flag0;
        // ---- what the task needs: tiles (i, k) and (j, k) for k < j, and (j, j) -------------
        if (tid == 0) {
            bool ok = true;
            for (int k = 0; k < j && ok; ++k)
                ok = wait_done(flags + tri_index(i, k), g.abort_flag, g.spin_limit) &&
                     wait_done(flags + tri_index(j, k), g.abort_flag, g.spin_limit);
            if (ok && i > j) ok = wait_done(flags + tri_index(j, j), g.abort_flag, g.spin_limit);
            s_ok = ok ? 1 : 0;
        }
        __syncthreads();
        if (!s_ok) continue;

        const int64_t n = in.n;
        const double *locs = g.locs + 2 * in.in0;
        float *tiles = g.tiles + in.tile0;
        auto tile_src = [&](int a, int b) {
            return QSrc{tiles + queue_tile_units(a, b, band), a - b <= band};
        };
        const double *linv_jj = g.linv + (in.linv0 + j) * te;
        if (i - j > band) {
            queue_task32(tiles, band, i, j, linv_jj, locs, n, in.mp, ldsq32, ldsr32);
        } else {
            // ---- FP64 tier: covariance block, written to the tile (column-major, coalesced) --
            double *Tij = reinterpret_cast<double *>(tiles + queue_tile_units(i, j, band));
            queue_covariance<double>(Tij, locs, n, i, j, in.mp);
            __syncthreads();
            // ---- left-looking update: A_ij -= sum_{k<j} L_ik L_jk^T (FP32 tiles promoted) --------
            if (i <= band) queue_update64<false>(Tij, tiles, band, i, j, ldsq, ldsr);   // FP64 operands only
            else queue_update64_mixed(Tij, tiles, band, i, j, ldsq, ldsr);
            __syncthreads();

            if (i == j) {
                // ---- forward-solve block: r_j = z_j - sum_{k<j} L_jk y_k ----------------------------
                double *rj = g.r + in.vec0 + (int64_t)j * kQTile;
                const double *ybase = g.y + in.vec0;
                if (tid < kQTile) {
                    double s = g.z[in.vec0 + (int64_t)j * kQTile + tid];
                    for (int k = 0; k < j; ++k) {
                        const QSrc L = tile_src(j, k);
                        const double *yk = ybase + (int64_t)k * kQTile;
                        if (L.f64) {
                            const double *Lp = static_cast<const double *>(L.p) + tid;
                            for (int t = 0; t < kQTile; ++t) s -= Lp[(int64_t)t * kQTile] * yk[t];
                        } else {
                            const float *Lp = static_cast<const float *>(L.p) + tid;
                            for (int t = 0; t < kQTile; ++t) s -= (double)Lp[(int64_t)t * kQTile] * yk[t];
                        }
                    }
                    rj[tid] = s;
                }
                __syncthreads();
                PotrfArgs pa;
                pa.a = Tij;
                pa.linv = g.linv + (in.linv0 + j) * te;
                pa.linv32 = nullptr;
                pa.r = rj;
                pa.y = g.y + in.vec0 + (int64_t)j * kQTile;
                pa.logdet_part = g.parts + in.part0 + j;
                pa.quad_part = g.parts + in.part0 + in.p + j;
                pa.info = g.info + tk.inst;
                pa.col_base = (int64_t)j * kQTile;
                pa.nb = kQTile;
                pa.nbp = kQTile;
                queue_potrf(pa);
                __syncthreads();
                if (j == in.p - 1 && tid == 0) {   // every part is visible (see the flags above)
                    double logdet = 0.0, quad = 0.0;
                    for (int k = 0; k < in.p; ++k) {
                        logdet += g.parts[in.part0 + k];
                        quad += g.parts[in.part0 + in.p + k];
                    }
                    const double dn = (double)n;
                    double *res = g.result + 3 * (int64_t)tk.inst;
                    res[0] = g.profile ? -0.5 * dn * (kQLog2Pi + 1.0) - 0.5 * dn * log(quad / dn) - 0.5 * logdet
                                       : -0.5 * dn * kQLog2Pi - 0.5 * logdet - 0.5 * quad;
                    res[1] = logdet;
                    res[2] = quad;
                }
            } else {
                // ---- L_ij = A_ij L_jj^-T ------------------------------------------------------------
                f64x4 acc[4][4];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) acc[a][b] = (f64x4){0.0, 0.0, 0.0, 0.0};
                queue_gemm<false>(acc, [&](int) { return QSrc{Tij, true}; }, [&](int) { return QSrc{linv_jj, true}; },
                                  1, false, ldsq, ldsr);
                acc_store(acc, Tij);
            }
        }
        // ---- done: every thread's stores made visible to the device, then the flag -----------
        __threadfence();
        __syncthreads();
        if (tid == 0) __hip_atomic_store(flags + tri_index(i, j), 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void fill_u32_kernel(uint32_t *p, uint32_t value, size_t count) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x)
        p[e] = value;
}

}  // namespace

void launch_fill_u32(uint32_t *p, uint32_t value, size_t count, hipStream_t stream) {
    if (count == 0) return;
    const unsigned blocks = (unsigned)std::min<size_t>((count + 255) / 256, 1024);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(blocks), dim3(256), 0, stream, p, value, count);
}

void launch_batch_order(const BatchInst *insts, int64_t count, int max_n, const double *locs_in,
                        const double *z_in, double *locs, double *zpad, bool order, bool lonlat,
                        hipStream_t stream) {
    if (count <= 0) return;
    int n2 = 2;
    while (n2 < max_n) n2 *= 2;
    hipLaunchKernelGGL(batch_order_kernel, dim3((unsigned)count), dim3(kOrderThreads),
                       (size_t)n2 * sizeof(uint64_t), stream, insts, locs_in, z_in, locs, zpad,
                       order ? 1 : 0, lonlat ? 1 : 0);
}

void launch_batch_queue(const QueueArgs &args, int workgroups, hipStream_t stream) {
    if (args.ntasks <= 0 || workgroups <= 0) return;
    hipLaunchKernelGGL(batch_queue_kernel, dim3((unsigned)workgroups), dim3(kQThreads), 0, stream, args);
}

}  // namespace mpgeo
