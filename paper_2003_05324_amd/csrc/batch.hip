// Batched evaluation of eq. (2) for many independent problems as one persistent kernel over a
// device task queue (many small likelihoods, Section VIII; the tile size question of
// Section V-C at the scale of a batch).
//
// Each problem is cut into 128 x 128 FP64 tiles and factored left-looking, one task per lower
// tile (Algorithm 1's operations regrouped by output tile):
//   T(i, j):  A_ij <- C(s_i, s_j; theta)                    (eq. (1), generated in place)
//             A_ij <- A_ij - sum_{k<j} L_ik L_jk^T          (the dsyrk / dgemm updates)
//             i == j:  r_j = z_j - sum_{k<j} L_jk y_k, then dpotrf of A_jj fused with L_jj^-1,
//                      y_j = L_jj^-1 r_j and the logdet / quadratic-form parts;
//                      the last diagonal tile also reduces the parts to ell(theta);
//             i >  j:  L_ij = A_ij L_jj^-T                  (dtrsm through the explicit inverse)
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

namespace mpgeo {

namespace {

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

// acc (+)= sum over pairs q < npairs of R_q Q_q^T, R_q = R0 + q * nbp^2 and Q_q likewise
// (column-major 128 x 128 tiles: R supplies the output rows, Q the output columns); the Q
// operand is negated when neg.  K runs through LDS in chunks of kQKc, double-buffered, the next
// chunk prefetched into registers.  Ends with a barrier (the LDS may be reused).
__device__ void queue_gemm(f64x4 (&acc)[4][4], const double *R0, const double *Q0, int npairs, bool neg,
                           double (*ldsq)[kQKc * kQLd], double (*ldsr)[kQKc * kQLd]) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    constexpr int64_t te = (int64_t)kQTile * kQTile;
    constexpr int cpp = kQTile / kQKc;                    // chunks per pair
    constexpr int NV = kQKc * kQTile / 2;                 // 16-byte vectors per chunk and operand
    constexpr int VP = NV / kQThreads;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wrow = (wave & 1) * 64, wcol = (wave >> 1) * 64;
    const int lr = lane & 15, lg = lane >> 4;
    const int nchunks = npairs * cpp;
    d2 rq[VP], rr[VP];
    auto load = [&](int c) {
        const int64_t off = (int64_t)(c / cpp) * te + (int64_t)((c % cpp) * kQKc) * kQTile;
#pragma unroll
        for (int v = 0; v < VP; ++v) {
            const int idx = v * kQThreads + tid;
            const int t = idx / (kQTile / 2), cv = idx % (kQTile / 2);
            rq[v] = *reinterpret_cast<const d2 *>(Q0 + off + (int64_t)t * kQTile + 2 * cv);
            rr[v] = *reinterpret_cast<const d2 *>(R0 + off + (int64_t)t * kQTile + 2 * cv);
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

// The diagonal-tile factorization and the covariance generation run out of line: their
// registers are not live together with the accumulators of the tile products.
__device__ __attribute__((noinline)) void queue_potrf(PotrfArgs pa) { potrf_tile_body<kQThreads>(pa); }

__device__ __attribute__((noinline)) void queue_covariance(double *T, const double *locs, int64_t n, int i,
                                                           int j, MaternParams mp) {
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
        T[e] = v;
    }
}

__global__ __launch_bounds__(kQThreads) void batch_queue_kernel(QueueArgs g) {
    __shared__ double ldsq[2][kQKc * kQLd];
    __shared__ double ldsr[2][kQKc * kQLd];
    __shared__ int s_task, s_skip, s_ok;
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

        // ---- covariance block, written to the tile (column-major, coalesced) ----------------
        const int64_t n = in.n;
        const double *locs = g.locs + 2 * in.in0;
        double *tiles = g.tiles + in.tile0 * te;
        double *Tij = tiles + tri_index(i, j) * te;
        queue_covariance(Tij, locs, n, i, j, in.mp);
        __syncthreads();
        f64x4 acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    acc[a][b][q] = Tij[(wrow + b * 16 + lr) + (int64_t)(wcol + a * 16 + lg + 4 * q) * kQTile];
        // ---- left-looking update: A_ij -= sum_{k<j} L_ik L_jk^T --------------------------------
        queue_gemm(acc, tiles + tri_index(i, 0) * te, tiles + tri_index(j, 0) * te, j, true, ldsq, ldsr);
        acc_store(acc, Tij);
        __syncthreads();

        if (i == j) {
            // ---- forward-solve block: r_j = z_j - sum_{k<j} L_jk y_k ----------------------------
            double *rj = g.r + in.vec0 + (int64_t)j * kQTile;
            const double *ybase = g.y + in.vec0;
            if (tid < kQTile) {
                double s = g.z[in.vec0 + (int64_t)j * kQTile + tid];
                for (int k = 0; k < j; ++k) {
                    const double *L = tiles + tri_index(j, k) * te + tid;
                    const double *yk = ybase + (int64_t)k * kQTile;
                    for (int t = 0; t < kQTile; ++t) s -= L[(int64_t)t * kQTile] * yk[t];
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
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = (f64x4){0.0, 0.0, 0.0, 0.0};
            queue_gemm(acc, Tij, g.linv + (in.linv0 + j) * te, 1, false, ldsq, ldsr);
            acc_store(acc, Tij);
        }
        // ---- done: every thread's stores made visible to the device, then the flag -----------
        __threadfence();
        __syncthreads();
        if (tid == 0) __hip_atomic_store(flags + tri_index(i, j), 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace

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
