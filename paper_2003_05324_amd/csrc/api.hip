// C-ABI entry points and the step-ordered tile engine of the mixed-precision
// log-likelihood (eq. (2) with the tile Cholesky of Algorithm 1).
//
// Per evaluation, on the context stream:
//   order (Z-order keys + sort)  ->  Matérn tiles in their tier precision
//   for k = 0 .. p-1:
//     POTRF(k) + L_kk^-1 + y_k                       (FP64, one workgroup)
//     panel X_i = A_ik L_kk^-T: FP64 band tiles, FP32 far tiles (matrix cores)
//     r_i -= X_i y_k and X_i back into its storage tile
//     trailing A_ij -= X_i X_j^T: FP64 launch for band tiles, FP32 launch for far tiles
//   reduce logdet and quad, assemble eq. (2)
// Tiles are kept resident in HBM; no host transfer happens inside the loop.
#include "common.h"
#include "../../include/mpgeo.h"
#include "tune_policy.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <thread>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace mpgeo;

namespace {

int status_from(hipError_t e) {
    if (e == hipSuccess) return MPGEO_OK;
    return e == hipErrorOutOfMemory ? MPGEO_E_NOMEM : MPGEO_E_DEVICE;
}

#define MPGEO_HIP(expr)                         \
    do {                                        \
        hipError_t _e = (expr);                 \
        if (_e != hipSuccess) {                 \
            (void)hipGetLastError();            \
            return status_from(_e);             \
        }                                       \
    } while (0)

#define MPGEO_TRY(expr)                         \
    do {                                        \
        int _s = (expr);                        \
        if (_s != MPGEO_OK) return _s;          \
    } while (0)

// Device buffer that only grows.  Growing frees the old block, so it first waits for every
// stream of the device: work already enqueued (another lane's evaluation, say) may still use it.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    int ensure(size_t b) {
        if (b <= bytes && ptr) return MPGEO_OK;
        if (ptr && hipDeviceSynchronize() != hipSuccess) (void)hipGetLastError();
        release();
        if (b == 0) return MPGEO_OK;
        hipError_t e = hipMalloc(&ptr, b);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            ptr = nullptr;
            bytes = 0;
            return MPGEO_E_NOMEM;
        }
        bytes = b;
        return MPGEO_OK;
    }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Tiles, precision tiers and per-step work lists for one (n, nb, band64, band32, band0).
struct Layout {
    int64_t n = 0;
    int nb = 0, nbp = 0, p = 0, band = -2;
    int edge = 0;                             // low tier (16-bit operands) iff i - j > edge
    int zband = 0;                            // zero tier (dropped tiles) iff i - j > zband
    int lowp = 0;                             // 0: none, 1: FP16, 2: BF16
    // precision map drawn from distances (dist64 > 0): the tier of each tile from the distance
    // between the bounding boxes of its two blocks of sites, instead of from i - j
    double dist64 = 0.0, dist32 = 0.0;
    int lowp_req = 0;                         // the plan's 16-bit format (distance map only)
    std::vector<signed char> tierv;           // per tri_index: 64, 32 or 16 (distance map only)
    std::vector<TileIJ> trsm64, trsm32;       // panel tiles per step by tier (distance map only)
    std::vector<int64_t> trsm64_b, trsm32_b;  // step k's section: [b[k], b[k+1])
    std::vector<int64_t> off;
    std::vector<TileIJ> all, list64, list32, list16;
    // per step k and tier (0: FP64, 1: FP32, 2: 16-bit operands): the list ranges of the bulk
    // update (tile columns j >= k+2) and of the lookahead column j = k+1, with their flops
    // The 16-bit tier is left-looking: bulk[2][k] is column k+2's 16-bit tiles, which take
    // panels 0 .. k in one pass (rows i > zband + k' skip the dropped panels k' < i - zband);
    // col[2][k] gives column k+1 its last panel k.  Tiles of later columns wait untouched.
    struct Range {
        int64_t b = 0, e = 0;
        double flops = 0.0;
        double panels = 0.0;   // bulk[2] only: 16-bit operand tiles read (rows i and row j)
    };
    std::vector<Range> bulk[3], col[3];
    // FP64 and FP32 bulk ranges end with column k+2's tiles: they start at next_b[q][k] and
    // take next_f[q][k] of the flops (the next lookahead column needs them first)
    std::vector<int64_t> next_b[2];
    std::vector<double> next_f[2];
    // bulk[2][k] indexes these: the 16-bit tiles step k's bulk pass updates and, per entry,
    // the first panel it takes (the pass takes panels first .. k)
    std::vector<TileIJ> bulk16;
    std::vector<int32_t> bulk16_k0;
    int wave16 = 0;                           // 16-bit bulk tiles that run at once (0: unknown)
    std::vector<char> needq;                  // panel k has a 16-bit copy (some later use)
    std::vector<double> trsm64_flops, trsm32_flops;
    int64_t n64 = 0, n32 = 0;                 // tiles per storage precision (FP32 holds tier 16)
    bool has_zero_tile = false;               // dropped tiles share one zero FP32 tile (index n32)

    bool same(int64_t n_, int nb_, int band_, int edge_, int zband_, int lowp_, double d64 = 0.0,
              double d32 = 0.0) const {
        return n == n_ && nb == nb_ && band == band_ && edge == edge_ && zband == zband_ &&
               lowp == lowp_ && dist64 == d64 && dist32 == d32;
    }
    bool distance_map() const { return !tierv.empty(); }
    // tier of tile (i, j): 64, 32, 16, or 0 for a dropped tile
    int tier(int i, int j) const {
        if (!tierv.empty()) return tierv[(size_t)tri_index(i, j)];
        const int d = i - j;
        return d > zband ? 0 : (d <= band ? 64 : (d <= edge ? 32 : 16));
    }
    static int slot(int t) { return t == 64 ? 0 : (t == 32 ? 1 : 2); }

    int64_t rows(int i) const { return std::min<int64_t>(nb, n - (int64_t)i * nb); }
    // panel tiles of step k that are not dropped: rows k+1 .. k+panel_count(k)
    int panel_count(int k) const { return std::max(0, std::min(p - 1 - k, zband)); }

    static int effective_zband(int64_t p_, int band0) { return (band0 < 0 || band0 > p_) ? (int)p_ : band0; }
    static int effective_band(int64_t p_, int band64, int band0 = -1) {
        const int b = (band64 < 0 || band64 > p_) ? (int)p_ : band64;
        return std::min(b, effective_zband(p_, band0));
    }
    static int effective_edge(int64_t p_, int band64, int band32, int band0 = -1) {
        const int b = effective_band(p_, band64, band0);
        const int e = (band32 < 0 || (int64_t)b + band32 > p_) ? (int)p_ : b + band32;
        return std::min(e, effective_zband(p_, band0));
    }

    // algorithmic flops of the update of tile (i, j) per unit of K (SYRK on the diagonal)
    double tile_flops(int i, int j) const {
        return (i == j) ? (double)rows(j) * (rows(j) + 1) : 2.0 * rows(i) * rows(j);
    }
    // ... and with panel k (K = rows(k))
    double update_flops(int i, int j, int k) const { return tile_flops(i, j) * rows(k); }

    // boxes: per tile row, {xmin, xmax, ymin, ymax} of its sites (distance map only)
    void build(int64_t n_, int nb_, int band64, int band32 = -1, int lowp_ = 0, int band0 = -1,
               const std::vector<double> *boxes = nullptr, double d64 = 0.0, double d32 = 0.0,
               int wave16_ = 0) {
        n = n_;
        wave16 = wave16_;
        nb = nb_;
        nbp = (nb + kTileQuantum - 1) / kTileQuantum * kTileQuantum;
        p = (int)((n + nb - 1) / nb);
        zband = effective_zband(p, band0);
        band = effective_band(p, band64, band0);
        edge = effective_edge(p, band64, band32, band0);
        lowp = (edge < std::min(zband, p - 1)) ? lowp_ : 0;
        dist64 = d64;
        dist32 = d32;
        lowp_req = lowp_;
        tierv.clear();
        trsm64.clear();
        trsm32.clear();
        trsm64_b.assign(p + 1, 0);
        trsm32_b.assign(p + 1, 0);
        if (boxes && d64 > 0.0) {
            // tile (i, j) is FP64 when its two blocks of sites come within d64 of each other (the
            // diagonal always), FP32 within d32 when a 16-bit tier is asked for, 16-bit beyond
            zband = p;
            band = 0;
            edge = p;
            lowp = 0;
            tierv.assign((size_t)p * (p + 1) / 2, 64);
            for (int i = 0; i < p; ++i)
                for (int j = 0; j < i; ++j) {
                    const double *a = boxes->data() + 4 * i, *b = boxes->data() + 4 * j;
                    const double dx = std::max(0.0, std::max(a[0] - b[1], b[0] - a[1]));
                    const double dy = std::max(0.0, std::max(a[2] - b[3], b[2] - a[3]));
                    const double d = std::sqrt(dx * dx + dy * dy);
                    const int t = d <= d64 ? 64 : ((lowp_ == 0 || d <= d32) ? 32 : 16);
                    tierv[(size_t)tri_index(i, j)] = (signed char)t;
                    if (t == 16) lowp = lowp_;
                }
            for (int k = 0; k < p; ++k) {
                for (int i = k + 1; i < p; ++i) (tier(i, k) == 64 ? trsm64 : trsm32).push_back({i, k});
                trsm64_b[k + 1] = (int64_t)trsm64.size();
                trsm32_b[k + 1] = (int64_t)trsm32.size();
            }
        }
        const int64_t nt = (int64_t)p * (p + 1) / 2;
        off.assign(nt, 0);
        all.clear();
        list64.clear();
        list32.clear();
        list16.clear();
        n64 = n32 = 0;
        const int64_t tile_elems = (int64_t)nbp * nbp;
        std::vector<int64_t> zero_tiles;
        for (int i = 0; i < p; ++i)
            for (int j = 0; j <= i; ++j) {
                const int t = tier(i, j);
                if (t == 0) {
                    zero_tiles.push_back(tri_index(i, j));
                    continue;
                }
                all.push_back({i, j});
                if (t == 64) off[tri_index(i, j)] = (n64++) * tile_elems;
                else off[tri_index(i, j)] = (n32++) * tile_elems;
            }
        has_zero_tile = !zero_tiles.empty();
        for (int64_t z : zero_tiles) off[z] = n32 * tile_elems;
        std::vector<TileIJ> *lists[3] = {&list64, &list32, &list16};
        for (int q = 0; q < 3; ++q) {
            bulk[q].assign(p, Range{});
            col[q].assign(p, Range{});
        }
        if (zband >= p) {
            // one list per tier: columns j = p-1 down to 1, rows ascending; the prefix with
            // j > k is exactly the trailing work of step k
            for (int j = p - 1; j >= 1; --j)
                for (int i = j; i < p; ++i) lists[slot(tier(i, j))]->push_back({i, j});
            std::vector<double> colf[3];
            std::vector<int64_t> cnt[3];
            for (int q = 0; q < 3; ++q) {
                colf[q].assign(p, 0.0);
                cnt[q].assign(p, 0);
            }
            for (int j = 1; j < p; ++j)
                for (int i = j; i < p; ++i) {
                    const int q = slot(tier(i, j));
                    colf[q][j] += tile_flops(i, j);
                    cnt[q][j]++;
                }
            for (int q = 0; q < 3; ++q) {
                std::vector<int64_t> pre(p + 1, 0);       // entries with j > k
                std::vector<double> suf(p + 1, 0.0);      // flops per unit K of columns > k
                for (int k = p - 1; k >= 0; --k) {
                    pre[k] = pre[k + 1] + (k + 1 < p ? cnt[q][k + 1] : 0);
                    suf[k] = suf[k + 1] + (k + 1 < p ? colf[q][k + 1] : 0.0);
                }
                for (int k = 0; k + 1 < p; ++k) {
                    const double rk = (double)rows(k);
                    bulk[q][k] = Range{0, pre[k + 1], suf[k + 1] * rk};
                    col[q][k] = Range{pre[k + 1], pre[k], colf[q][k + 1] * rk};
                }
            }
        } else {
            // dropped tiles: per step, only tiles with k < j <= i <= k + zband change, so each
            // step gets its own list section: the lookahead column first, then the bulk
            // (columns descending, rows ascending)
            for (int k = 0; k + 1 < p; ++k) {
                const int last = std::min(p - 1, k + zband);
                for (int q = 0; q < 3; ++q) {
                    col[q][k].b = (int64_t)lists[q]->size();
                    for (int i = k + 1; i <= last; ++i) {
                        const int t = tier(i, k + 1);
                        if (slot(t) != q || t == 0) continue;
                        lists[q]->push_back({i, k + 1});
                        col[q][k].flops += update_flops(i, k + 1, k);
                    }
                    col[q][k].e = bulk[q][k].b = (int64_t)lists[q]->size();
                    if (q == 2) {   // the 16-bit tier's bulk is set below (left-looking)
                        bulk[q][k].e = bulk[q][k].b;
                        continue;
                    }
                    for (int j = last; j >= k + 2; --j)
                        for (int i = j; i <= last; ++i) {
                            const int t = tier(i, j);
                            if (slot(t) != q || t == 0) continue;
                            lists[q]->push_back({i, j});
                            bulk[q][k].flops += update_flops(i, j, k);
                        }
                    bulk[q][k].e = (int64_t)lists[q]->size();
                }
            }
        }
        // left-looking 16-bit tier: step k's bulk pass brings column k+2 up to panel k (panels
        // [max(0, i - zband), k]).  All of its workgroups take equally long (k + 1 panels), so a
        // launch costs whole waves of them; when the last wave would run part-empty it is
        // filled with tiles of column k+3, which take panels 0 .. k now and only panel k+1 at
        // the next step (the tiles of one column then come first, taking one panel each).
        // Every tile still takes its panels one at a time in ascending order.
        bulk16.clear();
        bulk16_k0.clear();
        needq.assign(p, 0);
        std::vector<int> kmin_at(p, p);   // first panel any tile of step k's bulk takes
        std::vector<std::vector<int>> rows16(p), next16(p);   // per column: rows, next panel
        for (int64_t t = 0; t < (int64_t)list16.size(); ++t) rows16[list16[(size_t)t].j].push_back(list16[(size_t)t].i);
        for (int j = 0; j < p; ++j) {
            std::sort(rows16[j].begin(), rows16[j].end());
            next16[j].assign(rows16[j].size(), 0);
        }
        const bool fill = wave16 > 0 && zband >= p;
        for (int k = 0; k + 1 < p; ++k) {
            Range agg;
            agg.b = agg.e = (int64_t)bulk16.size();
            const int c = k + 2;
            if (c < p) {
                int64_t longs = 0;
                for (int pass = 0; pass < 2; ++pass)   // tiles begun at an earlier step first
                    for (size_t a = 0; a < rows16[c].size(); ++a) {
                        const int k0 = next16[c][a];
                        if ((pass == 0) != (k0 > 0)) continue;
                        bulk16.push_back({rows16[c][a], c});
                        bulk16_k0.push_back(k0);
                        next16[c][a] = k + 1;
                        if (k0 == 0) ++longs;
                    }
                if (fill && c + 1 < p && longs % wave16 != 0) {
                    const int64_t want = wave16 - longs % wave16;
                    for (size_t a = 0; a < rows16[c + 1].size() && (int64_t)a < want; ++a) {
                        bulk16.push_back({rows16[c + 1][a], c + 1});
                        bulk16_k0.push_back(0);
                        next16[c + 1][a] = k + 1;
                    }
                }
                agg.e = (int64_t)bulk16.size();
                int kmin = k + 1, kmin_col[2] = {k + 1, k + 1};
                for (int64_t t = agg.b; t < agg.e; ++t) {
                    const TileIJ ij = bulk16[(size_t)t];
                    const int k0 = std::max(bulk16_k0[(size_t)t], ij.i - zband);
                    for (int kk = k0; kk <= k; ++kk) agg.flops += update_flops(ij.i, ij.j, kk);
                    agg.panels += std::max(0, k + 1 - k0);
                    kmin = std::min(kmin, k0);
                    int &km = kmin_col[ij.j - c];
                    km = std::min(km, k0);
                }
                for (int q = 0; q < 2; ++q) agg.panels += std::max(0, k + 1 - kmin_col[q]);   // rows j
                if (agg.e > agg.b) kmin_at[k] = kmin;
            }
            bulk[2][k] = agg;
        }
        // panel k is an operand of the column update of step k or of a bulk pass of a later step
        int suffix_min = p;
        for (int k = p - 2; k >= 0; --k) {
            suffix_min = std::min(suffix_min, kmin_at[k]);
            needq[k] = lowp && (col[2][k].e > col[2][k].b || suffix_min <= k);
        }
        for (int q = 0; q < 2; ++q) {
            const std::vector<TileIJ> &lst = *lists[q];
            next_b[q].assign(p, 0);
            next_f[q].assign(p, 0.0);
            for (int k = 0; k + 1 < p; ++k) {
                int64_t a = bulk[q][k].e;
                while (a > bulk[q][k].b && lst[(size_t)a - 1].j == k + 2) --a;
                next_b[q][k] = a;
                for (int64_t t = a; t < bulk[q][k].e; ++t)
                    next_f[q][k] += update_flops(lst[(size_t)t].i, lst[(size_t)t].j, k);
            }
        }
        trsm64_flops.assign(p, 0.0);
        trsm32_flops.assign(p, 0.0);
        for (int k = 0; k < p; ++k)
            for (int i = k + 1; i <= k + panel_count(k); ++i) {
                const double f = (double)rows(i) * rows(k) * rows(k);   // triangular solve
                if (tier(i, k) == 64) trsm64_flops[k] += f;
                else trsm32_flops[k] += f;
            }
    }
    // panel k is quantised to the 16-bit factor copy
    bool lowp_step(int k) const { return lowp && k + 1 < p && needq[k]; }
};

enum StatClass {
    kStatCovgen, kStatOrder, kStatPotrf, kStatTrsm64, kStatTrsm32, kStatPanel, kStatUpdate64,
    kStatUpdate32, kStatFinal, kStatQuant, kStatUpdate16, kStatUpdate16Col, kStatCount
};
const char *kStatNames[kStatCount] = {"covgen", "morton_order", "potrf_tile", "trsm_fp64",
                                      "trsm_fp32", "panel_solve", "update_fp64", "update_fp32",
                                      "finalize", "quantize", "update_lowp", "update_lowp_col"};

// A class's tuned FP64 band (-1: all-FP64) and the largest error of its probes at that band,
// relative to the size of eq. (2)'s terms.
struct TunedBand {
    int band;
    double err;
};

}  // namespace

struct mpgeo_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t side = nullptr;            // lookahead stream (next panel's critical path)
    // Bulk trailing updates run on a stream whose CU mask leaves `reserved_cus` compute units
    // to the lookahead stream alone: the one-workgroup POTRF and the small FP64 TRSM of the
    // critical path then never wait for the wide update kernels to drain.  nullptr: the bulk
    // runs on `stream` with every CU.
    hipStream_t bulk = nullptr;
    // column k+2's FP64 and FP32 updates of each step, beside the rest of the bulk (nullptr:
    // on the bulk stream)
    hipStream_t next = nullptr;
    int reserved_cus = 0;
    int cus = 0;                           // compute units of the device
    size_t hbm_budget = 0;                 // tile bytes one evaluation may use (0: no cap)
    std::vector<hipEvent_t> sync_events;   // dependency events between the streams

    // at least `count` timing-free events for stream dependencies
    bool ensure_sync_events(size_t count) {
        while (sync_events.size() < count) {
            hipEvent_t e = nullptr;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                return false;
            }
            sync_events.push_back(e);
        }
        return true;
    }
    struct Pending {
        int cls;
        hipEvent_t a, b;
        double flops, bytes;
    };
    std::vector<Pending> pending;
    std::vector<hipEvent_t> spare;
    mpgeo_kernel_stat stats[kStatCount];
    bool timing = false;
    mpgeo_dataset *oneshot_ds = nullptr;   // workspace of the one-shot calls
    // batched evaluation: lanes (each its own streams, events and workspace) that run
    // independent instances concurrently, and the tile sizes the autotuner measured, keyed by
    // (half-octave bucket of n, precision plan)
    std::vector<mpgeo_ctx *> lanes;
    std::vector<mpgeo_dataset *> lane_ds;
    std::map<std::string, int> tuned_tile;
    std::map<std::string, TunedBand> tuned_band;   // MPGEO_TUNE_BAND: band and error per class
    DevBuf batch_res;                         // per-instance {loglik, logdet, quad, info}
    // the persistent task-queue batch: inputs, tiles, vectors and control words
    DevBuf q_in_locs, q_in_z, q_locs, q_vec, q_tiles, q_linv, q_parts, q_flags, q_ctrl,
        q_insts, q_tasks, q_res, q_info;

    hipEvent_t take_event() {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return e;
    }
    // launch wrapper: events around a launch when timing is on
    template <class F> void timed(int cls, double flops, double bytes, F &&launch) {
        timed_on(stream, cls, flops, bytes, launch);
    }
    template <class F> void timed_on(hipStream_t st, int cls, double flops, double bytes, F &&launch) {
        if (!timing) {
            launch();
            return;
        }
        hipEvent_t a = take_event(), b = take_event();
        if (!a || !b) {
            launch();
            return;
        }
        (void)hipEventRecord(a, st);
        launch();
        (void)hipEventRecord(b, st);
        pending.push_back({cls, a, b, flops, bytes});
    }
    void collect() {
        for (auto &pl : pending) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, pl.a, pl.b) == hipSuccess) {
                stats[pl.cls].launches += 1;
                stats[pl.cls].seconds += ms * 1e-3;
                stats[pl.cls].flops += pl.flops;
                stats[pl.cls].bytes += pl.bytes;
            } else {
                (void)hipGetLastError();
            }
            spare.push_back(pl.a);
            spare.push_back(pl.b);
        }
        pending.clear();
    }
    void reset_stats() {
        for (int c = 0; c < kStatCount; ++c) {
            std::memset(&stats[c], 0, sizeof(stats[c]));
            std::strncpy(stats[c].name, kStatNames[c], sizeof(stats[c].name) - 1);
        }
    }
};

struct mpgeo_dataset {
    mpgeo_ctx *ctx = nullptr;
    int64_t n = 0;
    uint32_t flags = 0;
    Layout layout;
    // ordered inputs
    DevBuf locs, z, perm, keys, locs_in, z_in;
    // tiles and work buffers
    DevBuf pool64, pool32, off, all, list64, list32, list16, bulk16, bulk16k0;
    DevBuf p64, p32, linv, linv32, q16, qscale;
    DevBuf r, y, parts, info, result;
    DevBuf tmp_a, tmp_b, tmp_c;
    DevBuf fp64tab, trsm64l, trsm32l;   // distance-drawn precision map
    DevBuf chk;                         // finiteness flag of device inputs
    bool has_factor = false;
    mpgeo_theta theta{};      // theta of the resident factor (theta1 = 1 for a profile evaluation)
    bool profile = false;     // the last evaluation used the profile likelihood
    double var_scale = 1.0;   // kriging variance scale: the variance estimate q~/n after a profile evaluation
};

namespace {

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

int check_theta(const mpgeo_theta &t) {
    return (finite_pos(t.sigma2) && finite_pos(t.beta) && finite_pos(t.nu)) ? MPGEO_OK : MPGEO_E_ARG;
}

int check_plan(const mpgeo_plan &pl) {
    if (pl.flags & MPGEO_GRAPH) return MPGEO_E_UNSUPPORTED;   // switched off (see the flag)
    if (pl.tile < 1 || pl.tile > kMaxTile) return MPGEO_E_ARG;
    if (pl.band64 < -1 || pl.band32 < -1 || pl.band0 < -1) return MPGEO_E_ARG;
    if (pl.lowp < 0 || pl.lowp > 2) return MPGEO_E_ARG;
    if (!(pl.dist64 >= 0.0) || !(pl.dist32 >= 0.0) || !std::isfinite(pl.dist64) || !std::isfinite(pl.dist32))
        return MPGEO_E_ARG;
    if (pl.dist64 > 0.0) {   // precision map drawn from distances: its own third-tier switch
        if (pl.band0 >= 0 || (pl.flags & MPGEO_DIST_GCD)) return MPGEO_E_ARG;
        if ((pl.dist32 > 0.0) != (pl.lowp != 0) || (pl.dist32 > 0.0 && pl.dist32 < pl.dist64))
            return MPGEO_E_ARG;
        return MPGEO_OK;
    }
    if (pl.dist32 > 0.0) return MPGEO_E_ARG;
    if ((pl.band32 >= 0) != (pl.lowp != 0)) return MPGEO_E_ARG;   // a third tier needs its format
    return MPGEO_OK;
}

bool all_finite(const double *a, size_t count) {
    for (size_t e = 0; e < count; ++e)
        if (!std::isfinite(a[e])) return false;
    return true;
}

// Non-finite entries among `count` device doubles: a reduction on the context stream, read
// back synchronously (inputs are checked once, when they enter the library).
int device_all_finite(mpgeo_dataset *ds, const double *a, int64_t count, bool *ok) {
    *ok = true;
    if (count <= 0) return MPGEO_OK;
    hipStream_t s = ds->ctx->stream;
    MPGEO_TRY(ds->chk.ensure(sizeof(int)));
    MPGEO_HIP(hipMemsetAsync(ds->chk.ptr, 0, sizeof(int), s));
    launch_find_nonfinite(a, count, 1, count, false, ds->chk.as<int>(), s);
    MPGEO_HIP(hipGetLastError());
    int flag = 0;
    MPGEO_HIP(hipMemcpyAsync(&flag, ds->chk.ptr, sizeof(int), hipMemcpyDeviceToHost, s));
    MPGEO_HIP(hipStreamSynchronize(s));
    *ok = flag == 0;
    return MPGEO_OK;
}

// Inputs of either kind: host arrays on the host, device arrays by the reduction above.
int check_finite(mpgeo_dataset *ds, const double *a, int64_t count, bool on_device) {
    if (!a || count <= 0) return MPGEO_OK;
    if (!on_device) return all_finite(a, (size_t)count) ? MPGEO_OK : MPGEO_E_ARG;
    bool ok = true;
    MPGEO_TRY(device_all_finite(ds, a, count, &ok));
    return ok ? MPGEO_OK : MPGEO_E_ARG;
}

// HBM bytes of a built layout's tiles: both pools (the shared zero tile of dropped tiles
// included) and, with a 16-bit tier, the 16-bit copy of the factor.
size_t layout_footprint(const Layout &L) {
    const size_t te = (size_t)L.nbp * L.nbp;
    const size_t q16 = L.lowp ? (size_t)L.p * (L.p + 1) / 2 * te * 2 : 0;
    return (size_t)L.n64 * te * sizeof(double) +
           ((size_t)L.n32 + (L.has_zero_tile ? 1 : 0)) * te * sizeof(float) + q16;
}

// The next plan of MPGEO_ESCALATE for a matrix of p tile rows: every reduced band widened,
// b -> 2b + 1 (band64, band32, band0), a band reaching the last tile row becoming -1; once the
// FP64 band covers the matrix the third tier goes too; a distance-drawn map becomes all-FP64.
// False when the plan is already all-FP64 with nothing dropped.
bool escalate_plan(mpgeo_plan &pl, int64_t p) {
    auto full = [&](int32_t b) { return b < 0 || (int64_t)b >= p - 1; };
    if (pl.dist64 > 0.0) {
        pl.dist64 = pl.dist32 = 0.0;
        pl.band64 = pl.band32 = pl.band0 = -1;
        pl.lowp = 0;
        return true;
    }
    if (full(pl.band64) && full(pl.band0)) return false;
    auto widen = [&](int32_t b) { return full(b) ? -1 : ((int64_t)2 * b + 1 >= p - 1 ? -1 : 2 * b + 1); };
    pl.band0 = widen(pl.band0);
    pl.band64 = widen(pl.band64);
    if (pl.band64 < 0) {
        pl.band32 = -1;
        pl.lowp = 0;
    } else if (pl.band32 >= 0) {
        pl.band32 = (int32_t)std::min<int64_t>((int64_t)2 * pl.band32 + 1, p);
    }
    return true;
}

TileMap tile_map(const mpgeo_dataset *ds) {
    const Layout &L = ds->layout;
    TileMap m;
    m.off = ds->off.as<int64_t>();
    m.pool64 = ds->pool64.as<double>();
    m.pool32 = ds->pool32.as<float>();
    m.band = L.band;
    m.fp64tab = L.distance_map() ? ds->fp64tab.as<signed char>() : nullptr;
    m.nbp = L.nbp;
    m.nb = L.nb;
    m.p = L.p;
    m.n = L.n;
    return m;
}

// Allocate tiles and tables for (n, plan) and upload the tables.
int prepare_layout(mpgeo_dataset *ds, const mpgeo_plan &pl) {
    Layout &L = ds->layout;
    const int64_t p_new = (ds->n + pl.tile - 1) / pl.tile;
    const int zband_eff = Layout::effective_zband(p_new, pl.band0);
    const int band_eff = Layout::effective_band(p_new, pl.band64, pl.band0);
    const int edge_eff = Layout::effective_edge(p_new, pl.band64, pl.band32, pl.band0);
    const int lowp_eff = (edge_eff < std::min<int64_t>(zband_eff, p_new - 1)) ? pl.lowp : 0;
    const bool dmap = pl.dist64 > 0.0;
    if (!dmap && !L.distance_map() && L.same(ds->n, pl.tile, band_eff, edge_eff, zband_eff, lowp_eff) &&
        ds->off.ptr)
        return MPGEO_OK;
    if (dmap && L.distance_map() && L.n == ds->n && L.nb == pl.tile && L.dist64 == pl.dist64 &&
        L.dist32 == pl.dist32 && L.lowp_req == pl.lowp && ds->off.ptr)
        return MPGEO_OK;
    std::vector<double> boxes;
    if (dmap) {
        // bounding box of each tile row's (ordered) sites, from a host copy of the locations
        if (!ds->locs.ptr) return MPGEO_E_ARG;
        std::vector<double> xy((size_t)ds->n * 2);
        MPGEO_HIP(hipMemcpy(xy.data(), ds->locs.ptr, xy.size() * sizeof(double), hipMemcpyDeviceToHost));
        const int64_t p = (ds->n + pl.tile - 1) / pl.tile;
        boxes.assign((size_t)p * 4, 0.0);
        for (int64_t i = 0; i < p; ++i) {
            double b[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
            for (int64_t a = i * pl.tile; a < std::min<int64_t>(ds->n, (i + 1) * pl.tile); ++a) {
                b[0] = std::min(b[0], xy[2 * a]);
                b[1] = std::max(b[1], xy[2 * a]);
                b[2] = std::min(b[2], xy[2 * a + 1]);
                b[3] = std::max(b[3], xy[2 * a + 1]);
            }
            std::copy(b, b + 4, boxes.begin() + 4 * i);
        }
    }
    const int nbp_new = (pl.tile + kTileQuantum - 1) / kTileQuantum * kTileQuantum;
    const int wave16 = pl.lowp ? lowp_wave_tiles(nbp_new, pl.lowp, ds->ctx->cus - ds->ctx->reserved_cus) : 0;
    {
        Layout fresh;
        fresh.build(ds->n, pl.tile, pl.band64, pl.band32, pl.lowp, pl.band0, dmap ? &boxes : nullptr,
                    pl.dist64, pl.dist32, wave16);
        // the context's HBM budget, checked before anything is allocated
        if (ds->ctx->hbm_budget > 0 && layout_footprint(fresh) > ds->ctx->hbm_budget) return MPGEO_E_NOMEM;
        L = std::move(fresh);
    }
    ds->has_factor = false;
    const size_t te = (size_t)L.nbp * L.nbp;
    const size_t tiles32 = (size_t)L.n32 + (L.has_zero_tile ? 1 : 0);
    MPGEO_TRY(ds->pool64.ensure(std::max<size_t>(1, (size_t)L.n64 * te * sizeof(double))));
    MPGEO_TRY(ds->pool32.ensure(std::max<size_t>(1, tiles32 * te * sizeof(float))));
    MPGEO_TRY(ds->off.ensure(L.off.size() * sizeof(int64_t)));
    MPGEO_TRY(ds->all.ensure(std::max<size_t>(1, L.all.size()) * sizeof(TileIJ)));
    MPGEO_TRY(ds->list64.ensure(std::max<size_t>(1, L.list64.size()) * sizeof(TileIJ)));
    MPGEO_TRY(ds->list32.ensure(std::max<size_t>(1, L.list32.size()) * sizeof(TileIJ)));
    MPGEO_TRY(ds->list16.ensure(std::max<size_t>(1, L.list16.size()) * sizeof(TileIJ)));
    MPGEO_TRY(ds->bulk16.ensure(std::max<size_t>(1, L.bulk16.size()) * sizeof(TileIJ)));
    MPGEO_TRY(ds->bulk16k0.ensure(std::max<size_t>(1, L.bulk16_k0.size()) * sizeof(int32_t)));
    if (L.lowp) {
        // 16-bit copy of the factor's tiles (slot tri_index(i, k)) and their scales
        const size_t slots = (size_t)L.p * (L.p + 1) / 2;
        MPGEO_TRY(ds->q16.ensure(slots * te * 2));
        MPGEO_TRY(ds->qscale.ensure((size_t)L.p * sizeof(float)));   // power of two per tile row
    }
    MPGEO_TRY(ds->p64.ensure(2 * (size_t)L.p * te * sizeof(double)));   // two steps in flight
    MPGEO_TRY(ds->p32.ensure(2 * (size_t)L.p * te * sizeof(float)));
    MPGEO_TRY(ds->linv.ensure((size_t)L.p * te * sizeof(double)));
    MPGEO_TRY(ds->linv32.ensure(te * sizeof(float)));
    const size_t vec = (size_t)L.p * L.nbp * sizeof(double);
    MPGEO_TRY(ds->r.ensure(vec));
    MPGEO_TRY(ds->y.ensure(vec));
    MPGEO_TRY(ds->parts.ensure(2 * (size_t)L.p * sizeof(double)));
    MPGEO_TRY(ds->info.ensure(sizeof(unsigned long long)));
    MPGEO_TRY(ds->result.ensure(4 * sizeof(double)));
    hipStream_t s = ds->ctx->stream;
    if (L.distance_map()) {
        MPGEO_TRY(ds->fp64tab.ensure(L.tierv.size()));
        std::vector<signed char> flag(L.tierv.size());
        for (size_t q = 0; q < flag.size(); ++q) flag[q] = L.tierv[q] == 64 ? 1 : 0;
        MPGEO_HIP(hipMemcpy(ds->fp64tab.ptr, flag.data(), flag.size(), hipMemcpyHostToDevice));
        MPGEO_TRY(ds->trsm64l.ensure(std::max<size_t>(1, L.trsm64.size()) * sizeof(TileIJ)));
        MPGEO_TRY(ds->trsm32l.ensure(std::max<size_t>(1, L.trsm32.size()) * sizeof(TileIJ)));
        if (!L.trsm64.empty())
            MPGEO_HIP(hipMemcpy(ds->trsm64l.ptr, L.trsm64.data(), L.trsm64.size() * sizeof(TileIJ),
                                hipMemcpyHostToDevice));
        if (!L.trsm32.empty())
            MPGEO_HIP(hipMemcpy(ds->trsm32l.ptr, L.trsm32.data(), L.trsm32.size() * sizeof(TileIJ),
                                hipMemcpyHostToDevice));
    }
    if (L.has_zero_tile)   // the shared tile every dropped tile maps to: zero, never written
        MPGEO_HIP(hipMemsetAsync(ds->pool32.as<float>() + (size_t)L.n32 * te, 0, te * sizeof(float), s));
    MPGEO_HIP(hipMemcpyAsync(ds->off.ptr, L.off.data(), L.off.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice, s));
    MPGEO_HIP(hipMemcpyAsync(ds->all.ptr, L.all.data(), L.all.size() * sizeof(TileIJ),
                             hipMemcpyHostToDevice, s));
    if (!L.list64.empty())
        MPGEO_HIP(hipMemcpyAsync(ds->list64.ptr, L.list64.data(), L.list64.size() * sizeof(TileIJ),
                                 hipMemcpyHostToDevice, s));
    if (!L.list32.empty())
        MPGEO_HIP(hipMemcpyAsync(ds->list32.ptr, L.list32.data(), L.list32.size() * sizeof(TileIJ),
                                 hipMemcpyHostToDevice, s));
    if (!L.list16.empty())
        MPGEO_HIP(hipMemcpyAsync(ds->list16.ptr, L.list16.data(), L.list16.size() * sizeof(TileIJ),
                                 hipMemcpyHostToDevice, s));
    if (!L.bulk16.empty()) {
        MPGEO_HIP(hipMemcpyAsync(ds->bulk16.ptr, L.bulk16.data(), L.bulk16.size() * sizeof(TileIJ),
                                 hipMemcpyHostToDevice, s));
        MPGEO_HIP(hipMemcpyAsync(ds->bulk16k0.ptr, L.bulk16_k0.data(),
                                 L.bulk16_k0.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    }
    MPGEO_HIP(hipStreamSynchronize(s));   // host vectors may change with the next build
    return MPGEO_OK;
}

// Copy caller inputs to the device (if on the host), order them, keep perm.
int load_inputs(mpgeo_dataset *ds, const double *locs, const double *z, uint32_t flags) {
    mpgeo_ctx *ctx = ds->ctx;
    hipStream_t s = ctx->stream;
    const int64_t n = ds->n;
    // sites and data must be finite (checked before they are used)
    const bool on_dev = (flags & MPGEO_INPUT_DEVICE) != 0;
    MPGEO_TRY(check_finite(ds, locs, 2 * n, on_dev));
    MPGEO_TRY(check_finite(ds, z, n, on_dev));
    MPGEO_TRY(ds->locs.ensure((size_t)n * 2 * sizeof(double)));
    MPGEO_TRY(ds->z.ensure((size_t)n * sizeof(double)));
    MPGEO_TRY(ds->perm.ensure((size_t)n * sizeof(int64_t)));
    const double *dl = locs;
    const double *dz = z;
    if (!(flags & MPGEO_INPUT_DEVICE)) {
        MPGEO_TRY(ds->locs_in.ensure((size_t)n * 2 * sizeof(double)));
        MPGEO_HIP(hipMemcpyAsync(ds->locs_in.ptr, locs, (size_t)n * 2 * sizeof(double),
                                 hipMemcpyHostToDevice, s));
        dl = ds->locs_in.as<double>();
        if (z) {
            MPGEO_TRY(ds->z_in.ensure((size_t)n * sizeof(double)));
            MPGEO_HIP(hipMemcpyAsync(ds->z_in.ptr, z, (size_t)n * sizeof(double),
                                     hipMemcpyHostToDevice, s));
            dz = ds->z_in.as<double>();
        }
    }
    if (flags & MPGEO_ORDER_MORTON) {
        int64_t n2 = 1024;
        while (n2 < n) n2 *= 2;
        MPGEO_TRY(ds->keys.ensure((size_t)n2 * sizeof(uint64_t)));
        ctx->timed(kStatOrder, 0.0, (double)n * 40.0, [&] {
            launch_morton_order(dl, dz, n, (flags & MPGEO_DIST_GCD) != 0, ds->keys.as<uint64_t>(), n2, ds->locs.as<double>(),
                                dz ? ds->z.as<double>() : nullptr, ds->perm.as<int64_t>(), s);
        });
        MPGEO_HIP(hipGetLastError());
    } else {
        MPGEO_HIP(hipMemcpyAsync(ds->locs.ptr, dl, (size_t)n * 2 * sizeof(double),
                                 hipMemcpyDeviceToDevice, s));
        if (dz)
            MPGEO_HIP(hipMemcpyAsync(ds->z.ptr, dz, (size_t)n * sizeof(double),
                                     hipMemcpyDeviceToDevice, s));
        std::vector<int64_t> id(n);
        for (int64_t i = 0; i < n; ++i) id[i] = i;
        MPGEO_HIP(hipMemcpyAsync(ds->perm.ptr, id.data(), (size_t)n * sizeof(int64_t),
                                 hipMemcpyHostToDevice, s));
        MPGEO_HIP(hipStreamSynchronize(s));
    }
    if (!z) MPGEO_HIP(hipMemsetAsync(ds->z.ptr, 0, (size_t)n * sizeof(double), s));
    return MPGEO_OK;
}

int run_covgen(mpgeo_dataset *ds, const mpgeo_theta &th) {
    mpgeo_ctx *ctx = ds->ctx;
    const Layout &L = ds->layout;
    MaternParams mp = make_matern_params(th.sigma2, th.beta, th.nu);
    mp.gcd = (ds->flags & MPGEO_DIST_GCD) ? 1 : 0;
    const TileMap map = tile_map(ds);
    const double evals = (double)L.n * (L.n + 1) / 2.0;
    const double bytes = (double)L.n64 * L.nb * L.nb * 8.0 + (double)L.n32 * L.nb * L.nb * 4.0;
    ctx->timed(kStatCovgen, evals, bytes, [&] {
        launch_covgen(map, ds->locs.as<double>(), ds->all.as<TileIJ>(), (int64_t)L.all.size(), mp,
                      ctx->stream);
    });
    MPGEO_HIP(hipGetLastError());
    return MPGEO_OK;
}

// Factor the resident tiles, fused with the forward solve of z, then reduce.
//
// Three streams: the bulk stream runs most of each step's trailing update (tile columns
// j >= k+3, and the 16-bit pass); a second stream runs column k+2's FP64 and FP32 updates,
// which the next lookahead step needs first, and column k+1's FP32 and 16-bit updates; the
// side stream runs the critical path one step ahead: the update of column k+1's FP64 tiles,
// then POTRF, panel TRSMs, quantiser and forward-solve step of k+1 (lookahead of depth 1).  Staging panels alternate between two buffers so step k+1's
// panel can be written while step k's updates still read step k's.  Dependencies:
//   F(k)        = POTRF + TRSM + panel solve of step k            (side stream)
//   U_col(k)    = update of column k+1 with panel k               (side; after U_next(k-1))
//   U_next(k)   = update of column k+2 with panel k               (second; after F(k), U_bulk(k-1))
//   U_bulk(k)   = update of columns >= k+3 with panel k           (bulk; after F(k))
// and F(k+1)'s panel TRSMs wait for U_bulk(k-1), the last reader of their staging buffer.
// The 16-bit tier's tiles wait instead: U_bulk(k) gives column k+2's 16-bit tiles panels
// 0 .. k at once from the 16-bit factor copy, and U_col(k+1) adds panel k+1.
int run_factor(mpgeo_dataset *ds, hipEvent_t ev_factored) {
    mpgeo_ctx *ctx = ds->ctx;
    hipStream_t s0 = ctx->stream;
    hipStream_t s1 = ctx->side;
    hipStream_t sb = ctx->bulk ? ctx->bulk : s0;   // bulk trailing updates
    hipStream_t sa = ctx->next ? ctx->next : sb;   // column k+2 of the FP64/FP32 bulk
    const Layout &L = ds->layout;
    const TileMap map = tile_map(ds);
    const int nbp = L.nbp, p = L.p;
    const size_t te = (size_t)nbp * nbp;
    double *r = ds->r.as<double>();
    double *y = ds->y.as<double>();
    double *logdet_part = ds->parts.as<double>();
    double *quad_part = logdet_part + p;
    unsigned long long *info = ds->info.as<unsigned long long>();
    if (!ctx->ensure_sync_events(4 * (size_t)p + 1)) return MPGEO_E_DEVICE;
    hipEvent_t ev_start = ctx->sync_events[0];
    hipEvent_t *ev_f = ctx->sync_events.data() + 1;       // F(k) done
    hipEvent_t *ev_bulk = ev_f + p;                        // U_bulk(k) done
    hipEvent_t *ev_next = ev_bulk + p;                     // U_next(k) done
    hipEvent_t *ev_col = ev_next + p;                      // column k+1's FP32 / 16-bit tiles done
    launch_fill_u64(info, ~0ull, 1, s0);   // no failing column yet
    launch_pad_vector(ds->z.as<double>(), r, L.n, L.nb, nbp, p, s0);
    if (L.lowp) launch_row_scale(map, ds->qscale.as<float>(), s0);   // from Sigma's diagonal
    MPGEO_HIP(hipEventRecord(ev_start, s0));
    MPGEO_HIP(hipStreamWaitEvent(s1, ev_start, 0));
    if (sb != s0) MPGEO_HIP(hipStreamWaitEvent(sb, ev_start, 0));
    if (sa != sb) MPGEO_HIP(hipStreamWaitEvent(sa, ev_start, 0));
    const double nbd = L.nb;
    const TileIJ *l64 = ds->list64.as<TileIJ>();
    const TileIJ *l32 = ds->list32.as<TileIJ>();
    const TileIJ *l16 = ds->list16.as<TileIJ>();
    const TileIJ *b16list = ds->bulk16.as<TileIJ>();
    const int32_t *b16k0 = ds->bulk16k0.as<int32_t>();
    void *q16 = ds->q16.ptr;                    // 16-bit factor copy, tile (i, k) at tri_index(i, k)
    float *qscale = ds->qscale.as<float>();     // power of two of each tile row (third tier)

    auto panel64 = [&](int k) { return ds->p64.as<double>() + (size_t)(k & 1) * p * te; };
    auto panel32 = [&](int k) { return ds->p32.as<float>() + (size_t)(k & 1) * p * te; };

    // F(k): POTRF, TRSM of the panel into staging (k & 1), panel solve of the forward solve;
    // potrf_step is its first part, which touches no staging buffer
    auto potrf_args = [&](int k) {
        PotrfArgs pa;
        pa.a = ds->pool64.as<double>() + L.off[tri_index(k, k)];
        pa.linv = ds->linv.as<double>() + (int64_t)k * te;
        pa.linv32 = ds->linv32.as<float>();
        pa.r = r + (int64_t)k * nbp;
        pa.y = y + (int64_t)k * nbp;
        pa.logdet_part = logdet_part + k;
        pa.quad_part = quad_part + k;
        pa.info = info;
        pa.col_base = (int64_t)k * L.nb;
        pa.nb = L.nb;
        pa.nbp = nbp;
        return pa;
    };
    auto potrf_step = [&](int k) {
        const PotrfArgs pa = potrf_args(k);
        const double rk = (double)L.rows(k);
        ctx->timed_on(s1, kStatPotrf, rk * rk * rk / 3.0, rk * rk * 8.0 * 3.0,
                      [&] { launch_potrf(pa, s1); });
    };
    // part 0: the FP64 panel TRSM (needs only the column's FP64 tiles and POTRF); part 1: the
    // FP32 panel TRSM, the quantiser and the panel solve
    auto panel_step = [&](int k, int part) {
        if (k + 1 >= p) return;
        const PotrfArgs pa = potrf_args(k);
        const int npanel = L.panel_count(k);            // panel tiles that are not dropped
        const int n64 = std::min(L.band, npanel);
        const int first32 = k + n64 + 1;
        const int n32 = npanel - n64;
        double *p64 = panel64(k);
        float *p32 = panel32(k);
        const bool quant = L.lowp_step(k);   // panel k gets a 16-bit copy
        if (L.distance_map()) {   // panel tiles of each precision as lists
            const int64_t b64 = L.trsm64_b[k], c64 = L.trsm64_b[k + 1] - b64;
            const int64_t b32 = L.trsm32_b[k], c32 = L.trsm32_b[k + 1] - b32;
            if (part == 0 && c64 > 0)
                ctx->timed_on(s1, kStatTrsm64, L.trsm64_flops[k], (double)c64 * nbd * nbd * 8.0 * 2.0, [&] {
                    launch_trsm(map, k, 0, (int)c64, true, pa.linv, pa.linv32, p64, p32, s1,
                                /*narrow=*/c64 <= 4, ds->trsm64l.as<TileIJ>() + b64);
                });
            if (part == 1 && c32 > 0)
                ctx->timed_on(s1, kStatTrsm32, L.trsm32_flops[k], (double)c32 * nbd * nbd * 4.0 * 2.0, [&] {
                    launch_trsm(map, k, 0, (int)c32, false, pa.linv, pa.linv32, p64, p32, s1,
                                false, ds->trsm32l.as<TileIJ>() + b32);
                });
        } else {
            if (part == 0 && n64 > 0)
                ctx->timed_on(s1, kStatTrsm64, L.trsm64_flops[k], (double)n64 * nbd * nbd * 8.0 * 2.0, [&] {
                    launch_trsm(map, k, k + 1, n64, true, pa.linv, pa.linv32, p64, p32, s1,
                                /*narrow=*/true);
                });
            if (part == 1 && n32 > 0)
                ctx->timed_on(s1, kStatTrsm32, L.trsm32_flops[k], (double)n32 * nbd * nbd * 4.0 * 2.0, [&] {
                    launch_trsm(map, k, first32, n32, false, pa.linv, pa.linv32, p64, p32, s1);
                });
        }
        if (part == 0) return;
        if (quant)   // 16-bit panel copy
            ctx->timed_on(s1, kStatQuant, 0.0, (double)npanel * nbd * nbd * 6.0, [&] {
                launch_quantize(map, k, k + 1, npanel, p32, qscale, q16, L.lowp, s1);
            });
        ctx->timed_on(s1, kStatPanel, 2.0 * npanel * nbd * nbd, (double)npanel * nbd * nbd * 16.0,
                      [&] { launch_panel_solve(map, k, npanel, p64, pa.y, r, s1); });
    };
    // update of list entries [b, e) of each tier with panel k on stream st; the 16-bit entries
    // take panels [k0, k] (the bulk pass: entries of the bulk16 list, each with its own k0; the
    // lookahead column: entries of list16, k0 = k).
    // Algorithmic bytes: every output tile read and written once, every operand tile it needs
    // read once (FP64/FP32: at most p - 1 - k distinct panel tiles, at most two per output
    // tile; 16-bit bulk: the operand tiles counted by the layout).
    auto update_range = [&](int k, int64_t b64, int64_t e64, int64_t b32, int64_t e32, int64_t b16,
                            int64_t e16, double f64, double f32, double f16, bool lookahead,
                            double panels16, hipStream_t st) {
        const double tile_elems = (double)nbd * nbd;
        auto panel_tiles = [&](int64_t count) { return (double)std::min<int64_t>(L.panel_count(k), 2 * count); };
        if (e16 > b16)
            ctx->timed_on(st, lookahead ? kStatUpdate16Col : kStatUpdate16, f16,
                          tile_elems * ((double)(e16 - b16) * 4.0 * 2.0 +
                                        (lookahead ? panel_tiles(e16 - b16) : panels16) * 2.0), [&] {
                if (lookahead)
                    launch_update_lowp(map, l16 + b16, e16 - b16, k, k + 1, L.zband, q16, qscale,
                                       L.lowp, st);
                else
                    launch_update_lowp(map, b16list + b16, e16 - b16, 0, k + 1, L.zband, q16, qscale,
                                       L.lowp, st, b16k0 + b16);
            });
        if (e64 > b64)
            ctx->timed_on(st, kStatUpdate64, f64,
                          tile_elems * ((double)(e64 - b64) * 8.0 * 2.0 + panel_tiles(e64 - b64) * 8.0), [&] {
                launch_update(map, l64 + b64, e64 - b64, true, panel64(k), panel32(k), st,
                              /*narrow=*/lookahead);   // the lookahead column
            });
        if (e32 > b32)
            ctx->timed_on(st, kStatUpdate32, f32,
                          tile_elems * ((double)(e32 - b32) * 4.0 * 2.0 + panel_tiles(e32 - b32) * 4.0), [&] {
                launch_update(map, l32 + b32, e32 - b32, false, panel64(k), panel32(k), st);
            });
    };

    potrf_step(0);
    panel_step(0, 0);
    panel_step(0, 1);
    MPGEO_HIP(hipEventRecord(ev_f[0], s1));
    for (int k = 0; k < p; ++k) {
        // U_next(k): column k+2's FP64 and FP32 tiles, after F(k) and U_bulk(k-1) (with no
        // stream of its own, it is part of the bulk launches below)
        const bool own_next = sa != sb;
        if (own_next) {
            MPGEO_HIP(hipStreamWaitEvent(sa, ev_f[k], 0));
            if (k >= 1) MPGEO_HIP(hipStreamWaitEvent(sa, ev_bulk[k - 1], 0));
            if (k + 1 < p)
                update_range(k, L.next_b[0][k], L.bulk[0][k].e, L.next_b[1][k], L.bulk[1][k].e, 0, 0,
                             L.next_f[0][k], L.next_f[1][k], 0.0, false, 0.0, sa);
            MPGEO_HIP(hipEventRecord(ev_next[k], sa));
            // column k+1's FP32 and 16-bit tiles take panel k here, beside POTRF(k+1) on the
            // side stream (they were brought up to panel k-1 by U_next(k-1) and step k-1's
            // 16-bit pass, both done once U_bulk(k-1) is)
            if (k + 1 < p)
                update_range(k, 0, 0, L.col[1][k].b, L.col[1][k].e, L.col[2][k].b, L.col[2][k].e, 0.0,
                             L.col[1][k].flops, L.col[2][k].flops, true, 0.0, sa);
            MPGEO_HIP(hipEventRecord(ev_col[k], sa));
        }
        // U_bulk(k): FP64 and FP32 columns >= k+3, then the 16-bit pass (column k+2), whose
        // long-running workgroups would otherwise hold the compute units the lookahead's
        // small launches wait for
        MPGEO_HIP(hipStreamWaitEvent(sb, ev_f[k], 0));
        if (k + 1 < p) {
            const int64_t e64 = own_next ? L.next_b[0][k] : L.bulk[0][k].e;
            const int64_t e32 = own_next ? L.next_b[1][k] : L.bulk[1][k].e;
            update_range(k, L.bulk[0][k].b, e64, L.bulk[1][k].b, e32, 0, 0,
                         L.bulk[0][k].flops - (own_next ? L.next_f[0][k] : 0.0),
                         L.bulk[1][k].flops - (own_next ? L.next_f[1][k] : 0.0), 0.0, false, 0.0, sb);
        }
        if (!own_next) MPGEO_HIP(hipEventRecord(ev_next[k], sb));
        if (k + 1 < p)
            update_range(k, 0, 0, 0, 0, L.bulk[2][k].b, L.bulk[2][k].e, 0.0, 0.0,
                         L.bulk[2][k].flops, false, L.bulk[2][k].panels, sb);
        MPGEO_HIP(hipEventRecord(ev_bulk[k], sb));
        if (k + 1 < p) {
            // Critical path: column k+1 takes panel k (its FP64 tiles, the diagonal tile among
            // them, once U_next(k-1) is done), then POTRF(k+1) and the FP64 panel TRSM, which
            // writes staging buffer (k+1) & 1 and so waits for U_bulk(k-1), its last reader (and
            // so also for step k-1's 16-bit pass); then, once the column's FP32 and 16-bit tiles
            // have taken panel k (on the second stream, or here without one), the rest of F(k+1).
            if (k >= 1) MPGEO_HIP(hipStreamWaitEvent(s1, ev_next[k - 1], 0));
            update_range(k, L.col[0][k].b, L.col[0][k].e, 0, 0, 0, 0, L.col[0][k].flops, 0.0, 0.0,
                         true, 0.0, s1);
            potrf_step(k + 1);
            if (k >= 1) MPGEO_HIP(hipStreamWaitEvent(s1, ev_bulk[k - 1], 0));
            panel_step(k + 1, 0);
            if (own_next)
                MPGEO_HIP(hipStreamWaitEvent(s1, ev_col[k], 0));
            else
                update_range(k, 0, 0, L.col[1][k].b, L.col[1][k].e, L.col[2][k].b, L.col[2][k].e, 0.0,
                             L.col[1][k].flops, L.col[2][k].flops, true, 0.0, s1);
            panel_step(k + 1, 1);
            MPGEO_HIP(hipEventRecord(ev_f[k + 1], s1));
        }
        MPGEO_HIP(hipGetLastError());
    }
    MPGEO_HIP(hipStreamWaitEvent(s0, ev_f[p - 1], 0));
    if (sb != s0) MPGEO_HIP(hipStreamWaitEvent(s0, ev_bulk[p - 1], 0));
    if (sa != s0) MPGEO_HIP(hipStreamWaitEvent(s0, sa != sb ? ev_col[p - 1] : ev_next[p - 1], 0));
    if (ev_factored) MPGEO_HIP(hipEventRecord(ev_factored, s0));
    ctx->timed(kStatFinal, 2.0 * p, 16.0 * p, [&] {
        launch_finalize(logdet_part, quad_part, p, L.n, ds->profile, ds->result.as<double>(), s0);
    });
    MPGEO_HIP(hipGetLastError());
    return MPGEO_OK;
}

// Read back {loglik, logdet, quad} and info into *out.
int read_result(mpgeo_dataset *ds, mpgeo_result *out) {
    hipStream_t s = ds->ctx->stream;
    double res[3];
    unsigned long long info = 0;
    MPGEO_HIP(hipMemcpyAsync(res, ds->result.ptr, sizeof(res), hipMemcpyDeviceToHost, s));
    MPGEO_HIP(hipMemcpyAsync(&info, ds->info.ptr, sizeof(info), hipMemcpyDeviceToHost, s));
    MPGEO_HIP(hipStreamSynchronize(s));
    out->loglik = res[0];
    out->logdet = res[1];
    out->quad = res[2];
    out->info = (info == ~0ull) ? -1 : (int64_t)info;
    return out->info >= 0 ? MPGEO_E_NOT_SPD : MPGEO_OK;
}

struct EventSet {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
    bool ok = true;
    EventSet() {
        for (auto &x : e)
            if (hipEventCreate(&x) != hipSuccess) {
                (void)hipGetLastError();
                x = nullptr;
                ok = false;
            }
    }
    ~EventSet() {
        for (auto &x : e)
            if (x) (void)hipEventDestroy(x);
    }
    double secs(int a, int b) const {
        float ms = 0.f;
        if (!ok || hipEventElapsedTime(&ms, e[a], e[b]) != hipSuccess) {
            (void)hipGetLastError();
            return 0.0;
        }
        return ms * 1e-3;
    }
};

// covgen + factor + reduce for a dataset whose ordered inputs are resident.
int evaluate(mpgeo_dataset *ds, const mpgeo_theta &th, const mpgeo_plan &pl, mpgeo_result *out,
             hipEvent_t ev_start_outer) {
    mpgeo_ctx *ctx = ds->ctx;
    hipStream_t s = ctx->stream;
    MPGEO_TRY(prepare_layout(ds, pl));
    // profile likelihood: the tiles hold the correlation matrix (theta1 = 1)
    ds->profile = (pl.flags & MPGEO_PROFILE) != 0;
    mpgeo_theta th_eval = th;
    if (ds->profile) th_eval.sigma2 = 1.0;
    EventSet ev;
    if (ev.ok) MPGEO_HIP(hipEventRecord(ev.e[0], s));
    MPGEO_TRY(run_covgen(ds, th_eval));
    if (ev.ok) MPGEO_HIP(hipEventRecord(ev.e[1], s));
    MPGEO_TRY(run_factor(ds, ev.ok ? ev.e[2] : nullptr));
    if (ev.ok) MPGEO_HIP(hipEventRecord(ev.e[3], s));
    const int st = read_result(ds, out);
    out->t_covgen = ev.secs(0, 1);
    out->t_factor = ev.secs(1, 2);
    out->t_solve = ev.secs(2, 3);
    if (ev_start_outer) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, ev_start_outer, ev.e[3]) == hipSuccess) out->t_total = ms * 1e-3;
        else (void)hipGetLastError();
    } else {
        out->t_total = ev.secs(0, 3);
    }
    ctx->collect();
    ds->has_factor = (st == MPGEO_OK);
    ds->theta = th_eval;
    ds->var_scale = ds->profile ? out->quad / (double)ds->layout.n : 1.0;
    out->band64 = pl.band64;
    out->band32 = pl.band32;
    out->band0 = pl.band0;
    out->escalations = 0;
    return st;
}

// evaluate(), repeated with wider bands while the factorization meets a non-positive pivot
// and the plan asks for it (MPGEO_ESCALATE; Section VIII-D-1: reduced precision next to the
// diagonal can cost positive definiteness)
int evaluate_escalating(mpgeo_dataset *ds, const mpgeo_theta &th, mpgeo_plan pl, mpgeo_result *out,
                        hipEvent_t ev_start_outer) {
    const int64_t p = (ds->n + pl.tile - 1) / pl.tile;
    for (int esc = 0;; ++esc) {
        const int st = evaluate(ds, th, pl, out, ev_start_outer);
        out->escalations = esc;
        if (st != MPGEO_E_NOT_SPD || !(pl.flags & MPGEO_ESCALATE) || !escalate_plan(pl, p)) return st;
    }
}

struct Device {
    explicit Device(int d) { ok = hipSetDevice(d) == hipSuccess; }
    bool ok;
};

// Simple kriging from the resident factor, enqueued on the dataset's stream without waiting:
// w = L^-T y (backward solve), pred_j = sum_a C(s0_j, s_a) w_a, and with var the prediction
// variances var_scale * (theta1 - |L^-1 c_j|^2).  New sites and outputs are device buffers.
int krige_enqueue(mpgeo_dataset *ds, int64_t m, const double *dnew, double *dpred, double *dvar,
                  double var_scale) {
    const Layout &L = ds->layout;
    hipStream_t s = ds->ctx->stream;
    const size_t vec = (size_t)L.p * L.nbp;
    MPGEO_TRY(ds->tmp_a.ensure(2 * vec * sizeof(double)));
    double *t = ds->tmp_a.as<double>();
    double *w = t + vec;
    launch_backward_solve(tile_map(ds), ds->linv.as<double>(), ds->y.as<double>(), t, w, s);
    MPGEO_HIP(hipGetLastError());
    MaternParams mp = make_matern_params(ds->theta.sigma2, ds->theta.beta, ds->theta.nu);
    mp.gcd = (ds->flags & MPGEO_DIST_GCD) ? 1 : 0;
    launch_krige_predict(ds->locs.as<double>(), L.n, L.nb, L.nbp, dnew, m, w, mp, dpred, s);
    MPGEO_HIP(hipGetLastError());
    if (dvar) {
        const int64_t ldc = (int64_t)vec;
        MPGEO_TRY(ds->tmp_c.ensure((size_t)ldc * m * sizeof(double) + (size_t)L.nbp * m * sizeof(double)));
        double *c = ds->tmp_c.as<double>();
        double *tmp = c + (size_t)ldc * m;
        launch_cross_cov(ds->locs.as<double>(), L.n, L.nb, L.nbp, L.p, dnew, m, mp, c, ldc, s);
        launch_forward_multi(tile_map(ds), ds->linv.as<double>(), c, ldc, m, tmp, s);
        launch_column_var(c, ldc, ldc, m, ds->theta.sigma2, var_scale, dvar, s);
        MPGEO_HIP(hipGetLastError());
    }
    return MPGEO_OK;
}

}  // namespace

extern "C" {

const char *mpgeo_status_string(int status) {
    switch (status) {
        case MPGEO_OK: return "ok";
        case MPGEO_E_ARG: return "invalid argument";
        case MPGEO_E_NOT_SPD: return "matrix is not positive definite";
        case MPGEO_E_NOMEM: return "device memory allocation failed";
        case MPGEO_E_DEVICE: return "HIP runtime error";
        case MPGEO_E_UNSUPPORTED: return "unsupported feature";
        case MPGEO_E_TOO_LARGE: return "problem exceeds the fixed scratch array of the allocation-free entry point";
        default: return "unknown status";
    }
}

size_t mpgeo_footprint_bytes(int64_t n, mpgeo_plan plan) {
    if (n < 1 || check_plan(plan) != MPGEO_OK) return 0;
    Layout L;
    if (plan.dist64 > 0.0) plan.band64 = -1;   // the map needs the sites: bound it by all-FP64
    L.build(n, plan.tile, plan.band64, plan.band32, plan.lowp, plan.band0);
    return layout_footprint(L);
}

// Reserved compute units for the critical path: MPGEO_RESERVED_CUS (default 0: none),
// spread over the mask so that they fall on different XCDs.
static void create_bulk_stream(mpgeo_ctx *c) {
    int reserve = 0;
    if (const char *env = std::getenv("MPGEO_RESERVED_CUS")) reserve = std::atoi(env);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    if (reserve <= 0 || reserve >= cus / 2) return;
    std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0u);
    for (int i = 0; i < cus; ++i) mask[(size_t)i / 32] |= 1u << (i % 32);
    const int stride = cus / reserve;
    for (int j = 0; j < reserve; ++j) {
        const int i = (j * stride + j) % cus;
        mask[(size_t)i / 32] &= ~(1u << (i % 32));
    }
    hipStream_t st = nullptr;
    if (hipExtStreamCreateWithCUMask(&st, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    c->bulk = st;
    c->reserved_cus = reserve;
}

int mpgeo_plan_tiers(int64_t n, mpgeo_plan plan, mpgeo_tier_summary *out) {
    if (!out || n < 1 || check_plan(plan) != MPGEO_OK || plan.dist64 > 0.0) return MPGEO_E_ARG;
    Layout L;
    L.build(n, plan.tile, plan.band64, plan.band32, plan.lowp, plan.band0);
    mpgeo_tier_summary info{};
    info.p = L.p;
    info.nbp = L.nbp;
    info.band64 = L.band;
    info.edge = L.edge;
    info.band0 = L.zband;
    info.lowp = L.lowp;
    for (int i = 0; i < L.p; ++i)
        for (int j = 0; j <= i; ++j) {
            const int t = L.tier(i, j);
            info.tiles[t == 64 ? 0 : t == 32 ? 1 : t == 16 ? 2 : 3]++;
        }
    for (int q = 0; q < 3; ++q)
        for (int k = 0; k + 1 < L.p; ++k) info.update_flops[q] += L.bulk[q][k].flops + L.col[q][k].flops;
    for (int k = 0; k < L.p; ++k) {
        info.trsm_flops[0] += L.trsm64_flops[k];
        info.trsm_flops[1] += L.trsm32_flops[k];
        const double r = (double)L.rows(k);
        info.potrf_flops += r * r * r / 3.0;
    }
    info.footprint_bytes = mpgeo_footprint_bytes(n, plan);
    *out = info;
    return MPGEO_OK;
}

// ---- the fixed device array of the allocation-free batch --------------------------------------
// Every work buffer of mpgeo_batch_loglik_noalloc is carved from `scratch`.  Host code never uses
// the array's name as an address (on the host it is only a stand-in for the symbol): its device
// address is resolved once per GPU, with that GPU current, when the first context on it is
// created, and kept here.
constexpr size_t kScratchBytes = (size_t)MPGEO_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];
static std::mutex g_scratch_mu;
static std::map<int, char *> g_scratch_ptr;   // device ordinal -> device address of `scratch`

static int scratch_setup(int device) {   // the device is current
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr.count(device)) return MPGEO_OK;
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) {
        (void)hipGetLastError();
        return MPGEO_E_DEVICE;
    }
    g_scratch_ptr[device] = static_cast<char *>(ptr);
    return MPGEO_OK;
}

static char *scratch_ptr(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    return it == g_scratch_ptr.end() ? nullptr : it->second;
}

int mpgeo_ctx_create(mpgeo_ctx **out, int device, void *hip_stream, size_t hbm_budget_bytes) {
    if (!out) return MPGEO_E_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess) {
        (void)hipGetLastError();
        return MPGEO_E_DEVICE;
    }
    if (device < 0 || device >= count) return MPGEO_E_ARG;
    MPGEO_HIP(hipSetDevice(device));
    MPGEO_TRY(scratch_setup(device));
    mpgeo_ctx *c = new mpgeo_ctx();
    c->device = device;
    c->hbm_budget = hbm_budget_bytes;
    if (hip_stream) {
        c->stream = static_cast<hipStream_t>(hip_stream);
    } else {
        hipError_t e = hipStreamCreate(&c->stream);   // blocking: ordered after the null stream
        if (e != hipSuccess) {
            (void)hipGetLastError();
            delete c;
            return MPGEO_E_DEVICE;
        }
        c->own_stream = true;
    }
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
        delete c;
        return MPGEO_E_DEVICE;
    }
    if (hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
        (void)hipGetLastError();
        c->cus = 0;
    }
    create_bulk_stream(c);
    if (!c->bulk && hipStreamCreateWithFlags(&c->next, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        c->next = nullptr;
    }
    c->reset_stats();
    *out = c;
    return MPGEO_OK;
}

int mpgeo_dataset_destroy(mpgeo_dataset *ds);

int mpgeo_ctx_destroy(mpgeo_ctx *ctx) {
    if (!ctx) return MPGEO_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->oneshot_ds) mpgeo_dataset_destroy(ctx->oneshot_ds);
    for (auto *d : ctx->lane_ds) mpgeo_dataset_destroy(d);
    for (auto *c : ctx->lanes) mpgeo_ctx_destroy(c);
    ctx->batch_res.release();
    ctx->collect();
    for (auto e : ctx->spare) (void)hipEventDestroy(e);
    for (auto e : ctx->sync_events) (void)hipEventDestroy(e);
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
    if (ctx->next) {
        (void)hipStreamSynchronize(ctx->next);
        (void)hipStreamDestroy(ctx->next);
    }
    if (ctx->bulk) {
        (void)hipStreamSynchronize(ctx->bulk);
        (void)hipStreamDestroy(ctx->bulk);
    }
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
    delete ctx;
    return MPGEO_OK;
}

int mpgeo_ctx_kernel_stats(mpgeo_ctx *ctx, mpgeo_kernel_stat *out, int max, int *count) {
    if (!ctx || !count || (max > 0 && !out)) return MPGEO_E_ARG;
    *count = kStatCount;
    for (int c = 0; c < kStatCount && c < max; ++c) out[c] = ctx->stats[c];
    return MPGEO_OK;
}

int mpgeo_ctx_reset_stats(mpgeo_ctx *ctx) {
    if (!ctx) return MPGEO_E_ARG;
    ctx->reset_stats();
    return MPGEO_OK;
}

int mpgeo_dataset_create(mpgeo_ctx *ctx, int64_t n, const double *locs, const double *z,
                         uint32_t flags, mpgeo_dataset **out) {
    if (!ctx || !out || !locs || n < 1 || n > (int64_t)0xFFFFFFFF) return MPGEO_E_ARG;
    *out = nullptr;
    Device dev(ctx->device);
    if (!dev.ok) return MPGEO_E_DEVICE;
    mpgeo_dataset *ds = new mpgeo_dataset();
    ds->ctx = ctx;
    ds->n = n;
    ds->flags = flags;
    const int st = load_inputs(ds, locs, z, flags);
    if (st != MPGEO_OK) {
        mpgeo_dataset_destroy(ds);
        return st;
    }
    *out = ds;
    return MPGEO_OK;
}

int mpgeo_dataset_destroy(mpgeo_dataset *ds) {
    if (!ds) return MPGEO_OK;
    (void)hipSetDevice(ds->ctx->device);
    (void)hipStreamSynchronize(ds->ctx->stream);
    for (DevBuf *b : {&ds->locs, &ds->z, &ds->perm, &ds->keys, &ds->locs_in, &ds->z_in,
                      &ds->pool64, &ds->pool32, &ds->off, &ds->all, &ds->list64, &ds->list32,
                      &ds->list16, &ds->bulk16, &ds->bulk16k0, &ds->q16, &ds->qscale,
                      &ds->p64, &ds->p32, &ds->linv, &ds->linv32, &ds->r, &ds->y, &ds->parts,
                      &ds->info, &ds->result, &ds->tmp_a, &ds->tmp_b, &ds->tmp_c, &ds->fp64tab,
                      &ds->trsm64l, &ds->trsm32l, &ds->chk})
        b->release();
    delete ds;
    return MPGEO_OK;
}

int mpgeo_dataset_loglik(mpgeo_dataset *ds, mpgeo_theta theta, mpgeo_plan plan, mpgeo_result *out) {
    if (!ds || !out) return MPGEO_E_ARG;
    out->info = -1;
    MPGEO_TRY(check_theta(theta));
    MPGEO_TRY(check_plan(plan));
    Device dev(ds->ctx->device);
    if (!dev.ok) return MPGEO_E_DEVICE;
    ds->ctx->timing = (plan.flags & MPGEO_TIMING) != 0;
    const int st = evaluate_escalating(ds, theta, plan, out, nullptr);
    ds->ctx->timing = false;
    return st;
}

int mpgeo_loglik(mpgeo_ctx *ctx, int64_t n, const double *locs, const double *z, mpgeo_theta theta,
                 mpgeo_plan plan, mpgeo_result *out) {
    if (!ctx || !out || !locs || !z || n < 1 || n > (int64_t)0xFFFFFFFF) return MPGEO_E_ARG;
    out->info = -1;
    MPGEO_TRY(check_theta(theta));
    MPGEO_TRY(check_plan(plan));
    Device dev(ctx->device);
    if (!dev.ok) return MPGEO_E_DEVICE;
    if (ctx->oneshot_ds && ctx->oneshot_ds->n != n) {
        // keep the large tile pools if the size matches; otherwise start over
        mpgeo_dataset_destroy(ctx->oneshot_ds);
        ctx->oneshot_ds = nullptr;
    }
    if (!ctx->oneshot_ds) {
        ctx->oneshot_ds = new mpgeo_dataset();
        ctx->oneshot_ds->ctx = ctx;
        ctx->oneshot_ds->n = n;
    }
    mpgeo_dataset *ds = ctx->oneshot_ds;
    ds->flags = plan.flags;
    ctx->timing = (plan.flags & MPGEO_TIMING) != 0;
    EventSet ev;
    if (ev.ok) MPGEO_HIP(hipEventRecord(ev.e[0], ctx->stream));
    int st = load_inputs(ds, locs, z, plan.flags);
    if (st == MPGEO_OK) st = evaluate_escalating(ds, theta, plan, out, ev.ok ? ev.e[0] : nullptr);
    ctx->timing = false;
    return st;
}

int mpgeo_dataset_perm(mpgeo_dataset *ds, int64_t *perm) {
    if (!ds || !perm) return MPGEO_E_ARG;
    Device dev(ds->ctx->device);
    MPGEO_HIP(hipMemcpy(perm, ds->perm.ptr, (size_t)ds->n * sizeof(int64_t), hipMemcpyDeviceToHost));
    return MPGEO_OK;
}

int mpgeo_dataset_covariance(mpgeo_dataset *ds, mpgeo_theta theta, mpgeo_plan plan) {
    if (!ds) return MPGEO_E_ARG;
    MPGEO_TRY(check_theta(theta));
    MPGEO_TRY(check_plan(plan));
    Device dev(ds->ctx->device);
    MPGEO_TRY(prepare_layout(ds, plan));
    mpgeo_theta th = theta;
    if (plan.flags & MPGEO_PROFILE) th.sigma2 = 1.0;   // the correlation matrix
    MPGEO_TRY(run_covgen(ds, th));
    ds->has_factor = false;
    MPGEO_HIP(hipStreamSynchronize(ds->ctx->stream));
    ds->ctx->collect();
    return MPGEO_OK;
}

int mpgeo_dataset_matrix(mpgeo_dataset *ds, double *out, int64_t ld) {
    if (!ds || !out || ld < ds->n || !ds->off.ptr) return MPGEO_E_ARG;
    Device dev(ds->ctx->device);
    const int64_t n = ds->n;
    hipStream_t s = ds->ctx->stream;
    MPGEO_TRY(ds->tmp_a.ensure((size_t)n * n * sizeof(double)));
    MPGEO_HIP(hipMemsetAsync(ds->tmp_a.ptr, 0, (size_t)n * n * sizeof(double), s));
    launch_export_dense(tile_map(ds), ds->tmp_a.as<double>(), n, ds->all.as<TileIJ>(),
                        (int64_t)ds->layout.all.size(), s);
    MPGEO_HIP(hipGetLastError());
    std::vector<double> host((size_t)n * n);
    MPGEO_HIP(hipMemcpyAsync(host.data(), ds->tmp_a.ptr, host.size() * sizeof(double),
                             hipMemcpyDeviceToHost, s));
    MPGEO_HIP(hipStreamSynchronize(s));
    for (int64_t c = 0; c < n; ++c)
        for (int64_t r = c; r < n; ++r) out[r + c * ld] = host[r + c * n];
    return MPGEO_OK;
}

int mpgeo_dataset_solution(mpgeo_dataset *ds, double *y) {
    if (!ds || !y || !ds->has_factor) return MPGEO_E_ARG;
    Device dev(ds->ctx->device);
    const Layout &L = ds->layout;
    hipStream_t s = ds->ctx->stream;
    MPGEO_TRY(ds->tmp_b.ensure((size_t)ds->n * sizeof(double)));
    launch_unpad_vector(ds->y.as<double>(), ds->tmp_b.as<double>(), L.n, L.nb, L.nbp, s);
    MPGEO_HIP(hipGetLastError());
    MPGEO_HIP(hipMemcpyAsync(y, ds->tmp_b.ptr, (size_t)ds->n * sizeof(double), hipMemcpyDeviceToHost, s));
    MPGEO_HIP(hipStreamSynchronize(s));
    return MPGEO_OK;
}

int mpgeo_dataset_krige(mpgeo_dataset *ds, int64_t m, const double *new_locs, double *pred,
                        double *var) {
    if (!ds || m < 0 || (m > 0 && (!new_locs || !pred))) return MPGEO_E_ARG;
    if (!ds->has_factor) return MPGEO_E_ARG;
    if (var && m > 65535) return MPGEO_E_ARG;
    if (m == 0) return MPGEO_OK;
    Device dev(ds->ctx->device);
    hipStream_t s = ds->ctx->stream;
    const bool on_dev = (ds->flags & MPGEO_INPUT_DEVICE) != 0;
    MPGEO_TRY(check_finite(ds, new_locs, 2 * m, on_dev));
    // new sites and outputs on the device
    const size_t need = (size_t)m * 2 * sizeof(double) + 2 * (size_t)m * sizeof(double);
    MPGEO_TRY(ds->tmp_b.ensure(need));
    double *dnew = ds->tmp_b.as<double>();
    double *dpred = dnew + 2 * m;
    double *dvar = dpred + m;
    if (on_dev) MPGEO_HIP(hipMemcpyAsync(dnew, new_locs, (size_t)m * 2 * sizeof(double), hipMemcpyDeviceToDevice, s));
    else MPGEO_HIP(hipMemcpyAsync(dnew, new_locs, (size_t)m * 2 * sizeof(double), hipMemcpyHostToDevice, s));
    MPGEO_TRY(krige_enqueue(ds, m, dnew, dpred, var ? dvar : nullptr, ds->var_scale));
    const hipMemcpyKind kind = on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    MPGEO_HIP(hipMemcpyAsync(pred, dpred, (size_t)m * sizeof(double), kind, s));
    if (var) MPGEO_HIP(hipMemcpyAsync(var, dvar, (size_t)m * sizeof(double), kind, s));
    MPGEO_HIP(hipStreamSynchronize(s));
    return MPGEO_OK;
}

int mpgeo_dataset_entries(mpgeo_dataset *ds, int64_t count, const int64_t *rows,
                          const int64_t *cols, double *out) {
    if (!ds || count < 0 || (count > 0 && (!rows || !cols || !out)) || !ds->off.ptr)
        return MPGEO_E_ARG;
    if (count == 0) return MPGEO_OK;
    for (int64_t q = 0; q < count; ++q)
        if (rows[q] < 0 || rows[q] >= ds->n || cols[q] < 0 || cols[q] >= ds->n) return MPGEO_E_ARG;
    Device dev(ds->ctx->device);
    hipStream_t s = ds->ctx->stream;
    const size_t ib = (size_t)count * sizeof(int64_t);
    MPGEO_TRY(ds->tmp_b.ensure(2 * ib + (size_t)count * sizeof(double)));
    char *base = ds->tmp_b.as<char>();
    int64_t *drows = reinterpret_cast<int64_t *>(base);
    int64_t *dcols = reinterpret_cast<int64_t *>(base + ib);
    double *dout = reinterpret_cast<double *>(base + 2 * ib);
    MPGEO_HIP(hipMemcpyAsync(drows, rows, ib, hipMemcpyHostToDevice, s));
    MPGEO_HIP(hipMemcpyAsync(dcols, cols, ib, hipMemcpyHostToDevice, s));
    launch_entries(tile_map(ds), count, drows, dcols, dout, s);
    MPGEO_HIP(hipGetLastError());
    MPGEO_HIP(hipMemcpyAsync(out, dout, (size_t)count * sizeof(double), hipMemcpyDeviceToHost, s));
    MPGEO_HIP(hipStreamSynchronize(s));
    return MPGEO_OK;
}

// The Nelder-Mead search of mpgeo_dataset_mle; with trace != NULL every evaluated theta (and
// its log-likelihood, -inf where not positive definite) is recorded in evaluation order.
static int dataset_mle(mpgeo_dataset *ds, mpgeo_theta start, mpgeo_plan plan, double xtol, double ftol,
                       int32_t max_evals, mpgeo_theta *theta_hat, double *loglik_hat, int32_t *evals_out,
                       int32_t *iters_out, mpgeo_theta *trace, double *trace_loglik) {
    if (!ds || max_evals < 4 || !(xtol >= 0.0) || !(ftol >= 0.0)) return MPGEO_E_ARG;
    MPGEO_TRY(check_theta(start));
    MPGEO_TRY(check_plan(plan));
    Device dev(ds->ctx->device);
    if (!dev.ok) return MPGEO_E_DEVICE;
    static const double lo[3] = {0.01, 0.001, 0.1};
    static const double hi[3] = {10.0, 2.0, 3.0};
    // the simplex lives in log-parameter space: (theta1, theta2, theta3), or (theta2, theta3)
    // for the profile likelihood, whose theta1 is then q~/n at the best point
    const bool profile = (plan.flags & MPGEO_PROFILE) != 0;
    const int dim = profile ? 2 : 3;
    const int first = profile ? 1 : 0;
    auto to_theta = [&](const double *u) {
        double t[3] = {1.0, 1.0, 1.0};
        for (int q = 0; q < dim; ++q)
            t[first + q] = std::min(std::max(std::exp(u[q]), lo[first + q]), hi[first + q]);
        return mpgeo_theta{t[0], t[1], t[2]};
    };
    int hard_error = MPGEO_OK;
    // objective: -loglik; a non-positive-definite point scores +infinity
    int traced = 0;
    auto f = [&](const double *u) -> double {
        mpgeo_result r{};
        const mpgeo_theta th = to_theta(u);
        const int st = evaluate_escalating(ds, th, plan, &r, nullptr);
        if (trace && traced < max_evals) {
            trace[traced] = th;
            if (trace_loglik) trace_loglik[traced] = (st == MPGEO_OK) ? r.loglik : -INFINITY;
            ++traced;
        }
        if (st == MPGEO_OK) return -r.loglik;
        if (st != MPGEO_E_NOT_SPD && hard_error == MPGEO_OK) hard_error = st;
        return INFINITY;
    };
    const int nv = dim + 1;
    double x[4][3] = {};
    double fv[4];
    const double start_t[3] = {start.sigma2, start.beta, start.nu};
    for (int v = 0; v < nv; ++v)
        for (int q = 0; q < dim; ++q)
            x[v][q] = std::log(start_t[first + q]) + ((v > 0 && q == v - 1) ? 0.1 : 0.0);
    int evals = 0, iters = 0;
    for (int v = 0; v < nv; ++v) {
        fv[v] = f(x[v]);
        ++evals;
    }
    const size_t row = sizeof(x[0]);
    while (evals < max_evals && hard_error == MPGEO_OK) {
        int order[4] = {0, 1, 2, 3};
        std::stable_sort(order, order + nv, [&](int a, int b) { return fv[a] < fv[b]; });
        double xs[4][3] = {}, fs[4];
        for (int v = 0; v < nv; ++v) {
            fs[v] = fv[order[v]];
            for (int q = 0; q < dim; ++q) xs[v][q] = x[order[v]][q];
        }
        std::memcpy(x, xs, sizeof(x));
        std::memcpy(fv, fs, sizeof(fv));
        double span = 0.0;
        for (int v = 1; v < nv; ++v)
            for (int q = 0; q < dim; ++q) span = std::max(span, std::fabs(x[v][q] - x[0][q]));
        if (span < xtol || (ftol > 0.0 && std::fabs(fv[dim] - fv[0]) <= ftol * std::fabs(fv[0]))) break;
        ++iters;
        const int w = dim;   // worst vertex
        double c[3] = {}, xr[3] = {}, xe[3] = {}, xc[3] = {};
        for (int q = 0; q < dim; ++q) {
            for (int v = 0; v < dim; ++v) c[q] += x[v][q];
            c[q] /= (double)dim;
        }
        for (int q = 0; q < dim; ++q) xr[q] = c[q] + (c[q] - x[w][q]);
        const double fr = f(xr);
        ++evals;
        if (fr < fv[0]) {
            for (int q = 0; q < dim; ++q) xe[q] = c[q] + 2.0 * (c[q] - x[w][q]);
            const double fe = f(xe);
            ++evals;
            if (fe < fr) {
                std::memcpy(x[w], xe, row);
                fv[w] = fe;
            } else {
                std::memcpy(x[w], xr, row);
                fv[w] = fr;
            }
            continue;
        }
        if (fr < fv[w - 1]) {
            std::memcpy(x[w], xr, row);
            fv[w] = fr;
            continue;
        }
        if (fr < fv[w]) {
            for (int q = 0; q < dim; ++q) xc[q] = c[q] + 0.5 * (xr[q] - c[q]);   // outside
            const double fc = f(xc);
            ++evals;
            if (fc <= fr) {
                std::memcpy(x[w], xc, row);
                fv[w] = fc;
                continue;
            }
        } else {
            for (int q = 0; q < dim; ++q) xc[q] = c[q] + 0.5 * (x[w][q] - c[q]);   // inside
            const double fc = f(xc);
            ++evals;
            if (fc < fv[w]) {
                std::memcpy(x[w], xc, row);
                fv[w] = fc;
                continue;
            }
        }
        for (int v = 1; v < nv; ++v) {   // shrink towards the best vertex
            for (int q = 0; q < dim; ++q) x[v][q] = x[0][q] + 0.5 * (x[v][q] - x[0][q]);
            fv[v] = f(x[v]);
            ++evals;
        }
    }
    if (hard_error != MPGEO_OK) return hard_error;
    int best = 0;
    for (int v = 1; v < nv; ++v)
        if (fv[v] < fv[best]) best = v;
    if (!std::isfinite(fv[best])) return MPGEO_E_NOT_SPD;
    mpgeo_theta th = to_theta(x[best]);
    mpgeo_result r{};
    MPGEO_TRY(evaluate_escalating(ds, th, plan, &r, nullptr));   // leave the factor of theta_hat resident
    if (profile) th.sigma2 = r.quad / (double)ds->layout.n;
    if (theta_hat) *theta_hat = th;
    if (loglik_hat) *loglik_hat = r.loglik;
    if (evals_out) *evals_out = evals;
    if (iters_out) *iters_out = iters;
    return MPGEO_OK;
}

int mpgeo_dataset_mle(mpgeo_dataset *ds, mpgeo_theta start, mpgeo_plan plan, double xtol,
                      double ftol, int32_t max_evals, mpgeo_theta *theta_hat, double *loglik_hat,
                      int32_t *evals_out, int32_t *iters_out) {
    return dataset_mle(ds, start, plan, xtol, ftol, max_evals, theta_hat, loglik_hat, evals_out, iters_out,
                       nullptr, nullptr);
}

int mpgeo_dataset_mle_trace(mpgeo_dataset *ds, mpgeo_theta start, mpgeo_plan plan, double xtol,
                            double ftol, int32_t max_evals, mpgeo_theta *theta_hat, double *loglik_hat,
                            int32_t *evals_out, int32_t *iters_out, mpgeo_theta *trace,
                            double *trace_loglik) {
    if (!trace) return MPGEO_E_ARG;
    return dataset_mle(ds, start, plan, xtol, ftol, max_evals, theta_hat, loglik_hat, evals_out, iters_out,
                       trace, trace_loglik);
}

int mpgeo_dataset_simulate(mpgeo_dataset *ds, mpgeo_theta theta, mpgeo_plan plan,
                           const double *eps, double *z_out) {
    if (!ds || !eps || !z_out || (plan.flags & MPGEO_PROFILE)) return MPGEO_E_ARG;
    MPGEO_TRY(check_theta(theta));
    MPGEO_TRY(check_plan(plan));
    Device dev(ds->ctx->device);
    if (!dev.ok) return MPGEO_E_DEVICE;
    hipStream_t s = ds->ctx->stream;
    const int64_t n = ds->n;
    const bool on_dev = (ds->flags & MPGEO_INPUT_DEVICE) != 0;
    MPGEO_TRY(check_finite(ds, eps, n, on_dev));
    // factor Sigma(theta) with a zero data vector (the dataset's z is kept aside)
    DevBuf saved_z;
    MPGEO_TRY(saved_z.ensure((size_t)n * sizeof(double)));
    MPGEO_HIP(hipMemcpyAsync(saved_z.ptr, ds->z.ptr, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s));
    MPGEO_HIP(hipMemsetAsync(ds->z.ptr, 0, (size_t)n * sizeof(double), s));
    mpgeo_result r{};
    int st = evaluate_escalating(ds, theta, plan, &r, nullptr);
    (void)hipMemcpyAsync(ds->z.ptr, saved_z.ptr, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, s);
    if (st != MPGEO_OK) {
        (void)hipStreamSynchronize(s);
        saved_z.release();
        ds->has_factor = false;
        return st;
    }
    const Layout &L = ds->layout;
    const size_t vec = (size_t)L.p * L.nbp;
    MPGEO_TRY(ds->tmp_a.ensure(2 * vec * sizeof(double) + 2 * (size_t)n * sizeof(double)));
    double *eps_phys = ds->tmp_a.as<double>();
    double *z_phys = eps_phys + vec;
    double *lin_a = z_phys + vec;
    double *lin_b = lin_a + n;
    MPGEO_HIP(hipMemcpyAsync(lin_a, eps, (size_t)n * sizeof(double),
                             on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    launch_permute(lin_a, lin_b, ds->perm.as<int64_t>(), n, false, s);        // ordered eps
    launch_pad_vector(lin_b, eps_phys, n, L.nb, L.nbp, L.p, s);
    launch_trmv(tile_map(ds), eps_phys, z_phys, s);
    launch_unpad_vector(z_phys, lin_b, n, L.nb, L.nbp, s);
    launch_permute(lin_b, lin_a, ds->perm.as<int64_t>(), n, true, s);         // caller order
    MPGEO_HIP(hipGetLastError());
    MPGEO_HIP(hipMemcpyAsync(z_out, lin_a, (size_t)n * sizeof(double),
                             on_dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s));
    MPGEO_HIP(hipStreamSynchronize(s));
    saved_z.release();
    return MPGEO_OK;
}

int mpgeo_factor_dense(mpgeo_ctx *ctx, int64_t n, const double *a, int64_t lda, const double *z,
                       mpgeo_plan plan, mpgeo_result *out) {
    if (!ctx || !out || !a || n < 1 || lda < n) return MPGEO_E_ARG;
    if ((plan.flags & MPGEO_PROFILE) && !z) return MPGEO_E_ARG;
    out->info = -1;
    MPGEO_TRY(check_plan(plan));
    if (plan.dist64 > 0.0) return MPGEO_E_ARG;   // a distance map needs sites
    Device dev(ctx->device);
    if (!dev.ok) return MPGEO_E_DEVICE;
    mpgeo_dataset ds;
    ds.ctx = ctx;
    ds.n = n;
    ds.profile = (plan.flags & MPGEO_PROFILE) != 0;
    hipStream_t s = ctx->stream;
    const bool on_dev = (plan.flags & MPGEO_INPUT_DEVICE) != 0;
    int st = MPGEO_OK;
    // the lower triangle and z must be finite
    if (!on_dev) {
        for (int64_t c = 0; c < n && st == MPGEO_OK; ++c)
            if (!all_finite(a + c * lda + c, (size_t)(n - c))) st = MPGEO_E_ARG;
        if (st == MPGEO_OK && z && !all_finite(z, (size_t)n)) st = MPGEO_E_ARG;
    } else {
        st = ds.chk.ensure(sizeof(int));
        int flag = 0;
        if (st == MPGEO_OK && hipMemsetAsync(ds.chk.ptr, 0, sizeof(int), s) != hipSuccess) st = MPGEO_E_DEVICE;
        if (st == MPGEO_OK) {
            launch_find_nonfinite(a, n, n, lda, true, ds.chk.as<int>(), s);
            if (z) launch_find_nonfinite(z, n, 1, n, false, ds.chk.as<int>(), s);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(&flag, ds.chk.ptr, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess)
                st = MPGEO_E_DEVICE;
            else if (flag) st = MPGEO_E_ARG;
        }
    }
    const double *da = a;
    if (st == MPGEO_OK && !on_dev) {
        st = ds.tmp_a.ensure((size_t)lda * n * sizeof(double));
        if (st == MPGEO_OK && hipMemcpyAsync(ds.tmp_a.ptr, a, (size_t)lda * n * sizeof(double),
                                             hipMemcpyHostToDevice, s) != hipSuccess)
            st = MPGEO_E_DEVICE;
        da = ds.tmp_a.as<double>();
    }
    if (st == MPGEO_OK) st = ds.z.ensure((size_t)n * sizeof(double));
    if (st == MPGEO_OK) {
        hipError_t e;
        if (!z) e = hipMemsetAsync(ds.z.ptr, 0, (size_t)n * sizeof(double), s);
        else e = hipMemcpyAsync(ds.z.ptr, z, (size_t)n * sizeof(double),
                                on_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
        if (e != hipSuccess) st = MPGEO_E_DEVICE;
    }
    // Algorithm 1 on the imported tiles; with MPGEO_ESCALATE, again with wider bands after a
    // non-positive pivot
    mpgeo_plan pl = plan;
    const int64_t p = (n + plan.tile - 1) / plan.tile;
    for (int esc = 0; st == MPGEO_OK; ++esc) {
        st = prepare_layout(&ds, pl);
        if (st != MPGEO_OK) break;
        ctx->timing = (pl.flags & MPGEO_TIMING) != 0;
        EventSet ev;
        if (ev.ok) (void)hipEventRecord(ev.e[0], s);
        launch_import_dense(tile_map(&ds), da, lda, ds.all.as<TileIJ>(), (int64_t)ds.layout.all.size(), s);
        if (ev.ok) (void)hipEventRecord(ev.e[1], s);
        st = status_from(hipGetLastError());
        if (st == MPGEO_OK) st = run_factor(&ds, ev.ok ? ev.e[2] : nullptr);
        if (ev.ok) (void)hipEventRecord(ev.e[3], s);
        if (st == MPGEO_OK) {
            st = read_result(&ds, out);
            out->t_covgen = ev.secs(0, 1);
            out->t_factor = ev.secs(1, 2);
            out->t_solve = ev.secs(2, 3);
            out->t_total = ev.secs(0, 3);
            out->band64 = pl.band64;
            out->band32 = pl.band32;
            out->band0 = pl.band0;
            out->escalations = esc;
        }
        ctx->collect();
        ctx->timing = false;
        if (st != MPGEO_E_NOT_SPD || !(pl.flags & MPGEO_ESCALATE) || !escalate_plan(pl, p)) break;
        st = MPGEO_OK;
    }
    (void)hipStreamSynchronize(s);
    for (DevBuf *b : {&ds.pool64, &ds.pool32, &ds.off, &ds.all, &ds.list64, &ds.list32, &ds.list16,
                      &ds.bulk16, &ds.bulk16k0, &ds.q16, &ds.qscale, &ds.p64,
                      &ds.p32, &ds.linv, &ds.linv32, &ds.r, &ds.y, &ds.parts, &ds.info, &ds.result,
                      &ds.tmp_a, &ds.z, &ds.chk})
        b->release();
    return st;
}

// ---- batched evaluation of independent instances ------------------------------------------
// Lanes are private contexts (own two streams, events and workspace); instances are dealt to
// them largest first so that each lane's buffers reach their final size early, and every
// evaluation is enqueued without a host synchronisation.  The tile size of an instance is the
// plan's, or, with plan.tile = 0, the autotuner's choice for its half-octave of n.

static int batch_lanes(mpgeo_ctx *ctx, int want) {
    while ((int)ctx->lanes.size() < want) {
        mpgeo_ctx *c = nullptr;
        MPGEO_TRY(mpgeo_ctx_create(&c, ctx->device, nullptr, ctx->hbm_budget));
        // Lanes overlap whole evaluations with each other; a third stream per lane only adds
        // small launches and queues (the hardware has few), so a lane's column k+2 updates
        // stay on its bulk stream.
        if (c->next) {
            (void)hipStreamDestroy(c->next);
            c->next = nullptr;
        }
        ctx->lanes.push_back(c);
        mpgeo_dataset *d = new mpgeo_dataset();
        d->ctx = c;
        ctx->lane_ds.push_back(d);
    }
    return MPGEO_OK;
}

// One evaluation enqueued on a lane; {loglik, logdet, quad, info bits} land in res_slot.  The
// lane's previous evaluation is waited for first: its work lists were uploaded from the host
// copy of the layout that this one rebuilds (so at most one evaluation per lane is in flight,
// and the lanes keep the device busy together).
static int batch_enqueue(mpgeo_dataset *ds, const mpgeo_instance &in, const mpgeo_plan &pl,
                         double *res_slot) {
    MPGEO_HIP(hipStreamSynchronize(ds->ctx->side));
    MPGEO_HIP(hipStreamSynchronize(ds->ctx->stream));
    ds->n = in.n;
    ds->flags = pl.flags | MPGEO_ORDER_MORTON;
    MPGEO_TRY(load_inputs(ds, in.locs, in.z, ds->flags));
    MPGEO_TRY(prepare_layout(ds, pl));
    ds->profile = (pl.flags & MPGEO_PROFILE) != 0;
    mpgeo_theta th = in.theta;
    if (ds->profile) th.sigma2 = 1.0;
    MPGEO_TRY(run_covgen(ds, th));
    MPGEO_TRY(run_factor(ds, nullptr));
    hipStream_t s = ds->ctx->stream;
    MPGEO_HIP(hipMemcpyAsync(res_slot, ds->result.ptr, 3 * sizeof(double), hipMemcpyDeviceToDevice, s));
    MPGEO_HIP(hipMemcpyAsync(res_slot + 3, ds->info.ptr, sizeof(double), hipMemcpyDeviceToDevice, s));
    ds->has_factor = false;   // the lane's workspace is reused by the next instance
    return MPGEO_OK;
}

static void batch_sync(mpgeo_ctx *ctx) {
    for (auto *c : ctx->lanes) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamSynchronize(c->stream);
    }
}

// Tile size for an instance: the plan's, else the fastest of the candidates measured on the
// first instance of its (half-octave of n, precision plan) class.  Candidates: one tile
// covering the problem when it fits, and 128, 256, 384, 512 below n.
constexpr double kTileTieMargin = 0.05;

static int batch_tile(mpgeo_ctx *ctx, const mpgeo_instance &in, mpgeo_plan pl, double *probe_out,
                      int *tile_out) {
    if (pl.tile > 0) {
        *tile_out = pl.tile;
        return MPGEO_OK;
    }
    const int bucket = (int)std::floor(2.0 * std::log2((double)in.n));
    const std::string key = std::to_string(bucket) + "/" + std::to_string(pl.band64) + "/" +
                            std::to_string(pl.band32) + "/" + std::to_string(pl.lowp) + "/" +
                            std::to_string(pl.flags & (MPGEO_PROFILE | MPGEO_DIST_GCD)) + "/" +
                            std::to_string(pl.band0);
    auto it = ctx->tuned_tile.find(key);
    if (it != ctx->tuned_tile.end()) {
        *tile_out = it->second;
        return MPGEO_OK;
    }
    std::vector<int> cand;
    cand.push_back((int)std::min<int64_t>(in.n, kMaxTile));
    for (int t : {128, 256, 384, 512})
        if (t < in.n && t != cand[0]) cand.push_back(t);
    mpgeo_dataset *ds = ctx->lane_ds[0];
    hipStream_t st = ctx->lanes[0]->stream;
    EventSet ev;
    std::vector<double> secs(cand.size(), INFINITY);
    for (size_t c = 0; c < cand.size(); ++c) {
        mpgeo_plan q = pl;
        q.tile = cand[c];
        MPGEO_TRY(batch_enqueue(ds, in, q, probe_out));   // warm-up (allocations, layout)
        batch_sync(ctx);
        for (int rep = 0; rep < 2; ++rep) {               // the faster of two timed runs
            if (ev.ok) MPGEO_HIP(hipEventRecord(ev.e[0], st));
            MPGEO_TRY(batch_enqueue(ds, in, q, probe_out));
            if (ev.ok) MPGEO_HIP(hipEventRecord(ev.e[1], st));
            batch_sync(ctx);
            secs[c] = std::min(secs[c], ev.secs(0, 1));
        }
    }
    // the largest tile within kTileTieMargin of the fastest: timing noise between near-equal
    // candidates then rarely flips the choice (a mixed plan's bands count tiles, so its l
    // follows the tile)
    const double fastest = *std::min_element(secs.begin(), secs.end());
    int best = 0;
    for (size_t c = 0; c < cand.size(); ++c)
        if (secs[c] <= fastest * (1.0 + kTileTieMargin) && cand[c] > best) best = cand[c];
    ctx->tuned_tile[key] = best;
    *tile_out = best;
    return MPGEO_OK;
}

// The band tuner (MPGEO_TUNE_BAND): its policy is in tune_policy.h.
static int batch_queue(mpgeo_ctx *ctx, int64_t count, const mpgeo_instance *inst, const mpgeo_plan &plan,
                       mpgeo_result *out, int32_t *tiles, char *arena, size_t arena_bytes,
                       const int32_t *bands);

// A class of the band tuner: band_class_key (n, smoothness, range), tile, path, flags.
static std::string band_class(const mpgeo_instance &in, const mpgeo_plan &pl, int tile, bool queue) {
    return band_class_key(in.n, in.theta.beta, in.theta.nu) + "/" + std::to_string(tile) + "/" +
           (queue ? "q" : "l") + "/" + std::to_string(pl.flags & (MPGEO_PROFILE | MPGEO_DIST_GCD));
}

// Tunes one class on its probe problems: each is evaluated all-FP64 and at every candidate band
// below its last tile row (one queue launch for all of them, or one lane evaluation each); the
// narrowest candidate at which every probe factors and stays within kTuneBandBar of its
// all-FP64 result (relative to its terms) is the class's band, the largest such error its
// error; all-FP64 (-1) when no candidate is.  Depends only on the probes' deterministic results.
static int band_probe(mpgeo_ctx *ctx, const std::vector<const mpgeo_instance *> &probes, mpgeo_plan pl, int tile,
                      bool queue, double *probe_out, TunedBand *tb) {
    int64_t pmax = 0;
    for (const mpgeo_instance *in : probes) pmax = std::max<int64_t>(pmax, (in->n + tile - 1) / tile);
    const std::vector<int> cand = band_candidates(pmax);
    const size_t np = probes.size(), nc = cand.size();
    std::vector<mpgeo_result> r(np * nc);   // [candidate][probe]
    pl.tile = tile;
    pl.flags &= ~(uint32_t)MPGEO_TUNE_BAND;
    if (queue) {
        std::vector<mpgeo_instance> all(np * nc);
        std::vector<int32_t> bands(np * nc);
        for (size_t c = 0; c < nc; ++c)
            for (size_t k = 0; k < np; ++k) {
                all[c * np + k] = *probes[k];
                bands[c * np + k] = cand[c];
            }
        const int st = batch_queue(ctx, (int64_t)all.size(), all.data(), pl, r.data(), nullptr, nullptr, 0, bands.data());
        if (st != MPGEO_OK && st != MPGEO_E_NOT_SPD) return st;
    } else {
        for (size_t c = 0; c < nc; ++c)
            for (size_t k = 0; k < np; ++k) {
                mpgeo_plan q = pl;
                q.band64 = cand[c];
                const int st = batch_enqueue(ctx->lane_ds[0], *probes[k], q, probe_out);
                batch_sync(ctx);
                if (st != MPGEO_OK) return st;
                double host[4];
                MPGEO_HIP(hipMemcpy(host, probe_out, sizeof(host), hipMemcpyDeviceToHost));
                unsigned long long info;
                std::memcpy(&info, host + 3, sizeof(info));
                mpgeo_result &o = r[c * np + k];
                o.loglik = host[0];
                o.logdet = host[1];
                o.quad = host[2];
                o.info = info == ~0ull ? -1 : (int64_t)info;
            }
    }
    std::vector<ProbeResult> pr(r.size());
    for (size_t e = 0; e < r.size(); ++e) pr[e] = ProbeResult{r[e].loglik, r[e].logdet, r[e].quad, r[e].info < 0};
    std::vector<int64_t> sizes(np);
    for (size_t k = 0; k < np; ++k) sizes[k] = probes[k]->n;
    choose_band(cand, sizes, pr, (pl.flags & MPGEO_PROFILE) != 0, &tb->band, &tb->err);
    return MPGEO_OK;
}

// The tuned band and class error of each instance (tile[i] its tile): classes not yet in the
// context are probed on their first kTuneProbes problems of this call, then kept for later
// batches.
static int tune_bands(mpgeo_ctx *ctx, int64_t count, const mpgeo_instance *inst, const mpgeo_plan &pl,
                      const std::vector<int> &tile, bool queue, double *probe_out, std::vector<int32_t> &band,
                      std::vector<double> &err) {
    std::vector<std::string> key((size_t)count);
    std::vector<std::string> order;   // new classes in order of first appearance
    std::map<std::string, std::vector<const mpgeo_instance *>> probes;
    std::map<std::string, int> probe_tile;
    for (int64_t i = 0; i < count; ++i) {
        key[(size_t)i] = band_class(inst[i], pl, tile[(size_t)i], queue);
        if (ctx->tuned_band.count(key[(size_t)i])) continue;
        auto &v = probes[key[(size_t)i]];
        if (v.empty()) {
            order.push_back(key[(size_t)i]);
            probe_tile[key[(size_t)i]] = tile[(size_t)i];
        }
        if ((int)v.size() < kTuneProbes) v.push_back(inst + i);
    }
    for (const std::string &k : order) {
        TunedBand tb;
        MPGEO_TRY(band_probe(ctx, probes[k], pl, probe_tile[k], queue, probe_out, &tb));
        ctx->tuned_band[k] = tb;
    }
    band.resize((size_t)count);
    err.resize((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        const TunedBand &tb = ctx->tuned_band[key[(size_t)i]];
        band[(size_t)i] = tb.band;
        err[(size_t)i] = tb.err;
    }
    return MPGEO_OK;
}

// The problems of a tuned batch to evaluate again all-FP64 for accuracy: factored at a band
// (not all-FP64) with an l too small against its terms for the class error err[i].
static std::vector<int64_t> accuracy_reruns(int64_t count, const mpgeo_instance *inst, const mpgeo_result *out,
                                            const std::vector<double> &err, bool profile) {
    std::vector<int64_t> redo;
    for (int64_t i = 0; i < count; ++i) {
        const mpgeo_result &o = out[i];
        if (needs_fp64_rerun(inst[i].n, o.loglik, o.logdet, o.quad, o.info < 0, o.band64, err[(size_t)i], profile))
            redo.push_back(i);
    }
    return redo;
}

// The persistent task-queue batch (MPGEO_BATCH_QUEUE): problems are packed into shared buffers
// in groups that fit in device memory, each group one ordering launch and one queue launch.
// The work buffers of a group come either from the context's growing buffers or from a fixed
// device array of `arena_bytes` at `arena` (nothing is
// allocated; every group must fit in the array, and what must start at zero is cleared by a
// fill kernel).
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static int64_t queue_p(int64_t n) { return (n + kQueueTile - 1) / kQueueTile; }

// FP64 band of a problem of n sites in tiles: the requested one, capped at p (every tile)
static int32_t queue_band(int64_t n, int32_t band) {
    const int64_t p = queue_p(n);
    return (int32_t)((band < 0 || band > p) ? p : band);
}

// bytes of the tiles of a problem: FP64 tiles 8 bytes per entry, FP32 tiles 4
static size_t queue_tile_bytes(int64_t n, int32_t band) {
    return (size_t)queue_tile_units(queue_p(n), 0, queue_band(n, band)) * sizeof(float);
}

// bytes of every work buffer a problem adds to a group (the fixed array's packing rule)
static size_t queue_prob_bytes(int64_t n, int32_t band) {
    const int64_t te = (int64_t)kQueueTile * kQueueTile;
    const int64_t p = queue_p(n), tl = p * (p + 1) / 2;
    return (size_t)n * 5 * sizeof(double) +                    // packed inputs, ordered sites
           (size_t)3 * p * kQueueTile * sizeof(double) +        // z, r, y (padded)
           queue_tile_bytes(n, band) + (size_t)p * te * sizeof(double) +   // tiles, diagonal inverses
           (size_t)2 * p * sizeof(double) +                     // logdet / quad parts
           (size_t)tl * (sizeof(int) + sizeof(BatchTask)) +     // done flags, tasks
           sizeof(BatchInst) + 3 * sizeof(double) + sizeof(unsigned long long);
}
constexpr size_t kQueueSlack = 13 * 256 + 2 * sizeof(int);     // alignment of 13 buffers, control

// Host side of one queued group (layout, task list, packed inputs: kept until the group's
// copies and launches have completed) and where its results land on the device.
struct QueueGroup {
    std::vector<BatchInst> bi;
    std::vector<BatchTask> tasks;
    std::vector<double> hl, hz;
    double *res = nullptr;               // loglik, logdet, quad per problem
    unsigned long long *info = nullptr;  // failing column per problem, all ones if none
    int *ctrl = nullptr;                 // task counter, abort flag
};

// Lays out problems inst[0 .. gc) (FP64 band of each in bands[]) as one group, uploads their
// inputs and enqueues the ordering launch and the queue launch on stream s without waiting.
static int queue_group_enqueue(mpgeo_ctx *ctx, hipStream_t s, const mpgeo_instance *const *inst, int64_t gc,
                               const int32_t *bands, const mpgeo_plan &plan, char *arena, size_t arena_bytes,
                               QueueGroup &G, int max_workgroups = 0) {
    const int64_t te = (int64_t)kQueueTile * kQueueTile;
    const bool fixed = arena != nullptr;
    G.bi.assign((size_t)gc, BatchInst{});
    int64_t pts = 0, tl = 0, lv = 0, vec = 0, prt = 0, units = 0;
    int max_n = 1, max_p = 1;
    for (int64_t q = 0; q < gc; ++q) {
        const mpgeo_instance &x = *inst[q];
        BatchInst &b = G.bi[(size_t)q];
        b.n = x.n;
        b.p = (int32_t)queue_p(x.n);
        b.band = queue_band(x.n, bands[q]);
        b.in0 = pts;
        b.tile0 = units;
        b.flag0 = tl;
        b.linv0 = lv;
        b.vec0 = vec;
        b.part0 = prt;
        b.mp = make_matern_params((plan.flags & MPGEO_PROFILE) ? 1.0 : x.theta.sigma2, x.theta.beta, x.theta.nu);
        b.mp.gcd = (plan.flags & MPGEO_DIST_GCD) ? 1 : 0;
        pts += x.n;
        tl += (int64_t)b.p * (b.p + 1) / 2;
        units += queue_tile_units(b.p, 0, b.band);
        lv += b.p;
        vec += (int64_t)b.p * kQueueTile;
        prt += 2 * (int64_t)b.p;
        max_n = std::max<int>(max_n, (int)x.n);
        max_p = std::max<int>(max_p, b.p);
    }
    // tasks: column by column; in a column the diagonal tiles of every problem, then the rest
    G.tasks.clear();
    G.tasks.reserve((size_t)tl);
    for (int j = 0; j < max_p; ++j) {
        for (int64_t q = 0; q < gc; ++q)
            if (j < G.bi[(size_t)q].p) G.tasks.push_back({(int32_t)q, j, j, 0});
        for (int64_t q = 0; q < gc; ++q)
            for (int i = j + 1; i < G.bi[(size_t)q].p; ++i) G.tasks.push_back({(int32_t)q, i, j, 0});
    }
    G.hl.assign((size_t)pts * 2, 0.0);
    G.hz.assign((size_t)pts, 0.0);
    for (int64_t q = 0; q < gc; ++q) {
        const mpgeo_instance &x = *inst[q];
        std::memcpy(G.hl.data() + 2 * G.bi[(size_t)q].in0, x.locs, (size_t)x.n * 2 * sizeof(double));
        std::memcpy(G.hz.data() + G.bi[(size_t)q].in0, x.z, (size_t)x.n * sizeof(double));
    }
    // ---- buffers -----------------------------------------------------------------------------------
    const size_t sz[13] = {G.hl.size() * sizeof(double), G.hz.size() * sizeof(double), G.hl.size() * sizeof(double),
                           3 * (size_t)vec * sizeof(double), (size_t)units * sizeof(float),
                           (size_t)lv * te * sizeof(double), (size_t)prt * sizeof(double),
                           (size_t)tl * sizeof(int), 2 * sizeof(int), (size_t)gc * sizeof(BatchInst),
                           G.tasks.size() * sizeof(BatchTask), (size_t)gc * 3 * sizeof(double),
                           (size_t)gc * sizeof(unsigned long long)};
    void *ptr[13];
    if (fixed) {   // carved from the fixed array, 256-byte aligned
        size_t off = 0;
        for (int q = 0; q < 13; ++q) {
            ptr[q] = arena + off;
            off += align256(sz[q]);
        }
        if (off > arena_bytes) return MPGEO_E_TOO_LARGE;   // (the packing rule keeps it inside)
    } else {   // grow only; growing waits for the device
        DevBuf *bufs[13] = {&ctx->q_in_locs, &ctx->q_in_z, &ctx->q_locs, &ctx->q_vec, &ctx->q_tiles,
                            &ctx->q_linv, &ctx->q_parts, &ctx->q_flags, &ctx->q_ctrl, &ctx->q_insts,
                            &ctx->q_tasks, &ctx->q_res, &ctx->q_info};
        for (int q = 0; q < 13; ++q) {
            MPGEO_TRY(bufs[q]->ensure(sz[q]));
            ptr[q] = bufs[q]->ptr;
        }
    }
    double *in_locs = static_cast<double *>(ptr[0]), *in_z = static_cast<double *>(ptr[1]);
    double *q_locs = static_cast<double *>(ptr[2]), *q_vec = static_cast<double *>(ptr[3]);
    int *q_flags = static_cast<int *>(ptr[7]), *q_ctrl = static_cast<int *>(ptr[8]);
    BatchInst *q_insts = static_cast<BatchInst *>(ptr[9]);
    BatchTask *q_tasks = static_cast<BatchTask *>(ptr[10]);
    G.res = static_cast<double *>(ptr[11]);
    G.info = static_cast<unsigned long long *>(ptr[12]);
    G.ctrl = q_ctrl;
    MPGEO_HIP(hipMemcpyAsync(in_locs, G.hl.data(), sz[0], hipMemcpyHostToDevice, s));
    MPGEO_HIP(hipMemcpyAsync(in_z, G.hz.data(), sz[1], hipMemcpyHostToDevice, s));
    MPGEO_HIP(hipMemcpyAsync(q_insts, G.bi.data(), sz[9], hipMemcpyHostToDevice, s));
    MPGEO_HIP(hipMemcpyAsync(q_tasks, G.tasks.data(), sz[10], hipMemcpyHostToDevice, s));
    if (fixed) {   // the array keeps the previous call's contents: clear flags, counter, info
        launch_fill_u32(reinterpret_cast<uint32_t *>(q_flags), 0u, (size_t)tl, s);
        launch_fill_u32(reinterpret_cast<uint32_t *>(q_ctrl), 0u, 2, s);
        launch_fill_u32(reinterpret_cast<uint32_t *>(G.info), ~0u, 2 * (size_t)gc, s);
        MPGEO_HIP(hipGetLastError());
    } else {
        MPGEO_HIP(hipMemsetAsync(q_flags, 0, sz[7], s));
        MPGEO_HIP(hipMemsetAsync(q_ctrl, 0, sz[8], s));
        MPGEO_HIP(hipMemsetAsync(G.info, 0xFF, sz[12], s));
    }
    launch_batch_order(q_insts, gc, max_n, in_locs, in_z, q_locs, q_vec,
                       true, (plan.flags & MPGEO_DIST_GCD) != 0, s);   // always ordered, as a lane would
    MPGEO_HIP(hipGetLastError());
    QueueArgs qa{};
    qa.tasks = q_tasks;
    qa.ntasks = (int64_t)G.tasks.size();
    qa.insts = q_insts;
    qa.locs = q_locs;
    qa.z = q_vec;
    qa.r = q_vec + vec;
    qa.y = q_vec + 2 * vec;
    qa.tiles = static_cast<float *>(ptr[4]);
    qa.linv = static_cast<double *>(ptr[5]);
    qa.parts = static_cast<double *>(ptr[6]);
    qa.flags = q_flags;
    qa.head = reinterpret_cast<unsigned *>(q_ctrl);
    qa.abort_flag = q_ctrl + 1;
    qa.info = G.info;
    qa.result = G.res;
    qa.profile = (plan.flags & MPGEO_PROFILE) ? 1 : 0;
    qa.spin_limit = 8 << 20;   // about 2 s of sleeps per wait
    const int cus = ctx->cus > 0 ? ctx->cus : 256;
    const int cap = max_workgroups > 0 ? std::min(max_workgroups, cus) : cus;
    const int wgs = (int)std::min<int64_t>((int64_t)G.tasks.size(), (int64_t)cap);
    launch_batch_queue(qa, wgs, s);
    MPGEO_HIP(hipGetLastError());
    return MPGEO_OK;
}

static int batch_queue(mpgeo_ctx *ctx, int64_t count, const mpgeo_instance *inst, const mpgeo_plan &plan,
                       mpgeo_result *out, int32_t *tiles, char *arena, size_t arena_bytes,
                       const int32_t *bands) {
    std::vector<int32_t> band((size_t)count);
    for (int64_t q = 0; q < count; ++q) band[(size_t)q] = bands ? bands[q] : plan.band64;
    const bool fixed = arena != nullptr;
    size_t budget = 0;
    if (fixed) {
        for (int64_t q = 0; q < count; ++q)
            if (queue_prob_bytes(inst[q].n, band[(size_t)q]) + kQueueSlack > arena_bytes)
                return MPGEO_E_TOO_LARGE;   // beyond the array
    } else {
        const int64_t te = (int64_t)kQueueTile * kQueueTile;
        size_t free_b = 0, total_b = 0;
        MPGEO_HIP(hipMemGetInfo(&free_b, &total_b));
        // tiles dominate: keep a group's tiles within half of the free memory (the buffers of an
        // earlier, larger group are reused)
        budget = std::max<size_t>(free_b / 2 + ctx->q_tiles.bytes, (size_t)te * 8 * 64);
        if (ctx->hbm_budget > 0) {   // the context's cap: every problem must fit in it alone
            budget = std::min(budget, ctx->hbm_budget);
            for (int64_t q = 0; q < count; ++q)
                if (queue_tile_bytes(inst[q].n, band[(size_t)q]) > budget) return MPGEO_E_NOMEM;
        }
    }
    hipStream_t s = ctx->stream;
    int status = MPGEO_OK;
    for (int64_t g0 = 0; g0 < count;) {
        // ---- group [g0, g1) ------------------------------------------------------------------------
        int64_t g1 = g0;
        size_t gbytes = kQueueSlack, tbytes = 0;
        if (fixed) {
            while (g1 < count && gbytes + queue_prob_bytes(inst[g1].n, band[(size_t)g1]) <= arena_bytes) {
                gbytes += queue_prob_bytes(inst[g1].n, band[(size_t)g1]);
                ++g1;
            }
        } else {
            while (g1 < count && (g1 == g0 || tbytes + queue_tile_bytes(inst[g1].n, band[(size_t)g1]) <= budget)) {
                tbytes += queue_tile_bytes(inst[g1].n, band[(size_t)g1]);
                ++g1;
            }
        }
        const int64_t gc = g1 - g0;
        std::vector<const mpgeo_instance *> members((size_t)gc);
        for (int64_t q = 0; q < gc; ++q) members[(size_t)q] = inst + g0 + q;
        QueueGroup G;
        MPGEO_TRY(queue_group_enqueue(ctx, s, members.data(), gc, band.data() + g0, plan, arena, arena_bytes, G));
        std::vector<double> res((size_t)gc * 3);
        std::vector<unsigned long long> info((size_t)gc);
        int ctrl[2] = {0, 0};
        MPGEO_HIP(hipMemcpyAsync(res.data(), G.res, res.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        MPGEO_HIP(hipMemcpyAsync(info.data(), G.info, info.size() * sizeof(unsigned long long),
                                 hipMemcpyDeviceToHost, s));
        MPGEO_HIP(hipMemcpyAsync(ctrl, G.ctrl, sizeof(ctrl), hipMemcpyDeviceToHost, s));
        MPGEO_HIP(hipStreamSynchronize(s));
        if (ctrl[1] != 0) return MPGEO_E_DEVICE;   // a wait timed out
        for (int64_t q = 0; q < gc; ++q) {
            mpgeo_result &o = out[g0 + q];
            o = mpgeo_result{};
            o.loglik = res[(size_t)q * 3];
            o.logdet = res[(size_t)q * 3 + 1];
            o.quad = res[(size_t)q * 3 + 2];
            o.info = (info[(size_t)q] == ~0ull) ? -1 : (int64_t)info[(size_t)q];
            o.band64 = G.bi[(size_t)q].band >= G.bi[(size_t)q].p - 1 ? -1 : G.bi[(size_t)q].band;
            o.band32 = o.band0 = -1;
            if (o.info >= 0) status = MPGEO_E_NOT_SPD;
            if (tiles) tiles[g0 + q] = kQueueTile;
        }
        g0 = g1;
    }
    return status;
}

// The queued batch with MPGEO_ESCALATE: problems that were not positive definite at their band
// run again, their bands widened b -> 2b + 1 (the step of escalate_plan) until they are or the
// band covers the matrix; each result then reports the band it was computed at and the number
// of widenings.
static int batch_queue_escalating(mpgeo_ctx *ctx, int64_t count, const mpgeo_instance *inst, const mpgeo_plan &plan,
                                  mpgeo_result *out, int32_t *tiles, char *arena, size_t arena_bytes,
                                  const int32_t *bands) {
    int st = batch_queue(ctx, count, inst, plan, out, tiles, arena, arena_bytes, bands);
    if (st != MPGEO_E_NOT_SPD || !(plan.flags & MPGEO_ESCALATE)) return st;
    std::vector<int32_t> band((size_t)count);
    std::vector<int32_t> esc((size_t)count, 0);
    for (int64_t q = 0; q < count; ++q) band[(size_t)q] = bands ? bands[q] : plan.band64;
    for (;;) {
        std::vector<int64_t> redo;
        for (int64_t q = 0; q < count; ++q) {
            const int64_t p = (inst[q].n + kQueueTile - 1) / kQueueTile;
            int32_t &b = band[(size_t)q];
            if (out[q].info < 0 || b < 0 || (int64_t)b >= p - 1) continue;   // done, or all-FP64 already
            b = ((int64_t)2 * b + 1 >= p - 1) ? -1 : 2 * b + 1;
            ++esc[(size_t)q];
            redo.push_back(q);
        }
        if (redo.empty()) break;
        std::vector<mpgeo_instance> sub(redo.size());
        std::vector<int32_t> sub_band(redo.size());
        std::vector<mpgeo_result> sub_out(redo.size());
        for (size_t r = 0; r < redo.size(); ++r) {
            sub[r] = inst[redo[r]];
            sub_band[r] = band[(size_t)redo[r]];
        }
        st = batch_queue(ctx, (int64_t)redo.size(), sub.data(), plan, sub_out.data(), nullptr, arena, arena_bytes,
                         sub_band.data());
        if (st != MPGEO_OK && st != MPGEO_E_NOT_SPD) return st;
        for (size_t r = 0; r < redo.size(); ++r) out[redo[r]] = sub_out[r];
    }
    st = MPGEO_OK;
    for (int64_t q = 0; q < count; ++q) {
        out[q].escalations = esc[(size_t)q];
        if (out[q].info >= 0) st = MPGEO_E_NOT_SPD;
    }
    return st;
}

// Arguments of the queued batch: a two-tier plan (FP64 band, FP32 beyond; or all FP64) at
// tile 128, each problem at most kQueueMaxN sites.
static int queue_plan_ok(const mpgeo_plan &plan) {
    const bool two_tier = plan.band32 == -1 && plan.lowp == 0 && plan.band0 == -1 && plan.dist64 == 0.0 &&
                          (plan.tile == 0 || plan.tile == kQueueTile);
    return two_tier ? MPGEO_OK : MPGEO_E_UNSUPPORTED;
}
static int queue_sizes_ok(int64_t count, const mpgeo_instance *inst) {
    for (int64_t i = 0; i < count; ++i)
        if (inst[i].n > kQueueMaxN) return MPGEO_E_UNSUPPORTED;
    return MPGEO_OK;
}

// The batch arguments every path checks: instances, theta, finite host inputs, the plan.
static int check_batch_args(mpgeo_ctx *ctx, int64_t count, const mpgeo_instance *inst, const mpgeo_plan &plan,
                            mpgeo_result *out) {
    if (!ctx || count < 0 || (count > 0 && (!inst || !out))) return MPGEO_E_ARG;
    if (plan.flags & (MPGEO_INPUT_DEVICE | MPGEO_TIMING)) return MPGEO_E_ARG;
    if ((plan.flags & MPGEO_ESCALATE) && !(plan.flags & MPGEO_BATCH_QUEUE)) return MPGEO_E_UNSUPPORTED;
    mpgeo_plan chk = plan;
    if (chk.tile == 0) chk.tile = 1;
    MPGEO_TRY(check_plan(chk));
    for (int64_t i = 0; i < count; ++i) {
        if (inst[i].n < 1 || inst[i].n > (int64_t)0xFFFFFFFF || !inst[i].locs || !inst[i].z)
            return MPGEO_E_ARG;
        MPGEO_TRY(check_theta(inst[i].theta));
        if (!all_finite(inst[i].locs, 2 * (size_t)inst[i].n) || !all_finite(inst[i].z, (size_t)inst[i].n))
            return MPGEO_E_ARG;
        out[i].info = -1;
    }
    return MPGEO_OK;
}

int mpgeo_batch_loglik(mpgeo_ctx *ctx, int64_t count, const mpgeo_instance *inst, mpgeo_plan plan,
                       mpgeo_result *out, int32_t *tiles) {
    MPGEO_TRY(check_batch_args(ctx, count, inst, plan, out));
    const bool tune_band = (plan.flags & MPGEO_TUNE_BAND) != 0;
    if (plan.flags & MPGEO_BATCH_QUEUE) {
        MPGEO_TRY(queue_plan_ok(plan));
        MPGEO_TRY(queue_sizes_ok(count, inst));
        if (count == 0) return MPGEO_OK;
        Device dev(ctx->device);
        if (!dev.ok) return MPGEO_E_DEVICE;
        if (!tune_band) return batch_queue_escalating(ctx, count, inst, plan, out, tiles, nullptr, 0, nullptr);
        std::vector<int32_t> bands;
        std::vector<double> err;
        MPGEO_TRY(tune_bands(ctx, count, inst, plan, std::vector<int>((size_t)count, kQueueTile), true, nullptr,
                             bands, err));
        int st = batch_queue_escalating(ctx, count, inst, plan, out, tiles, nullptr, 0, bands.data());
        if (st != MPGEO_OK && st != MPGEO_E_NOT_SPD) return st;
        const std::vector<int64_t> redo = accuracy_reruns(count, inst, out, err, (plan.flags & MPGEO_PROFILE) != 0);
        if (!redo.empty()) {
            std::vector<mpgeo_instance> sub(redo.size());
            std::vector<mpgeo_result> sub_out(redo.size());
            for (size_t r = 0; r < redo.size(); ++r) sub[r] = inst[redo[r]];
            mpgeo_plan fp64 = plan;
            fp64.band64 = -1;
            const int st2 = batch_queue(ctx, (int64_t)redo.size(), sub.data(), fp64, sub_out.data(), nullptr, nullptr,
                                        0, nullptr);
            if (st2 != MPGEO_OK && st2 != MPGEO_E_NOT_SPD) return st2;
            for (size_t r = 0; r < redo.size(); ++r) {
                const int esc = out[redo[r]].escalations;
                out[redo[r]] = sub_out[r];
                out[redo[r]].escalations = esc + 1;
            }
            st = MPGEO_OK;
            for (int64_t q = 0; q < count; ++q)
                if (out[q].info >= 0) st = MPGEO_E_NOT_SPD;
        }
        return st;
    }
    if (count == 0) return MPGEO_OK;
    Device dev(ctx->device);
    if (!dev.ok) return MPGEO_E_DEVICE;
    int nlanes = 4;
    if (const char *env = std::getenv("MPGEO_BATCH_LANES")) nlanes = std::max(1, std::atoi(env));
    nlanes = (int)std::min<int64_t>(nlanes, count);
    MPGEO_TRY(batch_lanes(ctx, nlanes));
    MPGEO_TRY(ctx->batch_res.ensure((size_t)(count + 1) * 4 * sizeof(double)));
    double *res = ctx->batch_res.as<double>();
    std::vector<int> tile((size_t)count);
    std::vector<int32_t> band((size_t)count, plan.band64);
    std::vector<double> err((size_t)count, 0.0);
    for (int64_t i = 0; i < count; ++i) {
        mpgeo_plan tp = plan;
        if (tune_band) {   // the tile is timed on the all-FP64 plan, the band then chosen for it
            tp.band64 = -1;
            tp.flags &= ~(uint32_t)MPGEO_TUNE_BAND;
        }
        const int st = batch_tile(ctx, inst[i], tp, res + 4 * count, &tile[(size_t)i]);
        if (st != MPGEO_OK) {
            batch_sync(ctx);
            return st;
        }
    }
    if (tune_band) {
        const int st = tune_bands(ctx, count, inst, plan, tile, false, res + 4 * count, band, err);
        if (st != MPGEO_OK) {
            batch_sync(ctx);
            return st;
        }
    }
    std::vector<int64_t> order((size_t)count);
    for (int64_t i = 0; i < count; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return inst[a].n > inst[b].n; });
    int status = MPGEO_OK;
    for (int64_t q = 0; q < count && status == MPGEO_OK; ++q) {
        const int64_t i = order[(size_t)q];
        mpgeo_plan pl = plan;
        pl.tile = tile[(size_t)i];
        pl.band64 = band[(size_t)i];
        pl.flags &= ~(uint32_t)MPGEO_TUNE_BAND;
        status = batch_enqueue(ctx->lane_ds[(size_t)(q % nlanes)], inst[i], pl, res + 4 * i);
    }
    batch_sync(ctx);
    if (status != MPGEO_OK) return status;
    std::vector<double> host((size_t)count * 4);
    MPGEO_HIP(hipMemcpy(host.data(), res, host.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < count; ++i) {
        const double *r = host.data() + 4 * i;
        unsigned long long info;
        std::memcpy(&info, r + 3, sizeof(info));
        out[i] = mpgeo_result{};
        out[i].loglik = r[0];
        out[i].logdet = r[1];
        out[i].quad = r[2];
        out[i].info = (info == ~0ull) ? -1 : (int64_t)info;
        const int64_t p = (inst[i].n + tile[(size_t)i] - 1) / tile[(size_t)i];
        out[i].band64 = band[(size_t)i] >= p - 1 ? -1 : band[(size_t)i];   // a band covering the matrix is all-FP64
        out[i].band32 = plan.band32;
        out[i].band0 = plan.band0;
        if (out[i].info >= 0) status = MPGEO_E_NOT_SPD;
        if (tiles) tiles[i] = tile[(size_t)i];
    }
    if (!tune_band) return status;
    const std::vector<int64_t> redo = accuracy_reruns(count, inst, out, err, (plan.flags & MPGEO_PROFILE) != 0);
    if (redo.empty()) return status;
    int est = MPGEO_OK;
    std::vector<char> again((size_t)count, 0);
    for (size_t q = 0; q < redo.size() && est == MPGEO_OK; ++q) {
        const int64_t i = redo[q];
        mpgeo_plan pl = plan;
        pl.tile = tile[(size_t)i];
        pl.band64 = -1;
        pl.flags &= ~(uint32_t)MPGEO_TUNE_BAND;
        again[(size_t)i] = 1;
        est = batch_enqueue(ctx->lane_ds[q % (size_t)nlanes], inst[i], pl, res + 4 * i);
    }
    batch_sync(ctx);
    if (est != MPGEO_OK) return est;
    MPGEO_HIP(hipMemcpy(host.data(), res, host.size() * sizeof(double), hipMemcpyDeviceToHost));
    status = MPGEO_OK;
    for (int64_t i = 0; i < count; ++i) {
        if (again[(size_t)i]) {
            const double *r = host.data() + 4 * i;
            unsigned long long info;
            std::memcpy(&info, r + 3, sizeof(info));
            out[i].loglik = r[0];
            out[i].logdet = r[1];
            out[i].quad = r[2];
            out[i].info = (info == ~0ull) ? -1 : (int64_t)info;
            out[i].band64 = -1;
            out[i].escalations += 1;
        }
        if (out[i].info >= 0) status = MPGEO_E_NOT_SPD;
    }
    return status;
}

// The persistent-queue batch with its work buffers in the GPU's fixed array: no device
// allocation (and no freeing) on any path of the call; the fill kernel clears what must start at
// zero, since the array keeps the previous call's contents.
int mpgeo_batch_loglik_noalloc(mpgeo_ctx *ctx, int64_t count, const mpgeo_instance *inst, mpgeo_plan plan,
                               mpgeo_result *out) {
    plan.flags |= MPGEO_BATCH_QUEUE;
    MPGEO_TRY(check_batch_args(ctx, count, inst, plan, out));
    if (plan.flags & MPGEO_TUNE_BAND) return MPGEO_E_UNSUPPORTED;   // its probes would allocate
    MPGEO_TRY(queue_plan_ok(plan));
    MPGEO_TRY(queue_sizes_ok(count, inst));
    if (count == 0) return MPGEO_OK;
    Device dev(ctx->device);
    if (!dev.ok) return MPGEO_E_DEVICE;
    char *ptr = scratch_ptr(ctx->device);
    if (!ptr) return MPGEO_E_DEVICE;
    return batch_queue_escalating(ctx, count, inst, plan, out, nullptr, ptr, kScratchBytes, nullptr);
}

// ---- serving loop ---------------------------------------------------------------------------
// Requests (dataset, theta) arrive over time; datasets keep their tiles resident on the device
// while they fit in the HBM budget (admission by their tile footprint, least recently used
// eviction of idle datasets); a dispatcher hands each ready request to a free lane as soon as
// its dataset is resident and not busy, without waiting for the others (continuous batching
// over the lanes), and records when each evaluation was dispatched and finished.

struct ServedDataset {
    int64_t n = 0;
    std::vector<double> locs, z;       // host copies (re-uploaded after an eviction)
    mpgeo_plan plan{};
    bool queued = false;               // likelihood requests go through the persistent queue
    size_t footprint = 0;
    mpgeo_dataset *ds = nullptr;       // resident device state, or nullptr
    bool busy = false;
    double last_used = -1.0;
};

struct ServedRequest {
    int32_t dataset;
    mpgeo_theta theta;
    double arrival;
    // kriging request: new sites (host copy), the caller's outputs, offset in the device arena
    int64_t m = 0;
    std::vector<double> sites;
    double *pred = nullptr, *var = nullptr;
    size_t arena = 0;
};

struct mpgeo_server {
    mpgeo_ctx *ctx = nullptr;
    size_t budget = 0;
    int nlanes = 0;
    std::vector<ServedDataset> sets;
    std::vector<ServedRequest> reqs;
    size_t resident_bytes = 0;
    DevBuf krige_arena;                // new sites, predictions and variances of kriging requests
};

int mpgeo_server_create(mpgeo_ctx *ctx, uint64_t hbm_budget_bytes, int32_t lanes, mpgeo_server **out) {
    if (!ctx || !out || lanes < 1 || lanes > 64) return MPGEO_E_ARG;
    *out = nullptr;
    Device dev(ctx->device);
    if (!dev.ok) return MPGEO_E_DEVICE;
    MPGEO_TRY(batch_lanes(ctx, lanes));
    mpgeo_server *srv = new mpgeo_server();
    srv->ctx = ctx;
    srv->budget = hbm_budget_bytes;
    srv->nlanes = lanes;
    *out = srv;
    return MPGEO_OK;
}

int mpgeo_server_add_dataset(mpgeo_server *srv, int64_t n, const double *locs, const double *z,
                             mpgeo_plan plan, int32_t *id) {
    if (!srv || !locs || !z || !id || n < 1 || n > (int64_t)0xFFFFFFFF) return MPGEO_E_ARG;
    if (plan.flags & (MPGEO_INPUT_DEVICE | MPGEO_TIMING)) return MPGEO_E_ARG;
    if (plan.flags & MPGEO_ESCALATE) return MPGEO_E_UNSUPPORTED;
    const bool queued = (plan.flags & MPGEO_BATCH_QUEUE) != 0;
    if (queued) {   // likelihood requests through the persistent queue: its plans and sizes only
        if (plan.tile == 0) plan.tile = kQueueTile;
        MPGEO_TRY(queue_plan_ok(plan));
        if (n > kQueueMaxN) return MPGEO_E_UNSUPPORTED;
    }
    MPGEO_TRY(check_plan(plan));
    if (!all_finite(locs, 2 * (size_t)n) || !all_finite(z, (size_t)n)) return MPGEO_E_ARG;
    ServedDataset d;
    d.n = n;
    d.locs.assign(locs, locs + 2 * n);
    d.z.assign(z, z + n);
    d.plan = plan;
    d.queued = queued;
    d.plan.flags &= ~(uint32_t)MPGEO_BATCH_QUEUE;   // the lane plan (kriging requests)
    d.footprint = mpgeo_footprint_bytes(n, d.plan);
    if (d.footprint > srv->budget) return MPGEO_E_NOMEM;   // could never be admitted
    srv->sets.push_back(std::move(d));
    *id = (int32_t)(srv->sets.size() - 1);
    return MPGEO_OK;
}

int mpgeo_server_submit(mpgeo_server *srv, int32_t dataset, mpgeo_theta theta, double arrival_s,
                        int64_t *ticket) {
    if (!srv || dataset < 0 || dataset >= (int32_t)srv->sets.size() || !(arrival_s >= 0.0))
        return MPGEO_E_ARG;
    MPGEO_TRY(check_theta(theta));
    ServedRequest rq;
    rq.dataset = dataset;
    rq.theta = theta;
    rq.arrival = arrival_s;
    srv->reqs.push_back(std::move(rq));
    if (ticket) *ticket = (int64_t)srv->reqs.size() - 1;
    return MPGEO_OK;
}

int mpgeo_server_submit_krige(mpgeo_server *srv, int32_t dataset, mpgeo_theta theta, int64_t m,
                              const double *new_locs, double *pred, double *var, double arrival_s,
                              int64_t *ticket) {
    if (!srv || dataset < 0 || dataset >= (int32_t)srv->sets.size() || !(arrival_s >= 0.0) || m < 1 ||
        !new_locs || !pred || (var && m > 65535))
        return MPGEO_E_ARG;
    MPGEO_TRY(check_theta(theta));
    if (!all_finite(new_locs, 2 * (size_t)m)) return MPGEO_E_ARG;
    ServedRequest rq;
    rq.dataset = dataset;
    rq.theta = theta;
    rq.arrival = arrival_s;
    rq.m = m;
    rq.sites.assign(new_locs, new_locs + 2 * m);
    rq.pred = pred;
    rq.var = var;
    srv->reqs.push_back(std::move(rq));
    if (ticket) *ticket = (int64_t)srv->reqs.size() - 1;
    return MPGEO_OK;
}

// release the device state of an idle dataset
static void server_evict(mpgeo_server *srv, ServedDataset &d) {
    if (!d.ds) return;
    mpgeo_dataset_destroy(d.ds);   // synchronises the lane stream it last ran on
    d.ds = nullptr;
    srv->resident_bytes -= d.footprint;
}

// make room for `need` bytes by evicting idle datasets, least recently used first
static bool server_admit(mpgeo_server *srv, size_t need) {
    while (srv->resident_bytes + need > srv->budget) {
        ServedDataset *victim = nullptr;
        for (auto &d : srv->sets)
            if (d.ds && !d.busy && (!victim || d.last_used < victim->last_used)) victim = &d;
        if (!victim) return false;
        server_evict(srv, *victim);
    }
    return true;
}

int mpgeo_server_run(mpgeo_server *srv, mpgeo_served *out) {
    if (!srv || (!srv->reqs.empty() && !out)) return MPGEO_E_ARG;
    mpgeo_ctx *ctx = srv->ctx;
    Device dev(ctx->device);
    if (!dev.ok) return MPGEO_E_DEVICE;
    const int64_t nreq = (int64_t)srv->reqs.size();
    if (nreq == 0) return MPGEO_OK;
    MPGEO_TRY(ctx->batch_res.ensure((size_t)nreq * 4 * sizeof(double)));
    double *res = ctx->batch_res.as<double>();
    // kriging requests: sites, predictions and variances in one device arena, sites uploaded now
    size_t arena = 0;
    for (auto &rq : srv->reqs) {
        rq.arena = arena;
        arena += 4 * (size_t)rq.m;
    }
    if (arena > 0) {
        MPGEO_TRY(srv->krige_arena.ensure(arena * sizeof(double)));
        for (auto &rq : srv->reqs)
            if (rq.m > 0)
                MPGEO_HIP(hipMemcpy(srv->krige_arena.as<double>() + rq.arena, rq.sites.data(),
                                    (size_t)rq.m * 2 * sizeof(double), hipMemcpyHostToDevice));
    }
    std::vector<int64_t> order((size_t)nreq);
    for (int64_t i = 0; i < nreq; ++i) order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int64_t a, int64_t b) { return srv->reqs[a].arrival < srv->reqs[b].arrival; });
    struct LaneState {
        int64_t req = -1;
        hipEvent_t done = nullptr;
    };
    std::vector<LaneState> lanes((size_t)srv->nlanes);
    for (auto &l : lanes)
        if (hipEventCreateWithFlags(&l.done, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            for (auto &m : lanes)
                if (m.done) (void)hipEventDestroy(m.done);
            return MPGEO_E_DEVICE;
        }
    for (int64_t i = 0; i < nreq; ++i) out[i] = mpgeo_served{};
    // the persistent queue: one batch of likelihood requests of queued datasets in flight at a
    // time, on the context's own stream (the lanes are sub-contexts with streams of their own)
    struct QueueState {
        bool busy = false;
        std::vector<int64_t> reqs;
        QueueGroup group;
        hipEvent_t done = nullptr;
    } qs;
    // the queue's persistent workgroups wait on dependencies between tasks: a quarter of the
    // compute units at most, so that the lanes' factorizations beside it keep the rest
    const int queue_wgs = std::max(8, (ctx->cus > 0 ? ctx->cus : 256) / 4);
    if (hipEventCreateWithFlags(&qs.done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        for (auto &l : lanes) (void)hipEventDestroy(l.done);
        return MPGEO_E_DEVICE;
    }
    std::deque<int64_t> ready;
    size_t next = 0;
    int64_t finished = 0;
    int status = MPGEO_OK;
    const auto t0 = std::chrono::steady_clock::now();
    auto now = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
    while (finished < nreq && status == MPGEO_OK) {
        const double t = now();
        while (next < order.size() && srv->reqs[order[next]].arrival <= t) ready.push_back(order[next++]);
        bool progressed = false;
        // completions
        for (auto &l : lanes) {
            if (l.req < 0) continue;
            const hipError_t q = hipEventQuery(l.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) {
                (void)hipGetLastError();
                status = MPGEO_E_DEVICE;
                break;
            }
            out[l.req].finish_s = now();
            srv->sets[srv->reqs[l.req].dataset].busy = false;
            l.req = -1;
            ++finished;
            progressed = true;
        }
        if (qs.busy && status == MPGEO_OK) {
            const hipError_t q = hipEventQuery(qs.done);
            if (q == hipSuccess) {
                int ctrl[2] = {0, 0};
                MPGEO_HIP(hipMemcpy(ctrl, qs.group.ctrl, sizeof(ctrl), hipMemcpyDeviceToHost));
                if (ctrl[1] != 0) status = MPGEO_E_DEVICE;   // a wait in the queue timed out
                const double tf = now();
                for (int64_t r : qs.reqs) out[r].finish_s = tf;
                finished += (int64_t)qs.reqs.size();
                qs.reqs.clear();
                qs.busy = false;
                progressed = true;
            } else if (q != hipErrorNotReady) {
                (void)hipGetLastError();
                status = MPGEO_E_DEVICE;
            }
        }
        // dispatch to the queue: every ready likelihood request of a queued dataset (with the
        // first one's distance and likelihood form), up to a quarter of the budget in tiles,
        // as one persistent launch
        if (!qs.busy && status == MPGEO_OK) {
            std::vector<mpgeo_instance> members;
            std::vector<int32_t> bands;
            uint32_t form = 0;
            size_t bytes = 0;
            for (auto it = ready.begin(); it != ready.end();) {
                const ServedRequest &rq = srv->reqs[*it];
                const ServedDataset &d = srv->sets[rq.dataset];
                const uint32_t f = d.plan.flags & (MPGEO_PROFILE | MPGEO_DIST_GCD);
                const size_t b = queue_tile_bytes(d.n, d.plan.band64);
                if (!d.queued || rq.m > 0 || (!members.empty() && (f != form || bytes + b > srv->budget / 4))) {
                    ++it;
                    continue;
                }
                form = f;
                bytes += b;
                mpgeo_theta th = rq.theta;
                if (f & MPGEO_PROFILE) th.sigma2 = 1.0;
                members.push_back(mpgeo_instance{d.n, d.locs.data(), d.z.data(), th});
                bands.push_back(d.plan.band64);
                qs.reqs.push_back(*it);
                it = ready.erase(it);
            }
            if (!members.empty()) {
                std::vector<const mpgeo_instance *> mp(members.size());
                for (size_t q = 0; q < members.size(); ++q) mp[q] = &members[q];
                mpgeo_plan qp{};
                qp.tile = kQueueTile;
                qp.flags = form;
                const double ts = now();
                for (int64_t r : qs.reqs) out[r].start_s = ts;
                status = queue_group_enqueue(ctx, ctx->stream, mp.data(), (int64_t)mp.size(), bands.data(), qp,
                                             nullptr, 0, qs.group, queue_wgs);
                for (size_t q = 0; q < qs.reqs.size() && status == MPGEO_OK; ++q) {
                    double *slot = res + 4 * qs.reqs[q];
                    if (hipMemcpyAsync(slot, qs.group.res + 3 * q, 3 * sizeof(double), hipMemcpyDeviceToDevice,
                                       ctx->stream) != hipSuccess ||
                        hipMemcpyAsync(slot + 3, qs.group.info + q, sizeof(double), hipMemcpyDeviceToDevice,
                                       ctx->stream) != hipSuccess) {
                        (void)hipGetLastError();
                        status = MPGEO_E_DEVICE;
                    }
                }
                if (status == MPGEO_OK && hipEventRecord(qs.done, ctx->stream) != hipSuccess) {
                    (void)hipGetLastError();
                    status = MPGEO_E_DEVICE;
                }
                qs.busy = status == MPGEO_OK;
                progressed = true;
            }
        }
        // dispatch: oldest ready request whose dataset is idle (and resident or admissible)
        for (int li = 0; li < srv->nlanes && status == MPGEO_OK; ++li) {
            LaneState &l = lanes[(size_t)li];
            if (l.req >= 0) continue;
            auto it = ready.begin();
            for (; it != ready.end(); ++it) {
                ServedDataset &d = srv->sets[srv->reqs[*it].dataset];
                if (d.busy || (d.queued && srv->reqs[*it].m == 0)) continue;
                if (d.ds || server_admit(srv, d.footprint)) break;
            }
            if (it == ready.end()) break;
            const int64_t r = *it;
            ready.erase(it);
            ServedRequest &rq = srv->reqs[r];
            ServedDataset &d = srv->sets[rq.dataset];
            mpgeo_ctx *lc = ctx->lanes[(size_t)li];
            if (!d.ds) {   // admission: resident device copy of the ordered inputs
                d.ds = new mpgeo_dataset();
                d.ds->ctx = lc;
                d.ds->n = d.n;
                d.ds->flags = d.plan.flags | MPGEO_ORDER_MORTON;
                srv->resident_bytes += d.footprint;
                status = load_inputs(d.ds, d.locs.data(), d.z.data(), d.ds->flags);
                if (status != MPGEO_OK) break;
            }
            if (d.ds->ctx != lc) {   // the dataset moves to this lane: order after its last use
                MPGEO_HIP(hipStreamSynchronize(d.ds->ctx->stream));
                d.ds->ctx = lc;
            }
            d.busy = true;
            d.last_used = now();
            out[r].start_s = d.last_used;
            mpgeo_plan pl = d.plan;
            status = prepare_layout(d.ds, pl);
            if (status != MPGEO_OK) break;
            d.ds->profile = (pl.flags & MPGEO_PROFILE) != 0;
            mpgeo_theta th = rq.theta;
            if (d.ds->profile) th.sigma2 = 1.0;
            status = run_covgen(d.ds, th);
            if (status == MPGEO_OK) status = run_factor(d.ds, nullptr);
            if (status == MPGEO_OK && rq.m > 0) {   // kriging from this factor, same lane
                d.ds->theta = th;
                double *a = srv->krige_arena.as<double>() + rq.arena;
                status = krige_enqueue(d.ds, rq.m, a, a + 2 * rq.m, rq.var ? a + 3 * rq.m : nullptr, 1.0);
            }
            if (status != MPGEO_OK) break;
            double *slot = res + 4 * r;
            MPGEO_HIP(hipMemcpyAsync(slot, d.ds->result.ptr, 3 * sizeof(double), hipMemcpyDeviceToDevice, lc->stream));
            MPGEO_HIP(hipMemcpyAsync(slot + 3, d.ds->info.ptr, sizeof(double), hipMemcpyDeviceToDevice, lc->stream));
            MPGEO_HIP(hipEventRecord(l.done, lc->stream));
            l.req = r;
            progressed = true;
        }
        if (!progressed) {
            // idle until the next arrival or a completion: short sleeps, no busy spin
            const double wake = next < order.size() ? srv->reqs[order[next]].arrival : INFINITY;
            const double dt = std::min(2e-4, std::max(0.0, wake - now()));
            if (dt > 0) std::this_thread::sleep_for(std::chrono::duration<double>(dt));
        }
    }
    for (auto *c : ctx->lanes) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamSynchronize(c->stream);
    }
    (void)hipStreamSynchronize(ctx->stream);
    for (auto &l : lanes) (void)hipEventDestroy(l.done);
    (void)hipEventDestroy(qs.done);
    if (status != MPGEO_OK) return status;
    std::vector<double> host((size_t)nreq * 4);
    MPGEO_HIP(hipMemcpy(host.data(), res, host.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < nreq; ++i) {
        const double *rr = host.data() + 4 * i;
        unsigned long long info;
        std::memcpy(&info, rr + 3, sizeof(info));
        out[i].loglik = rr[0];
        out[i].logdet = rr[1];
        out[i].quad = rr[2];
        out[i].info = (info == ~0ull) ? -1 : (int64_t)info;
        out[i].arrival_s = srv->reqs[(size_t)i].arrival;
        if (out[i].info >= 0) status = MPGEO_E_NOT_SPD;
        const ServedRequest &rq = srv->reqs[(size_t)i];
        if (rq.m > 0) {   // kriging outputs; a profile plan's variances take theta1 = q~ / n
            const double *a = srv->krige_arena.as<double>() + rq.arena;
            MPGEO_HIP(hipMemcpy(rq.pred, a + 2 * rq.m, (size_t)rq.m * sizeof(double), hipMemcpyDeviceToHost));
            if (rq.var) {
                MPGEO_HIP(hipMemcpy(rq.var, a + 3 * rq.m, (size_t)rq.m * sizeof(double), hipMemcpyDeviceToHost));
                if (srv->sets[(size_t)rq.dataset].plan.flags & MPGEO_PROFILE) {
                    const double scale = out[i].quad / (double)srv->sets[(size_t)rq.dataset].n;
                    for (int64_t j = 0; j < rq.m; ++j) rq.var[j] *= scale;
                }
            }
        }
    }
    srv->reqs.clear();
    return status;
}

int mpgeo_server_destroy(mpgeo_server *srv) {
    if (!srv) return MPGEO_OK;
    Device dev(srv->ctx->device);
    for (auto &d : srv->sets) server_evict(srv, d);
    srv->krige_arena.release();
    delete srv;
    return MPGEO_OK;
}

}  // extern "C"
