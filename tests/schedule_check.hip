// Host-side check of the factorization schedule built by the library's tile layout (no GPU
// work): the 16-bit tier's left-looking passes and the split of each step's FP64/FP32 update
// lists.  Built and run by test_schedule.py; exits non-zero on the first inconsistency.
//
// For every 16-bit tile (i, j), the bulk passes must apply panels max(0, i - zband) .. j - 2
// exactly once each, in ascending order, all before the lookahead step j - 1 adds panel j - 1;
// a pass of step k only touches columns k+2 and k+3; the flops of the passes add up to those
// of the plain schedule; when the layout knows the wave size, every pass that could be filled
// from the next column runs whole waves of full-length tiles.  The FP64/FP32 bulk list of step
// k must end with exactly the tiles of column k+2 (the part the next lookahead step waits for).
#include "../paper_2003_05324_amd/csrc/api.hip"

#include <cstdio>
#include <map>
#include <utility>

using namespace mpgeo;

static int check(int64_t n, int nb, int band64, int band32, int band0, int wave) {
    Layout L;
    L.build(n, nb, band64, band32, 1, band0, nullptr, 0.0, 0.0, wave);
    int bad = 0;
    auto fail = [&](const char *what, int k, int i, int j) {
        if (bad++ < 5) std::printf("  %s (step %d, tile %d,%d)\n", what, k, i, j);
    };
    std::map<std::pair<int, int>, int> next;   // next panel each 16-bit tile expects
    auto expected = [&](int i, int j) {
        auto it = next.find({i, j});
        return std::max(it == next.end() ? 0 : it->second, i - L.zband);
    };
    double flops = 0.0;
    for (int k = 0; k + 1 < L.p; ++k) {
        const Layout::Range &r = L.bulk[2][k];
        int64_t longs = 0, avail = 0;
        for (int64_t t = r.b; t < r.e; ++t) {
            const TileIJ ij = L.bulk16[(size_t)t];
            const int k0 = std::max((int)L.bulk16_k0[(size_t)t], ij.i - L.zband);
            if (L.tier(ij.i, ij.j) != 16) fail("not a 16-bit tile", k, ij.i, ij.j);
            if (ij.j != k + 2 && ij.j != k + 3) fail("column outside k+2 .. k+3", k, ij.i, ij.j);
            if (k0 != expected(ij.i, ij.j)) fail("panels out of order", k, ij.i, ij.j);
            // (an entry whose panels are all dropped so far takes none: the kernel skips it)
            if (k0 > k && ij.i - L.zband <= k) fail("empty pass entry", k, ij.i, ij.j);
            next[{ij.i, ij.j}] = k + 1;
            if (L.bulk16_k0[(size_t)t] == 0) ++longs;
        }
        flops += r.flops;
        if (k + 3 < L.p)
            for (int i = k + 3; i < L.p; ++i)
                if (L.tier(i, k + 3) == 16 && expected(i, k + 3) == 0) ++avail;
        if (wave > 0 && L.zband >= L.p && longs % wave != 0 && avail > 0)
            fail("pass not filled to whole waves", k, -1, -1);
        // the lookahead of step k adds panel k to column k+1: panels before k must be in
        for (int64_t t = L.col[2][k].b; t < L.col[2][k].e; ++t) {
            const TileIJ ij = L.list16[(size_t)t];
            if (ij.j != k + 1) fail("lookahead column", k, ij.i, ij.j);
            if (std::max(0, ij.i - L.zband) <= k - 1 && expected(ij.i, ij.j) != k)
                fail("column not complete before its lookahead", k, ij.i, ij.j);
        }
        for (int q = 0; q < 2; ++q) {
            const std::vector<TileIJ> &lst = q == 0 ? L.list64 : L.list32;
            double fa = 0.0;
            for (int64_t t = L.bulk[q][k].b; t < L.bulk[q][k].e; ++t) {
                const bool tail = t >= L.next_b[q][k];
                if (tail != (lst[(size_t)t].j == k + 2)) fail("column k+2 split", k, lst[(size_t)t].i, lst[(size_t)t].j);
                if (lst[(size_t)t].j < k + 2) fail("bulk column below k+2", k, lst[(size_t)t].i, lst[(size_t)t].j);
                if (tail) fa += L.update_flops(lst[(size_t)t].i, lst[(size_t)t].j, k);
            }
            if (std::abs(fa - L.next_f[q][k]) > 1e-9 * (1.0 + fa)) fail("column k+2 flops", k, -1, -1);
        }
    }
    double ref = 0.0;
    for (int j = 2; j < L.p; ++j)
        for (int i = j; i < L.p; ++i)
            if (L.tier(i, j) == 16) {
                const int lo = std::max(0, i - L.zband);
                if (lo <= j - 2 && expected(i, j) != j - 1) fail("tile not brought to panel j-2", -1, i, j);
                for (int kk = lo; kk <= j - 2; ++kk) ref += L.update_flops(i, j, kk);
            }
    if (std::abs(flops - ref) > 1e-12 * ref) fail("16-bit flops differ from the plain schedule", -1, -1, -1);
    std::printf("n %ld nb %d band64 %d band32 %d band0 %d wave %d: p %d, %zu pass entries, %s\n", (long)n, nb,
                band64, band32, band0, wave, L.p, L.bulk16.size(), bad ? "FAILED" : "ok");
    return bad;
}

// The escalation ladder of MPGEO_ESCALATE: bands b -> 2b + 1 until they reach the last tile
// row (then -1, and the third tier goes with the FP64 band); the all-FP64 plan cannot escalate.
static int check_escalation() {
    int bad = 0;
    auto expect = [&](const mpgeo_plan &pl, int b64, int b32, int lowp, int b0, const char *what) {
        if (pl.band64 != b64 || pl.band32 != b32 || pl.lowp != lowp || pl.band0 != b0) {
            std::printf("  escalation %s: got band64 %d band32 %d lowp %d band0 %d\n", what, pl.band64,
                        pl.band32, pl.lowp, pl.band0);
            ++bad;
        }
    };
    mpgeo_plan pl{};
    pl.tile = 160;
    pl.band64 = 0;
    pl.band32 = -1;
    pl.band0 = -1;
    const int64_t p = 10;   // n = 1,600, tile 160
    int steps = 0;
    const int want[] = {1, 3, 7, -1};
    while (escalate_plan(pl, p)) {
        if (steps < 4) expect(pl, want[steps], -1, 0, -1, "two tiers");
        ++steps;
    }
    if (steps != 4) {
        std::printf("  escalation took %d steps, want 4\n", steps);
        ++bad;
    }
    mpgeo_plan q{};
    q.tile = 512;
    q.band64 = 2;
    q.band32 = 8;
    q.lowp = 1;
    q.band0 = -1;
    if (!escalate_plan(q, 196)) ++bad;
    expect(q, 5, 17, 1, -1, "three tiers, first step");
    q.band64 = 100;
    if (!escalate_plan(q, 196)) ++bad;
    expect(q, -1, -1, 0, -1, "three tiers into all FP64");
    mpgeo_plan z{};
    z.tile = 100;
    z.band64 = -1;
    z.band32 = -1;
    z.band0 = 2;
    if (!escalate_plan(z, 31)) ++bad;
    expect(z, -1, -1, 0, 5, "dropped tiles");
    // the footprint of a built layout is the one the boundary reports
    for (int b : {-1, 0, 2}) {
        mpgeo_plan f{};
        f.tile = 512;
        f.band64 = b;
        f.band32 = b >= 0 ? 8 : -1;
        f.lowp = b >= 0 ? 1 : 0;
        f.band0 = -1;
        Layout L;
        L.build(99856, 512, f.band64, f.band32, f.lowp, f.band0);
        if (layout_footprint(L) != mpgeo_footprint_bytes(99856, f)) {
            std::printf("  footprint of band64 %d differs\n", b);
            ++bad;
        }
    }
    std::printf("escalation ladder and footprint: %s\n", bad ? "FAILED" : "ok");
    return bad;
}

// Tile offsets of the queued batch's mixed-precision layout: every tile (i, j) of a problem of
// p tile rows starts where the one before it (row-major lower order) ends, FP64 tiles taking
// 2 kQueueTile^2 four-byte units and FP32 tiles kQueueTile^2, the last ending at the total.
static int check_queue_offsets() {
    int bad = 0;
    const int64_t te = (int64_t)kQueueTile * kQueueTile;
    for (int p = 1; p <= 40; ++p)
        for (int band = 0; band <= p + 1; ++band) {
            int64_t expect = 0;
            for (int i = 0; i < p; ++i)
                for (int j = 0; j <= i; ++j) {
                    if (queue_tile_units(i, j, band) != expect) {
                        if (bad++ < 5) std::printf("  queue offset p %d band %d tile %d,%d\n", p, band, i, j);
                    }
                    expect += (i - j <= band ? 2 : 1) * te;
                }
            if (queue_tile_units(p, 0, band) != expect) {
                if (bad++ < 5) std::printf("  queue total p %d band %d\n", p, band);
            }
        }
    std::printf("queue tile offsets: %s\n", bad ? "FAILED" : "ok");
    return bad;
}

int main() {
    int bad = check_escalation() + check_queue_offsets();
    bad += check(99856, 512, 2, 8, -1, 64);     // the n ~ 1e5 three-tier plan on 256 compute units
    bad += check(99856, 512, 2, 8, -1, 32);
    bad += check(99856, 512, 2, 8, -1, 0);      // wave size unknown: no filling
    bad += check(99856, 512, 2, 8, -1, 1000);   // waves wider than any column
    bad += check(99856, 512, 2, 8, 40, 64);     // dropped tiles beyond 40: no filling
    bad += check(40000, 256, 2, 8, -1, 156);
    bad += check(40000, 512, 0, 1, -1, 32);
    bad += check(5000, 128, 1, 1, -1, 7);
    bad += check(5000, 128, 1, 1, 6, 7);
    bad += check(3001, 100, 0, 0, -1, 3);       // ragged last tile
    std::printf(bad ? "FAILED\n" : "all schedules consistent\n");
    return bad ? 1 : 0;
}
