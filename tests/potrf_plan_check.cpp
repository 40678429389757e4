// Host-side check of the blocked diagonal-tile factorization plan (potrf_plan.h), no GPU: every
// product stays inside the tile and its inverse, no launch holds more jobs than the kernel
// argument has room for, the products of one launch neither overlap each other's outputs nor
// write what another reads, no product reads its own output, nothing reads the strictly upper
// part of the tile or scratch that was not written first (both start as NaN), and replaying the
// plan in double precision gives the Cholesky factor and its inverse of a random symmetric
// positive-definite matrix (against a plain column Cholesky and forward substitution), with the
// inverse's strictly upper part zero and its FP32 copy complete.  Exits non-zero on a failure.
#include "../paper_2003_05324_amd/csrc/potrf_plan.h"

#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

using namespace mpgeo;

static int failures = 0;
static void fail(const char *what, int step, int job) {
    if (failures++ < 10) std::printf("  FAIL %s (step %d, job %d)\n", what, step, job);
}

struct Range { int buf; int64_t lo, hi; };   // element offsets [lo, hi] touched in a buffer (bounding)

static int check(int nbp, bool with32) {
    const int64_t te = (int64_t)nbp * nbp;
    const double nan = std::nan("");
    std::mt19937_64 rng(nbp);
    std::normal_distribution<double> gauss;
    std::vector<double> x(te), a0(te);
    for (auto &v : x) v = gauss(rng);
    for (int i = 0; i < nbp; ++i)   // a0 = x x^T + nbp I
        for (int j = 0; j < nbp; ++j) {
            double s = (i == j) ? nbp : 0.0;
            for (int t = 0; t < nbp; ++t) s += x[i + (int64_t)t * nbp] * x[j + (int64_t)t * nbp];
            a0[i + (int64_t)j * nbp] = s;
        }
    std::vector<double> A(te, nan), B(te, nan);
    std::vector<float> B32(te, NAN);
    for (int j = 0; j < nbp; ++j)
        for (int i = j; i < nbp; ++i) A[i + (int64_t)j * nbp] = a0[i + (int64_t)j * nbp];
    auto buf = [&](int b) -> std::vector<double> * { return b == kBufA ? &A : b == kBufB ? &B : nullptr; };
    const std::vector<PotrfStep> plan = potrf_blocked_plan(nbp, with32);
    const int P = kPotrfBlock;
    int si = 0;
    for (const PotrfStep &st : plan) {
        if (st.diag >= 0) {   // the single-workgroup factorization of one diagonal block
            const int64_t o = (int64_t)st.diag * P * (nbp + 1);
            std::vector<double> L((size_t)P * P, 0.0);
            for (int j = 0; j < P; ++j)
                for (int i = j; i < P; ++i) {
                    const double v = A[o + i + (int64_t)j * nbp];
                    if (std::isnan(v)) fail("diagonal block reads an unset entry", si, -1);
                    L[i + (size_t)j * P] = v;
                }
            for (int j = 0; j < P; ++j) {   // Cholesky of the block
                double d = L[j + (size_t)j * P];
                for (int t = 0; t < j; ++t) d -= L[j + (size_t)t * P] * L[j + (size_t)t * P];
                d = std::sqrt(d);
                L[j + (size_t)j * P] = d;
                for (int i = j + 1; i < P; ++i) {
                    double s = L[i + (size_t)j * P];
                    for (int t = 0; t < j; ++t) s -= L[i + (size_t)t * P] * L[j + (size_t)t * P];
                    L[i + (size_t)j * P] = s / d;
                }
            }
            for (int j = 0; j < P; ++j)
                for (int i = 0; i < P; ++i) {
                    if (i >= j) A[o + i + (int64_t)j * nbp] = L[i + (size_t)j * P];
                    B[o + i + (int64_t)j * nbp] = 0.0;
                }
            for (int c = 0; c < P; ++c)   // inverse, column c: L y = e_c
                for (int i = c; i < P; ++i) {
                    double s = (i == c) ? 1.0 : 0.0;
                    for (int t = c; t < i; ++t) s -= L[i + (size_t)t * P] * B[o + t + (int64_t)c * nbp];
                    B[o + i + (int64_t)c * nbp] = s / L[i + (size_t)i * P];
                }
            ++si;
            continue;
        }
        if ((int)st.jobs.size() > kPotrfMaxJobs || st.jobs.empty()) fail("job count", si, -1);
        std::vector<Range> writes, reads;
        for (size_t q = 0; q < st.jobs.size(); ++q) {
            const PotrfJob &j = st.jobs[q];
            if (j.m % 64 || j.n % 64 || j.k % 16 || j.m <= 0 || j.n <= 0) fail("shape", si, (int)q);
            auto inside = [&](int64_t o, int rows, int cols) {
                return o >= 0 && (o % nbp) + rows <= nbp && o / nbp + cols <= nbp;
            };
            if (!inside(j.c_off, j.m, j.n)) fail("output outside the tile", si, (int)q);
            writes.push_back({j.c_buf, j.c_off, j.c_off + (j.m - 1) + (int64_t)(j.n - 1) * nbp});
            if (j.a_buf != kBufNone) {
                const int acols = j.k > 0 ? j.k : j.n;
                if (!inside(j.a_off, j.m, acols)) fail("A operand outside the tile", si, (int)q);
                reads.push_back({j.a_buf, j.a_off, j.a_off + (j.m - 1) + (int64_t)(acols - 1) * nbp});
            }
            if (j.k > 0) {
                const bool ok = j.transb ? inside(j.b_off, j.n, j.k) : inside(j.b_off, j.k, j.n);
                if (!ok || j.b_buf == kBufNone) fail("B operand outside the tile", si, (int)q);
                reads.push_back({j.b_buf, j.b_off, j.b_off + (j.transb ? (j.n - 1) + (int64_t)(j.k - 1) * nbp
                                                                      : (j.k - 1) + (int64_t)(j.n - 1) * nbp)});
            }
        }
        // the device kernel's index arithmetic (subblock_kernel in potrf.hip, replayed): every
        // load and store of every lane stays inside its job's rectangles
        for (size_t q = 0; q < st.jobs.size(); ++q) {
            const PotrfJob &j = st.jobs[q];
            auto in_rect = [&](int64_t o, int64_t base, int rows, int cols) {
                const int64_t d = o - base;
                return d >= 0 && d % nbp < rows && d / nbp < cols && o < te;
            };
            const int mb = j.m / 64, nblk = mb * (j.n / 64);
            for (int local = 0; local < nblk; ++local)
                for (int wave = 0; wave < 4; ++wave)
                    for (int lane = 0; lane < 64; ++lane) {
                        const int r0 = (local % mb) * 64, c0 = (local / mb) * 64;
                        const int wr = r0 + (wave & 1) * 32, wc = c0 + (wave >> 1) * 32;
                        const int lr = lane & 15, lg = lane >> 4;
                        if (j.lower && wc >= wr + 32) continue;
                        if (j.a_buf == kBufNone || j.k == 0) {
                            for (int e = lane; e < 32 * 32; e += 64) {
                                const int i = wr + (e & 31), c = wc + (e >> 5);
                                if (!in_rect(j.c_off + i + (int64_t)c * nbp, j.c_off, j.m, j.n))
                                    fail("kernel copy index", si, (int)q);
                                if (j.a_buf != kBufNone && !in_rect(j.a_off + i + (int64_t)c * nbp, j.a_off, j.m, j.n))
                                    fail("kernel copy source index", si, (int)q);
                            }
                            continue;
                        }
                        for (int k0 = 0; k0 < j.k; k0 += 16)
                            for (int h = 0; h < 2; ++h)
                                for (int stp = 0; stp < 4; ++stp) {
                                    const int k = k0 + 4 * stp + lg;
                                    const int row = wr + 16 * h + lr, col = wc + 16 * h + lr;
                                    if (!in_rect(j.a_off + row + (int64_t)k * nbp, j.a_off, j.m, j.k))
                                        fail("kernel A index", si, (int)q);
                                    const bool okb = j.transb ? in_rect(j.b_off + col + (int64_t)k * nbp, j.b_off, j.n, j.k)
                                                              : in_rect(j.b_off + k + (int64_t)col * nbp, j.b_off, j.k, j.n);
                                    if (!okb) fail("kernel B index", si, (int)q);
                                }
                        for (int hi = 0; hi < 2; ++hi)
                            for (int hj = 0; hj < 2; ++hj)
                                for (int qq = 0; qq < 4; ++qq) {
                                    const int i = wr + 16 * hi + lr, c = wc + 16 * hj + lg + 4 * qq;
                                    if (!in_rect(j.c_off + i + (int64_t)c * nbp, j.c_off, j.m, j.n))
                                        fail("kernel C index", si, (int)q);
                                }
                    }
        }
        // the products of one launch are independent: blocks of outputs against everything else
        auto blocks_of = [&](int b, int64_t o, int rows, int cols) {
            std::vector<std::pair<int, int64_t>> out;
            for (int c = 0; c < cols; c += 64)
                for (int r = 0; r < rows; r += 64) out.push_back({b, o + r + (int64_t)c * nbp});
            return out;
        };
        for (size_t q = 0; q < st.jobs.size(); ++q) {
            const PotrfJob &j = st.jobs[q];
            auto wq = blocks_of(j.c_buf, j.c_off, j.m, j.n);
            for (size_t r = 0; r < st.jobs.size(); ++r) {
                const PotrfJob &o = st.jobs[r];
                std::vector<std::pair<int, int64_t>> other;
                if (r != q) {
                    auto w = blocks_of(o.c_buf, o.c_off, o.m, o.n);
                    other.insert(other.end(), w.begin(), w.end());
                }
                if (o.a_buf != kBufNone && !(o.k == 0 && r == q && o.a_off == o.c_off && o.a_buf == o.c_buf)) {
                    auto ra = blocks_of(o.a_buf, o.a_off, o.m, o.k > 0 ? o.k : o.n);
                    other.insert(other.end(), ra.begin(), ra.end());
                }
                if (o.k > 0) {
                    auto rb = o.transb ? blocks_of(o.b_buf, o.b_off, o.n, o.k) : blocks_of(o.b_buf, o.b_off, o.k, o.n);
                    other.insert(other.end(), rb.begin(), rb.end());
                }
                for (auto &x1 : wq)
                    for (auto &x2 : other)
                        if (x1 == x2) fail("a launch writes a 64 x 64 block another product touches", si, (int)q);
            }
        }
        // replay: all results computed from the state before the launch
        std::vector<double> A0 = A, Bs = B;
        for (size_t q = 0; q < st.jobs.size(); ++q) {
            const PotrfJob &j = st.jobs[q];
            std::vector<double> &C = *buf(j.c_buf);
            const std::vector<double> *src_a = j.a_buf == kBufA ? &A0 : j.a_buf == kBufB ? &Bs : nullptr;
            const std::vector<double> *src_b = j.b_buf == kBufA ? &A0 : j.b_buf == kBufB ? &Bs : nullptr;
            const std::vector<double> &C0 = j.c_buf == kBufA ? A0 : Bs;
            for (int c = 0; c < j.n; ++c)
                for (int r = 0; r < j.m; ++r) {
                    if (j.lower && c > r) continue;
                    const int64_t e = j.c_off + r + (int64_t)c * nbp;
                    double v;
                    if (!src_a) v = 0.0;
                    else if (j.k == 0) v = (*src_a)[j.a_off + r + (int64_t)c * nbp];
                    else {
                        double s = 0.0;
                        for (int t = 0; t < j.k; ++t) {
                            const double av = (*src_a)[j.a_off + r + (int64_t)t * nbp];
                            const double bv = j.transb ? (*src_b)[j.b_off + c + (int64_t)t * nbp]
                                                       : (*src_b)[j.b_off + t + (int64_t)c * nbp];
                            s += av * bv;
                        }
                        v = (j.beta == 0.0 ? 0.0 : j.beta * C0[e]) + j.alpha * s;
                    }
                    if (std::isnan(v)) fail("a product reads an unset entry", si, (int)q);
                    C[e] = v;
                    if (j.to32) B32[e] = (float)v;
                }
        }
        ++si;
    }
    // reference factor and inverse
    std::vector<double> L(te, 0.0), Linv(te, 0.0);
    for (int j = 0; j < nbp; ++j) {
        double d = a0[j + (int64_t)j * nbp];
        for (int t = 0; t < j; ++t) d -= L[j + (int64_t)t * nbp] * L[j + (int64_t)t * nbp];
        d = std::sqrt(d);
        L[j + (int64_t)j * nbp] = d;
        for (int i = j + 1; i < nbp; ++i) {
            double s = a0[i + (int64_t)j * nbp];
            for (int t = 0; t < j; ++t) s -= L[i + (int64_t)t * nbp] * L[j + (int64_t)t * nbp];
            L[i + (int64_t)j * nbp] = s / d;
        }
    }
    for (int c = 0; c < nbp; ++c)
        for (int i = c; i < nbp; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int t = c; t < i; ++t) s -= L[i + (int64_t)t * nbp] * Linv[t + (int64_t)c * nbp];
            Linv[i + (int64_t)c * nbp] = s / L[i + (int64_t)i * nbp];
        }
    double el = 0.0, eb = 0.0, upper = 0.0;
    for (int j = 0; j < nbp; ++j)
        for (int i = 0; i < nbp; ++i) {
            const int64_t e = i + (int64_t)j * nbp;
            if (i >= j) el = std::fmax(el, std::fabs(A[e] - L[e]) / std::fabs(L[j + (int64_t)j * nbp]));
            if (i >= j) eb = std::fmax(eb, std::fabs(B[e] - Linv[e]) * std::fabs(L[i + (int64_t)i * nbp]));
            else upper = std::fmax(upper, std::isnan(B[e]) ? INFINITY : std::fabs(B[e]));
            if (with32 && !(B32[e] == (float)B[e])) fail("FP32 copy of the inverse", -1, -1);
        }
    std::printf("nbp %d (FP32 copy %d): %zu launches, max |dL| %.2e, max |dL^-1| %.2e, max upper %.1e\n", nbp,
                with32 ? 1 : 0, plan.size(), el, eb, upper);
    if (!(el <= 1e-12) || !(eb <= 1e-12)) fail("factor or inverse differs from the plain algorithm", -1, -1);
    if (upper != 0.0) fail("strictly upper part of the inverse not zero", -1, -1);
    return failures;
}

int main() {
    check(256, true);
    check(512, true);
    check(512, false);
    if (failures) std::printf("%d failures\n", failures);
    return failures ? 1 : 0;
}
