// Host check of the FP64-band tuner's policy (tune_policy.h): the terms scale, the class key,
// the candidate bands, the choice of a class's band from its probes, and the all-FP64
// re-evaluation of a problem whose log-likelihood cancels.  Exits non-zero on the first failure.
#include "../paper_2003_05324_amd/csrc/tune_policy.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>

using namespace mpgeo;

static int failures = 0;
#define CHECK(cond)                                                         \
    do {                                                                    \
        if (!(cond)) {                                                      \
            std::printf("FAILED line %d: %s\n", __LINE__, #cond);           \
            ++failures;                                                     \
        }                                                                   \
    } while (0)

static bool close(double a, double b, double rel) { return std::fabs(a - b) <= rel * std::fabs(b); }

int main() {
    const double l2pi = std::log(2.0 * 3.14159265358979323846);
    // terms of eq. (2): n log 2 pi, |log det|, quad, halved; the profiled form uses n (log 2 pi + 1)
    // and n |log(quad / n)| in place of the last two
    CHECK(close(loglik_terms(100, -50.0, 80.0, false), 0.5 * (100 * l2pi + 50.0 + 80.0), 1e-15));
    CHECK(close(loglik_terms(100, 30.0, 80.0, false), 0.5 * (100 * l2pi + 30.0 + 80.0), 1e-15));
    CHECK(close(loglik_terms(100, -50.0, 400.0, true),
                0.5 * (100 * (l2pi + 1.0) + 100 * std::fabs(std::log(4.0)) + 50.0), 1e-15));
    // the terms bound |l| of the plain form: l = -(n log 2 pi + logdet + quad) / 2
    for (double ld : {-1e4, -10.0, 0.0, 50.0})
        for (double q : {1.0, 100.0, 1e4}) {
            const double l = -0.5 * (1000 * l2pi + ld + q);
            CHECK(std::fabs(l) <= loglik_terms(1000, ld, q, false) * (1 + 1e-15));
        }

    // class key: half-octave of n, smoothness to a quarter, range to a half-octave
    CHECK(band_class_key(1100, 0.1, 0.5) == band_class_key(1300, 0.1, 0.5));    // 2 log2 n: 20.2, 20.7
    CHECK(band_class_key(1000, 0.1, 0.5) != band_class_key(1100, 0.1, 0.5));    // 19.9 | 20.2
    CHECK(band_class_key(1000, 0.1, 0.5) != band_class_key(1000, 0.1, 1.5));
    CHECK(band_class_key(1000, 0.1, 0.5) == band_class_key(1000, 0.095, 0.55)); // 2 log2 beta: -6.6, -6.8
    CHECK(band_class_key(1000, 0.1, 0.5) != band_class_key(1000, 0.2, 0.5));

    // candidates below the last tile row, all-FP64 first
    CHECK((band_candidates(1) == std::vector<int>{-1}));
    CHECK((band_candidates(4) == std::vector<int>{-1, 0, 1, 2}));
    CHECK((band_candidates(10) == std::vector<int>{-1, 0, 1, 2, 4, 8}));

    // choice: two probes, candidates -1, 0, 1, 2; terms about 1e4 for both
    const std::vector<int> cand = band_candidates(4);
    const std::vector<int64_t> n{1000, 1200};
    const double ld = -5000.0, q = 1000.0;
    const double S0 = loglik_terms(1000, ld, q, false), S1 = loglik_terms(1200, ld, q, false);
    auto res = [&](double e0, double e1, bool ok1) {
        // res[c * np + k]: candidate c, probe k; errors relative to the terms
        std::vector<ProbeResult> r;
        const double base[2] = {-123.0, 456.0};
        const double errs[4][2] = {{0, 0}, {e0 * 50, e1 * 50}, {e0, e1}, {e0 / 10, e1 / 10}};
        for (int c = 0; c < 4; ++c)
            for (int k = 0; k < 2; ++k)
                r.push_back(ProbeResult{base[k] + errs[c][k] * (k ? S1 : S0), ld, q, c != 2 || k == 0 || ok1});
        return r;
    };
    int band;
    double err;
    // the narrowest band within the bar, with the larger of the two probes' errors
    choose_band(cand, n, res(1e-9, 0.8e-9, true), false, &band, &err);   // band 0: 5e-8, band 1: 1e-9
    CHECK(band == 0);
    CHECK(close(err, 5e-8, 1e-6));
    choose_band(cand, n, res(4e-8, 3e-8, true), false, &band, &err);     // band 0: 2e-6, band 1: 4e-8
    CHECK(band == 1);
    CHECK(close(err, 4e-8, 1e-6));
    // the second probe not positive definite at band 1: band 2
    choose_band(cand, n, res(4e-8, 3e-8, false), false, &band, &err);
    CHECK(band == 2);
    CHECK(close(err, 4e-9, 1e-6));
    // no candidate within the bar: all-FP64
    choose_band(cand, n, res(5e-6, 5e-6, true), false, &band, &err);
    CHECK(band == -1 && err == 0.0);
    // an error of exactly zero still counts the floor
    {
        std::vector<ProbeResult> r;
        for (int c = 0; c < 4; ++c)
            for (int k = 0; k < 2; ++k) r.push_back(ProbeResult{-7.0, ld, q, true});
        choose_band(cand, n, r, false, &band, &err);
        CHECK(band == 0 && err == kTuneErrFloor);
        // a probe that does not factor even all-FP64: all-FP64 for the class
        r[1].ok = false;
        choose_band(cand, n, r, false, &band, &err);
        CHECK(band == -1);
    }

    // re-evaluation: l cancelling against its terms is evaluated again, l of the terms' size not
    const double S = loglik_terms(1600, -5000.0, 1600.0, false);
    CHECK(needs_fp64_rerun(1600, 1e-3, -5000.0, 1600.0, true, 0, 1e-8, false));
    CHECK(!needs_fp64_rerun(1600, 0.5 * S, -5000.0, 1600.0, true, 0, 1e-8, false));
    // the threshold: 3 err S > 1e-5 |l|
    const double lthr = kTuneMargin * 1e-7 * S / kTuneTarget;
    CHECK(needs_fp64_rerun(1600, 0.99 * lthr, -5000.0, 1600.0, true, 2, 1e-7, false));
    CHECK(!needs_fp64_rerun(1600, 1.01 * lthr, -5000.0, 1600.0, true, 2, 1e-7, false));
    // not for all-FP64 results, failed factorizations or classes without an error
    CHECK(!needs_fp64_rerun(1600, 1e-3, -5000.0, 1600.0, true, -1, 1e-8, false));
    CHECK(!needs_fp64_rerun(1600, 1e-3, -5000.0, 1600.0, false, 0, 1e-8, false));
    CHECK(!needs_fp64_rerun(1600, 1e-3, -5000.0, 1600.0, true, 0, 0.0, false));

    if (failures) return 1;
    std::printf("tuner policy: all checks passed\n");
    return 0;
}
