// Host-side policy of the FP64-band tuner of batched evaluation (MPGEO_TUNE_BAND): the classes
// of problems, the candidate bands, the choice of a class's band from its probes' results, and
// the all-FP64 re-evaluation of a problem whose log-likelihood cancels.  Plain host code, shared
// by the library and by a host check program.
//
// The bar on a candidate's error is relative to the size of the terms that eq. (2) sums (the
// sizes of n log 2 pi, log|Sigma| and z^T Sigma^-1 z, halved), not to l itself: l passes through
// zero where those terms cancel (smooth fields of long range), while the rounding error of a
// mixed factorization scales with the terms.  The relative accuracy of l is then kept by
// evaluating again all-FP64 a problem whose l comes out too small against its terms for its
// class's error.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>
#include <vector>

namespace mpgeo {

constexpr int kTuneBands[] = {0, 1, 2, 4, 8};   // candidate FP64 bands (tiles), narrowest first
constexpr double kTuneBandBar = 1e-7;           // largest probe error, relative to the terms
constexpr int kTuneProbes = 2;                  // problems of a class evaluated per candidate
constexpr double kTuneTarget = 1e-5;            // relative accuracy of l that is kept
constexpr double kTuneMargin = 3.0;             // safety factor on the class's error
constexpr double kTuneErrFloor = 1e-9;          // a class error measured as zero counts this much

// Half the summed sizes of eq. (2)'s terms (of the profiled form when profile).
inline double loglik_terms(int64_t n, double logdet, double quad, bool profile) {
    const double dn = (double)n, l2pi = 1.8378770664093454836;   // log 2 pi
    if (profile) return 0.5 * (dn * (l2pi + 1.0) + dn * std::fabs(std::log(quad / dn)) + std::fabs(logdet));
    return 0.5 * (dn * l2pi + std::fabs(logdet) + std::fabs(quad));
}

// Class of a problem: half-octave of n, smoothness to a quarter, range to a half-octave (the two
// set Sigma's conditioning, hence how narrow a band stays within the bar); the caller appends
// what else must match (tile, path, flags).  The variance does not enter: it scales Sigma.
inline std::string band_class_key(int64_t n, double beta, double nu) {
    const int bucket = (int)std::floor(2.0 * std::log2((double)n));
    const int nu_q = (int)std::lround(4.0 * nu);
    const int beta_h = (int)std::lround(2.0 * std::log2(beta));
    return std::to_string(bucket) + "/" + std::to_string(nu_q) + "/" + std::to_string(beta_h);
}

// Candidate bands for probes of at most pmax tile rows: all-FP64 (-1) first, then the
// candidates below the last tile row (a band reaching it is all-FP64 again).
inline std::vector<int> band_candidates(int64_t pmax) {
    std::vector<int> cand{-1};
    for (int b : kTuneBands)
        if (b < pmax - 1) cand.push_back(b);
    return cand;
}

// One probe evaluation: l, log|Sigma|, z^T Sigma^-1 z and whether it factored.
struct ProbeResult {
    double loglik, logdet, quad;
    bool ok;
};

// The class's band from res[c * np + k] (candidate c of cand, probe k of sizes n[k]): the
// narrowest candidate at which every probe factors and stays within kTuneBandBar of its
// all-FP64 result (relative to its terms), with the largest such error (at least
// kTuneErrFloor); all-FP64 (-1, error 0) when none is, or when a probe does not factor even
// all-FP64.
inline void choose_band(const std::vector<int> &cand, const std::vector<int64_t> &n,
                        const std::vector<ProbeResult> &res, bool profile, int *band, double *err) {
    const size_t np = n.size(), nc = cand.size();
    *band = -1;
    *err = 0.0;
    for (size_t k = 0; k < np; ++k)
        if (!res[k].ok) return;
    for (size_t c = 1; c < nc; ++c) {
        double worst = 0.0;
        bool ok = true;
        for (size_t k = 0; k < np && ok; ++k) {
            const ProbeResult &f = res[k], &m = res[c * np + k];
            ok = m.ok;
            worst = std::max(worst, std::fabs(m.loglik - f.loglik) / loglik_terms(n[k], f.logdet, f.quad, profile));
        }
        if (ok && worst <= kTuneBandBar) {
            *band = cand[c];
            *err = std::max(worst, kTuneErrFloor);
            return;
        }
    }
}

// Whether a problem computed at a tuned band (band >= 0, factored) must be evaluated again
// all-FP64: its l is too small against its terms for the class's error err.
inline bool needs_fp64_rerun(int64_t n, double loglik, double logdet, double quad, bool factored, int band,
                             double err, bool profile) {
    if (!factored || band < 0 || err <= 0.0) return false;
    return kTuneMargin * err * loglik_terms(n, logdet, quad, profile) > kTuneTarget * std::fabs(loglik);
}

}  // namespace mpgeo
