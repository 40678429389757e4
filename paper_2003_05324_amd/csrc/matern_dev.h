// Device evaluation of the Matern covariance (eq. (1), Section IV-B) and of site distances,
// shared by the tile generator, the kriging kernels and the persistent batched kernel.
//
// K_nu for general smoothness: nu = mu + nl with mu in [-1/2, 1/2).  K_mu and K_mu+1
// come from Temme's series (J. Comput. Phys. 19, 1975) for x <= 2 and, for x > 2, from
// the ratios of the minimal solution u_k = U(mu + 1/2 + k, 2 mu + 1, 2x) of Kummer's
// contiguous recurrence, computed by backward (Miller) recurrence and normalised with
// Temme's identity sum_k (1/2+mu)_k (1/2-mu)_k / k! u_k = (2x)^(-mu-1/2) (the approach of
// Temme 1975 and Thompson & Barnett 1987).  Forward recurrence in the order then reaches
// nu.  Half-integer smoothness 1/2, 3/2, 5/2 uses the elementary closed forms.
#pragma once
#include "common.h"
#include "rgamma_coeffs.h"

namespace mpgeo {

namespace {

constexpr double kPi = 3.14159265358979323846;

// Gamma1(mu) = (1/Gamma(1-mu) - 1/Gamma(1+mu)) / (2 mu) and
// Gamma2(mu) = (1/Gamma(1-mu) + 1/Gamma(1+mu)) / 2 from the power series of 1/Gamma(1+x).
__device__ inline void temme_gammas(double mu, double &g1, double &g2) {
    const double m2 = mu * mu;
    double odd = 0.0, even = 0.0;
#pragma unroll
    for (int j = MPGEO_RGAMMA_NCOEF - 1; j >= 0; --j) {
        if (j & 1) odd = odd * m2 + kRGammaCoef[j];
        else even = even * m2 + kRGammaCoef[j];
    }
    g1 = -odd;
    g2 = even;
}

// K_mu(x), K_mu+1(x) for |mu| <= 1/2 and 0 < x <= 2 (Temme's series).
__device__ void bessel_k_small(double mu, double x, double &k0, double &k1) {
    double g1, g2;
    temme_gammas(mu, g1, g2);
    const double gp = 1.0 / (g2 - mu * g1);   // Gamma(1 + mu)
    const double gm = 1.0 / (g2 + mu * g1);   // Gamma(1 - mu)
    const double lg = log(2.0 / x);
    const double sig = mu * lg;
    const double fact = (mu == 0.0) ? 1.0 : (kPi * mu) / sinpi(mu);
    const double fact2 = (sig == 0.0) ? 1.0 : sinh(sig) / sig;
    double f = fact * (cosh(sig) * g1 + fact2 * lg * g2);
    const double e = exp(sig);                // (2/x)^mu
    double p = 0.5 * e * gp;
    double q = 0.5 / e * gm;
    double c = 1.0;
    const double d = 0.25 * x * x;
    double s0 = f, s1 = p;
    const double m2 = mu * mu;
    for (int k = 1; k < 64; ++k) {
        const double dk = (double)k;
        f = (dk * f + p + q) / (dk * dk - m2);
        c *= d / dk;
        p /= (dk - mu);
        q /= (dk + mu);
        const double h = p - dk * f;
        const double t0 = c * f, t1 = c * h;
        s0 += t0;
        s1 += t1;
        if (fabs(t0) < 1e-17 * fabs(s0) && fabs(t1) < 1e-17 * fabs(s1)) break;
    }
    k0 = s0;
    k1 = s1 * 2.0 / x;
}

// e^x K_mu(x), e^x K_mu+1(x) for |mu| < 1/2 and x > 2.
__device__ void bessel_k_large_scaled(double mu, double x, double &k0s, double &k1s) {
    const double m2 = mu * mu;
    int kmax = 20 + (int)(130.0 / x);
    if (kmax > 90) kmax = 90;
    // C_k = (1/2 + mu)_k (1/2 - mu)_k / k!  at k = kmax
    double ck = 1.0;
    for (int t = 1; t <= kmax; ++t) {
        const double h = t - 0.5;
        ck *= (h * h - m2) / t;
    }
    double up1 = 0.0, u = 1.0;   // u_{k+1}, u_k (unnormalised), starting at k = kmax
    double s = ck * u;
    for (int k = kmax; k >= 1; --k) {
        const double kh = k + 0.5;
        const double um1 = 2.0 * (k + x) * u - (kh * kh - m2) * up1;
        up1 = u;
        u = um1;
        const double hm = k - 0.5;
        ck *= k / (hm * hm - m2);   // C_{k-1}
        s += ck * u;
    }
    k0s = sqrt(kPi / (2.0 * x)) / (s / u);
    k1s = k0s / x * (x + mu + 0.5 + (m2 - 0.25) * up1 / u);
}

// The quantities of the two K_mu evaluations above that depend on the smoothness only, formed
// once per workgroup (in LDS) so that the per-entry loops multiply instead of divide:
//   Miller:  C_k = prod_{t <= k} ((t - 1/2)^2 - mu^2) / t and 1 / ((k - 1/2)^2 - mu^2);
//   Temme:   Gamma1, Gamma2, Gamma(1 + mu), Gamma(1 - mu), pi mu / sin(pi mu), and
//            1 / (k^2 - mu^2), 1 / (k - mu), 1 / (k + mu), 1 / k.
struct MaternTable {
    static constexpr int kMiller = 91;   // k = 0 .. 90 (the largest start of the recurrence)
    static constexpr int kSeries = 64;   // k = 1 .. 63 (the series' longest run)
    double ck[kMiller], ia[kMiller];
    double isq[kSeries], im[kSeries], ip[kSeries], ik[kSeries];
    double g1, g2, gp, gm, fact;
};

// Built by all threads of the workgroup; the caller synchronises before use.
__device__ inline void matern_table_build(double mu, MaternTable &t) {
    const double m2 = mu * mu;
    for (int k = threadIdx.x; k < MaternTable::kMiller; k += blockDim.x) {
        const double h = k - 0.5;
        t.ia[k] = (k == 0) ? 0.0 : 1.0 / (h * h - m2);
        double c = 1.0;
        for (int q = 1; q <= k; ++q) {
            const double hq = q - 0.5;
            c *= (hq * hq - m2) / q;
        }
        t.ck[k] = c;
    }
    for (int k = threadIdx.x; k < MaternTable::kSeries; k += blockDim.x) {
        const double dk = (double)k;
        t.isq[k] = (k == 0) ? 0.0 : 1.0 / (dk * dk - m2);
        t.im[k] = (k == 0) ? 0.0 : 1.0 / (dk - mu);
        t.ip[k] = (k == 0) ? 0.0 : 1.0 / (dk + mu);
        t.ik[k] = (k == 0) ? 0.0 : 1.0 / dk;
    }
    if (threadIdx.x == 0) {
        temme_gammas(mu, t.g1, t.g2);
        t.gp = 1.0 / (t.g2 - mu * t.g1);
        t.gm = 1.0 / (t.g2 + mu * t.g1);
        t.fact = (mu == 0.0) ? 1.0 : (kPi * mu) / sinpi(mu);
    }
}

// bessel_k_small with the smoothness-only quantities from the table.
__device__ inline void bessel_k_small_tab(double mu, double x, const MaternTable &t, double &k0, double &k1) {
    const double lg = log(2.0 / x);
    const double sig = mu * lg;
    const double fact2 = (sig == 0.0) ? 1.0 : sinh(sig) / sig;
    double f = t.fact * (cosh(sig) * t.g1 + fact2 * lg * t.g2);
    const double e = exp(sig);
    double p = 0.5 * e * t.gp;
    double q = 0.5 / e * t.gm;
    double c = 1.0;
    const double d = 0.25 * x * x;
    double s0 = f, s1 = p;
    for (int k = 1; k < MaternTable::kSeries; ++k) {
        const double dk = (double)k;
        f = (dk * f + p + q) * t.isq[k];
        c *= d * t.ik[k];
        p *= t.im[k];
        q *= t.ip[k];
        const double h = p - dk * f;
        const double t0 = c * f, t1 = c * h;
        s0 += t0;
        s1 += t1;
        if (fabs(t0) < 1e-17 * fabs(s0) && fabs(t1) < 1e-17 * fabs(s1)) break;
    }
    k0 = s0;
    k1 = s1 * 2.0 / x;
}

// bessel_k_large_scaled with C_kmax and the recurrence's reciprocals from the table.
__device__ inline void bessel_k_large_scaled_tab(double mu, double x, const MaternTable &t, double &k0s,
                                                 double &k1s) {
    const double m2 = mu * mu;
    int kmax = 20 + (int)(130.0 / x);
    if (kmax > 90) kmax = 90;
    double ck = t.ck[kmax];
    double up1 = 0.0, u = 1.0;
    double s = ck * u;
    for (int k = kmax; k >= 1; --k) {
        const double kh = k + 0.5;
        const double um1 = 2.0 * (k + x) * u - (kh * kh - m2) * up1;
        up1 = u;
        u = um1;
        ck *= k * t.ia[k];   // C_{k-1}
        s += ck * u;
    }
    k0s = sqrt(kPi / (2.0 * x)) / (s / u);
    k1s = k0s / x * (x + mu + 0.5 + (m2 - 0.25) * up1 / u);
}

// C(r; theta) of eq. (1); C(0) = sigma2 (the r -> 0 limit).  With a table (general
// smoothness; a table must be given then), the K_mu loops take their smoothness-only factors
// from it.
template <bool kTable>
__device__ inline double matern_cov_impl(double r, const MaternParams &mp, const MaternTable *tab) {
    if (r == 0.0) return mp.sigma2;
    const double x = r / mp.beta;
    switch (mp.mode) {
        case 1: return mp.sigma2 * exp(-x);
        case 2: return mp.sigma2 * (1.0 + x) * exp(-x);
        case 3: return mp.sigma2 * (1.0 + x + x * x * (1.0 / 3.0)) * exp(-x);
        default: break;
    }
    if (x > 745.0) return 0.0;
    const double mu = mp.mu;
    double k0, k1;
    bool scaled;
    if (mu == -0.5) {          // K_{-1/2} = K_{1/2} = sqrt(pi/2x) e^-x, K_{1/2}(1 + 1/x) next
        k0 = sqrt(kPi / (2.0 * x));
        k1 = k0 * (1.0 + 1.0 / x);
        scaled = true;
    } else if (x <= 2.0) {
        if constexpr (kTable) bessel_k_small_tab(mu, x, *tab, k0, k1);
        else bessel_k_small(mu, x, k0, k1);
        scaled = false;
    } else {
        if constexpr (kTable) bessel_k_large_scaled_tab(mu, x, *tab, k0, k1);
        else bessel_k_large_scaled(mu, x, k0, k1);
        scaled = true;
    }
    for (int i = 1; i <= mp.nl; ++i) {
        const double k2 = (2.0 * (mu + i) / x) * k1 + k0;
        k0 = k1;
        k1 = k2;
    }
    if (scaled) return mp.pref * exp(mp.nu * log(x) - x) * k0;
    return mp.pref * pow(x, mp.nu) * k0;
}

__device__ inline double matern_cov(double r, const MaternParams &mp) {
    return matern_cov_impl<false>(r, mp, nullptr);
}
__device__ inline double matern_cov_tab(double r, const MaternParams &mp, const MaternTable &tab) {
    return matern_cov_impl<true>(r, mp, &tab);
}

constexpr double kDegToRad = 3.14159265358979323846 / 180.0;

// Great-circle distance by the haversine formula, from latitudes in radians (with their
// cosines) and the longitude difference in degrees:
//   a = sin^2(dlat / 2) + cos(lat1) cos(lat2) sin^2(dlon / 2),  d = 2 R asin(sqrt(min(a, 1))).
__device__ inline double haversine(double dlon_deg, double lat1, double cos1, double lat2, double cos2) {
    const double sp = sin(0.5 * (lat2 - lat1));
    const double sl = sin(0.5 * (dlon_deg * kDegToRad));
    double a = sp * sp + (cos1 * cos2) * (sl * sl);
    a = a < 1.0 ? a : 1.0;
    return 2.0 * kEarthRadiusKm * asin(sqrt(a));
}

// Distance between two sites: Euclidean, or great-circle for (lon, lat) in degrees.
__device__ inline double site_distance(double x1, double y1, double x2, double y2, int gcd) {
    if (gcd) {
        const double p1 = y1 * kDegToRad, p2 = y2 * kDegToRad;
        return haversine(x2 - x1, p1, cos(p1), p2, cos(p2));
    }
    const double dx = x1 - x2, dy = y1 - y2;
    return sqrt(dx * dx + dy * dy);
}

}  // namespace

}  // namespace mpgeo
