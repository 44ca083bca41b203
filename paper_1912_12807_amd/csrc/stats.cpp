// Host FP64 detection statistics.
//
// In white noise a normalised power is a unit exponential, so a sum of H
// independent powers is Gamma(H, 1) distributed with survival
//   Q(H, S) = exp(-S) sum_{j<H} S^j / j!.
// A single-trial significance sigma corresponds to the Gaussian upper-tail
// probability p = erfc(sigma / sqrt 2) / 2; the detection threshold T_H is the
// root of Q(H, T_H) = p, and a measured sum S maps back to the sigma whose
// Gaussian tail equals Q(H, S). Everything is done in log space so that very
// strong signals (Q far below the double range) keep a finite sigma.
#include "fdas_internal.h"

#include <cmath>

namespace fdas {

static constexpr double kPi = 3.14159265358979323846264338327950288;

// log j! for the harmonic counts of a search (the same std::lgamma values,
// computed once).
static double log_factorial(int j) {
    static const struct Table {
        double v[65];
        Table() {
            for (int i = 0; i < 65; ++i) v[i] = std::lgamma(i + 1.0);
        }
    } t;
    return j < 65 ? t.v[j] : std::lgamma(j + 1.0);
}

// log Q(H, S). At or above the mean (S >= H) from the H terms S^j / j! of the
// finite series scaled by the largest, j = H - 1: each term is the next one
// times j / S, so only two logarithms are needed.
double log_gamma_sf(int H, double S) {
    if (S <= 0.0) return 0.0;
    const double ls = std::log(S);
    if (S < H) {
        // below the mean Q is close to 1: log1p of minus the lower tail
        // P(H, S) = exp(-S) sum_{j >= H} S^j / j!, whose terms shrink by S / j
        double term = 1.0, acc = 1.0;   // scaled by S^H / H!
        for (int j = H + 1; j < H + 400; ++j) {
            term *= S / j;
            acc += term;
            if (term < 1e-17 * acc) break;
        }
        return std::log1p(-std::exp(-S + H * ls - log_factorial(H) + std::log(acc)));
    }
    double acc = 1.0, r = 1.0;
    for (int j = H - 1; j > 0; --j) {   // terms j - 1 down to 0
        r *= j / S;
        acc += r;
    }
    return -S + ((H - 1) * ls - log_factorial(H - 1)) + std::log(acc);
}

// d/dS log Q(H, S) = -(S^(H-1)/(H-1)!) exp(-S) / Q(H, S).
static double dlog_gamma_sf(int H, double S, double logq) {
    return -std::exp((H - 1) * std::log(S) - log_factorial(H - 1) - S - logq);
}

// log of the Gaussian upper tail, log(erfc(s / sqrt 2) / 2), for any s.
double log_gauss_tail(double s) {
    if (s < 0.0) return std::log1p(-0.5 * std::erfc(-s / std::sqrt(2.0)));   // tail near 1
    if (s < 25.0) return std::log(0.5 * std::erfc(s / std::sqrt(2.0)));
    // asymptotic series of the Mills ratio: tail = phi(s)/s * sum (-1)^n (2n-1)!! / s^(2n)
    double inv2 = 1.0 / (s * s);
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 30; ++n) {
        double nt = -term * (2.0 * n - 1.0) * inv2;
        if (std::fabs(nt) > std::fabs(term)) break;
        term = nt;
        sum += term;
        if (std::fabs(term) < 1e-18) break;
    }
    return -0.5 * s * s - std::log(s * std::sqrt(2.0 * kPi)) + std::log(sum);
}

// d/ds log tail = -phi(s) / tail(s).
static double dlog_gauss_tail(double s, double logt) {
    return -std::exp(-0.5 * s * s - 0.5 * std::log(2.0 * kPi) - logt);
}

double threshold(int H, double sigma) {
    const double logp = log_gauss_tail(sigma);
    // bracket, then safeguarded Newton on g(T) = log Q(H, T) - log p (decreasing in T)
    double lo = 0.0, hi = std::fmax(1.0, (double)H);
    while (log_gamma_sf(H, hi) > logp) hi *= 2.0;
    double t = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
        double lq = log_gamma_sf(H, t);
        double g = lq - logp;
        if (g > 0) lo = t; else hi = t;
        double d = dlog_gamma_sf(H, t, lq);
        double tn = t - g / d;
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (std::fabs(tn - t) <= 1e-15 * std::fabs(t)) { t = tn; break; }
        t = tn;
    }
    return t;
}

double sigma_of(int H, double power) {
    const double lq = log_gamma_sf(H, power);
    // solve log_gauss_tail(s) = lq; start from the leading-order inversion.
    // Safeguarded Newton (bisection when a step leaves the bracket); once a
    // Newton step is below 1e-7 one more step reaches the rounding level of
    // the tail evaluation (waiting for steps below 1e-14 instead left it
    // hovering there between the brackets for dozens of iterations)
    double s = (lq < -1.0) ? std::sqrt(std::fmax(0.0, -2.0 * lq - std::log(-4.0 * kPi * lq))) : 0.0;
    double lo = -40.0, hi = 1e5;
    bool close = false;
    for (int it = 0; it < 200; ++it) {
        const double lt = log_gauss_tail(s);
        const double g = lt - lq;       // decreasing in s
        if (g > 0) lo = s; else hi = s;
        const double d = dlog_gauss_tail(s, lt);
        double sn = s - g / d;
        const bool newton = sn > lo && sn < hi;
        if (close) {                    // the final step
            if (newton) s = sn;
            break;
        }
        if (!newton) sn = 0.5 * (lo + hi);
        const double step = std::fabs(sn - s);
        s = sn;
        if (step <= 1e-14 * std::fmax(1.0, std::fabs(s))) break;
        close = newton && step <= 1e-7 * std::fmax(1.0, std::fabs(s));
    }
    return s;
}

}  // namespace fdas

extern "C" double fdas_threshold(int32_t harm, double sigma) {
    if (harm < 1 || !std::isfinite(sigma)) return NAN;
    return fdas::threshold(harm, sigma);
}

extern "C" double fdas_sigma(int32_t harm, double power) {
    if (harm < 1 || !std::isfinite(power)) return NAN;
    return fdas::sigma_of(harm, power);
}
