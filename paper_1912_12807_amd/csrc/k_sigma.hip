// Significance of every candidate record, in FP64 on the device.
//
// The same arithmetic as the host functions of the detection statistics: a
// stage-H sum S of unit-exponential powers has the Gamma(H, 1) survival
// Q(H, S) = exp(-S) sum_{j<H} S^j / j!, and the reported sigma is the s whose
// Gaussian upper tail erfc(s / sqrt 2) / 2 equals Q, found in log space by
// safeguarded Newton steps. Running it here keeps long candidate lists (many
// trial DMs at a low threshold) from spending most of a search on the host.
#include "fdas_internal.h"

namespace fdas {

__device__ static double dev_log_gamma_sf(int H, double S) {
    if (S <= 0.0) return 0.0;
    const double ls = log(S);
    if (S < H) {
        // below the mean: log1p of minus the lower tail exp(-S) sum_{j>=H} S^j / j!
        double term = 1.0, acc = 1.0;
        for (int j = H + 1; j < H + 400; ++j) {
            term *= S / j;
            acc += term;
            if (term < 1e-17 * acc) break;
        }
        return log1p(-exp(-S + H * ls - lgamma(H + 1.0) + log(acc)));
    }
    // the H terms scaled by the largest (j = H - 1), each the next times j / S
    double acc = 1.0, r = 1.0;
    for (int j = H - 1; j > 0; --j) {
        r *= j / S;
        acc += r;
    }
    return -S + ((H - 1) * ls - lgamma((double)H)) + log(acc);
}

__device__ static double dev_log_gauss_tail(double s) {
    constexpr double kLogSqrt2Pi = 0.91893853320467274178;   // log sqrt(2 pi)
    if (s < 0.0) return log1p(-0.5 * erfc(-s * 0.70710678118654752440));
    if (s < 25.0) return log(0.5 * erfc(s * 0.70710678118654752440));
    // asymptotic series of the Mills ratio
    const double inv2 = 1.0 / (s * s);
    double term = 1.0, sum = 1.0;
    for (int n = 1; n < 30; ++n) {
        const double nt = -term * (2.0 * n - 1.0) * inv2;
        if (fabs(nt) > fabs(term)) break;
        term = nt;
        sum += term;
        if (fabs(term) < 1e-18) break;
    }
    return -0.5 * s * s - log(s) - kLogSqrt2Pi + log(sum);
}

__device__ static double dev_sigma(int H, double power) {
    constexpr double kPi = 3.14159265358979323846;
    constexpr double kLogSqrt2Pi = 0.91893853320467274178;
    const double lq = dev_log_gamma_sf(H, power);
    double s = (lq < -1.0) ? sqrt(fmax(0.0, -2.0 * lq - log(-4.0 * kPi * lq))) : 0.0;
    double lo = -40.0, hi = 1e5;
    bool close = false;
    for (int it = 0; it < 200; ++it) {
        const double lt = dev_log_gauss_tail(s);
        const double g = lt - lq;
        if (g > 0) lo = s; else hi = s;
        const double d = -exp(-0.5 * s * s - kLogSqrt2Pi - lt);
        double sn = s - g / d;
        const bool newton = sn > lo && sn < hi;
        if (close) {
            if (newton) s = sn;
            break;
        }
        if (!newton) sn = 0.5 * (lo + hi);
        const double step = fabs(sn - s);
        s = sn;
        if (step <= 1e-14 * fmax(1.0, fabs(s))) break;
        close = newton && step <= 1e-7 * fmax(1.0, fabs(s));
    }
    return s;
}

// records [0, min(state[0], cap)): every record of the call, launched once
// after its last compaction
__global__ __launch_bounds__(256) void k_cand_sigma(DevCand *__restrict__ rec, const int64_t *__restrict__ state,
                                                    int64_t cap) {
    const int64_t end = state[0] < cap ? state[0] : cap;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < end; i += (int64_t)gridDim.x * 256)
        rec[i].sigma = dev_sigma(1 << rec[i].s, (double)rec[i].power);
}

hipError_t launch_cand_sigma(DevCand *rec, const int64_t *state, int64_t cap, hipStream_t st) {
    hipLaunchKernelGGL(k_cand_sigma, dim3(256), dim3(256), 0, st, rec, state, cap);
    return hipGetLastError();
}

}  // namespace fdas
