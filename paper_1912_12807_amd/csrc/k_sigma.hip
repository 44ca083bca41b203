// Significance of every candidate record, in FP32 on the device.
//
// A stage-H sum S of unit-exponential powers has the Gamma(H, 1) survival
// Q(H, S) = exp(-S) sum_{j<H} S^j / j!, and the reported sigma is the s whose
// Gaussian upper tail erfc(s / sqrt 2) / 2 equals Q, found in log space by
// safeguarded Newton steps (the same formulation as the host FP64 statistics,
// evaluated here in single precision).
//
// Error against the host FP64 value: log Q carries an absolute rounding error
// of about ulp(S) (the -S term dominates for strong signals), and d sigma /
// d log Q is about -1/sigma, so sigma is off by about ulp(S)/sigma ~ 1e-7 sigma
// (S ~ sigma^2 / 2); below sigma ~ 25 the erfc evaluation adds a few ulp. The
// records are therefore within 1e-5 (relative, or absolute below 1) of the
// host statistics, which the tests check over all stages and over powers up to
// the 10^6 of strong RFI tones. Thresholds, which decide candidates, stay FP64
// on the host (rounded once to FP32 for the comparison on the device).
#include "fdas_internal.h"

namespace fdas {

// log Q(H, S)
__device__ static float sf_log_gamma(int H, float S) {
    if (S <= 0.0f) return 0.0f;
    const float ls = logf(S);
    if (S < (float)H) {
        // below the mean: log1p of minus the lower tail exp(-S) sum_{j>=H} S^j / j!
        // (terms scaled by S^H / H!, each the previous times S / j)
        float term = 1.0f, acc = 1.0f;
        for (int j = H + 1; j < H + 200; ++j) {
            term *= S / (float)j;
            acc += term;
            if (term < 1e-8f * acc) break;
        }
        return log1pf(-expf(-S + (float)H * ls - lgammaf((float)H + 1.0f) + logf(acc)));
    }
    // the H terms scaled by the largest (j = H - 1), each the next times j / S
    float acc = 1.0f, r = 1.0f;
    for (int j = H - 1; j > 0; --j) {
        r *= (float)j / S;
        acc += r;
    }
    return -S + ((float)(H - 1) * ls - lgammaf((float)H)) + logf(acc);
}

// log(erfc(s / sqrt 2) / 2)
__device__ static float sf_log_gauss_tail(float s) {
    constexpr float kLogSqrt2Pi = 0.918938533f;   // log sqrt(2 pi)
    constexpr float kInvSqrt2 = 0.707106781f;
    if (s < 0.0f) return log1pf(-0.5f * erfcf(-s * kInvSqrt2));
    if (s < 9.0f) return logf(0.5f * erfcf(s * kInvSqrt2));
    // asymptotic series of the Mills ratio: tail = phi(s)/s sum (-1)^n (2n-1)!! / s^(2n)
    const float inv2 = 1.0f / (s * s);
    float term = 1.0f, sum = 1.0f;
    for (int n = 1; n < 20; ++n) {
        const float nt = -term * (2.0f * n - 1.0f) * inv2;
        if (fabsf(nt) > fabsf(term)) break;
        term = nt;
        sum += term;
        if (fabsf(term) < 1e-9f) break;
    }
    return -0.5f * s * s - logf(s) - kLogSqrt2Pi + logf(sum);
}

__device__ static float sf_sigma(int H, float power) {
    constexpr float kPi = 3.14159265f;
    constexpr float kLogSqrt2Pi = 0.918938533f;
    const float lq = sf_log_gamma(H, power);
    float s = (lq < -1.0f) ? sqrtf(fmaxf(0.0f, -2.0f * lq - logf(-4.0f * kPi * lq))) : 0.0f;
    float lo = -40.0f, hi = 1e5f;
    for (int it = 0; it < 100; ++it) {
        const float lt = sf_log_gauss_tail(s);
        const float g = lt - lq;              // decreasing in s
        if (g > 0.0f) lo = s; else hi = s;
        const float d = -expf(-0.5f * s * s - kLogSqrt2Pi - lt);
        float sn = s - g / d;
        if (!(sn > lo && sn < hi)) sn = 0.5f * (lo + hi);
        const float step = fabsf(sn - s);
        s = sn;
        if (step <= 2e-7f * fmaxf(1.0f, fabsf(s)) || hi - lo <= 2e-7f * fmaxf(1.0f, fabsf(s))) break;
    }
    return s;
}

// records [0, min(state[0], cap)): every record of the call, launched once
// after its last compaction
__global__ __launch_bounds__(256) void k_cand_sigma(DevCand *__restrict__ rec, const int64_t *__restrict__ state,
                                                    int64_t cap) {
    const int64_t end = state[0] < cap ? state[0] : cap;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < end; i += (int64_t)gridDim.x * 256)
        rec[i].sigma = (double)sf_sigma(1 << rec[i].s, rec[i].power);
}

hipError_t launch_cand_sigma(DevCand *rec, const int64_t *state, int64_t cap, hipStream_t st) {
    hipLaunchKernelGGL(k_cand_sigma, dim3(256), dim3(256), 0, st, rec, state, cap);
    return hipGetLastError();
}

}  // namespace fdas
