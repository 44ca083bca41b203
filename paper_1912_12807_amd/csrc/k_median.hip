// K2: per-series normalisation by the lower median of the power spectrum.
//
// norm = s_(floor((M'-1)/2)) / ln 2, where s is the ascending order of the
// M' = N/2 - 1 powers |A_k|^2, k = 1..N/2-1 (the median of a unit exponential
// is ln 2, so white-noise powers become unit-mean). The order statistic is
// found exactly by a three-pass radix select on the IEEE bits of the
// non-negative float32 powers (bits 30..20, 19..9, 8..0): each pass counts the
// values that share the prefix found so far into buckets of the next bits and
// keeps the bucket that holds the wanted rank.
//
// A pass is spread over the whole chip: every workgroup histograms one chunk
// of one series in LDS and adds its non-zero buckets to the series' global
// histogram; a one-wave-per-series kernel then selects the bucket, advances
// the prefix and the rank, and clears the histogram for the next pass.
#include "dft_small.h"
#include "fdas_internal.h"

namespace fdas {

static constexpr int kHistThreads = 256;
static constexpr int kHistChunk = 8192;     // powers per histogram workgroup
static constexpr int kBins = 2048;

__device__ __forceinline__ float power_bits_f(float2 a) { return __fmaf_rn(a.x, a.x, __fmul_rn(a.y, a.y)); }
__device__ __forceinline__ uint32_t power_bits(float2 a) { return __float_as_uint(power_bits_f(a)); }

// state[b] = {prefix, mask, rank, 0}; hist[b][*] = 0.
__global__ __launch_bounds__(256) void k_med_init(uint32_t *__restrict__ hist, uint4 *__restrict__ state,
                                                  int64_t half) {
    const int b = blockIdx.x;
    for (int i = threadIdx.x; i < kBins; i += blockDim.x) hist[(int64_t)b * kBins + i] = 0;
    if (threadIdx.x == 0) state[b] = make_uint4(0u, 0u, (uint32_t)((half - 2) / 2), 0u);
}

// Histogram of bits [sh, sh + width) of the powers in one chunk of bins 1..half-1
// whose higher bits equal the series' prefix.
__global__ __launch_bounds__(kHistThreads) void k_med_hist(const float2 *__restrict__ spec, int64_t spitch,
                                                           int64_t half, const uint4 *__restrict__ state,
                                                           uint32_t *__restrict__ hist, int sh, int width) {
    __shared__ uint32_t h[kBins];
    const int b = blockIdx.y;
    const int nb = 1 << width;
    for (int i = threadIdx.x; i < nb; i += kHistThreads) h[i] = 0;
    __syncthreads();
    const uint4 s = state[b];
    const float2 *A = spec + (int64_t)b * spitch;
    const int64_t k0 = 1 + (int64_t)blockIdx.x * kHistChunk;
    const int64_t k1 = min(half, k0 + kHistChunk);
    for (int64_t k = k0 + threadIdx.x; k < k1; k += kHistThreads) {
        const uint32_t u = power_bits(A[k]);
        if ((u & s.y) == s.x) atomicAdd(&h[(u >> sh) & (nb - 1)], 1u);
    }
    __syncthreads();
    uint32_t *g = hist + (int64_t)b * kBins;
    for (int i = threadIdx.x; i < nb; i += kHistThreads) {
        const uint32_t v = h[i];
        if (v) atomicAdd(&g[i], v);
    }
}

// One wave per series: the bucket that holds the rank; on the last pass the
// median is complete and the scale is written.
__global__ __launch_bounds__(64) void k_med_select(uint32_t *__restrict__ hist, uint4 *__restrict__ state,
                                                   int sh, int width, int last, float *__restrict__ scale,
                                                   double *__restrict__ norm) {
    __shared__ uint32_t s_bucket, s_below;
    const int b = blockIdx.x;
    const int lane = threadIdx.x;
    const int nb = 1 << width;
    const int per = nb / 64;
    uint32_t *g = hist + (int64_t)b * kBins;
    const uint4 s = state[b];
    uint32_t local = 0;
    for (int i = 0; i < per; ++i) local += g[lane * per + i];
    uint32_t incl = local;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    const uint32_t excl = incl - local;
    if (excl <= s.z && s.z < incl) {
        uint32_t acc = excl;
        for (int i = 0; i < per; ++i) {
            const uint32_t c = g[lane * per + i];
            if (s.z < acc + c) {
                s_bucket = (uint32_t)(lane * per + i);
                s_below = acc;
                break;
            }
            acc += c;
        }
    }
    __syncthreads();
    for (int i = lane; i < kBins; i += 64) g[i] = 0;
    if (lane == 0) {
        const uint32_t prefix = s.x | (s_bucket << sh);
        const uint32_t mask = s.y | ((uint32_t)(nb - 1) << sh);
        state[b] = make_uint4(prefix, mask, s.z - s_below, 0u);
        if (last) {
            const float med = __uint_as_float(prefix);
            const double nrm = (double)med / 0.69314718055994530942;
            norm[b] = nrm;
            scale[b] = med > 0.0f ? (float)sqrt(1.0 / nrm) : 0.0f;
        }
    }
}

size_t median_scratch_bytes(int nseries) {
    return (size_t)nseries * (kBins * sizeof(uint32_t) + sizeof(uint4));
}

hipError_t launch_median_scale(const float2 *spec, int64_t spitch, int64_t half, int nseries,
                               float *scale, double *norm, void *scratch, hipStream_t st) {
    if (half < 2 || nseries < 1 || nseries > 65535) return hipErrorInvalidValue;
    uint32_t *hist = static_cast<uint32_t *>(scratch);
    uint4 *state = reinterpret_cast<uint4 *>(hist + (size_t)nseries * kBins);
    hipLaunchKernelGGL(k_med_init, dim3(nseries), dim3(256), 0, st, hist, state, half);
    const int64_t nchunk = (half - 1 + kHistChunk - 1) / kHistChunk;
    const int shifts[3] = {20, 9, 0};
    const int widths[3] = {11, 11, 9};
    for (int pass = 0; pass < 3; ++pass) {
        hipLaunchKernelGGL(k_med_hist, dim3((unsigned)nchunk, nseries), dim3(kHistThreads), 0, st, spec, spitch,
                           half, state, hist, shifts[pass], widths[pass]);
        hipLaunchKernelGGL(k_med_select, dim3(nseries), dim3(64), 0, st, hist, state, shifts[pass], widths[pass],
                           pass == 2 ? 1 : 0, scale, norm);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- local medians
//
// Red-noise ("local") normalisation: blocks [b_i, b_{i+1}) of at most 200 bins
// (host table), m_i = lower median of the block's powers / ln 2 at the block
// centre c_i = (b_i + b_{i+1} - 1)/2, m(k) linear between neighbouring centres
// (constant outside), A_k <- A_k / sqrt(m(k)).

// One wave per (block, series): each lane holds up to 4 powers; the median is the
// element whose count of smaller values is <= rank < count of smaller or equal.
__global__ __launch_bounds__(64) void k_block_median(const float2 *__restrict__ spec, int64_t spitch,
                                                     const int32_t *__restrict__ bstart, int nblk,
                                                     float *__restrict__ med) {
    __shared__ float s_p[256];
    const int i = blockIdx.x, b = blockIdx.y, lane = threadIdx.x;
    const int lo = bstart[i], w = bstart[i + 1] - lo;
    const float2 *A = spec + (int64_t)b * spitch + lo;
    float v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int k = lane + 64 * q;
        v[q] = k < w ? power_bits_f(A[k]) : __builtin_inff();
        s_p[k] = v[q];
    }
    __syncthreads();
    const int rank = (w - 1) / 2;
    float found = -1.f;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (lane + 64 * q >= w) continue;
        int less = 0, leq = 0;
        for (int k = 0; k < w; ++k) {
            const float u = s_p[k];
            less += u < v[q];
            leq += u <= v[q];
        }
        if (less <= rank && rank < leq) found = v[q];
    }
    // every lane that holds a copy of the median value found the same value
    const float m = __shfl(found, __ffsll((unsigned long long)__ballot(found >= 0.f)) - 1, 64);
    if (lane == 0) med[(int64_t)b * nblk + i] = m / 0.69314718055994530942f;
}

__global__ __launch_bounds__(256) void k_local_apply(float2 *__restrict__ spec, int64_t spitch, int64_t half,
                                                     const int32_t *__restrict__ bstart, int nblk,
                                                     const float *__restrict__ med, float *__restrict__ scale) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int b = blockIdx.y;
    if (k > half) return;
    float2 *A = spec + (int64_t)b * spitch;
    if (k == 0 || k == half) {
        A[k] = make_float2(0.f, 0.f);
        if (k == 0 && scale) scale[b] = 1.0f;
        return;
    }
    // block j holding k: bstart[j] <= k < bstart[j + 1]
    int lo = 0, hi = nblk;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bstart[mid] <= k) lo = mid; else hi = mid;
    }
    const float *m = med + (int64_t)b * nblk;
    const float ck = (float)k;
    const float cj = 0.5f * (float)(bstart[lo] + bstart[lo + 1] - 1);
    int i0 = ck >= cj ? lo : lo - 1;          // centres c_i0 <= k < c_i0+1
    float mk;
    if (i0 < 0) {
        mk = m[0];
    } else if (i0 >= nblk - 1) {
        mk = m[nblk - 1];
    } else {
        const float c0 = 0.5f * (float)(bstart[i0] + bstart[i0 + 1] - 1);
        const float c1 = 0.5f * (float)(bstart[i0 + 1] + bstart[i0 + 2] - 1);
        mk = m[i0] + (m[i0 + 1] - m[i0]) * ((ck - c0) / (c1 - c0));
    }
    const float2 a = A[k];
    if (mk > 0.f) {
        const float r = 1.0f / sqrtf(mk);
        A[k] = make_float2(a.x * r, a.y * r);
    } else {
        A[k] = make_float2(0.f, 0.f);
    }
}

hipError_t launch_local_norm(float2 *spec, int64_t spitch, int64_t half, int nseries, const int32_t *bstart,
                             int nblk, float *med, float *scale, hipStream_t st) {
    if (half < 2 || nseries < 1 || nseries > 65535 || nblk < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_block_median, dim3((unsigned)nblk, (unsigned)nseries), dim3(64), 0, st, spec, spitch,
                       bstart, nblk, med);
    hipLaunchKernelGGL(k_local_apply, dim3((unsigned)((half + 1 + 255) / 256), (unsigned)nseries), dim3(256), 0,
                       st, spec, spitch, half, bstart, nblk, med, scale);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_scale(float *__restrict__ scale, int n, float v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) scale[i] = v;
}

hipError_t launch_fill_scale(float *scale, int nseries, float value, hipStream_t st) {
    if (nseries < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fill_scale, dim3((nseries + 255) / 256), dim3(256), 0, st, scale, nseries, value);
    return hipGetLastError();
}

}  // namespace fdas
