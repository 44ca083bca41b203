// K2: per-series normalisation by the lower median of the power spectrum.
//
// norm = s_(floor((M'-1)/2)) / ln 2, where s is the ascending order of the
// M' = N/2 - 1 powers |A_k|^2, k = 1..N/2-1 (the median of a unit exponential
// is ln 2, so white-noise powers become unit-mean). The order statistic is
// found exactly by a three-pass radix select on the IEEE bits of the
// non-negative float32 powers (bits 30..20, 19..9, 8..0): each pass builds an
// LDS histogram of the values that share the prefix found so far and picks
// the bucket that holds the wanted rank. One workgroup per series.
#include "dft_small.h"
#include "fdas_internal.h"

namespace fdas {

static constexpr int kMedThreads = 1024;

__device__ __forceinline__ uint32_t power_bits(float2 a) {
    return __float_as_uint(__fmaf_rn(a.x, a.x, __fmul_rn(a.y, a.y)));
}

__global__ __launch_bounds__(kMedThreads) void k_median_scale(const float2 *__restrict__ spec,
                                                              int64_t spitch, int64_t half,
                                                              float *__restrict__ scale,
                                                              double *__restrict__ norm) {
    __shared__ uint32_t hist[2048];
    __shared__ uint32_t s_bucket;
    __shared__ uint32_t s_below;
    const float2 *A = spec + (int64_t)blockIdx.x * spitch;
    const int tid = threadIdx.x;
    const int64_t count = half - 1;                 // bins 1..half-1
    uint32_t rank = (uint32_t)((count - 1) / 2);
    uint32_t prefix = 0, pmask = 0;
    const int shifts[3] = {20, 9, 0};
    const int widths[3] = {11, 11, 9};
    for (int pass = 0; pass < 3; ++pass) {
        const int sh = shifts[pass];
        const int nb = 1 << widths[pass];
        for (int i = tid; i < nb; i += kMedThreads) hist[i] = 0;
        __syncthreads();
        for (int64_t k = 1 + tid; k < half; k += kMedThreads) {
            uint32_t u = power_bits(A[k]);
            if ((u & pmask) == prefix) atomicAdd(&hist[(u >> sh) & (nb - 1)], 1u);
        }
        __syncthreads();
        if (tid < 64) {
            // lane l owns bins [l*per, (l+1)*per)
            const int per = nb / 64;
            uint32_t local = 0;
            for (int i = 0; i < per; ++i) local += hist[tid * per + i];
            uint32_t incl = local;
            for (int off = 1; off < 64; off <<= 1) {
                uint32_t v = __shfl_up(incl, off, 64);
                if (tid >= off) incl += v;
            }
            const uint32_t excl = incl - local;
            const bool mine = (excl <= rank) && (rank < incl);
            if (mine) {
                uint32_t acc = excl;
                for (int i = 0; i < per; ++i) {
                    uint32_t h = hist[tid * per + i];
                    if (rank < acc + h) {
                        s_bucket = (uint32_t)(tid * per + i);
                        s_below = acc;
                        break;
                    }
                    acc += h;
                }
            }
        }
        __syncthreads();
        prefix |= s_bucket << sh;
        pmask |= (uint32_t)(nb - 1) << sh;
        rank -= s_below;
        __syncthreads();
    }
    if (tid == 0) {
        const float med = __uint_as_float(prefix);
        const double nrm = (double)med / 0.69314718055994530942;
        norm[blockIdx.x] = nrm;
        scale[blockIdx.x] = med > 0.0f ? (float)sqrt(1.0 / nrm) : 0.0f;
    }
}

hipError_t launch_median_scale(const float2 *spec, int64_t spitch, int64_t half, int nseries,
                               float *scale, double *norm, hipStream_t st) {
    if (half < 2 || nseries < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_median_scale, dim3(nseries), dim3(kMedThreads), 0, st, spec, spitch, half,
                       scale, norm);
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
