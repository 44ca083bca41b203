// K0: incoherent dedispersion of 8-bit filterbank data into trial-DM series
// (the paper's Section 2, step 2; DM plans of Tables 2-3).
//
// For one range of trial DMs with downsampling factor D:
//   y_c[j]   = sum_{d<D} x[j D + d][c]                (boxcar, j < n = nsamp / D)
//   out_i[j] = sum_c y_c[j + delta_i,c]                (y_c = D m_c past n)
// with m_c = floor((sum_t x[t][c] + nsamp/2) / nsamp) the channel's rounded mean
// with the integer delays delta_i,c computed on the host. Inputs are 8-bit, so
// every sum is an integer below 2^24 and float32 holds it exactly: the result
// does not depend on the summation order.
//
// k_fil_downsample transposes the time-major file layout into channel-major
// rows while summing D samples (64 channels x 64 outputs per block, through
// LDS); k_downsample_rows derives a coarser range's rows from the previous
// range's (DM plans double D from range to range). k_dedisperse<G> gives each
// block 256 consecutive outputs of G trial DMs: per chunk of 16 channels it
// stages, for every channel, the input span that the G delays touch in LDS
// (256 + spread floats, read once from HBM/L2 and coalesced), then every
// thread adds G LDS values per channel into G register accumulators.
#include "fdas_internal.h"

namespace fdas {

static constexpr int kDdT = 256;      // outputs per dedispersion block
static constexpr int kDdCh = 16;      // channels staged per LDS chunk

__global__ __launch_bounds__(256) void k_fil_downsample(const uint8_t *__restrict__ x, int64_t nsamp, int nchan,
                                                        int D, float *__restrict__ y, int64_t ypitch) {
    __shared__ float tile[64][65];
    const int c0 = blockIdx.y * 64;
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int64_t n = nsamp / D;
    const int c = c0 + tx;
    for (int jj = ty; jj < 64; jj += 4) {
        const int64_t j = j0 + jj;
        uint32_t acc = 0;
        if (c < nchan && j < n) {
            const uint8_t *p = x + j * D * nchan + c;
            for (int d = 0; d < D; ++d) acc += p[(int64_t)d * nchan];
        }
        tile[tx][jj] = (float)acc;
    }
    __syncthreads();
    for (int cc = ty; cc < 64; cc += 4) {
        const int c2 = c0 + cc;
        const int64_t j = j0 + tx;
        if (c2 < nchan && j < n) y[(int64_t)c2 * ypitch + j] = tile[cc][tx];
    }
}

// sums[c] += sum over a strip of 4096 samples of x[t][c] (sums zeroed beforehand).
__global__ __launch_bounds__(256) void k_channel_sums(const uint8_t *__restrict__ x, int64_t nsamp, int nchan,
                                                      unsigned long long *__restrict__ sums) {
    __shared__ uint32_t part[4][64];
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + tx;
    const int64_t t0 = (int64_t)blockIdx.y * 4096;
    const int64_t t1 = min(nsamp, t0 + 4096);
    uint32_t acc = 0;
    if (c < nchan)
        for (int64_t t = t0 + ty; t < t1; t += 4) acc += x[t * nchan + c];
    part[ty][tx] = acc;
    __syncthreads();
    if (ty == 0 && c < nchan)
        atomicAdd(sums + c, (unsigned long long)(part[0][tx] + part[1][tx] + part[2][tx] + part[3][tx]));
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long *__restrict__ v, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) v[i] = 0ull;
}

// m_c = floor((sums[c] + nsamp/2) / nsamp), as float.
__global__ __launch_bounds__(256) void k_channel_pad(const unsigned long long *__restrict__ sums, int64_t nsamp,
                                                     int nchan, float *__restrict__ pad) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c < nchan) pad[c] = (float)((sums[c] + (unsigned long long)(nsamp / 2)) / (unsigned long long)nsamp);
}

// out[c][j] = sum_{k<f} in[c][j f + k], j < n_out.
__global__ __launch_bounds__(256) void k_downsample_rows(const float *__restrict__ in, int64_t ipitch,
                                                         int64_t n_out, int f, float *__restrict__ out,
                                                         int64_t opitch) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= n_out) return;
    const float *p = in + (int64_t)c * ipitch + j * f;
    float s = 0.f;
    for (int k = 0; k < f; ++k) s += p[k];
    out[(int64_t)c * opitch + j] = s;
}

template <int G>
__global__ __launch_bounds__(kDdT) void k_dedisperse(const float *__restrict__ y, int64_t ypitch, int64_t n,
                                                     int nchan, const float *__restrict__ pad, float D,
                                                     const int32_t *__restrict__ delays, int ndm,
                                                     int span_max, float *__restrict__ out, int64_t opitch) {
    extern __shared__ float stage[];            // [kDdCh][kDdT + span_max]
    __shared__ int s_del[G][kDdCh];
    __shared__ int s_min[kDdCh];
    const int t = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * kDdT;
    const int dm0 = blockIdx.y * G;
    const int width = kDdT + span_max;
    float acc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] = 0.f;
    for (int c0 = 0; c0 < nchan; c0 += kDdCh) {
        const int nc = min(kDdCh, nchan - c0);
        for (int k = t; k < G * kDdCh; k += kDdT) {
            const int g = k / kDdCh, cc = k % kDdCh;
            const int i = min(dm0 + g, ndm - 1);  // padding DMs repeat the last one (outputs not written)
            s_del[g][cc] = cc < nc ? delays[(int64_t)i * nchan + c0 + cc] : 0;
        }
        __syncthreads();
        if (t < kDdCh) {
            int m = s_del[0][t];
#pragma unroll
            for (int g = 1; g < G; ++g) m = min(m, s_del[g][t]);
            s_min[t] = m;
        }
        __syncthreads();
        for (int cc = 0; cc < nc; ++cc) {
            const float *row = y + (int64_t)(c0 + cc) * ypitch;
            const float past = D * pad[c0 + cc];
            const int64_t base = j0 + s_min[cc];
            for (int k = t; k < width; k += kDdT) {
                const int64_t idx = base + k;
                stage[cc * width + k] = idx < n ? row[idx] : past;
            }
        }
        __syncthreads();
        for (int cc = 0; cc < nc; ++cc) {
            const float *srow = stage + cc * width + t - s_min[cc];
#pragma unroll
            for (int g = 0; g < G; ++g) acc[g] += srow[s_del[g][cc]];
        }
        __syncthreads();
    }
    const int64_t j = j0 + t;
    if (j < n) {
#pragma unroll
        for (int g = 0; g < G; ++g)
            if (dm0 + g < ndm) out[(int64_t)(dm0 + g) * opitch + j] = acc[g];
    }
}

hipError_t launch_fil_downsample(const uint8_t *x, int64_t nsamp, int nchan, int D, float *y, int64_t ypitch,
                                 hipStream_t st) {
    const int64_t n = nsamp / D;
    if (n < 1 || nchan < 1 || (n + 63) / 64 > 0x7fffffffLL || (nchan + 63) / 64 > 65535) return hipErrorInvalidValue;
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)((nchan + 63) / 64));
    hipLaunchKernelGGL(k_fil_downsample, grid, dim3(256), 0, st, x, nsamp, nchan, D, y, ypitch);
    return hipGetLastError();
}

hipError_t launch_channel_pad(const uint8_t *x, int64_t nsamp, int nchan, unsigned long long *sums, float *pad,
                              hipStream_t st) {
    if (nsamp < 1 || nchan < 1 || (nchan + 63) / 64 > 0x7fffffff || (nsamp + 4095) / 4096 > 65535)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_u64, dim3((nchan + 255) / 256), dim3(256), 0, st, sums, nchan);
    dim3 grid((unsigned)((nchan + 63) / 64), (unsigned)((nsamp + 4095) / 4096));
    hipLaunchKernelGGL(k_channel_sums, grid, dim3(256), 0, st, x, nsamp, nchan, sums);
    hipLaunchKernelGGL(k_channel_pad, dim3((nchan + 255) / 256), dim3(256), 0, st, sums, nsamp, nchan, pad);
    return hipGetLastError();
}

hipError_t launch_downsample_rows(const float *in, int64_t ipitch, int64_t n_out, int f, int nchan, float *out,
                                  int64_t opitch, hipStream_t st) {
    if (n_out < 1 || nchan < 1 || nchan > 65535 || f < 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)((n_out + 255) / 256), (unsigned)nchan);
    hipLaunchKernelGGL(k_downsample_rows, grid, dim3(256), 0, st, in, ipitch, n_out, f, out, opitch);
    return hipGetLastError();
}

size_t dedisperse_lds_bytes(int span_max) { return (size_t)kDdCh * (kDdT + span_max) * sizeof(float); }

hipError_t launch_dedisperse(const float *y, int64_t ypitch, int64_t n, int nchan, const float *pad, int D,
                             const int32_t *delays, int ndm, int G, int span_max, float *out, int64_t opitch,
                             hipStream_t st) {
    const size_t lds = dedisperse_lds_bytes(span_max);
    if (n < 1 || nchan < 1 || ndm < 1 || span_max < 0 || lds > 64 * 1024) return hipErrorInvalidValue;
    dim3 grid((unsigned)((n + kDdT - 1) / kDdT), (unsigned)((ndm + G - 1) / G));
    if (grid.y > 65535) return hipErrorInvalidValue;
    switch (G) {
    case 16: hipLaunchKernelGGL(k_dedisperse<16>, grid, dim3(kDdT), lds, st, y, ypitch, n, nchan, pad, (float)D, delays, ndm, span_max, out, opitch); break;
    case 8: hipLaunchKernelGGL(k_dedisperse<8>, grid, dim3(kDdT), lds, st, y, ypitch, n, nchan, pad, (float)D, delays, ndm, span_max, out, opitch); break;
    case 4: hipLaunchKernelGGL(k_dedisperse<4>, grid, dim3(kDdT), lds, st, y, ypitch, n, nchan, pad, (float)D, delays, ndm, span_max, out, opitch); break;
    case 2: hipLaunchKernelGGL(k_dedisperse<2>, grid, dim3(kDdT), lds, st, y, ypitch, n, nchan, pad, (float)D, delays, ndm, span_max, out, opitch); break;
    case 1: hipLaunchKernelGGL(k_dedisperse<1>, grid, dim3(kDdT), lds, st, y, ypitch, n, nchan, pad, (float)D, delays, ndm, span_max, out, opitch); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fdas
