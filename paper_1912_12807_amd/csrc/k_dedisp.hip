// K0: incoherent dedispersion of 8-bit filterbank data into trial-DM series
// (the paper's Section 2, step 2; DM plans of Tables 2-3).
//
// For one range of trial DMs with downsampling factor D:
//   y_c[j]   = sum_{d<D} x[j D + d][c]                (boxcar, j < n = nsamp / D)
//   out_i[j] = sum_c y_c[j + delta_i,c]                (y_c = p_c past n)
// with p_c = floor((D sum_t x[t][c] + nsamp/2) / nsamp) the channel's rounded boxcar mean
// with the integer delays delta_i,c computed on the host. Inputs are 8-bit, so
// every sum is an integer below 2^24 and float32 holds it exactly: the result
// does not depend on the summation order.
//
// k_fil_downsample transposes the time-major file layout into channel-major
// rows while summing D samples (64 channels x 64 outputs per block, through
// LDS), and on its first call adds up each channel's samples for the padding
// mean; k_downsample_rows derives a coarser range's rows from the previous
// range's (DM plans double D from range to range). k_dedisperse<G> gives each
// block 256 consecutive outputs of G trial DMs: per chunk of channels it
// stages, for every channel, the input span that the G delays touch in LDS
// (256 + spread floats, read once from L2 and coalesced), then every thread
// adds G LDS values per channel into G register accumulators; the delays are
// wave-uniform scalar loads.
#include "fdas_internal.h"

#include <algorithm>

namespace fdas {

static constexpr int kDdT = 256;      // outputs per dedispersion block
static constexpr int kDdChan = 16;    // channels staged per LDS chunk

// With sums set, the block also adds its channels' sample totals to sums[c].
__global__ __launch_bounds__(256) void k_fil_downsample(const uint8_t *__restrict__ x, int64_t nsamp, int nchan,
                                                        int D, float *__restrict__ y, int64_t ypitch,
                                                        unsigned long long *__restrict__ sums) {
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
    if (sums && ty == 0 && c < nchan) {
        uint32_t tot = 0;                          // at most 64 D 255 < 2^32 for D < 2^18
        for (int jj = 0; jj < 64; ++jj) tot += (uint32_t)tile[tx][jj];
        atomicAdd(sums + c, (unsigned long long)tot);
    }
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long *__restrict__ v, int n) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) v[i] = 0ull;
}

// p_c = floor((D sums[c] + nsamp/2) / nsamp): the channel's boxcar mean, rounded.
__global__ __launch_bounds__(256) void k_channel_pad(const unsigned long long *__restrict__ sums, int64_t nsamp,
                                                     int D, int nchan, float *__restrict__ pad) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c < nchan)
        pad[c] = (float)(((unsigned long long)D * sums[c] + (unsigned long long)(nsamp / 2)) /
                         (unsigned long long)nsamp);
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

// delays: [nchan][ndm_pad] (per channel, non-decreasing in DM; entries past ndm
// repeat the last DM). Per chunk of ch channels, every channel's span
// [j0 + delta(dm0), j0 + 255 + delta(dm0 + G - 1)] is staged in LDS together with
// the chunk's G x ch delays (LDS too: scalar loads would share the LDS wait
// counter and stall the reads).
template <int G, int W>
__global__ __launch_bounds__(kDdT) void k_dedisperse(const float *__restrict__ y, int64_t ypitch, int64_t n,
                                                     int nchan, const float *__restrict__ pad,
                                                     const int32_t *__restrict__ delays, int ndm, int ndm_pad,
                                                     int chan_split, float *__restrict__ out, int64_t opitch) {
    // fixed-size stage: its LDS address and row stride are compile-time constants,
    // so a read costs one address add (lane + trial offset) and the LDS read
    __shared__ float stage[kDdChan][W];
    __shared__ int s_off[kDdChan * G];
    const int t = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * kDdT;
    const int dm0 = blockIdx.y * G;
    // blockIdx.z takes channels [c_lo, c_hi); several splits add into a zeroed output
    const int c_lo = blockIdx.z * chan_split;
    const int c_hi = min(nchan, c_lo + chan_split);
    float acc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] = 0.f;
    for (int c0 = c_lo; c0 < c_hi; c0 += kDdChan) {
        const int nc = min(kDdChan, c_hi - c0);
        // byte offset of trial g relative to the group's first trial
        for (int k = t; k < nc * G; k += kDdT) {
            const int32_t *dl = delays + (int64_t)(c0 + k / G) * ndm_pad + dm0;
            s_off[k] = (dl[k % G] - dl[0]) * (int)sizeof(float);
        }
        for (int cc = 0; cc < nc; ++cc) {
            const int c = c0 + cc;
            const int64_t base = j0 + delays[(int64_t)c * ndm_pad + dm0];
            const float *row = y + (int64_t)c * ypitch;
            const float past = pad[c];
            for (int k = t; k < W; k += kDdT) {
                const int64_t idx = base + k;
                stage[cc][k] = idx < n ? row[idx] : past;
            }
        }
        __syncthreads();
        for (int cc = 0; cc < nc; ++cc) {
            int off[G];
            if constexpr (G >= 4) {
                const int4 *o4 = reinterpret_cast<const int4 *>(s_off + cc * G);
#pragma unroll
                for (int q = 0; q < G / 4; ++q) {
                    const int4 v = o4[q];
                    off[4 * q] = v.x;
                    off[4 * q + 1] = v.y;
                    off[4 * q + 2] = v.z;
                    off[4 * q + 3] = v.w;
                }
            } else {
#pragma unroll
                for (int g = 0; g < G; ++g) off[g] = s_off[cc * G + g];
            }
            const char *p = reinterpret_cast<const char *>(&stage[cc][t]);
            float v[G];
#pragma unroll
            for (int g = 0; g < G; ++g) v[g] = *reinterpret_cast<const float *>(p + off[g]);
#pragma unroll
            for (int g = 0; g < G; ++g) acc[g] += v[g];
        }
        __syncthreads();
    }
    const int64_t j = j0 + t;
    if (j < n) {
        if (gridDim.z == 1) {
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (dm0 + g < ndm) out[(int64_t)(dm0 + g) * opitch + j] = acc[g];
        } else {
            // partial sums are integers below 2^24: float addition is exact in any order
#pragma unroll
            for (int g = 0; g < G; ++g)
                if (dm0 + g < ndm) atomicAdd(out + (int64_t)(dm0 + g) * opitch + j, acc[g]);
        }
    }
}

__global__ __launch_bounds__(256) void k_zero_rows(float *__restrict__ out, int64_t opitch, int64_t n) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j < n) out[(int64_t)blockIdx.y * opitch + j] = 0.f;
}

hipError_t launch_fil_downsample(const uint8_t *x, int64_t nsamp, int nchan, int D, float *y, int64_t ypitch,
                                 unsigned long long *sums, hipStream_t st) {
    const int64_t n = nsamp / D;
    if (n < 1 || nchan < 1 || (n + 63) / 64 > 0x7fffffffLL || (nchan + 63) / 64 > 65535) return hipErrorInvalidValue;
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)((nchan + 63) / 64));
    hipLaunchKernelGGL(k_fil_downsample, grid, dim3(256), 0, st, x, nsamp, nchan, D, y, ypitch, sums);
    return hipGetLastError();
}

hipError_t launch_zero_sums(unsigned long long *sums, int nchan, hipStream_t st) {
    if (nchan < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_u64, dim3((nchan + 255) / 256), dim3(256), 0, st, sums, nchan);
    return hipGetLastError();
}

hipError_t launch_channel_pad(const unsigned long long *sums, int64_t nsamp, int D, int nchan, float *pad,
                              hipStream_t st) {
    if (nsamp < 1 || nchan < 1 || D < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_channel_pad, dim3((nchan + 255) / 256), dim3(256), 0, st, sums, nsamp, D, nchan, pad);
    return hipGetLastError();
}

hipError_t launch_downsample_rows(const float *in, int64_t ipitch, int64_t n_out, int f, int nchan, float *out,
                                  int64_t opitch, hipStream_t st) {
    if (n_out < 1 || nchan < 1 || nchan > 65535 || f < 1) return hipErrorInvalidValue;
    dim3 grid((unsigned)((n_out + 255) / 256), (unsigned)nchan);
    hipLaunchKernelGGL(k_downsample_rows, grid, dim3(256), 0, st, in, ipitch, n_out, f, out, opitch);
    return hipGetLastError();
}

int dedisperse_width(int span_max) {
    for (int w : {288, 384, 512, 768, 1024})
        if (kDdT + span_max <= w) return w;
    return 0;
}

hipError_t launch_dedisperse(const float *y, int64_t ypitch, int64_t n, int nchan, const float *pad,
                             const int32_t *delays, int ndm, int ndm_pad, int G, int span_max, float *out,
                             int64_t opitch, hipStream_t st) {
    const int W = dedisperse_width(span_max);
    if (n < 1 || nchan < 1 || ndm < 1 || span_max < 0 || !W || ndm_pad < ndm || ndm_pad % G)
        return hipErrorInvalidValue;
    dim3 grid((unsigned)((n + kDdT - 1) / kDdT), (unsigned)(ndm_pad / G));
    if (grid.y > 65535 || ndm > 65535) return hipErrorInvalidValue;
    // split the channels over blocks until the launch has about 8192 blocks
    // (small ranges otherwise leave most of the chip idle)
    const int64_t blocks = (int64_t)grid.x * grid.y;
    int splits = (int)std::min<int64_t>((nchan + kDdChan - 1) / kDdChan, (8192 + blocks - 1) / blocks);
    splits = std::max(1, std::min(splits, 64));
    const int chan_split = ((nchan + splits - 1) / splits + kDdChan - 1) / kDdChan * kDdChan;
    grid.z = (unsigned)((nchan + chan_split - 1) / chan_split);
    if (grid.z > 1) {
        hipLaunchKernelGGL(k_zero_rows, dim3((unsigned)((n + 255) / 256), (unsigned)ndm), dim3(256), 0, st, out,
                           opitch, n);
    }
#define FDAS_DD(GG, WW)                                                                                        \
    hipLaunchKernelGGL((k_dedisperse<GG, WW>), grid, dim3(kDdT), 0, st, y, ypitch, n, nchan, pad,              \
                       delays, ndm, ndm_pad, chan_split, out, opitch)
#define FDAS_DDW(GG)                                                                                           \
    switch (W) {                                                                                               \
    case 288: FDAS_DD(GG, 288); break;                                                                         \
    case 384: FDAS_DD(GG, 384); break;                                                                         \
    case 512: FDAS_DD(GG, 512); break;                                                                         \
    case 768: FDAS_DD(GG, 768); break;                                                                         \
    default: FDAS_DD(GG, 1024); break;                                                                         \
    }
    switch (G) {
    case 16: FDAS_DDW(16); break;
    case 8: FDAS_DDW(8); break;
    case 4: FDAS_DDW(4); break;
    case 2: FDAS_DDW(2); break;
    case 1: FDAS_DDW(1); break;
    default: return hipErrorInvalidValue;
    }
#undef FDAS_DDW
#undef FDAS_DD
    return hipGetLastError();
}

}  // namespace fdas
