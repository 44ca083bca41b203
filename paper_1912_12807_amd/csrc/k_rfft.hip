// K1: real-to-complex FFT of each series.
//
// A_k = sum_n x_n exp(-2 pi i k n / N), k = 0..N/2, for a batch of float32
// series (the "FFT of the dedispersed series" step of the pipeline, paper
// Section 2, step 3). The N real samples are read as N/2 complex values
// z_n = x_2n + i x_2n+1, transformed by a batched Stockham autosort FFT of
// length M = N/2 (one launch per radix-32 pass after one of radix 2 to 16,
// every pass reading and writing coalesced rows), and split into the real
// spectrum by
//   A_k = E_k + exp(-2 pi i k / N) O_k,  E_k = (Z_k + conj Z_{M-k}) / 2,
//   O_k = (Z_k - conj Z_{M-k}) / (2 i),  Z_M = Z_0.
// Twiddles come from sincospi of exactly representable arguments 2 j / n
// (powers of two of a pass's base twiddle; the others are products of them).
#include "dft_small.h"
#include "fdas_internal.h"

namespace fdas {

// One Stockham pass: butterfly j reads in[j + r M/R], writes out[(j - k) R + k + r Ns],
// k = j mod Ns, after twiddling input r by exp(DIR 2 pi i k r / (Ns R)).
// offs (optional, first pass only): series b starts at in + offs[b] complex values.
template <int R, int DIR>
__global__ __launch_bounds__(256) void k_stockham_pass(const float2 *__restrict__ in,
                                                       float2 *__restrict__ out, int64_t M,
                                                       int64_t Ns, int64_t pin, int64_t pout,
                                                       const int64_t *__restrict__ offs) {
    const int64_t nb = M / R;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nb) return;
    const float2 *src = in + (offs ? offs[blockIdx.y] : (int64_t)blockIdx.y * pin);
    float2 *dst = out + (int64_t)blockIdx.y * pout;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[j + r * nb];
    const int64_t k = j & (Ns - 1);
    if (Ns > 1) {
        // twiddle w^r, w = exp(DIR 2 pi i k / (Ns R)): the powers w^(2^b) from
        // sincospi of exactly representable arguments, every other power as
        // w^(r - 2^b) w^(2^b) for the lowest set bit b of r (at most log2 R
        // rounded products deep)
        const float base = (float)DIR * (float)k * (2.0f / (float)(Ns * R));
        float2 w[R];
#pragma unroll
        for (int r = 1; r < R; ++r) {
            if ((r & (r - 1)) == 0) {
                w[r] = expipi(base * (float)r);
            } else {
                const int low = r & -r;
                w[r] = cmul(w[r - low], w[low]);
            }
        }
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], w[r]);
    }
    dft_r<R, DIR>(v);
    const int64_t o = (j - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[o + r * Ns] = v[r];
}

__global__ __launch_bounds__(256) void k_rfft_post(const float2 *__restrict__ Z, int64_t zpitch,
                                                   float2 *__restrict__ A, int64_t apitch, int64_t M) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > M) return;
    const float2 *z = Z + (int64_t)blockIdx.y * zpitch;
    const float2 a = z[k == M ? 0 : k];
    const float2 c = z[k == 0 ? 0 : M - k];
    const float2 e = make_float2(0.5f * (a.x + c.x), 0.5f * (a.y - c.y));
    const float2 o = make_float2(0.5f * (a.y + c.y), -0.5f * (a.x - c.x));
    const float2 w = expipi(-(float)k / (float)M);   // exp(-2 pi i k / N), N = 2M
    A[(int64_t)blockIdx.y * apitch + k] = cadd(e, cmul(o, w));
}

template <int R>
static void pass(const float2 *in, float2 *out, int64_t M, int64_t Ns, int64_t pin, int64_t pout,
                 int nseries, const int64_t *offs, hipStream_t st) {
    const int64_t nb = M / R;
    dim3 grid((unsigned)((nb + 255) / 256), (unsigned)nseries);
    hipLaunchKernelGGL((k_stockham_pass<R, -1>), grid, dim3(256), 0, st, in, out, M, Ns, pin, pout, offs);
}

hipError_t launch_rfft(const float *x, int64_t n, int nseries, float2 *w0, float2 *w1,
                       float2 *spec, int64_t spitch, hipStream_t st, const int64_t *offs) {
    const int64_t M = n / 2;
    if (M < 4 || (M & (M - 1)) || nseries < 1 || nseries > 65535) return hipErrorInvalidValue;
    int p = 0;
    while ((int64_t(1) << p) < M) ++p;
    // radix sequence: a leading 2, 4, 8 or 16 absorbs p mod 5, then radix 32
    // (each pass is one read and one write of the batch: 2^17 points take 4
    // passes, 2^22 take 5)
    const float2 *src = reinterpret_cast<const float2 *>(x);
    int64_t pin = M;
    float2 *bufs[2] = {w0, w1};
    int which = 0;
    int64_t Ns = 1;
    const int rem = p % 5;
    if (rem) {
        switch (rem) {
        case 1: pass<2>(src, bufs[which], M, Ns, pin, M, nseries, offs, st); break;
        case 2: pass<4>(src, bufs[which], M, Ns, pin, M, nseries, offs, st); break;
        case 3: pass<8>(src, bufs[which], M, Ns, pin, M, nseries, offs, st); break;
        default: pass<16>(src, bufs[which], M, Ns, pin, M, nseries, offs, st); break;
        }
        offs = nullptr;
        Ns <<= rem;
        src = bufs[which];
        which ^= 1;
        pin = M;
    }
    while (Ns < M) {
        pass<32>(src, bufs[which], M, Ns, pin, M, nseries, offs, st);
        offs = nullptr;
        Ns *= 32;
        src = bufs[which];
        which ^= 1;
        pin = M;
    }
    dim3 grid((unsigned)((M + 1 + 255) / 256), (unsigned)nseries);
    hipLaunchKernelGGL(k_rfft_post, grid, dim3(256), 0, st, src, M, spec, spitch, M);
    return hipGetLastError();
}

}  // namespace fdas
