// K1: real-to-complex FFT of each series, staged in LDS.
//
// A_k = sum_n x_n exp(-2 pi i k n / N), k = 0..N/2, for a batch of float32
// series (the "FFT of the dedispersed series" step of the pipeline, paper
// Section 2, step 3). The N real samples are read as M = N/2 complex values
// z_n = x_2n + i x_2n+1, transformed by a complex FFT of length M and split
// into the real spectrum by
//   A_k = E_k + exp(-2 pi i k / N) O_k,  E_k = (Z_k + conj Z_{M-k}) / 2,
//   O_k = (Z_k - conj Z_{M-k}) / (2 i),  Z_M = Z_0.
// M may be any product of powers of 2, 3 and 5.
//
// Every transform runs in LDS: a workgroup stages T lines of P points (at most
// kLdsPoints complex values, 64 KB), transforms each line by Stockham passes
// of radix 8, 4, 2, 5 and 3 (every pass reads its butterflies' points into
// registers, then writes them back after a barrier, so one buffer suffices),
// and writes the lines out. Points of a line sit at an XOR-swizzled slot
// (the low 4 bits of the index XOR a function of the next bits and the line)
// so that the stride-R writes of the first passes and the line-interleaved
// loads spread over the LDS banks.
//   * M <= kLdsPoints: one workgroup per series does the whole FFT and the
//     real split (both Z_k and Z_{M-k} are in LDS): one read and one write.
//   * larger M = M1 M2 (four-step): pass 1 transforms columns n2 of
//     z[n1 M2 + n2] over n1 (length M1, T consecutive columns per workgroup),
//     multiplies by exp(-2 pi i n2 k1 / M) and writes Y[k1 M2 + n2]; pass 2
//     transforms rows k1 of Y over n2 (length M2) and splits them into A:
//     a workgroup holds T/2 consecutive rows and their T/2 mirror rows
//     M1 - k1, where the partners Z_{M-k} of its outputs lie. Each pass reads
//     and writes every point once, T (pass 1) or T/2 (pass 2) consecutive
//     complex values per access group. (With T = 1, possible only for odd
//     factors, pass 2 writes Z[k1 + M1 k2] and a last pass splits Z into A.)
// Twiddles come from sincospi of 2 j / n (exact for power-of-two n).
#include "dft_small.h"
#include "fdas_internal.h"

namespace fdas {

static constexpr int kFftThreads = 512;
static constexpr int kLdsPoints = 8192;   // complex values staged per workgroup (64 KB)
static constexpr int kMaxPasses = 24;

// Radices of an in-LDS transform of length P (the product of the radices).
struct FftPlan {
    int P;
    int npass;
    int radix[kMaxPasses];
};

// Slot of point n of line t: the low 4 bits of n XOR (n / 16 + 5 t) within
// complete groups of 16 (a permutation of each group), n itself in a trailing
// partial group.
__device__ __forceinline__ int swz(int n, int t, int P) {
    return ((n | 15) < P) ? (n ^ (((n >> 4) + 5 * t) & 15)) : n;
}

// v[q] *= w^q, w = expipi(x): w from sincospi, w^2 and w^4 from sincospi of the
// exactly doubled arguments, the other powers as products of these
template <int R>
__device__ __forceinline__ void twiddle(float2 *v, float x) {
    float2 w[R];
#pragma unroll
    for (int q = 1; q < R; ++q) {
        if ((q & (q - 1)) == 0) {
            w[q] = expipi(x * (float)q);
        } else {
            const int low = q & -q;
            w[q] = cmul(w[q - low], w[low]);
        }
    }
#pragma unroll
    for (int q = 1; q < R; ++q) v[q] = cmul(v[q], w[q]);
}

// The same pass with P, R and Ns known at compile time (power-of-two P):
// index arithmetic by shifts and masks.
template <int P, int R, int NS>
__device__ __forceinline__ void fft_pass_c(float2 *buf, int T) {
    constexpr int nb = P / R;
    const int total = T * nb;
    constexpr int MAXB = (kLdsPoints / R + kFftThreads - 1) / kFftThreads;
    float2 v[MAXB][R];
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        const int idx = (int)threadIdx.x + m * kFftThreads;
        if (idx < total) {
            const int t = idx / nb, i = idx % nb;
            const float2 *src = buf + t * P;
#pragma unroll
            for (int q = 0; q < R; ++q) v[m][q] = src[swz(i + q * nb, t, P)];
            if constexpr (NS > 1) twiddle<R>(v[m], -2.0f / (float)(NS * R) * (float)(i % NS));
            dft_r<R, -1>(v[m]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        const int idx = (int)threadIdx.x + m * kFftThreads;
        if (idx < total) {
            const int t = idx / nb, i = idx % nb;
            const int k = i % NS;
            float2 *dst = buf + t * P;
            const int o = (i - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) dst[swz(o + q * NS, t, P)] = v[m][q];
        }
    }
    __syncthreads();
}

// radix-8 passes, then one of radix 4 or 2 for the remaining factor
template <int P, int NS = 1>
__device__ __forceinline__ void lds_fft_pow2(float2 *buf, int T) {
    if constexpr (NS < P) {
        constexpr int left = P / NS;
        constexpr int R = left >= 8 ? 8 : left;
        fft_pass_c<P, R, NS>(buf, T);
        lds_fft_pow2<P, NS * R>(buf, T);
    }
}

// One Stockham pass of radix R with stride Ns over T lines of P points
// (line t at buf + t P): butterfly i of a line reads points i + q P/R, twiddles
// input q by exp(-2 pi i k q / (Ns R)), k = i mod Ns, and writes output q to
// (i - k) R + k + q Ns.
template <int R>
__device__ __forceinline__ void fft_pass(float2 *buf, int P, int T, int Ns) {
    const int nb = P / R;
    const int total = T * nb;
    constexpr int MAXB = (kLdsPoints / R + kFftThreads - 1) / kFftThreads;
    float2 v[MAXB][R];
    const float scale = -2.0f / (float)(Ns * R);
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        const int idx = (int)threadIdx.x + m * kFftThreads;
        if (idx < total) {
            const int t = idx / nb, i = idx - t * nb;
            const float2 *src = buf + t * P;
#pragma unroll
            for (int q = 0; q < R; ++q) v[m][q] = src[swz(i + q * nb, t, P)];
            const int k = i % Ns;
            if (Ns > 1) twiddle<R>(v[m], scale * (float)k);
            dft_r<R, -1>(v[m]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < MAXB; ++m) {
        const int idx = (int)threadIdx.x + m * kFftThreads;
        if (idx < total) {
            const int t = idx / nb, i = idx - t * nb;
            const int k = i % Ns;
            float2 *dst = buf + t * P;
            const int o = (i - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) dst[swz(o + q * Ns, t, P)] = v[m][q];
        }
    }
    __syncthreads();
}

// Forward FFT of T lines of P points staged in buf (natural order in and out,
// swizzled slots).
__device__ __forceinline__ void lds_fft(float2 *buf, const FftPlan &fp, int T) {
    int Ns = 1;
    for (int p = 0; p < fp.npass; ++p) {
        const int R = fp.radix[p];
        switch (R) {
        case 8: fft_pass<8>(buf, fp.P, T, Ns); break;
        case 4: fft_pass<4>(buf, fp.P, T, Ns); break;
        case 2: fft_pass<2>(buf, fp.P, T, Ns); break;
        case 5: fft_pass<5>(buf, fp.P, T, Ns); break;
        default: fft_pass<3>(buf, fp.P, T, Ns); break;
        }
        Ns *= R;
    }
}

// PC > 0: a power-of-two length known at compile time; 0: the plan's length
template <int PC>
__device__ __forceinline__ void run_fft(float2 *buf, const FftPlan &fp, int T) {
    if constexpr (PC > 0) lds_fft_pow2<PC>(buf, T);
    else lds_fft(buf, fp, T);
}

// A_k from Z (Z_M = Z_0): E_k + exp(-2 pi i k / N) O_k.
__device__ __forceinline__ float2 real_split(float2 a, float2 c, int64_t k, int64_t M) {
    const float2 e = make_float2(0.5f * (a.x + c.x), 0.5f * (a.y - c.y));
    const float2 o = make_float2(0.5f * (a.y + c.y), -0.5f * (a.x - c.x));
    // exp(-2 pi i k / N) = expipi(-k / M): an exact argument for power-of-two M
    const float2 w = expipi(-(float)k / (float)M);
    return cadd(e, cmul(o, w));
}

// series b of a batch: at z + offs[b] (ragged) or z + b M (complex values)
__device__ __forceinline__ const float2 *series_at(const float2 *z, const int64_t *offs, int b, int64_t M) {
    return z + (offs ? offs[b] : (int64_t)b * M);
}

// M <= kLdsPoints: one workgroup per series, FFT and real split in LDS.
template <int PC>
__global__ __launch_bounds__(kFftThreads) void k_rfft_lds(const float2 *__restrict__ z,
                                                          const int64_t *__restrict__ offs, FftPlan fp,
                                                          float2 *__restrict__ A, int64_t apitch) {
    extern __shared__ __align__(16) float2 fbuf[];
    const int b = blockIdx.x;
    const int M = PC > 0 ? PC : fp.P;
    const float2 *src = series_at(z, offs, b, M);
    for (int n = threadIdx.x; n < M; n += kFftThreads) fbuf[swz(n, 0, M)] = src[n];
    __syncthreads();
    run_fft<PC>(fbuf, fp, 1);
    float2 *dst = A + (int64_t)b * apitch;
    for (int k = threadIdx.x; k <= M; k += kFftThreads) {
        const float2 a = fbuf[swz(k == M ? 0 : k, 0, M)];
        const float2 c = fbuf[swz(k == 0 ? 0 : M - k, 0, M)];
        dst[k] = real_split(a, c, k, M);
    }
}

// Four-step pass 1: T columns n2 = n2_0..n2_0+T-1 of series b, transform over
// n1 (length M1), twiddle, Y[k1 M2 + n2].
template <int PC>
__global__ __launch_bounds__(kFftThreads) void k_fft_cols(const float2 *__restrict__ z,
                                                          const int64_t *__restrict__ offs, FftPlan fp,
                                                          int M2, int lgT, int64_t tiles_per_series,
                                                          int64_t total_tiles, float2 *__restrict__ Y) {
    const int T = 1 << lgT;
    extern __shared__ __align__(16) float2 fbuf[];
    // consecutive tiles of a series run on one XCD: their T-wide column groups
    // share the L2 lines of every row
    const int64_t w = blockIdx.x;
    const int64_t per_xcd = (total_tiles + 7) / 8;
    const int64_t g = (w & 7) * per_xcd + (w >> 3);
    if (g >= total_tiles) return;
    const int b = (int)(g / tiles_per_series);
    const int n20 = (int)(g - (int64_t)b * tiles_per_series) * T;
    const int M1 = PC > 0 ? PC : fp.P;
    const int64_t M = (int64_t)M1 * M2;
    const float2 *src = series_at(z, offs, b, M) + n20;
    for (int e = threadIdx.x; e < T * M1; e += kFftThreads) {
        const int t = e & (T - 1), n1 = e >> lgT;
        fbuf[t * M1 + swz(n1, t, M1)] = src[(int64_t)n1 * M2 + t];
    }
    __syncthreads();
    run_fft<PC>(fbuf, fp, T);
    float2 *dst = Y + (int64_t)b * M + n20;
    for (int e = threadIdx.x; e < T * M1; e += kFftThreads) {
        const int t = e & (T - 1), k1 = e >> lgT;
        const int m = (n20 + t) * k1;                       // twiddle exp(-2 pi i n2 k1 / M), n2 k1 < M
        const float2 tw = expipi(-2.0f * (float)m / (float)M);
        dst[(int64_t)k1 * M2 + t] = cmul(fbuf[t * M1 + swz(k1, t, M1)], tw);
    }
}

// Four-step pass 2 without the split (T = 1): T rows k1 = k10..k10+T-1 of Y,
// transform over n2 (length M2), Z[k1 + M1 k2] into the spectrum rows.
template <int PC>
__global__ __launch_bounds__(kFftThreads) void k_fft_rows(const float2 *__restrict__ Y, FftPlan fp, int M1,
                                                          int lgT, int64_t tiles_per_series, int64_t total_tiles,
                                                          float2 *__restrict__ Z, int64_t zpitch) {
    const int T = 1 << lgT;
    extern __shared__ __align__(16) float2 fbuf[];
    const int64_t w = blockIdx.x;
    const int64_t per_xcd = (total_tiles + 7) / 8;
    const int64_t g = (w & 7) * per_xcd + (w >> 3);
    if (g >= total_tiles) return;
    const int b = (int)(g / tiles_per_series);
    const int k10 = (int)(g - (int64_t)b * tiles_per_series) * T;
    const int M2 = PC > 0 ? PC : fp.P;
    const int64_t M = (int64_t)M1 * M2;
    const float2 *src = Y + (int64_t)b * M + (int64_t)k10 * M2;
    for (int e = threadIdx.x; e < T * M2; e += kFftThreads) {
        const int t = e / M2, n2 = e - t * M2;
        fbuf[t * M2 + swz(n2, t, M2)] = src[e];
    }
    __syncthreads();
    run_fft<PC>(fbuf, fp, T);
    float2 *dst = Z + (int64_t)b * zpitch + k10;
    for (int e = threadIdx.x; e < T * M2; e += kFftThreads) {
        const int t = e & (T - 1), k2 = e >> lgT;
        dst[(int64_t)k2 * M1 + t] = fbuf[t * M2 + swz(k2, t, M2)];
    }
}

// Four-step pass 2 fused with the real split. Output k = k1 + M1 k2 needs
// Z_{M-k}, which lies in row (M1 - k1) mod M1 at k2' = M2 - 1 - k2 (k1 > 0) or
// (M2 - k2) mod M2 (k1 = 0). So the T lines of a workgroup hold T/2 "lower"
// rows r = r0..r0+T/2-1 (r <= M1/2) in lines 0..T/2-1 and their mirrors
// (M1 - r) mod M1 in lines T/2..T-1: after the row transforms every output of
// these rows has both its points in LDS and A is written directly. A mirror
// equal to its own row (r = 0, r = M1/2) is written from the lower line only;
// the row-0 line also writes A_M (Z_M = Z_0).
template <int PC>
__global__ __launch_bounds__(kFftThreads) void k_fft_rows_split(const float2 *__restrict__ Y, FftPlan fp, int M1,
                                                                int lgT, int64_t tiles_per_series,
                                                                int64_t total_tiles, float2 *__restrict__ A,
                                                                int64_t apitch) {
    const int T = 1 << lgT, H = T >> 1;
    extern __shared__ __align__(16) float2 fbuf[];
    const int64_t w = blockIdx.x;
    const int64_t per_xcd = (total_tiles + 7) / 8;
    const int64_t g = (w & 7) * per_xcd + (w >> 3);
    if (g >= total_tiles) return;
    const int b = (int)(g / tiles_per_series);
    const int r0 = (int)(g - (int64_t)b * tiles_per_series) * H;
    const int M2 = PC > 0 ? PC : fp.P;
    const int64_t M = (int64_t)M1 * M2;
    const int rmax = M1 / 2;   // last lower row
    const float2 *src = Y + (int64_t)b * M;
    // line t: its row, or -1 past the last lower row
    auto row_of = [&](int t) -> int {
        const int r = r0 + (t & (H - 1));
        if (r > rmax) return -1;
        return t < H ? r : (r == 0 ? 0 : M1 - r);
    };
    for (int e = threadIdx.x; e < T * M2; e += kFftThreads) {
        const int t = e / M2, n2 = e - t * M2;
        const int row = row_of(t);
        if (row >= 0) fbuf[t * M2 + swz(n2, t, M2)] = src[(int64_t)row * M2 + n2];
    }
    __syncthreads();
    run_fft<PC>(fbuf, fp, T);
    float2 *dst = A + (int64_t)b * apitch;
    for (int e = threadIdx.x; e < T * M2; e += kFftThreads) {
        const int t = e & (T - 1), k2 = e >> lgT;
        const int r = r0 + (t & (H - 1));
        if (r > rmax || (t >= H && (r == 0 || 2 * r == M1))) continue;
        const int row = t < H ? r : M1 - r;
        const int pt = t ^ H;                                        // the mirror row's line
        const int p2 = row == 0 ? (k2 == 0 ? 0 : M2 - k2) : M2 - 1 - k2;
        const float2 zk = fbuf[t * M2 + swz(k2, t, M2)];
        const float2 zm = fbuf[pt * M2 + swz(p2, pt, M2)];
        const int64_t k = row + (int64_t)M1 * k2;
        dst[k] = real_split(zk, zm, k, M);
        if (row == 0 && k2 == 0) dst[M] = real_split(zk, zk, M, M);
    }
}

// Real split in place after the T = 1 pass 2: one thread per pair (k, M - k)
// reads Z_k and Z_{M-k} from the spectrum row and writes A_k and A_{M-k}
// (k = 0: A_0 and A_M from Z_0), so every point is read once.
__global__ __launch_bounds__(256) void k_rfft_split_pairs(float2 *__restrict__ A, int64_t apitch, int64_t M) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (2 * k > M) return;
    float2 *a = A + (int64_t)blockIdx.y * apitch;
    const float2 zk = a[k];
    const float2 zm = a[k == 0 ? 0 : M - k];
    a[k] = real_split(zk, zm, k, M);
    if (k == 0) a[M] = real_split(zk, zk, M, M);
    else if (2 * k != M) a[M - k] = real_split(zm, zk, M - k, M);
}

namespace {

bool smooth5(int64_t m) {
    if (m < 1) return false;
    for (int f : {2, 3, 5})
        while (m % f == 0) m /= f;
    return m == 1;
}

bool radix_plan(int P, FftPlan &fp) {
    fp.P = P;
    fp.npass = 0;
    int m = P;
    for (int r : {8, 4, 2, 5, 3}) {
        while (m % r == 0) {
            if (fp.npass == kMaxPasses) return false;
            fp.radix[fp.npass++] = r;
            m /= r;
        }
    }
    return m == 1;
}

struct FourStep {
    int M1, M2;   // column and row lengths, M = M1 M2
    int T1, T2;   // columns per workgroup of pass 1, lines per workgroup of pass 2
};

// Widest power-of-two tile (at most 64 lines) of lines of P points that fits
// in LDS.
int tile_lines(int64_t P) {
    int t = 1;
    while (t < 64 && P * (2 * t) <= kLdsPoints) t *= 2;
    return t;
}

// Split M into M1 x M2 (both 5-smooth, at most kLdsPoints): the widest tile
// T that divides both and fits in LDS for both (T1 = T consecutive columns in
// pass 1), then the most even split. Pass 2 stages as many lines as fit (T2,
// no divisibility needed: rows and mirrors are paired); T2 = 1 (M2 > 4096)
// leaves the split to a pass of its own. (Choosing the split for the fewest
// short runs per pass instead measured slower: 0.22 against 0.19 ms of FFT
// on 128 series of 2^18 samples.)
bool four_step_split(int64_t M, FourStep &fs) {
    int64_t best = -1;
    for (int64_t a = 1; a <= kLdsPoints; ++a) {
        if (M % a || !smooth5(a)) continue;
        const int64_t c = M / a;
        if (c > kLdsPoints) continue;
        const int64_t mx = std::max<int64_t>(a, c);
        int t = 1;
        while (t < 64 && mx * (2 * t) <= kLdsPoints && (a % (2 * t)) == 0 && (c % (2 * t)) == 0) t *= 2;
        // prefer the widest tiles, then the most even split
        const int64_t score = (int64_t)t * (1 << 20) - mx;
        if (score > best) {
            best = score;
            fs = FourStep{(int)a, (int)c, t, tile_lines(c)};
        }
    }
    return best >= 0;
}

}  // namespace

bool fft_length_supported(int64_t n) {
    const int64_t M = n / 2;
    if (n < 8 || (n & 1) || !smooth5(M)) return false;
    if (M <= kLdsPoints) return true;
    FourStep fs;
    return four_step_split(M, fs);
}

// Launch KERNEL<P> for a power-of-two length P known at compile time, or
// KERNEL<0> with the plan's radices.
#define FDAS_FFT_DISPATCH(KERNEL, P, ...)                                           \
    switch (P) {                                                                    \
    case 8: hipLaunchKernelGGL(KERNEL<8>, __VA_ARGS__); break;                      \
    case 16: hipLaunchKernelGGL(KERNEL<16>, __VA_ARGS__); break;                    \
    case 32: hipLaunchKernelGGL(KERNEL<32>, __VA_ARGS__); break;                    \
    case 64: hipLaunchKernelGGL(KERNEL<64>, __VA_ARGS__); break;                    \
    case 128: hipLaunchKernelGGL(KERNEL<128>, __VA_ARGS__); break;                  \
    case 256: hipLaunchKernelGGL(KERNEL<256>, __VA_ARGS__); break;                  \
    case 512: hipLaunchKernelGGL(KERNEL<512>, __VA_ARGS__); break;                  \
    case 1024: hipLaunchKernelGGL(KERNEL<1024>, __VA_ARGS__); break;                \
    case 2048: hipLaunchKernelGGL(KERNEL<2048>, __VA_ARGS__); break;                \
    case 4096: hipLaunchKernelGGL(KERNEL<4096>, __VA_ARGS__); break;                \
    case 8192: hipLaunchKernelGGL(KERNEL<8192>, __VA_ARGS__); break;                \
    default: hipLaunchKernelGGL(KERNEL<0>, __VA_ARGS__); break;                     \
    }

hipError_t launch_rfft(const float *x, int64_t n, int nseries, float2 *w0,
                       float2 *spec, int64_t spitch, hipStream_t st, const int64_t *offs) {
    const int64_t M = n / 2;
    if (n < 8 || (n & 1) || nseries < 1 || nseries > 65535 || !smooth5(M)) return hipErrorInvalidValue;
    const float2 *z = reinterpret_cast<const float2 *>(x);
    if (M <= kLdsPoints) {
        FftPlan fp;
        if (!radix_plan((int)M, fp)) return hipErrorInvalidValue;
        FDAS_FFT_DISPATCH(k_rfft_lds, (int)M, dim3(nseries), dim3(kFftThreads), (size_t)M * sizeof(float2), st, z,
                          offs, fp, spec, spitch);
        return hipGetLastError();
    }
    FourStep fs;
    if (!four_step_split(M, fs)) return hipErrorInvalidValue;
    const int M1 = fs.M1, M2 = fs.M2;
    FftPlan f1, f2;
    if (!radix_plan(M1, f1) || !radix_plan(M2, f2)) return hipErrorInvalidValue;
    auto lg = [](int t) {
        int l = 0;
        while ((1 << l) < t) ++l;
        return l;
    };
    {
        const int T = fs.T1;
        const int64_t tps = M2 / T, total = tps * nseries;
        FDAS_FFT_DISPATCH(k_fft_cols, M1, dim3((unsigned)(8 * ((total + 7) / 8))), dim3(kFftThreads),
                          (size_t)T * M1 * sizeof(float2), st, z, offs, f1, M2, lg(T), tps, total, w0);
    }
    const int T = fs.T2;
    if (T >= 2) {
        // rows and their mirrors together: the split needs no pass of its own
        const int64_t tps = (M1 / 2 + T / 2) / (T / 2), total = tps * nseries;
        FDAS_FFT_DISPATCH(k_fft_rows_split, M2, dim3((unsigned)(8 * ((total + 7) / 8))), dim3(kFftThreads),
                          (size_t)T * M2 * sizeof(float2), st, w0, f2, M1, lg(T), tps, total, spec, spitch);
        return hipGetLastError();
    }
    {
        const int64_t tps = M1 / T, total = tps * nseries;
        FDAS_FFT_DISPATCH(k_fft_rows, M2, dim3((unsigned)(8 * ((total + 7) / 8))), dim3(kFftThreads),
                          (size_t)T * M2 * sizeof(float2), st, w0, f2, M1, lg(T), tps, total, spec, spitch);
    }
    dim3 grid((unsigned)((M / 2 + 1 + 255) / 256), (unsigned)nseries);
    hipLaunchKernelGGL(k_rfft_split_pairs, grid, dim3(256), 0, st, spec, spitch, M);
    return hipGetLastError();
}
#undef FDAS_FFT_DISPATCH

}  // namespace fdas
