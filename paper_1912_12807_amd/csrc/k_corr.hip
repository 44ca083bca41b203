// K4: f-fdot power plane by overlap-save correlation with the template bank.
//
// For every series, drift row z and half-bin R = 2 k0 + p, the plane holds
//   P = |sum_d A^_{k0+d} t_{z,p}[d]|^2,
// the matched-filter power of a sinusoid drifting by z bins over the
// observation (the acceleration search of the paper's Section 2, step 4,
// bounded by zmax as in Section 3.2). The correlation runs in the Fourier
// domain of the spectrum: a workgroup loads one length-L segment of the
// spectrum, FFTs it once (kept in registers, scaled by sqrt(1/norm)), and for
// each of its z rows and both parities multiplies by the precomputed kernel
// spectrum T_{z,p} (L2-resident), inverse-FFTs and squares. L - 2 mseg outputs
// per segment are valid (mseg = template half-width of the bank).
//
// FFT layout: L points over T = L/8 threads, thread t holding points t + q T
// (q = 0..7) in natural order before every pass. Stockham radix-8 passes with
// Ns = 1, 8, 64, then a radix-(L/512) pass, exchange through padded LDS (one
// pad word per 8, separate re/im arrays, ping-pong buffers, one barrier per
// exchange); after the last pass each thread again holds t + q T, so plane
// rows are written as coalesced float2 (p = 0, p = 1) pairs.
//
// Work is split so that each XCD (workgroup id mod 8) only touches one group
// of z rows: its slice of the template bank stays in that XCD's L2.
#include "dft_small.h"
#include "fdas_internal.h"

namespace fdas {

template <int L>
struct Corr {
    static constexpr int T = L / 8;          // threads per workgroup
    static constexpr int R4 = L / 512;       // radix of the fourth pass (1: none)
    static constexpr int LDSZ = L + L / 8;   // padded floats per array
    static constexpr int RS = 9 * T / 8;     // padded stride between a thread's points
    static constexpr int NTW4 = R4 > 1 ? (8 / R4) * (R4 - 1) : 1;
};

template <int L>
struct Twiddles {
    float2 p2[7], p3[7], p4[Corr<L>::NTW4];
};

template <int L>
__device__ __forceinline__ void make_twiddles(Twiddles<L> &tw, int t) {
    const int k2 = t & 7, k3 = t & 63;
#pragma unroll
    for (int r = 1; r < 8; ++r) {
        tw.p2[r - 1] = expipi((float)(k2 * r) / 32.0f);     // exp(2 pi i k r / 64)
        tw.p3[r - 1] = expipi((float)(k3 * r) / 256.0f);    // exp(2 pi i k r / 512)
    }
    constexpr int R4 = Corr<L>::R4;
    if constexpr (R4 > 1) {
        constexpr int B = 8 / R4;
#pragma unroll
        for (int u = 0; u < B; ++u) {
            const int k = t + u * Corr<L>::T;                // < 512
#pragma unroll
            for (int r = 1; r < R4; ++r)
                tw.p4[u * (R4 - 1) + r - 1] = expipi((float)(2 * k * r) / (float)L);
        }
    }
}

// write v[r] at wbase + r*WS of buffer sel, barrier, read the thread's points back
template <int L, int WS>
__device__ __forceinline__ void exchange(float2 *v, float *lds, int &sel, int wbase, int rbase) {
    float *re = lds + sel * 2 * Corr<L>::LDSZ;
    float *im = re + Corr<L>::LDSZ;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        re[wbase + r * WS] = v[r].x;
        im[wbase + r * WS] = v[r].y;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = make_float2(re[rbase + q * Corr<L>::RS], im[rbase + q * Corr<L>::RS]);
    sel ^= 1;
}

struct LdsAddr {
    int w1, w2, w3, rd;
};

template <int L, int DIR>
__device__ __forceinline__ void fft_block(float2 *v, float *lds, int &sel, const Twiddles<L> &tw,
                                          const LdsAddr &a) {
    // pass 1: radix 8, Ns = 1
    dft8<DIR>(v);
    exchange<L, 1>(v, lds, sel, a.w1, a.rd);
    // pass 2: radix 8, Ns = 8
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = ctw<DIR>(v[r], tw.p2[r - 1]);
    dft8<DIR>(v);
    exchange<L, 9>(v, lds, sel, a.w2, a.rd);
    // pass 3: radix 8, Ns = 64
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = ctw<DIR>(v[r], tw.p3[r - 1]);
    dft8<DIR>(v);
    constexpr int R4 = Corr<L>::R4;
    if constexpr (R4 > 1) {
        exchange<L, 72>(v, lds, sel, a.w3, a.rd);
        // pass 4: radix R4, Ns = 512, butterflies u use points v[u + r * (8 / R4)]
        constexpr int B = 8 / R4;
#pragma unroll
        for (int u = 0; u < B; ++u) {
            float2 w[R4 > 1 ? R4 : 1];
#pragma unroll
            for (int r = 0; r < R4; ++r) w[r] = v[u + r * B];
#pragma unroll
            for (int r = 1; r < R4; ++r) w[r] = ctw<DIR>(w[r], tw.p4[u * (R4 - 1) + r - 1]);
            dft_r<R4, DIR>(w);
#pragma unroll
            for (int r = 0; r < R4; ++r) v[u + r * B] = w[r];
        }
    }
}

template <int L, bool PYR>
__global__ __launch_bounds__(L / 8) void k_corr_power(const float2 *__restrict__ spec, int64_t spitch,
                                                      const float *__restrict__ scale,
                                                      const float2 *__restrict__ bank, CorrGeom g,
                                                      int nseries, float *__restrict__ plane,
                                                      int64_t pitch, int64_t sstride,
                                                      float *__restrict__ pyr, int64_t psstride,
                                                      const int32_t *__restrict__ blk_lo,
                                                      const int32_t *__restrict__ blk_of_row) {
    constexpr int T = Corr<L>::T;
    __shared__ float lds[4 * Corr<L>::LDSZ];
    const int t = threadIdx.x;

    // XCD-aware decomposition: xcd = id mod 8 serves z group (xcd mod G)
    const int w = blockIdx.x;
    const int xcd = w & 7;
    const int G = g.zgroups;
    const int per = 8 / G;
    const int zg = xcd & (G - 1);
    const int64_t unit = (int64_t)(w >> 3) * per + xcd / G;
    if (unit >= (int64_t)nseries * g.nseg) return;
    const int b = (int)(unit / g.nseg);
    const int s = (int)(unit - (int64_t)b * g.nseg);
    const int z0 = zg * g.NZ / G, z1 = (zg + 1) * g.NZ / G;
    const int64_t ks = g.rlo + (int64_t)s * g.Lv;   // first output bin of the segment

    Twiddles<L> tw;
    make_twiddles<L>(tw, t);
    LdsAddr a;
    a.w1 = 9 * t;
    a.w2 = (t >> 3) * 72 + (t & 7);
    a.w3 = (t >> 6) * 576 + (t & 63) + ((t & 63) >> 3);
    a.rd = t + (t >> 3);
    int sel = 0;

    // segment s[n] = A[ks - mseg + n], zero outside bins 1..half-1
    const float2 *A = spec + (int64_t)b * spitch;
    const float sc = scale[b];
    float2 S[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t k = ks - g.mseg + t + q * T;
        S[q] = (k >= 1 && k < g.half) ? A[k] : make_float2(0.0f, 0.0f);
    }
    fft_block<L, -1>(S, lds, sel, tw, a);
#pragma unroll
    for (int q = 0; q < 8; ++q) S[q] = make_float2(S[q].x * sc, S[q].y * sc);

    float *out = plane + (int64_t)b * sstride + 2 * (ks - g.rlo);
    float *pout = PYR ? pyr + (int64_t)b * psstride + 2 * (ks - g.rlo) : nullptr;
    int blk = 0, blk_end = 0;
    float m0[8], m1[8];
    if constexpr (PYR) {
        blk = blk_of_row[z0];
        blk_end = blk_lo[blk + 1];
#pragma unroll
        for (int q = 0; q < 8; ++q) m0[q] = m1[q] = 0.0f;
    }
    for (int zi = z0; zi < z1; ++zi) {
        float p0[8];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            const float2 *Tz = bank + (int64_t)(2 * zi + p) * L;
            float2 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) v[q] = cmul(S[q], Tz[t + q * T]);
            fft_block<L, 1>(v, lds, sel, tw, a);
            if (p == 0) {
#pragma unroll
                for (int q = 0; q < 8; ++q) p0[q] = v[q].x * v[q].x + v[q].y * v[q].y;
            } else {
                float *row = out + (int64_t)zi * pitch;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int i = t + q * T;
                    const float p1 = v[q].x * v[q].x + v[q].y * v[q].y;
                    if (i < g.Lv && ks + i < g.half)
                        *reinterpret_cast<float2 *>(row + 2 * i) = make_float2(p0[q], p1);
                    if constexpr (PYR) {
                        m0[q] = fmaxf(m0[q], p0[q]);
                        m1[q] = fmaxf(m1[q], p1);
                    }
                }
                if constexpr (PYR) {
                    if (zi + 1 == blk_end) {
                        float *prow = pout + (int64_t)blk * pitch;
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const int i = t + q * T;
                            if (i < g.Lv && ks + i < g.half)
                                *reinterpret_cast<float2 *>(prow + 2 * i) = make_float2(m0[q], m1[q]);
                            m0[q] = m1[q] = 0.0f;
                        }
                        ++blk;
                        if (zi + 1 < z1) blk_end = blk_lo[blk + 1];
                    }
                }
            }
        }
    }
}

void row_blocks(int NZ, int G, int bz, std::vector<int32_t> &lo, std::vector<int32_t> &of_row) {
    lo.clear();
    of_row.assign(NZ, 0);
    for (int gi = 0; gi < G; ++gi) {
        const int z0 = gi * NZ / G, z1 = (gi + 1) * NZ / G;
        const int n = z1 - z0;
        if (n <= 0) continue;
        const int nb = (n + bz - 1) / bz;
        for (int k = 0; k < nb; ++k) {
            const int a = z0 + k * n / nb, e = z0 + (k + 1) * n / nb;
            for (int r = a; r < e; ++r) of_row[r] = (int32_t)lo.size();
            lo.push_back(a);
        }
    }
    lo.push_back(NZ);
}

template <int L>
static void launch_l(const float2 *spec, int64_t spitch, const float *scale, const float2 *bank,
                     const CorrGeom &g, int nseries, float *plane, int64_t pitch, int64_t sstride,
                     float *pyr, int64_t psstride, const RowBlocks &rb, int64_t nwg, hipStream_t st) {
    if (pyr)
        hipLaunchKernelGGL((k_corr_power<L, true>), dim3((unsigned)nwg), dim3(L / 8), 0, st, spec, spitch,
                           scale, bank, g, nseries, plane, pitch, sstride, pyr, psstride, rb.lo, rb.of_row);
    else
        hipLaunchKernelGGL((k_corr_power<L, false>), dim3((unsigned)nwg), dim3(L / 8), 0, st, spec, spitch,
                           scale, bank, g, nseries, plane, pitch, sstride, pyr, psstride, rb.lo, rb.of_row);
}

hipError_t launch_corr_power(const float2 *spec, int64_t spitch, const float *scale,
                             const float2 *bank, const CorrGeom &g, int nseries, float *plane,
                             int64_t pitch, int64_t series_stride, float *pyr,
                             int64_t pyr_series_stride, const RowBlocks &rb, hipStream_t st) {
    if (nseries < 1 || g.nseg < 1 || g.Lv < 1 || (g.zgroups & (g.zgroups - 1)) || g.zgroups > 8 ||
        g.zgroups < 1 || (pitch & 1) || (pyr && (!rb.lo || !rb.of_row || rb.nblk < 1)))
        return hipErrorInvalidValue;
    const int64_t units = (int64_t)nseries * g.nseg;
    const int per = 8 / g.zgroups;
    const int64_t nwg = 8 * ((units + per - 1) / per);
    if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
    switch (g.L) {
    case 512: launch_l<512>(spec, spitch, scale, bank, g, nseries, plane, pitch, series_stride, pyr, pyr_series_stride, rb, nwg, st); break;
    case 1024: launch_l<1024>(spec, spitch, scale, bank, g, nseries, plane, pitch, series_stride, pyr, pyr_series_stride, rb, nwg, st); break;
    case 2048: launch_l<2048>(spec, spitch, scale, bank, g, nseries, plane, pitch, series_stride, pyr, pyr_series_stride, rb, nwg, st); break;
    case 4096: launch_l<4096>(spec, spitch, scale, bank, g, nseries, plane, pitch, series_stride, pyr, pyr_series_stride, rb, nwg, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fdas
