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
// Ns = 1, 8, 64, then a radix-(L/512) pass, exchange through LDS (8-byte
// complex values, a bank-conflict-free layout per exchange, ping-pong
// buffers, one barrier per exchange); after the last pass each thread again holds
// t + q T, so plane rows are written with coalesced stores.
//
// Work is split so that each XCD (workgroup id mod 8) only touches one group
// of z rows: its slice of the template bank stays in that XCD's L2.
#include "dft_small.h"
#include "fdas_internal.h"

#include <algorithm>
#include <cstdlib>

namespace fdas {

template <int L>
struct Corr {
    static constexpr int T = L / 8;          // threads per workgroup
    static constexpr int R4 = L / 512;       // radix of the fourth pass (1: none)
    static constexpr int LDSZ = L + L / 8;   // complex slots per buffer (largest padded layout)
    // read strides between a thread's points t + q T in the three exchange layouts
    static constexpr int RS1 = T + T / 32;   // layout 1: point p at p + p/32
    static constexpr int RS2 = T + T / 8;    // layout 2: point p at p + 8 (p/64)
    static constexpr int RS3 = T;            // layout 3: point p at p
};

template <int L>
struct Twiddles {
    // pass-4 twiddles are kept for the first butterfly only: the butterfly u
    // twiddle exp(2 pi i (t + u T) r / L) is that of u = 0 rotated by
    // exp(i pi u r / 4), since T / L = 1/8
    float2 p2[7], p3[7], p4[Corr<L>::R4 > 1 ? Corr<L>::R4 - 1 : 1];
};

__device__ __forceinline__ float max_nonneg(float a, float b) {
    return __uint_as_float(max(__float_as_uint(a), __float_as_uint(b)));
}

// a * exp(i pi K / 4) for a compile-time K
template <int K>
__device__ __forceinline__ float2 rot8(float2 a) {
    constexpr float h = 0.70710678118654752440f;
    constexpr int k = K & 7;
    if constexpr (k == 0) return a;
    else if constexpr (k == 1) return make_float2(h * (a.x - a.y), h * (a.x + a.y));
    else if constexpr (k == 2) return make_float2(-a.y, a.x);
    else if constexpr (k == 3) return make_float2(h * (-a.x - a.y), h * (a.x - a.y));
    else if constexpr (k == 4) return make_float2(-a.x, -a.y);
    else if constexpr (k == 5) return make_float2(h * (a.y - a.x), h * (-a.x - a.y));
    else if constexpr (k == 6) return make_float2(a.y, -a.x);
    else return make_float2(h * (a.x + a.y), h * (a.y - a.x));
}

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
#pragma unroll
        for (int r = 1; r < R4; ++r) tw.p4[r - 1] = expipi((float)(2 * t * r) / (float)L);
    }
}

// twiddle of butterfly U, input R of pass 4, for direction DIR applied to a
template <int L, int DIR, int U, int R>
__device__ __forceinline__ float2 pass4_twiddle(float2 a, const Twiddles<L> &tw) {
    const float2 w = rot8<U * R>(tw.p4[R - 1]);
    return ctw<DIR>(a, w);
}

template <int L, int DIR, int U, int R4, int B>
__device__ __forceinline__ void pass4_butterfly(float2 *v, const Twiddles<L> &tw) {
    float2 w[R4];
#pragma unroll
    for (int r = 0; r < R4; ++r) w[r] = v[U + r * B];
    if constexpr (R4 >= 2) w[1] = pass4_twiddle<L, DIR, U, 1>(w[1], tw);
    if constexpr (R4 >= 4) {
        w[2] = pass4_twiddle<L, DIR, U, 2>(w[2], tw);
        w[3] = pass4_twiddle<L, DIR, U, 3>(w[3], tw);
    }
    if constexpr (R4 >= 8) {
        w[4] = pass4_twiddle<L, DIR, U, 4>(w[4], tw);
        w[5] = pass4_twiddle<L, DIR, U, 5>(w[5], tw);
        w[6] = pass4_twiddle<L, DIR, U, 6>(w[6], tw);
        w[7] = pass4_twiddle<L, DIR, U, 7>(w[7], tw);
    }
    dft_r<R4, DIR>(w);
#pragma unroll
    for (int r = 0; r < R4; ++r) v[U + r * B] = w[r];
}

// write v[r] at wbase + r*WS of buffer sel, barrier, read the thread's points
// back from rbase + q*RS.
//
// Points are exchanged as 8-byte complex values (one LDS instruction each).
// Each exchange has its own layout, chosen so that each half wave's 32 lanes
// (an 8-byte access covers two 4-byte banks) hit 32 distinct bank pairs both
// when writing the pass outputs (position 8t + r after pass 1, 64(t/8) + t%8
// + 8r after pass 2, 512(t/64) + t%64 + 64r after pass 3) and when reading
// t + qT back: point p is stored at p + p/32 (exchange 1), p + 8(p/64)
// (exchange 2) and p (exchange 3).
template <int L, int WS, int RS>
__device__ __forceinline__ void exchange(float2 *v, float *lds, int &sel, int wbase, int rbase) {
    float2 *cx = reinterpret_cast<float2 *>(lds) + sel * Corr<L>::LDSZ;
#pragma unroll
    for (int r = 0; r < 8; ++r) cx[wbase + r * WS] = v[r];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = cx[rbase + q * RS];
    sel ^= 1;
}

struct LdsAddr {
    int w1, w2, w3, r1, r2, r3;
};

template <int L, int DIR>
__device__ __forceinline__ void fft_block(float2 *v, float *lds, int &sel, const Twiddles<L> &tw,
                                          const LdsAddr &a) {
    // pass 1: radix 8, Ns = 1
    dft8<DIR>(v);
    exchange<L, 1, Corr<L>::RS1>(v, lds, sel, a.w1, a.r1);
    // pass 2: radix 8, Ns = 8
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = ctw<DIR>(v[r], tw.p2[r - 1]);
    dft8<DIR>(v);
    exchange<L, 8, Corr<L>::RS2>(v, lds, sel, a.w2, a.r2);
    // pass 3: radix 8, Ns = 64
#pragma unroll
    for (int r = 1; r < 8; ++r) v[r] = ctw<DIR>(v[r], tw.p3[r - 1]);
    dft8<DIR>(v);
    constexpr int R4 = Corr<L>::R4;
    if constexpr (R4 > 1) {
        exchange<L, 64, Corr<L>::RS3>(v, lds, sel, a.w3, a.r3);
        // pass 4: radix R4, Ns = 512, butterflies u use points v[u + r * (8 / R4)]
        constexpr int B = 8 / R4;
        pass4_butterfly<L, DIR, 0, R4, B>(v, tw);
        if constexpr (B >= 2) pass4_butterfly<L, DIR, 1, R4, B>(v, tw);
        if constexpr (B >= 4) {
            pass4_butterfly<L, DIR, 2, R4, B>(v, tw);
            pass4_butterfly<L, DIR, 3, R4, B>(v, tw);
        }
    }
}


// PYR: 0 no block maxima, 1 one maximum per column (half bin), 2 one per bin
// (both parities).
template <int L, int PYR>
__device__ __forceinline__ void corr_power(const float2 *__restrict__ spec, int64_t spitch,
                                           const float *__restrict__ scale,
                                           const float2 *__restrict__ bank, CorrGeom g,
                                           int nseries, float *__restrict__ plane,
                                           int64_t pitch, int64_t sstride,
                                           bmax_t *__restrict__ pyr, int64_t psstride,
                                           const int32_t *__restrict__ blk_lo,
                                           const int32_t *__restrict__ blk_of_row) {
    constexpr int T = Corr<L>::T;
    __shared__ __align__(16) float lds[4 * Corr<L>::LDSZ];
    const int t = threadIdx.x;

    // XCD-aware decomposition: xcd = id mod 8 serves z group (xcd mod G)
    const int w = blockIdx.x;
    const int xcd = w & 7;
    const int G = g.zgroups;
    const int per = 8 / G;
    const int zg = xcd & (G - 1);
    const int64_t unit = (int64_t)(w >> 3) * per + xcd / G;
    // the group's own segmentation (its widest template)
    const int nseg = g.gnseg[zg], Lv = g.gLv[zg], mseg = g.gmseg[zg];
    if (unit >= (int64_t)nseries * nseg) return;
    const int b = (int)(unit / nseg);
    const int s = (int)(unit - (int64_t)b * nseg);
    const int z0 = g.zb[zg], z1 = g.zb[zg + 1];
    const int64_t ks = g.rlo + (int64_t)s * Lv;   // first output bin of the segment

    Twiddles<L> tw;
    make_twiddles<L>(tw, t);
    LdsAddr a;
    a.w1 = 8 * t + (t >> 2);                 // pass-1 output 8t + r in layout 1
    a.w2 = 72 * (t >> 3) + (t & 7);          // pass-2 output 64(t/8) + t%8 + 8r in layout 2
    a.w3 = 512 * (t >> 6) + (t & 63);        // pass-3 output 512(t/64) + t%64 + 64r in layout 3
    a.r1 = t + (t >> 5);
    a.r2 = t + 8 * (t >> 6);
    a.r3 = t;
    int sel = 0;

    // segment s[n] = A[ks - mseg + n], zero outside bins 1..half-1
    const float2 *A = spec + (int64_t)b * spitch;
    const float sc = scale[b];
    float2 S[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const int64_t k = ks - mseg + t + q * T;
        S[q] = (k >= 1 && k < g.half) ? A[k] : make_float2(0.0f, 0.0f);
    }
    fft_block<L, -1>(S, lds, sel, tw, a);
#pragma unroll
    for (int q = 0; q < 8; ++q) S[q] = make_float2(S[q].x * sc, S[q].y * sc);

    float *out = plane + (int64_t)b * sstride + 2 * (ks - g.rlo);
    // block-maxima row: pitch/2 halves per block (PYR 2: one half per bin);
    // pitch 16-bit words (PYR 1: per column, the 8-bit codes of blocks k and
    // k + 1)
    const int64_t ppitch = PYR == 2 ? pitch / 2 : pitch;
    bmax_t *pout = PYR ? pyr + (int64_t)b * psstride + (PYR == 2 ? 1 : 2) * (ks - g.rlo) : nullptr;
    int blk = 0, blk_end = 0;
    // PYR 2: the running maximum of both parities of each bin. PYR 1: per
    // bin one register with the upper 16 bits of each parity's running
    // maximum power (parity p in half p), and the previous block's codes of
    // both columns of two bins per register (16 bits each): the registers
    // this saves fit the instance in 4 waves per SIMD
    float m0[8];
    uint32_t m01[8], pv[4];
    if constexpr (PYR != 0) {
        blk = blk_of_row[z0];
        blk_end = blk_lo[blk + 1];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            m0[q] = 0.0f;
            m01[q] = 0u;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) pv[q] = 0u;
    }
    // Kernel spectra and plane rows go through buffer resources: a
    // workgroup-uniform base and scalar offset plus the lane's fixed 32-bit
    // offset, so loads and stores need no per-lane address arithmetic (the
    // kernel is bound by VALU issue). The row resource covers the segment's
    // 2 Lv columns.
    const __amdgpu_buffer_rsrc_t bank_rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float2 *>(bank), (short)0, (int)(2 * g.NZ * L * (int)sizeof(float2)), kBufferRsrcWord3);
    const int t_bank = t * (int)sizeof(float2);
    const int t_row = 2 * t * (int)sizeof(float);
    for (int zi = z0; zi < z1; ++zi) {
        const __amdgpu_buffer_rsrc_t row_rs = __builtin_amdgcn_make_buffer_rsrc(
            out + (int64_t)zi * pitch, (short)0, 2 * Lv * (int)sizeof(float), kBufferRsrcWord3);
        // up to L 2048 the parity-0 powers wait in registers and both
        // parities of a bin are stored as one 8-byte pair (whole lines, half
        // the store instructions); at L 4096 that would cost the registers of
        // a wave, so each parity is stored as it is computed
        constexpr bool kPairStore = L <= 2048;
        float pw0[8];
#pragma unroll
        for (int p = 0; p < 2; ++p) {
            float2 v[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int soff = ((2 * zi + p) * L + q * T) * (int)sizeof(float2);
                v[q] = cmul(S[q], __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(
                                                                bank_rs, t_bank, soff, 0)));
            }
            fft_block<L, 1>(v, lds, sel, tw, a);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int i = t + q * T;
                const float pw = __fmaf_rn(v[q].x, v[q].x, __fmul_rn(v[q].y, v[q].y));
                if constexpr (kPairStore) {
                    if (p == 0) {
                        pw0[q] = pw;
                    } else if (i < Lv && ks + i < g.half) {
                        typedef unsigned int u32x2 __attribute__((__vector_size__(8)));
                        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, make_float2(pw0[q], pw)),
                                                              row_rs, t_row, 2 * q * T * (int)sizeof(float), 0);
                    }
                } else if (i < Lv && ks + i < g.half) {
                    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, pw), row_rs,
                                                          t_row + p * (int)sizeof(float),
                                                          2 * q * T * (int)sizeof(float), 0);
                }
                // powers are >= +0, so their bit patterns order like their
                // values: an integer maximum needs no NaN canonicalisation
                // (a float maximum costs two instructions per power here)
                if constexpr (PYR == 2) {
                    // both parities in one 3-input maximum (the parity-0 power
                    // waits in pw0 anyway when pairs are stored)
                    if constexpr (kPairStore) {
                        if (p == 1) m0[q] = max_nonneg(m0[q], max_nonneg(pw0[q], pw));
                    } else {
                        m0[q] = max_nonneg(m0[q], pw);
                    }
                } else if constexpr (PYR == 1) {
                    // half p of m01 = max(half p, upper 16 bits of pw): one
                    // 16-bit maximum with sub-dword operand selection (the
                    // truncated bits are restored as all ones at the block end,
                    // so the bound stays at or above every power)
                    if (p == 0)
                        asm("v_max_u16_sdwa %0, %1, %0 dst_sel:WORD_0 dst_unused:UNUSED_PRESERVE "
                            "src0_sel:WORD_1 src1_sel:WORD_0"
                            : "+v"(m01[q])
                            : "v"(pw));
                    else
                        asm("v_max_u16_sdwa %0, %1, %0 dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE "
                            "src0_sel:WORD_1 src1_sel:WORD_1"
                            : "+v"(m01[q])
                            : "v"(pw));
                }
            }
        }
        if constexpr (PYR != 0) {
            if (zi + 1 == blk_end) {
                bmax_t *prow = pout + (int64_t)blk * ppitch;
                // PYR 1 code pairs: word k of a column holds the codes of
                // blocks k (low byte) and k + 1 (high byte; 0 above the last
                // block). Block k's code goes to word k - 1 (high byte) and
                // word k (low byte). Inside a z group one workgroup has both
                // codes of a word and stores both columns' words of a bin as
                // one 32-bit value, one block late; across a group boundary
                // each group's workgroup stores its own bytes.
                const bool first = blk_lo[blk] == z0;           // first block of the group
                const bool last = zi + 1 == z1;                 // last block of the group
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int i = t + q * T;
                    // PYR 1: cur = c0 | c1 << 8, the codes of the bin's columns
                    // (each parity's maximum with its truncated low 16 bits
                    // set: at or above the true maximum)
                    const uint32_t cur = PYR == 1 ? bound_code(__uint_as_float((m01[q] << 16) | 0xffffu)) |
                                                        (bound_code(__uint_as_float(m01[q] | 0xffffu)) << 8)
                                                  : 0u;
                    if (i < Lv && ks + i < g.half) {
                        if constexpr (PYR == 2) {
                            prow[i] = bound_half(m0[q]);
                        } else {
                            // columns 2i and 2i + 1: words 2i and 2i + 1 of the
                            // row; the bin's two words are the bytes
                            // [p0, c0, p1, c1] of the previous codes and cur (one
                            // permute)
                            const uint32_t prev = (q & 1) ? pv[q >> 1] >> 16 : pv[q >> 1];
                            uint8_t *w = reinterpret_cast<uint8_t *>(prow + 2 * i);
                            uint8_t *wp = reinterpret_cast<uint8_t *>(prow - ppitch + 2 * i);
                            if (!first) {
                                *reinterpret_cast<uint32_t *>(wp) = __builtin_amdgcn_perm(cur, prev, 0x05010400u);
                            } else if (z0 > 0) {
                                wp[1] = (uint8_t)cur;
                                wp[3] = (uint8_t)(cur >> 8);
                            }
                            if (last) {
                                if (z1 == g.NZ) {
                                    *reinterpret_cast<uint32_t *>(w) = __builtin_amdgcn_perm(0u, cur, 0x0c010c00u);
                                } else {
                                    w[0] = (uint8_t)cur;
                                    w[2] = (uint8_t)(cur >> 8);
                                }
                            }
                        }
                    }
                    // cur's two code bytes into half q & 1 of pv[q / 2] by a
                    // byte permute, which reads bytes 0 and 1 of cur only: on
                    // gfx950 the compiler packs the two codes with one
                    // instruction whose bits 16..31 are not zero in practice
                    // (merged with masks and ORs, they spoiled the other bin's
                    // codes and the harmonic sums took 370 instead of 43 ms)
                    if constexpr (PYR == 1)
                        pv[q >> 1] = __builtin_amdgcn_perm(pv[q >> 1], cur, (q & 1) ? 0x01000504u : 0x07060100u);
                    m0[q] = 0.0f;
                    m01[q] = 0u;
                }
                ++blk;
                if (zi + 1 < z1) blk_end = blk_lo[blk + 1];
            }
        }
    }
}

#define FDAS_K4_PARAMS                                                                                \
    const float2 *__restrict__ spec, int64_t spitch, const float *__restrict__ scale,                  \
        const float2 *__restrict__ bank, CorrGeom g, int nseries, float *__restrict__ plane,           \
        int64_t pitch, int64_t sstride, bmax_t *__restrict__ pyr, int64_t psstride,                    \
        const int32_t *__restrict__ blk_lo, const int32_t *__restrict__ blk_of_row
#define FDAS_K4_ARGS spec, spitch, scale, bank, g, nseries, plane, pitch, sstride, pyr, psstride, blk_lo, blk_of_row

template <int L, int PYR>
__global__ __launch_bounds__(L / 8) void k_corr_power(FDAS_K4_PARAMS) {
    corr_power<L, PYR>(FDAS_K4_ARGS);
}

// Per-column maxima: the two parities' running maxima share a register as
// 16-bit halves, and the previous block's codes of two bins share one, which
// fits the instance in 4 waves per SIMD (as many as LDS allows). With them in
// 24 registers of their own it needed 152 and ran at 3 waves. At L 1024 (a
// different pass layout) 4 waves would spill registers, so that instance
// keeps 3.
template <int L>
__global__ __launch_bounds__(L / 8) __attribute__((amdgpu_waves_per_eu(L == 1024 ? 3 : 4, L == 1024 ? 3 : 4))) void k_corr_power_cols(
    FDAS_K4_PARAMS) {
    corr_power<L, 1>(FDAS_K4_ARGS);
}
#undef FDAS_K4_PARAMS
#undef FDAS_K4_ARGS

void zgroup_bounds(int NZ, double dz, int K, int L, int G, int32_t *zb) {
    const int Z = (NZ - 1) / 2;
    // valid outputs per segment of a group over rows a..e - 1 (its widest
    // drift sets the template half-width)
    auto valid = [&](int a, int e) {
        const int zmax = std::max(std::abs(a - Z), std::abs(e - 1 - Z));
        return L - 2 * half_width(zmax * dz, K);
    };
    // greedy cover with groups of time <= t; the smallest t that needs at most
    // G groups (bisection over t)
    auto cover = [&](double t, int32_t *b) {
        int n = 0;
        b[0] = 0;
        while (b[n] < NZ) {
            if (n == G) return false;
            int e = b[n] + 1;
            while (e < NZ && (double)(e + 1 - b[n]) / valid(b[n], e + 1) <= t) ++e;
            b[++n] = e;
        }
        // fewer groups than G: split the longest until there are G
        while (n < G) {
            int w = 0;
            for (int i = 1; i < n; ++i)
                if (b[i + 1] - b[i] > b[w + 1] - b[w]) w = i;
            for (int i = n + 1; i > w + 1; --i) b[i] = b[i - 1];
            b[w + 1] = b[w] + (b[w + 2] - b[w]) / 2;
            ++n;
        }
        return true;
    };
    double lo = 0.0, hi = (double)NZ;   // hi: one group per row is always feasible below this
    int32_t b[kMaxZGroups + 2];
    for (int i = 0; i <= G; ++i) zb[i] = i * NZ / G;
    for (int it = 0; it < 60; ++it) {
        const double t = 0.5 * (lo + hi);
        if (cover(t, b)) {
            hi = t;
            for (int i = 0; i <= G; ++i) zb[i] = b[i];
        } else {
            lo = t;
        }
    }
}

void row_blocks(const int32_t *zb, int G, int bz, std::vector<int32_t> &lo, std::vector<int32_t> &of_row) {
    const int NZ = zb[G];
    lo.clear();
    of_row.assign(NZ, 0);
    for (int gi = 0; gi < G; ++gi) {
        const int z0 = zb[gi], z1 = zb[gi + 1];
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

void fraction_ranges(int NZ, int numharm, const std::vector<int32_t> &lo,
                     const std::vector<int32_t> &of_row, std::vector<int32_t> &frange) {
    const int Z = (NZ - 1) / 2;
    const int nblk = (int)lo.size() - 1;
    auto frow = [&](int zq, int j) {
        const int az = zq < 0 ? -zq : zq;
        const int r = (2 * az * j + numharm) / (2 * numharm);
        return zq < 0 ? -r : r;
    };
    frange.assign((size_t)nblk * numharm, 0);
    for (int k = 0; k < nblk; ++k) {
        const int zqa = lo[k] - Z, zqb = lo[k + 1] - 1 - Z;
        for (int j = 1; j <= numharm; ++j) {
            const int a = of_row[frow(zqa, j) + Z], e = of_row[frow(zqb, j) + Z];
            frange[(size_t)k * numharm + j - 1] = a | ((e - a) << 24);
        }
    }
}

void bound_offsets(int numharm, const std::vector<int32_t> &frange, int64_t ppitch,
                   std::vector<int32_t> &boff) {
    const int nblk = (int)(frange.size() / numharm);
    const int W = 2 * numharm + 2;
    const uint32_t rowb = (uint32_t)ppitch * (uint32_t)sizeof(bmax_t);
    boff.assign((size_t)nblk * W, 0);
    for (int k = 0; k < nblk; ++k) {
        int32_t *o = &boff[(size_t)k * W];
        int32_t wide = 0;
        for (int j = 0; j < numharm; ++j) {
            const int32_t f = frange[(size_t)k * numharm + j];
            const uint32_t a = (uint32_t)(f & 0xffffff), n = (uint32_t)f >> 24;
            o[j] = (int32_t)(a * rowb);
            // the code pair of block a holds a + 1's code in its high byte: a
            // byte selector that keeps it where the range has a + 1
            o[numharm + j] = n > 0 ? 0x0c010c00 : 0x0c0c0c00;
            if (n > 1) wide = 1;
        }
        o[2 * numharm + 1] = wide;
    }
}

template <int L>
static void launch_l(const float2 *spec, int64_t spitch, const float *scale, const float2 *bank,
                     const CorrGeom &g, int nseries, float *plane, int64_t pitch, int64_t sstride,
                     bmax_t *pyr, int64_t psstride, const RowBlocks &rb, int64_t nwg, hipStream_t st) {
    const int mode = pyr ? (rb.pair ? 2 : 1) : 0;
#define FDAS_K4(KERNEL)                                                                             \
    hipLaunchKernelGGL(KERNEL, dim3((unsigned)nwg), dim3(L / 8), 0, st, spec, spitch, scale, bank, g, \
                       nseries, plane, pitch, sstride, pyr, psstride, rb.lo, rb.of_row)
    if (mode == 0) FDAS_K4((k_corr_power<L, 0>));
    else if (mode == 1) FDAS_K4((k_corr_power_cols<L>));
    else FDAS_K4((k_corr_power<L, 2>));
#undef FDAS_K4
}

hipError_t launch_corr_power(const float2 *spec, int64_t spitch, const float *scale,
                             const float2 *bank, const CorrGeom &g, int nseries, float *plane,
                             int64_t pitch, int64_t series_stride, bmax_t *pyr,
                             int64_t pyr_series_stride, const RowBlocks &rb, hipStream_t st) {
    // buffer resources take 32-bit byte ranges: the bank and a segment's row
    if ((int64_t)2 * g.NZ * g.L * 8 > 0x7fffffffLL)
        return hipErrorInvalidValue;
    if (nseries < 1 || (g.zgroups & (g.zgroups - 1)) || g.zgroups > kMaxZGroups || g.zgroups < 1 ||
        g.zgroups > g.NZ || (pitch & 1) || g.zb[0] != 0 || g.zb[g.zgroups] != g.NZ ||
        (pyr && (!rb.lo || !rb.of_row || rb.nblk < 1 || rb.ppitch != (rb.pair ? pitch / 2 : pitch))))
        return hipErrorInvalidValue;
    int maxseg = 0;
    for (int i = 0; i < g.zgroups; ++i) {
        if (g.zb[i + 1] <= g.zb[i] || g.gLv[i] < 1 || g.gLv[i] != g.L - 2 * g.gmseg[i] || g.gmseg[i] > g.mseg ||
            g.gnseg[i] < 1 || (int64_t)g.gnseg[i] * g.gLv[i] < g.half - g.rlo)
            return hipErrorInvalidValue;
        maxseg = std::max(maxseg, g.gnseg[i]);
    }
    const int64_t units = (int64_t)nseries * maxseg;
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
