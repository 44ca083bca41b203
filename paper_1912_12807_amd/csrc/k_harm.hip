// K5: harmonic sums and their maxima over drift; K6: ordered compaction of
// the maxima above threshold; and the argmax over drift of each candidate.
//
// A periodic signal puts power at harmonics k = 1..H of its fundamental
// (r_f, z_f), i.e. at (k r_f, k z_f). Indexing a trial by its H-th harmonic
// (R half bins, z index Zq), the k-th harmonic sits at
//   R_k = floor((2 R k + H) / (2 H)),  Zq_k = sgn(Zq) floor((2 |Zq| k + H) / (2 H)),
// and S_H(R, Zq) = sum_k P(R_k, Zq_k). The candidate list handed to the
// sifting step (paper, Section 2, step 5) keeps, per stage H in 1, 2, 4, ...,
// numharm and column R in [2 rlo H, N-1], M_H(R) = max over Zq of S_H when it
// exceeds the stage threshold.
//
// Since the k-th of H harmonics equals the 2k-th of 2H, every stage is a
// prefix of one chain over the fractions j / numharm:
//   S_1 = P(j = nh), S_2h = S_h + sum over odd k < 2h of P(j = k nh / 2h).
// K5 gives each lane one column R and walks Zq; the row offsets of the
// gathers are wave-uniform (scalar), the column offsets per lane constant.
#include "dft_small.h"
#include "fdas_internal.h"

#include <climits>

namespace fdas {

template <int NH>
struct Stages {
    static constexpr int NS = NH == 1 ? 1 : NH == 2 ? 2 : NH == 4 ? 3 : NH == 8 ? 4 : NH == 16 ? 5 : 6;
};

// Stage sums of one cell from the gathered fractions P[j - 1], j = 1..NH.
template <int NH>
__device__ __forceinline__ void stage_chain(const float *P, float *Ss) {
    float S = P[NH - 1];
    Ss[0] = S;
    int s = 1;
#pragma unroll
    for (int h = 2; h <= NH; h *= 2, ++s) {
#pragma unroll
        for (int k = 1; k < h; k += 2) S += P[k * (NH / h) - 1];
        Ss[s] = S;
    }
}

// The same chain over the raw half bits of bounds: each step adds the half to
// the FP32 sum with one mixed-precision fused multiply-add (h x 1 + S rounds
// once, exactly as S + (float)h), so it orders the bounds exactly like
// stage_chain and needs no separate conversions.
template <int NH>
__device__ __forceinline__ void stage_chain_h(const uint16_t *Ph, float *Ss) {
    // a one the compiler cannot see through: with a literal 1 it turns the
    // multiply-add back into a conversion and an addition
    const float one = __uint_as_float(0x3f800000u | __builtin_amdgcn_mbcnt_lo(0u, 0u));
    float S = half_bits_to_float(Ph[NH - 1]);
    Ss[0] = S;
    int s = 1;
#pragma unroll
    for (int h = 2; h <= NH; h *= 2, ++s) {
#pragma unroll
        for (int k = 1; k < h; k += 2) S = __builtin_fmaf(half_bits_to_float(Ph[k * (NH / h) - 1]), one, S);
        Ss[s] = S;
    }
}

// The larger of the two 8-bit codes of a 16-bit word w, the high one only
// where the byte selector sel keeps it: the permute spreads the codes into
// the two 16-bit halves of a register (sel 0x0c010c00; 0x0c0c0c00 zeroes the
// high code) and one packed maximum compares them. Bits above the low half of
// the result are not zero; code_half_bits drops them.
__device__ __forceinline__ uint32_t max_code(uint32_t w, uint32_t sel) {
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    const u16x2 a = __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(0u, w, sel));
    const u16x2 m = __builtin_elementwise_max(a, __builtin_shufflevector(a, a, 1, 0));
    return __builtin_bit_cast(uint32_t, m);
}
// Half bits of a code's value: (1 + (c mod 32) / 32) 2^(c / 32) has half
// exponent c / 32 + 15 and mantissa (c mod 32) << 5, i.e. (c << 5) + 0x3c00
// (c <= 255 keeps it below 0x7c00, and bits of c above 15 leave the half).
__device__ __forceinline__ uint16_t code_half_bits(uint32_t c) { return (uint16_t)((c << 5) + 0x3c00u); }

// Column offsets R_j - 2 rlo and the mask of fractions some searched stage needs.
template <int NH>
__device__ __forceinline__ uint32_t column_offsets(int64_t R, int64_t rlo, int64_t *col) {
    uint32_t need = 0;
#pragma unroll
    for (int j = 1; j <= NH; ++j) {
        const int64_t Rj = (2 * R * j + NH) / (2 * NH);
        col[j - 1] = Rj - 2 * rlo;
        const int hmin = NH >> __builtin_ctz(j);     // smallest stage using fraction j
        if (R >= 2 * rlo * hmin) need |= 1u << (j - 1);
    }
    return need;
}

template <int NH>
__device__ __forceinline__ void gather(const float *__restrict__ pb, int64_t pitch, int Z, int zq,
                                       const int64_t *col, uint32_t need, float *P) {
    const int az = zq < 0 ? -zq : zq;
    const int sg = zq < 0 ? -1 : 1;
#pragma unroll
    for (int j = 1; j <= NH; ++j) {
        const int zj = sg * ((2 * az * j + NH) / (2 * NH));
        P[j - 1] = (need >> (j - 1)) & 1u ? pb[(int64_t)(zj + Z) * pitch + col[j - 1]] : 0.0f;
    }
}

// Row of fraction j for drift index zq (wave-uniform).
template <int NH>
__device__ __forceinline__ int frac_row(int zq, int j) {
    const int az = zq < 0 ? -zq : zq;
    const int r = (2 * az * j + NH) / (2 * NH);
    return zq < 0 ? -r : r;
}

// One lane per column R. As Zq sweeps -Z..Z, the row of fraction j changes
// only every ~NH/j steps, so each fraction's value stays in a register and is
// reloaded only when its (wave-uniform) row changes: about (NH+1)/2 loads per
// cell instead of NH. The next sweep step's loads are issued before the
// current step is summed. Column tiles are assigned so that each XCD (workgroup
// id mod 8) works through a contiguous run of tiles of one series, whose
// fraction strips overlap in its L2.
template <int NH>
__global__ __launch_bounds__(256) void k_harmsum(const float *__restrict__ plane, int64_t pitch,
                                                 int64_t sstride, int64_t NR, int64_t rlo, int Z,
                                                 float *__restrict__ maxv, int16_t *__restrict__ zarg,
                                                 int64_t mpitch, int64_t tiles_per_series, int64_t total_tiles,
                                                 int xcd_runs, int zq_lo, int zq_hi, int merge) {
    constexpr int NS = Stages<NH>::NS;
    const int64_t w = blockIdx.x;
    int64_t g = w;
    if (xcd_runs) {
        const int64_t per_xcd = (total_tiles + 7) / 8;
        g = (w & 7) * per_xcd + (w >> 3);
    }
    if (g >= total_tiles) return;
    const int b = (int)(g / tiles_per_series);
    const int64_t c = (g - (int64_t)b * tiles_per_series) * 256 + threadIdx.x;
    if (c >= mpitch) return;
    float *mo = maxv + (int64_t)b * NS * mpitch + c;
    int16_t *za = zarg + (int64_t)b * NS * mpitch + c;
    if (c >= NR) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            mo[s * mpitch] = 0.0f;
            za[s * mpitch] = 0;
        }
        return;
    }
    const int64_t R = c + 2 * rlo;
    int64_t col[NH];
    const uint32_t need = column_offsets<NH>(R, rlo, col);
    const float *pb = plane + (int64_t)b * sstride + (int64_t)Z * pitch;   // row Zq = 0
    // maxima and their smallest maximising Zq (the sweep runs upward in Zq and
    // a later row replaces the maximum only when strictly larger)
    float mx[NS];
    int az[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        mx[s] = 0.0f;
        az[s] = zq_lo;
    }

    if (merge) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            mx[s] = mo[s * mpitch];
            az[s] = za[s * mpitch];
        }
    }
    float cur[NH];
    int row[NH];
#pragma unroll
    for (int j = 1; j <= NH; ++j) {
        row[j - 1] = frac_row<NH>(zq_lo, j);
        cur[j - 1] = (need >> (j - 1)) & 1u ? pb[(int64_t)row[j - 1] * pitch + col[j - 1]] : 0.0f;
    }
    for (int zq = zq_lo; zq <= zq_hi; ++zq) {
        float nxt[NH];
#pragma unroll
        for (int j = 1; j <= NH; ++j) nxt[j - 1] = cur[j - 1];
        if (zq < zq_hi) {
#pragma unroll
            for (int j = 1; j <= NH; ++j) {
                const int r = frac_row<NH>(zq + 1, j);
                if (r != row[j - 1]) {
                    row[j - 1] = r;
                    nxt[j - 1] = (need >> (j - 1)) & 1u ? pb[(int64_t)r * pitch + col[j - 1]] : 0.0f;
                }
            }
        }
        float Ss[NS];
        stage_chain<NH>(cur, Ss);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (Ss[s] > mx[s]) {
                mx[s] = Ss[s];
                az[s] = zq;
            }
        }
#pragma unroll
        for (int j = 0; j < NH; ++j) cur[j] = nxt[j];
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const bool on = R >= 2 * rlo * (1 << s);
        mo[s * mpitch] = on ? mx[s] : 0.0f;
        za[s * mpitch] = (int16_t)(on ? az[s] : 0);
    }
}

// Bounded variant: lane = column R, loop over drift blocks. For fraction j the
// rows a block's sums read, frac_row(zq, j) for zq in the block, lie in row
// blocks a..e (a host table, packed as a | (e - a) << 24, read through scalar
// loads since every index is wave-uniform); the largest block maximum among
// them bounds every value the fraction contributes. Maxima per bin cover both
// half-bin columns of a bin as halves rounded up; maxima per column are 8-bit
// codes rounded up (bound_code), the codes of blocks k and k + 1 in one
// 16-bit word, so one gather covers a range of one or two blocks. The stage
// chain of these bounds (same order as the exact chain, each step rounding
// like an FP32 addition) bounds every exact stage sum of the block, so a block
// whose bounds stay at or below all searched stages' thresholds cannot hold a
// candidate and is skipped. A block that some lane of the wave cannot rule out
// is summed exactly by those lanes (the others masked off), with the row
// bookkeeping shared by the wave.
//
// A range spans one or two row blocks in all but rare cases: the loads of
// the first and second block of every fraction (maxima per bin) or the one
// code pair (per column) are independent and in flight together, and only
// longer ranges take a further loop. Block-maxima addresses are a uniform
// per-series base plus a 32-bit byte offset per lane (one series' maxima stay
// below 4 GiB). The kernel is bound by the issue of these gathers (about seven
// texture-addresser cycles per 64-lane gather of one cache line), so what
// counts is gathers times lines: 16-bit entries, one per column.

// consecutive column tiles per XCD run of the bounded sums
constexpr int kBoundXcdRun = 4;

template <int NH>
struct BoundCfg {
    // series per lane: the wave-uniform block bookkeeping is shared by SB series
    static constexpr int SB = NH <= 8 ? 2 : 1;
};

__device__ __forceinline__ float load_at(const bmax_t *base, uint32_t byte_off) {
    return half_bits_to_float(*reinterpret_cast<const bmax_t *>(reinterpret_cast<const char *>(base) + byte_off));
}
__device__ __forceinline__ uint16_t load_bits_at(const bmax_t *base, uint32_t byte_off) {
    return *reinterpret_cast<const bmax_t *>(reinterpret_cast<const char *>(base) + byte_off);
}

// Tile g of one set of series: series group g / tiles_per_series (SB series),
// 256 columns from (g mod tiles_per_series) * 256. PW: block maxima per column
// as 32-bit pair words (the halves of blocks k and k + 1); otherwise one half
// per bin (both half-bin columns).
template <int NH, bool PW>
__device__ __forceinline__ void harm_bound_tile(const float *__restrict__ plane, int64_t pitch,
                                                int64_t sstride, const bmax_t *__restrict__ pyr,
                                                int64_t psstride, const int32_t *__restrict__ blk_lo,
                                                const int32_t *__restrict__ frange, int nblk, int64_t NR,
                                                int64_t rlo, int Z, const float *__restrict__ thr,
                                                float *__restrict__ maxv, int16_t *__restrict__ zarg,
                                                int64_t mpitch, int64_t tiles_per_series, int64_t g,
                                                int64_t ppitch, int nseries) {
    constexpr int NS = Stages<NH>::NS;
    constexpr int SB = BoundCfg<NH>::SB;
    const int grp = (int)(g / tiles_per_series);
    const int b0 = grp * SB;
    const int64_t c = (g - (int64_t)grp * tiles_per_series) * 256 + threadIdx.x;
    if (c >= mpitch) return;
    if (c >= NR) {
#pragma unroll
        for (int m = 0; m < SB; ++m) {
            if (b0 + m >= nseries) break;
            float *mo = maxv + (int64_t)(b0 + m) * NS * mpitch + c;
            int16_t *za = zarg + (int64_t)(b0 + m) * NS * mpitch + c;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                mo[s * mpitch] = 0.0f;
                za[s * mpitch] = 0;
            }
        }
        return;
    }
    const int64_t R = c + 2 * rlo;
    uint32_t need;
    // byte offset of each fraction's block-maxima column (clamped to a valid
    // column when unused)
    uint32_t cb[NH];
    {
        int64_t col[NH];
        need = column_offsets<NH>(R, rlo, col);
#pragma unroll
        for (int j = 0; j < NH; ++j) {
            const int64_t cc = col[j] < 0 ? 0 : col[j];
            cb[j] = (uint32_t)(PW ? cc : cc >> 1) * (uint32_t)sizeof(bmax_t);
        }
    }
    // each series' block maxima (below 4 GiB): a pointer (halves per bin) or a
    // buffer resource (code pairs per column)
    const bmax_t *yb[SB];
    __amdgpu_buffer_rsrc_t rs[SB];
#pragma unroll
    for (int m = 0; m < SB; ++m) {
        const int bm = b0 + m < nseries ? b0 + m : nseries - 1;   // spare lanes re-read the last series
        yb[m] = pyr + (int64_t)bm * psstride;
        rs[m] = __builtin_amdgcn_make_buffer_rsrc(const_cast<bmax_t *>(yb[m]), (short)0,
                                                  (int)(uint32_t)(psstride * (int64_t)sizeof(bmax_t)),
                                                  kBufferRsrcWord3);
    }
    const uint32_t rowb = (uint32_t)ppitch * (uint32_t)sizeof(bmax_t);   // bytes per row block
    const int32_t *boff = frange + nblk * NH;   // gather offsets of the bound tests
    float th[NS];
    bool valid[NS];
    // code pairs saturate at kCodeMax: a threshold at or above it could not be
    // told from a saturated bound, so every block is then summed exactly
    bool all_hot = false;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        th[s] = thr[s];
        valid[s] = R >= 2 * rlo * (1 << s);
        if (PW) all_hot |= !(th[s] < kCodeMax);
    }
    // Exact maxima over the column's hot blocks and their smallest maximising
    // Zq: a column's maximum above threshold lies in a block that is hot for
    // that column (every other block's sums are at or below its bound, itself
    // at or below the threshold), and hot blocks are summed in increasing Zq
    // with strictly larger values only replacing the maximum. Stage maxima at
    // or below the threshold are not candidates, whatever blocks they cover. The Zq of two stages share a register as 16-bit
    // halves (the block tests need the registers).
    constexpr int NP = (NS + 1) / 2;
    float mx[SB][NS];
    uint32_t azp[SB][NP];
#pragma unroll
    for (int m = 0; m < SB; ++m) {
#pragma unroll
        for (int s = 0; s < NS; ++s) mx[m][s] = 0.0f;
#pragma unroll
        for (int h = 0; h < NP; ++h) azp[m][h] = 0u;
    }
    for (int k0 = 0; k0 < nblk; k0 += kBoundChunk) {
        // pass 1: per series, a wave-uniform mask of the blocks some lane cannot rule out
        // per series, a wave-uniform mask of the blocks some lane cannot rule
        // out, and each lane's own mask of the blocks it cannot rule out
        uint64_t hotmask[SB], lanehot[SB];
#pragma unroll
        for (int m = 0; m < SB; ++m) hotmask[m] = lanehot[m] = 0;
        const int kend = nblk - k0 < kBoundChunk ? nblk - k0 : kBoundChunk;
        for (int kk = 0; kk < kend; ++kk) {
            if constexpr (PW) {
                // Code pairs per column: one gather per fraction and block,
                // none under a branch, through buffer resources with the row
                // block's byte offset from a host table as the scalar offset
                // and the lane's column as the vector offset (no lane computes
                // an address): o[j] is the byte offset of the code pair of row
                // block a; o[NH + j] the byte selector that keeps block a + 1's
                // code where the range has it and zeroes it otherwise. Codes
                // order like their values, so a range's bound is the larger
                // code. Fractions that no searched stage of this lane needs are
                // gathered and summed like the others: they only enter the sums
                // of stages the lane does not search.
                const int32_t *bt = boff + (k0 + kk) * (2 * NH + 2);
                int32_t o[2 * NH + 2];
#pragma unroll
                for (int i = 0; i < 2 * NH + 2; ++i) o[i] = bt[i];
                uint16_t B[SB][NH];   // half bits of the fractions' bounds
                uint32_t w[SB][NH];
#pragma unroll
                for (int j = 0; j < NH; ++j) {
#pragma unroll
                    for (int m = 0; m < SB; ++m) w[m][j] = __builtin_amdgcn_raw_buffer_load_b16(rs[m], cb[j], o[j], 0);
                }
#pragma unroll
                for (int m = 0; m < SB; ++m) {
#pragma unroll
                    for (int j = 0; j < NH; ++j) B[m][j] = code_half_bits(max_code(w[m][j], (uint32_t)o[NH + j]));
                }
                if (o[2 * NH + 1]) {
                    // ranges over three or more row blocks (wave-uniform, rare):
                    // blocks a + 2 .. e, the low code of their pairs
                    const int32_t *fr = frange + (k0 + kk) * NH;
#pragma unroll
                    for (int j = 0; j < NH; ++j) {
                        const int n = fr[j] >> 24;
                        for (int k = 2; k <= n; ++k) {
                            const int32_t off = o[j] + k * (int32_t)rowb;
#pragma unroll
                            for (int m = 0; m < SB; ++m) {
                                const uint16_t v = code_half_bits(__builtin_amdgcn_raw_buffer_load_b16(rs[m], cb[j], off, 0) & 0xffu);
                                B[m][j] = B[m][j] > v ? B[m][j] : v;
                            }
                        }
                    }
                }
#pragma unroll
                for (int m = 0; m < SB; ++m) {
                    float U[NS];
                    stage_chain_h<NH>(B[m], U);
                    bool hot = false;
#pragma unroll
                    for (int s = 0; s < NS; ++s) hot |= valid[s] && (U[s] > th[s]);
                    hot |= all_hot;
                    if (hot) lanehot[m] |= 1ull << kk;
                    if (__any(hot)) hotmask[m] |= 1ull << kk;
                }
            } else {
                const int32_t *fr = frange + (k0 + kk) * NH;
                // The first row block of every range, and the second only where
                // the range has one (a wave-uniform test; about a third of the
                // ranges at 6-row blocks and 16 harmonics). The block's ranges are
                // read before the first test: inside the tests each would be a
                // scalar load of its own that the next gathers wait for. The
                // gathers keep their raw half bits, so no conversion sits in a
                // branch where it would wait for all earlier loads, and both
                // blocks' bits merge by an integer maximum (non-negative halves
                // order like their bits).
                float B[SB][NH];
                int wide = 0;
                {
                    int32_t fv[NH];
    #pragma unroll
                    for (int j = 0; j < NH; ++j) fv[j] = fr[j];
                    uint16_t Bb[SB][NH], Cb[SB][NH];
                    // a zero the compiler cannot see through: with a literal 0 it
                    // folds the merge into the branch, where it waits for every
                    // earlier gather
                    const uint16_t zero = (uint16_t)__builtin_amdgcn_mbcnt_lo(0u, 0u);
    #pragma unroll
                    for (int j = 0; j < NH; ++j) {
                        const int32_t f = fv[j];
                        const int n = f >> 24;
                        wide |= n > 1;
                        const uint32_t o0 = (uint32_t)(f & 0xffffff) * rowb + cb[j];
    #pragma unroll
                        for (int m = 0; m < SB; ++m) {
                            Bb[m][j] = load_bits_at(yb[m], o0);
                            Cb[m][j] = zero;
                        }
                        if (n > 0) {
    #pragma unroll
                            for (int m = 0; m < SB; ++m) Cb[m][j] = load_bits_at(yb[m], o0 + rowb);
                        }
                    }
    #pragma unroll
                    for (int m = 0; m < SB; ++m) {
    #pragma unroll
                        for (int j = 0; j < NH; ++j)
                            B[m][j] = half_bits_to_float(Bb[m][j] > Cb[m][j] ? Bb[m][j] : Cb[m][j]);
                    }
                }
                if (wide) {
                    // ranges over three or more row blocks (wave-uniform, rare)
    #pragma unroll
                    for (int j = 0; j < NH; ++j) {
                        const int32_t f = fr[j];
                        const int n = f >> 24;
                        for (int k = 2; k <= n; ++k) {
                            const uint32_t o = (uint32_t)((f & 0xffffff) + k) * rowb + cb[j];
    #pragma unroll
                            for (int m = 0; m < SB; ++m) B[m][j] = fmaxf(B[m][j], load_at(yb[m], o));
                        }
                    }
                }
    #pragma unroll
                for (int m = 0; m < SB; ++m) {
    #pragma unroll
                    for (int j = 0; j < NH; ++j) B[m][j] = ((need >> j) & 1u) ? B[m][j] : 0.0f;
                    float U[NS];
                    stage_chain<NH>(B[m], U);
                    bool hot = false;
    #pragma unroll
                    for (int s = 0; s < NS; ++s) hot |= valid[s] && (U[s] > th[s]);
                    if (hot) lanehot[m] |= 1ull << kk;
                    if (__any(hot)) hotmask[m] |= 1ull << kk;
                }
            }
        }
        // pass 2: exact sums of the hot blocks
        uint64_t any_hot = 0;
#pragma unroll
        for (int m = 0; m < SB; ++m) any_hot |= hotmask[m];
        if (!any_hot) continue;
        int64_t col[NH];
        (void)column_offsets<NH>(R, rlo, col);
#pragma unroll
        for (int m = 0; m < SB; ++m) {
            if (b0 + m >= nseries) break;
            const float *pb = plane + (int64_t)(b0 + m) * sstride;
            uint64_t hm = hotmask[m];
            while (hm) {
                const int kk = __builtin_ctzll(hm), kb = k0 + kk;
                hm &= hm - 1;
                // only the lanes whose own bound is hot sum the block: a lane
                // whose bounds stay at or below every threshold holds no
                // candidate in it, and its maxima matter only above them
                if (!((lanehot[m] >> kk) & 1u)) continue;
                const int zqa = blk_lo[kb] - Z, zqb = blk_lo[kb + 1] - 1 - Z;
                // as the exhaustive sweep: fraction values stay in registers and
                // are reloaded only when their (wave-uniform) row changes, the
                // next row's loads issued before the current row is summed
                const float *pz = pb + (int64_t)Z * pitch;     // row Zq = 0
                float cur[NH];
                int rowj[NH];
#pragma unroll
                for (int j = 1; j <= NH; ++j) {
                    rowj[j - 1] = frac_row<NH>(zqa, j);
                    cur[j - 1] = (need >> (j - 1)) & 1u ? pz[(int64_t)rowj[j - 1] * pitch + col[j - 1]] : 0.0f;
                }
                for (int zq = zqa; zq <= zqb; ++zq) {
                    float nxt[NH];
#pragma unroll
                    for (int j = 0; j < NH; ++j) nxt[j] = cur[j];
                    if (zq < zqb) {
#pragma unroll
                        for (int j = 1; j <= NH; ++j) {
                            const int r = frac_row<NH>(zq + 1, j);
                            if (r != rowj[j - 1]) {
                                rowj[j - 1] = r;
                                nxt[j - 1] = (need >> (j - 1)) & 1u ? pz[(int64_t)r * pitch + col[j - 1]] : 0.0f;
                            }
                        }
                    }
                    float Ss[NS];
                    stage_chain<NH>(cur, Ss);
#pragma unroll
                    for (int s = 0; s < NS; ++s) {
                        if (Ss[s] > mx[m][s]) {
                            mx[m][s] = Ss[s];
                            const uint32_t sh = 16u * (s & 1);
                            azp[m][s >> 1] = (azp[m][s >> 1] & ~(0xffffu << sh)) | ((uint32_t)(uint16_t)zq << sh);
                        }
                    }
#pragma unroll
                    for (int j = 0; j < NH; ++j) cur[j] = nxt[j];
                }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < SB; ++m) {
        if (b0 + m >= nseries) break;
        float *mo = maxv + (int64_t)(b0 + m) * NS * mpitch + c;
        int16_t *za = zarg + (int64_t)(b0 + m) * NS * mpitch + c;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            mo[s * mpitch] = valid[s] ? mx[m][s] : 0.0f;
            za[s * mpitch] = (int16_t)(valid[s] ? (azp[m][s >> 1] >> (16u * (s & 1))) & 0xffffu : 0u);
        }
    }
}

template <int NH, bool PW>
__global__ __launch_bounds__(256) void k_harm_bound(const float *__restrict__ plane, int64_t pitch,
                                                    int64_t sstride, const bmax_t *__restrict__ pyr,
                                                    int64_t psstride, const int32_t *__restrict__ blk_lo,
                                                    const int32_t *__restrict__ frange, int nblk,
                                                    int64_t NR, int64_t rlo, int Z,
                                                    const float *__restrict__ thr,
                                                    float *__restrict__ maxv, int16_t *__restrict__ zarg,
                                                    int64_t mpitch, int64_t tiles_per_series,
                                                    int64_t total_tiles, int64_t ppitch, int nseries) {
    // Items (series group, column tile) in series-major order go to the XCDs
    // (workgroup id mod 8) in runs of kBoundXcdRun consecutive tiles: the
    // whole chip sweeps one series at a time, so the fractions' re-reads of
    // its block maxima meet in the shared last-level cache, while each XCD
    // still gets neighbouring tiles whose fraction strips overlap in its L2
    // (one contiguous share of the items per XCD, one series each at 8 series
    // per launch, took 45.7 ms of harmonic sums on 32 x 2^23 series at 16
    // harmonics, runs of 1, 4 and 16 tiles 43.7, 43.2 and 43.3 ms). The grid is
    // a whole number of 8 kBoundXcdRun workgroups.
    const int64_t w = blockIdx.x;
    const int64_t i = w >> 3;
    const int64_t g = ((i / kBoundXcdRun) * 8 + (w & 7)) * kBoundXcdRun + i % kBoundXcdRun;
    if (g >= total_tiles) return;
    harm_bound_tile<NH, PW>(plane, pitch, sstride, pyr, psstride, blk_lo, frange, nblk, NR, rlo, Z, thr, maxv,
                            zarg, mpitch, tiles_per_series, g, ppitch, nseries);
}

// A pointer read from memory is generic for the compiler (flat loads with
// 64-bit lane addresses); this marks it as global memory again.
template <typename T>
__device__ __forceinline__ T *global_ptr(T *p) {
    typedef __attribute__((address_space(1))) T global_T;
    return (T *)(global_T *)(uintptr_t)p;
}

// The same over a work list: the XCD of workgroup w (w mod 8) walks its runs
// of every item in list order (the host puts the items with the most drift
// blocks first, so the launch ends on cheap tiles); item i's run on XCD x is
// its tiles x run_i ... (x + 1) run_i - 1, so each XCD still sweeps
// neighbouring tiles. The item of a workgroup is found by bisection of the
// run starts (wave-uniform scalar loads).
template <int NH>
__global__ __launch_bounds__(256) void k_harm_bound_list(const HarmItem *__restrict__ items,
                                                         const int64_t *__restrict__ starts, int n,
                                                         const float *__restrict__ thr) {
    const int64_t w = blockIdx.x;
    const int64_t l = w >> 3;
    int lo = 0, hi = n;   // starts[lo] <= l < starts[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (starts[mid] <= l) lo = mid;
        else hi = mid;
    }
    const HarmItem &it = items[lo];
    const int64_t run = starts[lo + 1] - starts[lo];
    const int64_t g = (w & 7) * run + (l - starts[lo]);
    if (g >= it.ntiles) return;
    if (it.pair)
        harm_bound_tile<NH, false>(global_ptr(it.plane), it.pitch, it.sstride, global_ptr(it.pyr), it.psstride,
                                   global_ptr(it.blk_lo), global_ptr(it.frange), it.nblk, it.NR, it.rlo, it.Z,
                                   thr, global_ptr(it.maxv), global_ptr(it.zarg), it.mpitch, it.tiles_per_series,
                                   g, it.ppitch, it.nseries);
    else
        harm_bound_tile<NH, true>(global_ptr(it.plane), it.pitch, it.sstride, global_ptr(it.pyr), it.psstride,
                                  global_ptr(it.blk_lo), global_ptr(it.frange), it.nblk, it.NR, it.rlo, it.Z,
                                  thr, global_ptr(it.maxv), global_ptr(it.zarg), it.mpitch, it.tiles_per_series,
                                  g, it.ppitch, it.nseries);
}

// Block maxima of a caller-supplied plane (what K4 writes while it builds the
// plane). With pair, pyr[b][k][i] covers columns 2i and 2i+1 as a half rounded
// up; otherwise column c of row block k holds the 16-bit word of the
// bound_code()s of the maxima of blocks k (low byte) and k + 1 (high byte, 0
// above the last block).
__device__ __forceinline__ float block_max_of(const float *src, int64_t pitch, int r0, int r1, int pair) {
    float mx = 0.0f;
    for (int r = r0; r < r1; ++r) {
        const float *q = src + (int64_t)r * pitch;
        mx = fmaxf(mx, pair ? fmaxf(q[0], q[1]) : q[0]);
    }
    return mx;
}

__global__ __launch_bounds__(256) void k_block_max(const float *__restrict__ plane, int64_t pitch,
                                                   int64_t sstride, int64_t NR,
                                                   const int32_t *__restrict__ blk_lo, int nblk,
                                                   bmax_t *__restrict__ pyr, int64_t psstride, int pair,
                                                   int64_t ppitch) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int k = blockIdx.y, b = blockIdx.z;
    const int64_t ncol = pair ? NR / 2 : NR;
    if (i >= ncol || k >= nblk) return;
    const float *src = plane + (int64_t)b * sstride + (pair ? 2 * i : i);
    const float mk = block_max_of(src, pitch, blk_lo[k], blk_lo[k + 1], pair);
    bmax_t *row = pyr + (int64_t)b * psstride + (int64_t)k * ppitch;
    if (pair) {
        row[i] = bound_half(mk);
    } else {
        const uint32_t c1 = k + 1 < nblk ? bound_code(block_max_of(src, pitch, blk_lo[k + 1], blk_lo[k + 2], 0)) : 0u;
        row[i] = (bmax_t)(bound_code(mk) | (c1 << 8));
    }
}

hipError_t launch_block_max(const float *plane, int64_t pitch, int64_t series_stride, int64_t NR,
                            const RowBlocks &rb, int nseries, bmax_t *pyr, int64_t pyr_series_stride,
                            hipStream_t st) {
    const int64_t ncol = rb.pair ? NR / 2 : NR;
    if (nseries < 1 || nseries > 65535 || rb.nblk < 1 || rb.nblk > 65535 || !rb.lo || (pitch & 1) ||
        (NR & 1) || rb.ppitch < ncol || (rb.ppitch & 31) ||
        pyr_series_stride < rb.nblk * rb.ppitch)
        return hipErrorInvalidValue;
    dim3 grid((unsigned)((ncol + 255) / 256), (unsigned)rb.nblk, (unsigned)nseries);
    hipLaunchKernelGGL(k_block_max, grid, dim3(256), 0, st, plane, pitch, series_stride, NR, rb.lo,
                       rb.nblk, pyr, pyr_series_stride, rb.pair ? 1 : 0, rb.ppitch);
    return hipGetLastError();
}

// ------------------------------------------------------------------ compaction

static constexpr int kCB = 4096;   // elements per compaction block: 256 threads x 16

__device__ __forceinline__ int block_exclusive_scan(int v, int *tmp, int &total) {
    // 256 threads: wave inclusive scans, then the wave totals
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(incl, off, 64);
        if (lane >= off) incl += o;
    }
    if (lane == 63) tmp[wid] = incl;
    __syncthreads();
    int base = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < 4; ++w) {
        const int x = tmp[w];
        if (w < wid) base += x;
        total += x;
    }
    __syncthreads();
    return base + incl - v;
}

template <bool SCATTER>
__global__ __launch_bounds__(256) void k_compact(const float *__restrict__ maxv,
                                                 const int16_t *__restrict__ zarg, int64_t nelem,
                                                 int64_t mpitch, int ns, int b0,
                                                 const float *__restrict__ thr,
                                                 int32_t *__restrict__ counts,
                                                 const int64_t *__restrict__ offsets,
                                                 DevCand *__restrict__ out, int64_t cap) {
    __shared__ int tmp[4];
    // the scatter pass skips the blocks the counting pass found empty (most of
    // them: candidates are rare), without reading their maxima
    if (SCATTER && counts[blockIdx.x] == 0) return;
    const int64_t e0 = (int64_t)blockIdx.x * kCB + (int64_t)threadIdx.x * 16;
    float v[16];
    int row = 0;
    float th = INFINITY;
    if (e0 < nelem) {
        row = (int)(e0 / mpitch);          // mpitch is a multiple of 16: one row per thread
        th = thr[row % ns];
        const float4 *p = reinterpret_cast<const float4 *>(maxv + e0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float4 x = p[i];
            v[4 * i] = x.x;
            v[4 * i + 1] = x.y;
            v[4 * i + 2] = x.z;
            v[4 * i + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int i = 0; i < 16; ++i) v[i] = 0.0f;
    }
    int cnt = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) cnt += v[i] > th;
    int total;
    const int pre = block_exclusive_scan(cnt, tmp, total);
    if (!SCATTER) {
        if (threadIdx.x == 0) counts[blockIdx.x] = total;
        return;
    }
    if (cnt == 0) return;
    int64_t o = offsets[blockIdx.x] + pre;
    const int64_t c0 = e0 - (int64_t)row * mpitch;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (v[i] > th) {
            if (o < cap) {
                DevCand d;
                d.b = b0 + row / ns;
                d.s = row % ns;
                d.c = (int32_t)(c0 + i);
                d.zq = zarg[e0 + i];
                d.power = v[i];
                d.pad = 0;
                d.sigma = 0.0;
                out[o] = d;
            }
            ++o;
        }
    }
}

// Exclusive scan of the block counts, offset by the running total in state[0].
// The 1024 threads sweep the counts in tiles of 4096, four consecutive counts
// per thread (one coalesced 16-byte load), each tile scanned by wave shuffles
// and then across the 16 wave totals.
__global__ __launch_bounds__(1024) void k_scan_counts(const int32_t *__restrict__ counts,
                                                      int64_t nblk, int64_t *__restrict__ offsets,
                                                      int64_t *__restrict__ state) {
    __shared__ int64_t wsum[16];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    const int64_t base0 = state[0];
    int64_t carry = base0;
    for (int64_t i0 = 0; i0 < nblk; i0 += 4096) {
        const int64_t i = i0 + 4 * (int64_t)t;
        int c[4];
        if (i + 3 < nblk) {
            const int4 v = *reinterpret_cast<const int4 *>(counts + i);
            c[0] = v.x;
            c[1] = v.y;
            c[2] = v.z;
            c[3] = v.w;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) c[q] = i + q < nblk ? counts[i + q] : 0;
        }
        const int64_t sum = (int64_t)c[0] + c[1] + c[2] + c[3];
        int64_t incl = sum;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int64_t o = __shfl_up(incl, off, 64);
            if (lane >= off) incl += o;
        }
        if (lane == 63) wsum[wid] = incl;
        __syncthreads();
        int64_t wbase = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < 16; ++w) {
            const int64_t x = wsum[w];
            if (w < wid) wbase += x;
            tot += x;
        }
        __syncthreads();   // wsum is rewritten by the next tile
        int64_t run = carry + wbase + incl - sum;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (i + q < nblk) offsets[i + q] = run;
            run += c[q];
        }
        carry += tot;
    }
    __syncthreads();   // every thread has read state[0]
    if (t == 0) {
        state[1] = base0;
        state[0] = carry;
    }
}

template <int NH>
static void launch_harm_nh(const float *plane, int64_t pitch, int64_t sstride, int64_t NR,
                           int64_t rlo, int Z, int nseries, float *maxv, int16_t *zarg, int64_t mpitch,
                           int order, hipStream_t st) {
    const int64_t tps = (mpitch + 255) / 256;
    const int64_t total = tps * nseries;
    const int64_t nwg = 8 * ((total + 7) / 8);
    const int xcd_runs = order == 1 ? 1 : 0;
    if (order == 3 && Z > 0) {
        // negative drift half, then the positive half merged into the same maxima
        hipLaunchKernelGGL(k_harmsum<NH>, dim3((unsigned)nwg), dim3(256), 0, st, plane, pitch, sstride,
                           NR, rlo, Z, maxv, zarg, mpitch, tps, total, 0, -Z, 0, 0);
        hipLaunchKernelGGL(k_harmsum<NH>, dim3((unsigned)nwg), dim3(256), 0, st, plane, pitch, sstride,
                           NR, rlo, Z, maxv, zarg, mpitch, tps, total, 0, 1, Z, 1);
    } else {
        hipLaunchKernelGGL(k_harmsum<NH>, dim3((unsigned)nwg), dim3(256), 0, st, plane, pitch, sstride,
                           NR, rlo, Z, maxv, zarg, mpitch, tps, total, xcd_runs, -Z, Z, 0);
    }
}

hipError_t launch_harmsum(const float *plane, int64_t pitch, int64_t series_stride, int64_t NR,
                          int64_t rlo, int Z, int numharm, int nseries, float *maxv, int16_t *zarg,
                          int64_t mpitch, int order, hipStream_t st) {
    if (nseries < 1 || mpitch < NR || (mpitch & 15) || (mpitch + 255) / 256 * nseries > 0x7fffff00LL ||
        order < 1 || order > 3 || !zarg || Z > 32767)
        return hipErrorInvalidValue;
    switch (numharm) {
    case 1: launch_harm_nh<1>(plane, pitch, series_stride, NR, rlo, Z, nseries, maxv, zarg, mpitch, order, st); break;
    case 2: launch_harm_nh<2>(plane, pitch, series_stride, NR, rlo, Z, nseries, maxv, zarg, mpitch, order, st); break;
    case 4: launch_harm_nh<4>(plane, pitch, series_stride, NR, rlo, Z, nseries, maxv, zarg, mpitch, order, st); break;
    case 8: launch_harm_nh<8>(plane, pitch, series_stride, NR, rlo, Z, nseries, maxv, zarg, mpitch, order, st); break;
    case 16: launch_harm_nh<16>(plane, pitch, series_stride, NR, rlo, Z, nseries, maxv, zarg, mpitch, order, st); break;
    case 32: launch_harm_nh<32>(plane, pitch, series_stride, NR, rlo, Z, nseries, maxv, zarg, mpitch, order, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int NH>
static void launch_bound_nh(const float *plane, int64_t pitch, int64_t sstride, const bmax_t *pyr,
                            int64_t psstride, const RowBlocks &rb, int64_t NR, int64_t rlo, int Z,
                            int nseries, const float *thr, float *maxv, int16_t *zarg, int64_t mpitch,
                            hipStream_t st) {
    const int64_t tps = (mpitch + 255) / 256;
    const int64_t groups = (nseries + BoundCfg<NH>::SB - 1) / BoundCfg<NH>::SB;
    const int64_t total = tps * groups;
    const int64_t unit = 8 * kBoundXcdRun;
    const int64_t nwg = unit * ((total + unit - 1) / unit);
    if (rb.pair)
        hipLaunchKernelGGL((k_harm_bound<NH, false>), dim3((unsigned)nwg), dim3(256), 0, st, plane, pitch,
                           sstride, pyr, psstride, rb.lo, rb.frange, rb.nblk, NR, rlo, Z, thr, maxv, zarg, mpitch,
                           tps, total, rb.ppitch, nseries);
    else
        hipLaunchKernelGGL((k_harm_bound<NH, true>), dim3((unsigned)nwg), dim3(256), 0, st, plane, pitch,
                           sstride, pyr, psstride, rb.lo, rb.frange, rb.nblk, NR, rlo, Z, thr, maxv, zarg, mpitch,
                           tps, total, rb.ppitch, nseries);
}

hipError_t launch_harmsum_bounded(const float *plane, int64_t pitch, int64_t series_stride,
                                  const bmax_t *pyr, int64_t pyr_series_stride, const RowBlocks &rb,
                                  int64_t NR, int64_t rlo, int Z, int numharm, int nseries,
                                  const float *thr_dev, float *maxv, int16_t *zarg, int64_t mpitch,
                                  hipStream_t st) {
    // block-maxima offsets within one series are 32-bit in the kernel
    if (nseries < 1 || mpitch < NR || (mpitch & 15) || (mpitch + 255) / 256 * nseries > 0x7fffff00LL ||
        !pyr || !rb.lo || !rb.frange || rb.nblk < 1 || rb.frange_nh != numharm ||
        bounded_table_bytes(rb.nblk, numharm) > kBoundTableMax || pyr_series_stride > kMaxPyrSeriesStride ||
        !zarg || Z > 32767 || (rb.ppitch & 31) || rb.ppitch < (rb.pair ? NR / 2 : NR) || rb.table_ppitch != rb.ppitch ||
        pyr_series_stride < rb.nblk * rb.ppitch)
        return hipErrorInvalidValue;
#define FDAS_BOUND(NHV) launch_bound_nh<NHV>(plane, pitch, series_stride, pyr, pyr_series_stride, rb, NR, rlo, Z, nseries, thr_dev, maxv, zarg, mpitch, st)
    switch (numharm) {
    case 1: FDAS_BOUND(1); break;
    case 2: FDAS_BOUND(2); break;
    case 4: FDAS_BOUND(4); break;
    case 8: FDAS_BOUND(8); break;
    case 16: FDAS_BOUND(16); break;
    case 32: FDAS_BOUND(32); break;
    default: return hipErrorInvalidValue;
    }
#undef FDAS_BOUND
    return hipGetLastError();
}

template <int NH>
static void launch_bound_list_nh(const HarmItem *items, const int64_t *starts, int n, int64_t runs,
                                 const float *thr, hipStream_t st) {
    hipLaunchKernelGGL(k_harm_bound_list<NH>, dim3((unsigned)(8 * runs)), dim3(256), 0, st, items, starts, n, thr);
}

int64_t harm_items_layout(HarmItem *items, int n, int numharm, int64_t *starts) {
    int sb = 0;
    switch (numharm) {
    case 1: sb = BoundCfg<1>::SB; break;
    case 2: sb = BoundCfg<2>::SB; break;
    case 4: sb = BoundCfg<4>::SB; break;
    case 8: sb = BoundCfg<8>::SB; break;
    case 16: sb = BoundCfg<16>::SB; break;
    case 32: sb = BoundCfg<32>::SB; break;
    default: return -1;
    }
    if (n < 1) return -1;
    starts[0] = 0;
    for (int i = 0; i < n; ++i) {
        HarmItem &it = items[i];
        if (!it.plane || it.nseries < 1 || it.mpitch < it.NR || (it.mpitch & 15) ||
            (it.mpitch + 255) / 256 * it.nseries > 0x7ffffff0LL || !it.pyr || !it.blk_lo || !it.frange ||
            it.nblk < 1 || bounded_table_bytes(it.nblk, numharm) > kBoundTableMax ||
            it.psstride > kMaxPyrSeriesStride || !it.maxv || !it.zarg || it.Z < 0 || it.Z > 32767 ||
            (it.ppitch & 31) || it.ppitch < (it.pair ? it.NR / 2 : it.NR) || it.psstride < it.nblk * it.ppitch)
            return -1;
        it.tiles_per_series = (it.mpitch + 255) / 256;
        it.ntiles = it.tiles_per_series * ((it.nseries + sb - 1) / sb);
        starts[i + 1] = starts[i] + (it.ntiles + 7) / 8;
    }
    return starts[n] > 0x0fffffffLL ? -1 : starts[n];
}

hipError_t launch_harmsum_bounded_list(const HarmItem *items_dev, const int64_t *starts_dev, int n,
                                       int64_t runs, int numharm, const float *thr_dev, hipStream_t st) {
    if (n < 1 || runs < 1 || runs > 0x0fffffffLL || !items_dev || !starts_dev || !thr_dev)
        return hipErrorInvalidValue;
    switch (numharm) {
    case 1: launch_bound_list_nh<1>(items_dev, starts_dev, n, runs, thr_dev, st); break;
    case 2: launch_bound_list_nh<2>(items_dev, starts_dev, n, runs, thr_dev, st); break;
    case 4: launch_bound_list_nh<4>(items_dev, starts_dev, n, runs, thr_dev, st); break;
    case 8: launch_bound_list_nh<8>(items_dev, starts_dev, n, runs, thr_dev, st); break;
    case 16: launch_bound_list_nh<16>(items_dev, starts_dev, n, runs, thr_dev, st); break;
    case 32: launch_bound_list_nh<32>(items_dev, starts_dev, n, runs, thr_dev, st); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

__global__ void k_zero_state(int64_t *state) {
    if (threadIdx.x < 2) state[threadIdx.x] = 0;
}

hipError_t launch_zero_state(int64_t *state, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_state, dim3(1), dim3(64), 0, st, state);
    return hipGetLastError();
}

int64_t compact_blocks(int64_t nelem) { return (nelem + kCB - 1) / kCB; }

hipError_t launch_compact(const float *maxv, const int16_t *zarg, int64_t nelem, int64_t mpitch, int nstages,
                          int b0,
                          const float *thr_dev, int32_t *counts, int64_t *offsets, int64_t *state,
                          DevCand *out, int64_t cap, hipStream_t st) {
    if ((mpitch & 15) || nelem % mpitch) return hipErrorInvalidValue;
    const int64_t nblk = compact_blocks(nelem);
    if (nblk > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_compact<false>, dim3((unsigned)nblk), dim3(256), 0, st, maxv, zarg, nelem, mpitch,
                       nstages, b0, thr_dev, counts, offsets, out, cap);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, counts, nblk, offsets, state);
    hipLaunchKernelGGL(k_compact<true>, dim3((unsigned)nblk), dim3(256), 0, st, maxv, zarg, nelem, mpitch,
                       nstages, b0, thr_dev, counts, offsets, out, cap);
    return hipGetLastError();
}

}  // namespace fdas
