// Internal declarations shared by the host runtime and the kernel launchers.
#pragma once

#include "../../include/fdas.h"

#include <complex>
#include <cstdint>
#include <functional>
#include <new>
#include <stdexcept>
#include <vector>

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#else
#include <hip/hip_runtime_api.h>
#include <hip/hip_vector_types.h>
#endif

// Host exceptions (allocation failures, threads that cannot start) never
// cross the C ABI: an entry point's body runs between these two macros and
// such a failure becomes a status code (FDAS_E_NOMEM for allocations).
#define FDAS_ENTRY_TRY try {
#define FDAS_ENTRY_CATCH(handler, ctx)                                     \
    }                                                                      \
    catch (const std::bad_alloc &) {                                       \
        return handler(ctx, FDAS_E_NOMEM, "host memory allocation failed"); \
    }                                                                      \
    catch (const std::exception &x) {                                      \
        return handler(ctx, FDAS_E_DEVICE, x.what());                      \
    }                                                                      \
    catch (...) {                                                          \
        return handler(ctx, FDAS_E_DEVICE, "unexpected host error");       \
    }

namespace fdas {

// Runs fn(w) for w = 0..n-1 on up to n host threads, the caller's included.
// Shares whose thread cannot be started run on the caller; an exception of fn
// is caught in the thread that raised it. False if any share threw.
bool run_parallel(int n, const std::function<void(int)> &fn);
// entry-point error handler without a plan: the status alone
inline fdas_status status_only(const void *, fdas_status s, const char *) { return s; }

// ---------------------------------------------------------------- host FP64 math
std::complex<double> fresnel(double x);
std::complex<double> response(double q, double z);
int half_width(double z, int K);
void unit_taps(double z, int parity, int K, std::vector<std::complex<double>> &taps, int &d0);
void kernel_spectrum(double z, int parity, int K, int L, int mseg, float *out_interleaved);
double log_gamma_sf(int H, double S);
double log_gauss_tail(double s);
double threshold(int H, double sigma);
double sigma_of(int H, double power);

// 16-point Gauss-Legendre nodes and weights on [-1, 1] (FP64, Newton on P_16).
struct GaussLegendre16 {
    double x[16], w[16];
};
const GaussLegendre16 &gauss_legendre16();

// ---------------------------------------------------------------- device records
// One thresholded column maximum, in (series, stage, column) order.
struct DevCand {
    int32_t b;       // series within the batch
    int32_t s;       // stage index: H = 1 << s
    int32_t c;       // column: R = c + 2 rlo
    int32_t zq;      // smallest maximising z index
    float power;     // M_H(R)
    int32_t pad;
    double sigma;    // significance of power at stage H (filled by launch_cand_sigma)
};

// ---------------------------------------------------------------- launchers
// K1: real FFT of nseries series of n samples: n even, >= 8, with n/2 a product of
// powers of 2, 3 and 5 (fft_length_supported).
bool fft_length_supported(int64_t n);
// x: [nseries][n] float32; w0: scratch [nseries][n/2] complex (unused when
// n/2 <= 8192); spec: [nseries][spitch] complex receiving A_k for k = 0..n/2.
// offs (device, optional): series b starts at x + 2 offs[b] floats (ragged batches);
// otherwise series b starts at x + b n.
hipError_t launch_rfft(const float *x, int64_t n, int nseries, float2 *w0,
                       float2 *spec, int64_t spitch, hipStream_t st, const int64_t *offs = nullptr);

// state[0] = state[1] = 0 (a kernel, so that captured graphs hold no memset node).
hipError_t launch_zero_state(int64_t *state, hipStream_t st);

// K2: lower median of |A_k|^2 (k = 1..n/2-1) per series -> norm (FP64) and the
// amplitude scale sqrt(1/norm) (0 when the median is 0). scratch: device
// memory of median_scratch_bytes(nseries) bytes (histograms and select state).
size_t median_scratch_bytes(int nseries);
hipError_t launch_median_scale(const float2 *spec, int64_t spitch, int64_t half, int nseries,
                               float *scale, double *norm, void *scratch, hipStream_t st);
// Local (red-noise) normalisation in place: bstart[0..nblk] block starts (bstart[0]
// = 1, bstart[nblk] = half, widths <= 256); med: scratch of nseries * nblk floats;
// scale[b] is set to 1 (the spectrum itself carries the normalisation).
hipError_t launch_local_norm(float2 *spec, int64_t spitch, int64_t half, int nseries, const int32_t *bstart,
                             int nblk, float *med, float *scale, hipStream_t st);
// scale[0..nseries) = value (the fixed-variance normalisation).
hipError_t launch_fill_scale(float *scale, int nseries, float value, hipStream_t st);

// K4: overlap-save correlation with the template bank and power. The z rows
// are split into zgroups contiguous groups (one per XCD); group i covers rows
// zb[i] .. zb[i + 1] - 1 and segments the spectrum by its own widest
// template: half-width gmseg[i], gLv[i] = L - 2 gmseg[i] valid outputs per
// segment, gnseg[i] segments per series.
constexpr int kMaxZGroups = 8;
struct CorrGeom {
    int L;            // segment length (512, 1024, 2048 or 4096)
    int mseg;         // largest template half-width (of the widest group)
    int64_t half;     // n/2
    int64_t rlo;      // lowest searched bin
    int NZ;           // z rows
    int zgroups;      // z rows are split in this many groups (1, 2, 4, 8)
    int zb[kMaxZGroups + 1];
    int gmseg[kMaxZGroups], gLv[kMaxZGroups], gnseg[kMaxZGroups];
};
// Row boundaries zb[0..G] of the G z groups of K4 for NZ rows at spacing dz
// (templates of half-width half_width(z, K), segments of length L): contiguous
// groups chosen so that the plane kernel's time is as even as possible over
// the groups (one per XCD), a group's time being its rows divided by its
// valid outputs per segment. Every group keeps at least one row.
void zgroup_bounds(int NZ, double dz, int K, int L, int G, int32_t *zb);
// Drift-row blocks for the block maxima ("pyramid"): block k covers rows
// [lo[k], lo[k+1]); blocks never straddle a z group of K4. of_row[r] is the
// block of row r. Both tables live in device memory.
struct RowBlocks {
    const int32_t *lo = nullptr;      // nblk + 1 entries
    const int32_t *of_row = nullptr;  // NZ entries
    const int32_t *frange = nullptr;  // [nblk][frange_nh]: row blocks a..e that fraction j of
                                      // block k reads, packed a | (e - a) << 24
    // frange is followed by the bound test's gather table for code pairs in
    // rows of table_ppitch words (bound_offsets()), [nblk][2 frange_nh + 2]
    int nblk = 0;
    int frange_nh = 0;
    int64_t table_ppitch = 0;
    bool pair = false;                // maxima per bin (both parities, one half each) instead of
                                      // per column (a 16-bit word each: the 8-bit codes of
                                      // blocks k and k + 1)
    int64_t ppitch = 0;               // 16-bit entries per row block of the maxima (a multiple
                                      // of 32): pitch / 2 per bin, pitch per column
};
// Host construction of the row-block partition for the NZ = zb[G] rows of G z
// groups (boundaries zb) with blocks of at most bz rows (as even as possible
// inside each group).
void row_blocks(const int32_t *zb, int G, int bz, std::vector<int32_t> &lo, std::vector<int32_t> &of_row);
// Host table of the row blocks each harmonic fraction of each block reads.
void fraction_ranges(int NZ, int numharm, const std::vector<int32_t> &lo,
                     const std::vector<int32_t> &of_row, std::vector<int32_t> &frange);
// Host table of what the bound test of block k gathers for fraction j from
// code pairs per column (maxima rows of ppitch 16-bit words): entry [k][j] is
// the byte offset of row block a (the first of the fraction's range),
// [k][numharm + j] the byte selector (v_perm) that keeps block a + 1's code
// where the range has it (0x0c010c00) and drops it where the range is block a
// alone (0x0c0c0c00), [k][2 numharm + 1] non-zero if some range has three or
// more blocks. Maxima per bin are gathered by offsets the kernel derives from
// frange.
void bound_offsets(int numharm, const std::vector<int32_t> &frange, int64_t ppitch,
                   std::vector<int32_t> &boff);
constexpr int kBoundChunk = 64;   // blocks per pass of the bound test (one 64-bit hot mask)
// Fourth word of a raw buffer resource on this GPU family (32-bit data
// format; the base, stride 0 and the byte range come from the caller).
constexpr int kBufferRsrcWord3 = 0x00020000;
// Block maxima are stored as IEEE half bits rounded upward (+inf above the
// largest half), so every stored value still bounds the powers of its block.
using bmax_t = uint16_t;
// Limits of the bounded harmonic sums: row-block tables of at most 48 KiB, and
// block maxima of one series below 4 GiB (32-bit byte offsets in the kernel).
constexpr size_t kBoundTableMax = 48 * 1024;
constexpr int64_t kMaxPyrSeriesStride = ((int64_t)1 << 31) - 1;   // halves
inline size_t bounded_table_bytes(int nblk, int numharm) {
    return (size_t)(nblk + 1 + (size_t)nblk * numharm + (size_t)nblk * (2 * numharm + 2)) * sizeof(int32_t);
}

// K4. If pyr is not null, K4 also writes the block maxima, rounded up: with
// rb.pair the maximum over the rows of block k and columns 2i and 2i+1 as a
// half at pyr[b][k][i] (rows of pitch / 2 halves); otherwise, per column c, a
// 16-bit word at pyr[b][k][c] (rows of pitch words) holding bound_code() of
// the maxima of blocks k (low byte) and k + 1 (high byte; 0 for the last
// block).
hipError_t launch_corr_power(const float2 *spec, int64_t spitch, const float *scale,
                             const float2 *bank, const CorrGeom &g, int nseries, float *plane,
                             int64_t pitch, int64_t series_stride, bmax_t *pyr,
                             int64_t pyr_series_stride, const RowBlocks &rb, hipStream_t st);

// K5: harmonic sums and maxima over z for every column and stage.
// maxv: [nseries][nstages][mpitch] (zero where a stage is not searched);
// zarg, same layout: the smallest Zq reaching the maximum (|Zq| <= 32767).
// order: 1 each XCD sweeps a contiguous run of tiles, 2 all XCDs sweep the
// tiles in launch order, 3 as 2 but in two launches over the drift halves
// (Zq <= 0, then Zq > 0 merged), which halves the live plane per series.
hipError_t launch_harmsum(const float *plane, int64_t pitch, int64_t series_stride, int64_t NR,
                          int64_t rlo, int Z, int numharm, int nseries, float *maxv, int16_t *zarg,
                          int64_t mpitch, int order, hipStream_t st);

// Block maxima of a caller-supplied plane (what K4 writes alongside its plane).
hipError_t launch_block_max(const float *plane, int64_t pitch, int64_t series_stride, int64_t NR,
                            const RowBlocks &rb, int nseries, bmax_t *pyr, int64_t pyr_series_stride,
                            hipStream_t st);

// K5 with block bounds: per column and drift block, the stage chain over the
// block maxima bounds every exact stage sum of the block from above (FP32
// addition is monotone); only blocks where some searched stage's bound
// exceeds its threshold are summed exactly. maxv (and zarg) is exact wherever
// it exceeds the threshold (elsewhere it only stays at or below it), so the
// candidates equal those of launch_harmsum bit for bit.
hipError_t launch_harmsum_bounded(const float *plane, int64_t pitch, int64_t series_stride,
                                  const bmax_t *pyr, int64_t pyr_series_stride, const RowBlocks &rb,
                                  int64_t NR, int64_t rlo, int Z, int numharm, int nseries,
                                  const float *thr_dev, float *maxv, int16_t *zarg, int64_t mpitch,
                                  hipStream_t st);

// One entry of a bounded-sum work list: the arguments of
// launch_harmsum_bounded for one set of series (its plane, block maxima and
// maxima regions), plus its place in the merged launch. A work list lets one
// launch cover the planes of several groups of a ragged batch, whose separate
// launches each end in a partly idle tail.
struct HarmItem {
    const float *plane;
    int64_t pitch, sstride;
    const bmax_t *pyr;
    int64_t psstride, ppitch;
    const int32_t *blk_lo, *frange;
    float *maxv;
    int16_t *zarg;
    int64_t mpitch, NR, rlo;
    int64_t tiles_per_series;   // set by harm_items_layout
    int64_t ntiles;             // set by harm_items_layout
    int32_t nblk, Z, pair, nseries;
};
// Checks every item as launch_harmsum_bounded checks its arguments, fills in
// the tile counts and writes starts[0..n]: the merged launch gives each XCD
// (workgroup id mod 8) one contiguous run of starts[i+1] - starts[i] tiles
// of item i, items in list order. Returns starts[n] (tiles per XCD), or -1 if
// an item is invalid.
int64_t harm_items_layout(HarmItem *items, int n, int numharm, int64_t *starts);
// The merged bounded sums over a work list already in device memory
// (items_dev[n], starts_dev[n + 1] from harm_items_layout; runs = starts[n]).
hipError_t launch_harmsum_bounded_list(const HarmItem *items_dev, const int64_t *starts_dev, int n,
                                       int64_t runs, int numharm, const float *thr_dev, hipStream_t st);

// K6: ordered compaction of maxv > thr[stage] into records in (b, s, c) order,
// with the drift index from zarg.
// The batch may be processed in series chunks: state[0] (device int64) is the
// running record count over the chunks done so far, and after the call
// state[1] holds this chunk's first record index. Records at index >= cap are
// counted but not written. counts/offsets: scratch of compact_blocks() entries.
int64_t compact_blocks(int64_t nelem);
hipError_t launch_compact(const float *maxv, const int16_t *zarg, int64_t nelem, int64_t mpitch,
                          int nstages, int b0, const float *thr_dev, int32_t *counts, int64_t *offsets,
                          int64_t *state, DevCand *out, int64_t cap, hipStream_t st);

// FP64 significance of the records [0, min(state[0], cap)) of the call
// (the host statistics' arithmetic).
hipError_t launch_cand_sigma(DevCand *rec, const int64_t *state, int64_t cap, hipStream_t st);

// K0: dedispersion. x: time-major uint8 [nsamp][nchan]; y: channel-major float
// rows [nchan][ypitch] of boxcar sums over D samples (n = nsamp / D outputs).
// With sums set (zeroed by launch_zero_sums), the channels' sample totals are
// added to sums[c].
hipError_t launch_fil_downsample(const uint8_t *x, int64_t nsamp, int nchan, int D, float *y, int64_t ypitch,
                                 unsigned long long *sums, hipStream_t st);
hipError_t launch_zero_sums(unsigned long long *sums, int nchan, hipStream_t st);
// pad[c] = floor((D sums[c] + nsamp/2) / nsamp).
hipError_t launch_channel_pad(const unsigned long long *sums, int64_t nsamp, int D, int nchan, float *pad,
                              hipStream_t st);
// out[c][j] = sum_{k<f} in[c][j f + k] for j < n_out, c < nchan.
hipError_t launch_downsample_rows(const float *in, int64_t ipitch, int64_t n_out, int f, int nchan, float *out,
                                  int64_t opitch, hipStream_t st);
// LDS row width (floats) that launch_dedisperse stages for a delay spread
// span_max (0 if the spread is too wide for groups of more than one trial).
int dedisperse_width(int span_max);
// out[i][j] = sum_c y[c][j + delays[c][i]] (pad[c] past n - 1), groups of G trial
// DMs per block (G in 1, 2, 4, 8, 16), 16 channels per LDS stage. delays:
// [nchan][ndm_pad], non-decreasing in i, ndm_pad a multiple of G with entries
// past ndm repeating the last DM; span_max bounds delays[c][i0 + G - 1] -
// delays[c][i0] over groups and channels.
hipError_t launch_dedisperse(const float *y, int64_t ypitch, int64_t n, int nchan, const float *pad,
                             const int32_t *delays, int ndm, int ndm_pad, int G, int span_max, float *out,
                             int64_t opitch, hipStream_t st);

// K7/K8: refinement objective (see fdas_refine_eval), its gradients and the
// ascent. One wave per point; the window of 2 m + 1 bins is staged in LDS, so
// every point must have m <= max_m <= kRefineMaxM (others give NaN).
constexpr int kRefineMaxM = 2000;
hipError_t launch_refine_eval(const float2 *spec, int64_t spitch, int64_t nbins, int nseries, const float *scale,
                              const fdas_refine_point *pts, int64_t n, int max_m, float *power, float *dpdr,
                              float *dpdz, hipStream_t st);
hipError_t launch_refine_grad(const float2 *spec, int64_t spitch, int64_t nbins, int nseries, const float *scale,
                              const fdas_refine_point *pts, int64_t n, int max_m, const float *grad_power,
                              float *grad_r, float *grad_z, float *grad_spec, hipStream_t st);
hipError_t launch_refine_ascent(const float2 *spec, int64_t spitch, int64_t nbins, int nseries, const float *scale,
                                fdas_refine_point *pts, int64_t n, int max_m, double dz, int iters, float *power,
                                hipStream_t st);

}  // namespace fdas
