/*
 * fdas.h - C ABI of the MI355X (gfx950) Fourier-domain acceleration search.
 *
 * The library searches a batch of dedispersed time series for periodic
 * signals whose frequency drifts linearly over the observation: the pipeline
 * steps "FFT the dedispersed series" and "search the spectrum for periodic
 * signals with a frequency derivative bounded by zmax" (paper, Section 2,
 * steps 3-4; zmax is the knob measured in Section 3.2, Table 4), followed by
 * the candidate list that the sifting step (Section 2, step 5) consumes.
 *
 * The paper names these steps but does not state their mathematics. This
 * library computes, per series b of length N (even) sampled at tsamp:
 *   A_k   = sum_n x_n exp(-2 pi i k n / N), k = 0..N/2            (real FFT)
 *   norm  = lower median of |A_k|^2 over k = 1..N/2-1, divided by ln 2
 *           (or N * fixed_var), A^_k = A_k / sqrt(norm), A^_0 = A^_{N/2} = 0
 *   P(r,z)= |sum_k A^_k conj rho(r-k, z)|^2 / E over |k - r| <= ceil(|z|/2)+K,
 *           rho(q,z) = int_0^1 exp(2 pi i [q u + z (u^2-u)/2]) du, E the tap
 *           energy; r = R/2 (half bins) at mid-observation, z = Zq*dz total drift
 *   S_H   = sum_{k=1..H} P(round_half_up(R k/H), round_half_away(Zq k/H))
 *   M_H(R)= max over Zq of S_H; a candidate is (b, H, R, Zq*) with
 *           M_H(R) > T_H, where a sum of H unit exponentials exceeds T_H with
 *           probability erfc(sigma/sqrt 2)/2 (single trial).
 * H runs over 1, 2, 4, ..., numharm; R over [2 rlo H, N-1], rlo = ceil(flo T)
 * (at least 1), T = N tsamp; Zq over [-zmax/dz, zmax/dz].
 *
 * Conventions: every pointer argument named *_dev is device memory of the
 * current HIP device, *_host is host memory. Calls return an fdas_status and
 * never abort or throw across the ABI (a failed host allocation inside a call
 * returns FDAS_E_NOMEM, with the message in fdas_last_error when a plan is
 * given). A plan is not thread safe: use one
 * plan per host thread / stream. Calls that take a stream enqueue their work
 * on it (NULL = the default stream) and return only after the work is done.
 */
#ifndef FDAS_H
#define FDAS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdas_plan_s *fdas_plan;

typedef enum {
    FDAS_OK = 0,
    FDAS_E_INVAL = -1,        /* bad argument; nothing was launched */
    FDAS_E_NOMEM = -2,        /* device or host allocation failed */
    FDAS_E_DEVICE = -3,       /* a HIP call failed; sticky on the plan */
    FDAS_E_TRUNC = -4,        /* more candidates than the caller's capacity */
    FDAS_E_UNSUPPORTED = -5   /* valid but not supported (e.g. N/2 with a prime factor above 5) */
} fdas_status;

/* FDAS_NORM_LOCAL (red-noise normalisation): bins 1..N/2-1 are cut into blocks
 * starting at b_0 = 1 of width min(200, 6 + floor(b_i / 30)); each block's lower
 * median power / ln 2 sits at the block centre, the mean-power estimate m(k)
 * interpolates linearly between centres (constant outside them) and
 * A^_k = A_k / sqrt(m(k)). fdas_spectrum then returns the normalised spectra. */
typedef enum { FDAS_NORM_MEDIAN = 0, FDAS_NORM_FIXED = 1, FDAS_NORM_LOCAL = 2 } fdas_norm;

typedef struct {
    double  flo_hz;              /* lowest searched frequency, Hz (default 1.0) */
    int32_t K;                   /* template half-width margin in bins (default 16) */
    int32_t norm;                /* fdas_norm (default FDAS_NORM_MEDIAN) */
    double  fixed_var;           /* FDAS_NORM_FIXED: norm = N * fixed_var (default 1.0) */
    int64_t max_workspace_bytes; /* cap on the power-plane workspace (0 = automatic) */
    int64_t max_candidates;      /* initial device candidate capacity (0 = 1<<20) */
    int32_t seg_len;             /* overlap-save segment length L, 512..4096 (0 = automatic) */
    int32_t profile;             /* nonzero: time every phase with HIP events (fdas_profile_read) */
    int32_t harm_order;          /* harmonic-sum tile order: 0 automatic, 1 each XCD sweeps its own
                                    series, 2 all XCDs sweep one series at a time, 3 as 2 in two
                                    drift halves (results never depend on it) */
    int32_t harm_bound;          /* 0: harmonic sums skip drift blocks whose block-maximum bound
                                    rules out a candidate (exact; default), 1: sum every cell */
    int32_t harm_block;          /* drift rows per bound block (0 = automatic) */
    int32_t harm_pair;           /* 0: automatic (per bin up to 8 harmonics, per column above);
                                    1: block maxima per column (tighter bound, twice the memory);
                                    2: per bin, covering both half-bin columns */
    int32_t autotune;            /* 1: on the first search of each shape (nsamp, zmax, numharm),
                                    time candidate seg_len / harm_block / harm_pair on that data
                                    and keep the fastest (results agree to FP32 rounding) */
    int32_t graph;               /* 1: fdas_search and fdas_search_ragged capture their launches
                                    in a hipGraph and replay it when a call with the same input
                                    pointer and shapes repeats (sigma and offsets may change);
                                    ignored while profile is set */
    int32_t fail_alloc;          /* test hook: n > 0 makes the n-th device or pinned-host allocation made
                                    for the plan (counted from fdas_plan_create on) fail as if memory
                                    were exhausted, returning FDAS_E_NOMEM; the plan stays usable
                                    (default 0: off) */
    int32_t reserved[3];         /* must be zero */
} fdas_plan_opts;

/* One candidate. r = r_idx/2 and z = z_idx*dz are the Fourier frequency
 * (bins, mid-observation) and drift (bins) of the harm-th harmonic; the
 * fundamental is r_fund = r_idx/(2 harm), z_fund = z_idx*dz/harm,
 * f_hz = r_fund/T, fdot_hz_s = z_fund/T^2. power = M_H(R) in units of the
 * mean noise power; sigma is its single-trial Gaussian-equivalent significance. */
typedef struct {
    int32_t series;
    int32_t harm;
    int64_t r_idx;
    int32_t z_idx;
    float   power;
    double  sigma;
    double  r_fund;
    double  z_fund;
    double  f_hz;
    double  fdot_hz_s;
} fdas_cand;

/* Fill *opts with the defaults listed above. */
void fdas_plan_opts_default(fdas_plan_opts *opts);

/* Create a plan on the current HIP device for series of up to max_nsamp
 * samples, batches of up to max_series series, drifts up to zmax (a whole
 * multiple of dz) and up to numharm harmonics (1, 2, 4, 8, 16 or 32). The
 * plan owns its device workspace and FP64-built response-template bank.
 * opts may be NULL (defaults). On success *out is a new plan; on failure
 * *out is NULL. Errors: FDAS_E_INVAL, FDAS_E_NOMEM, FDAS_E_DEVICE. */
fdas_status fdas_plan_create(fdas_plan *out, int64_t max_nsamp, int32_t max_series,
                             double zmax, double dz, int32_t numharm,
                             const fdas_plan_opts *opts);

/* Destroy a plan and free its device memory (NULL is ignored). */
void fdas_plan_destroy(fdas_plan p);

/* Search series_dev (device, float32, contiguous [nseries][nsamp]).
 * Writes min(total, cap) candidates to out_host, sorted by (series, harm,
 * r_idx), and the total count to *n_total. Returns FDAS_E_TRUNC if total >
 * cap (the first cap records in that order are written). zmax/dz/numharm may
 * differ from the plan's (the template bank is rebuilt when zmax or dz
 * change) but numharm may not exceed the plan's, nor nsamp/nseries its
 * maxima. Errors: FDAS_E_INVAL when nsamp is odd, nsamp > max_nsamp, the
 * searched band is empty, zmax is not a whole multiple of dz, numharm is not
 * a power of two <= 32, sigma <= 0 or not finite, tsamp <= 0;
 * FDAS_E_UNSUPPORTED when nsamp / 2 is not a product of powers of 2, 3 and 5
 * or exceeds 2^26 (a 2100.224 s file sampled at 250 us, 8400896 samples, is
 * searched as its first 8398080 samples, nsamp / 2 = 2^7 3^8 5, or padded by
 * the caller to 8437500). NaN samples are not
 * checked: they propagate into the powers. The caller keeps ownership of
 * all buffers; the plan keeps no caller pointer after return. */
fdas_status fdas_search(fdas_plan p, const float *series_dev, int64_t nsamp, int32_t nseries,
                        double tsamp, double zmax, double dz, int32_t numharm, double sigma,
                        fdas_cand *out_host, int64_t cap, int64_t *n_total, void *stream);

/* Search a ragged batch: series i (float32, device) starts at series_dev +
 * offsets[i] (an even element offset) and has nsamp[i] samples taken every
 * tsamp[i] seconds, searched to drift zmax[i] (a whole multiple of dz; 0 is
 * allowed). offsets, nsamp, tsamp and zmax are host arrays of nseries
 * entries; dz, numharm and sigma are common. Series of the same (nsamp,
 * search band, zmax) are searched together as one batch. Output and errors as
 * fdas_search (records sorted by (series, harm, r_idx), series = index i);
 * every nsamp[i] must be at most the plan's max_nsamp, nseries at most its
 * max_series, and one series' plane must fit the plan's workspace (always
 * true for zmax[i] up to the plan's zmax). The caller guarantees that every
 * series lies inside its buffer. A truncated result (FDAS_E_TRUNC) holds the
 * first cap records of the complete sorted list. */
fdas_status fdas_search_ragged(fdas_plan p, const float *series_dev, const int64_t *offsets,
                               const int64_t *nsamp, const double *tsamp, const double *zmax,
                               int32_t nseries, double dz, int32_t numharm, double sigma,
                               fdas_cand *out_host, int64_t cap, int64_t *n_total, void *stream);

/* Autotuner results as text, one line per shape:
 * "nsamp zsteps numharm seg_len harm_block harm_pair". fdas_tuning_export
 * writes at most cap bytes (including the terminating NUL) and sets *len to
 * the full length; fdas_tuning_import adds lines in the same format (a
 * tuning file kept by the caller), replacing entries of the same shape. */
fdas_status fdas_tuning_export(fdas_plan p, char *buf, int64_t cap, int64_t *len);
fdas_status fdas_tuning_import(fdas_plan p, const char *text);

/* ------------------------------------------------------------------ sifting
 *
 * Sifting of a candidate list (the paper's Section 2, step 5), on each
 * candidate's fundamental frequency f_hz and significance sigma:
 *   order: sigma descending, then series, harm, r_idx ascending;
 *   duplicates: walking that order, a candidate within tol_bins / min(T_a, T_b)
 *     Hz of an already kept candidate joins the first such kept candidate,
 *     otherwise it is kept (T = r_fund / f_hz, the observation length);
 *   harmonics: walking the kept candidates in order, B is dropped when a
 *     stronger surviving A has |f_B - rho f_A| <= rho tol_bins / min(T_A, T_B)
 *     for rho = n or 1/n, 2 <= n <= max_ratio.
 * Host only; any mix of series (e.g. all trial DMs of one observation).
 */
typedef struct {
    int64_t index;       /* surviving candidate: its position in the input list */
    int32_t hits;        /* candidates it stands for (itself and its duplicates) */
    int32_t series_lo;   /* smallest and largest series index among them */
    int32_t series_hi;
    int32_t reserved;
} fdas_sifted;

/* Survivors in sifted order into out (cap entries; *n_out = their number,
 * FDAS_E_TRUNC when cap is smaller). Every candidate needs f_hz > 0, r_fund > 0
 * and a finite sigma (FDAS_E_INVAL otherwise). */
fdas_status fdas_sift(const fdas_cand *cands, int64_t n, double tol_bins, int32_t max_ratio,
                      fdas_sifted *out, int64_t cap, int64_t *n_out);

/* ------------------------------------------------------------------ dedispersion
 *
 * Incoherent dedispersion of 8-bit filterbank data into time series at trial
 * DMs (the paper's Section 2, step 2, with DM plans like its Tables 2-3). For
 * a range with downsampling factor D and trial DM d:
 *   y_c[j] = sum_{s<D} x[j D + s][c],  j < nsamp / D,
 *   delta_c = floor(4.148808e3 d (f_c^-2 - f_hi^-2) / (D tsamp) + 1/2)   (FP64),
 *   out[j] = sum_c y_c[j + delta_c],   y_c read as p_c past its end,
 *   p_c = floor((D sum_t x[t][c] + nsamp/2) / nsamp)  (rounded boxcar mean),
 * with f_c = f0 + c df (MHz) and f_hi the highest channel frequency. All sums
 * are integers below 2^24 (nchan D 255 < 2^24 is required), exact in float32.
 */
typedef struct {
    double  dm_start;   /* pc cm^-3, >= 0 */
    double  dm_step;    /* >= 0 */
    int32_t ndm;        /* trial DMs dm_start + i dm_step, i < ndm */
    int32_t downsamp;   /* D >= 1, dividing nsamp */
} fdas_dm_range;

/* Dedisperse fil_dev (device uint8 [nsamp][nchan], time-major as filterbank
 * files store it) for every range. out_dev (device float32) receives, range
 * after range, [ndm][nsamp / D] series, so that it is directly a packed batch
 * for fdas_search_ragged (series i of range r at offset
 * sum_{r' < r} ndm_r' nsamp / D_r' + i nsamp / D_r, sampled every D_r tsamp).
 * out_elems: capacity of out_dev in floats. Uses the plan's stream handling
 * and workspace (grown as needed); the plan's series limits do not apply. */
fdas_status fdas_dedisperse(fdas_plan p, const uint8_t *fil_dev, int64_t nsamp, int32_t nchan, double tsamp,
                            double f0_mhz, double df_mhz, const fdas_dm_range *ranges, int32_t nranges,
                            float *out_dev, int64_t out_elems, void *stream);

/* ------------------------------------------------------------------ refinement
 *
 * Refinement maximises the correlation power of a candidate over continuous
 * (r, z) near its grid cell (the search of the paper's Section 2, steps 4-5,
 * reports grid cells only). For a point with window (k0, m) on the normalised
 * spectrum a_k (a_k = 0 outside bins 1..nbins-1):
 *   c(r, z) = sum_{k=k0-m}^{k0+m} a_k conj rho(r - k, z),   P = |c|^2,
 *   rho(q, z) = int_0^1 exp(2 pi i [q u + z (u^2 - u)/2]) du,
 * the window staying fixed while (r, z) move, so that P is smooth in (r, z).
 */
typedef struct {
    int32_t series;   /* spectrum row */
    int32_t m;        /* window half-width, 0 <= m <= max_m <= 2000 */
    int64_t k0;       /* window centre bin; |r - k0| <= 64 */
    double  r;        /* Fourier frequency in bins (mid-observation) */
    double  z;        /* drift in bins over the observation, |z| <= 8192 */
} fdas_refine_point;

/* P, dP/dr and dP/dz of n points (all device arrays). spec_dev: complex64
 * [nseries][spitch] (interleaved re, im) spectra; scale_dev (may be NULL):
 * float [nseries], a_k = scale[series] * spec[series][k]. power_dev receives P,
 * dpdr_dev / dpdz_dev (may be NULL) the derivatives. Points whose fields are
 * out of range (series, m > max_m, |r - k0|, |z|) receive NaN. */
fdas_status fdas_refine_eval(const float *spec_dev, int64_t spitch, int64_t nbins, int32_t nseries,
                             const float *scale_dev, const fdas_refine_point *pts_dev, int64_t n,
                             int32_t max_m, float *power_dev, float *dpdr_dev, float *dpdz_dev,
                             void *stream);

/* Backward of fdas_refine_eval for upstream gradients grad_power_dev [n]:
 * grad_r = g dP/dr, grad_z = g dP/dz (each may be NULL) and, if grad_spec_dev
 * is not NULL, adds g dP/dRe(spec_k) + i g dP/dIm(spec_k) = 2 g s c rho(r - k, z)
 * to grad_spec_dev (complex64 [nseries][spitch], same layout as spec_dev) for
 * every window bin in 1..nbins-1 (atomically: points may share bins). */
fdas_status fdas_refine_grad(const float *spec_dev, int64_t spitch, int64_t nbins, int32_t nseries,
                             const float *scale_dev, const fdas_refine_point *pts_dev, int64_t n,
                             int32_t max_m, const float *grad_power_dev, float *grad_r_dev,
                             float *grad_z_dev, float *grad_spec_dev, void *stream);

/* Refine n candidates of a batch of series: the plan computes the normalised
 * spectra of series_dev (device float32 [nseries][nsamp]) as fdas_search does,
 * then runs, per point, iters steps of
 *   (r, z) += (3/(2 pi^2) dP/dr, 90/pi^2 dP/dz) / P
 * (the Newton step at a peak of |rho|^2, whose curvatures in r and z are
 * -2 pi^2/3 and -pi^2/90 per unit power), clamped to |r - r0| <= 1 and
 * |z - z0| <= 2 dz around the start (r0, z0). pts_host (host, n entries): on
 * input series, r and z of each start; k0 = nearest bin to r0 and
 * m = ceil((|z0| + 2 dz)/2) + K + 1 are set by the call; on output r and z hold
 * the refined point. power_host (host, n floats) receives P there. */
fdas_status fdas_refine(fdas_plan p, const float *series_dev, int64_t nsamp, int32_t nseries, double dz,
                        int32_t iters, fdas_refine_point *pts_host, float *power_host, int64_t n,
                        void *stream);

/* The window fdas_refine uses for a start (r0, z0): k0 = floor(r0 + 1/2),
 * m = ceil((|z0| + 2 dz)/2) + K + 1 (host, no device work). */
fdas_status fdas_refine_window(double r0, double z0, double dz, int32_t K, int64_t *k0, int32_t *m);

/* The normalised power plane of each series: plane_dev (device, float32)
 * receives [nseries][NZ][NR] with NZ = 2 zmax/dz + 1 rows (z = (row - zmax/dz)
 * dz) and NR = nsamp - 2 rlo columns (column c holds R = c + 2 rlo).
 * plane_elems is the buffer size in floats and must be at least
 * nseries*NZ*NR. Same argument rules as fdas_search. */
fdas_status fdas_plane(fdas_plan p, const float *series_dev, int64_t nsamp, int32_t nseries,
                       double tsamp, double zmax, double dz, float *plane_dev,
                       int64_t plane_elems, void *stream);

/* Harmonic sums, thresholding and candidates of a caller-supplied plane in
 * the layout fdas_plane writes (device, float32 [nseries][NZ][NR]). Output
 * as fdas_search. Lets callers search planes they built themselves. */
fdas_status fdas_harmsum(fdas_plan p, const float *plane_dev, int64_t nsamp, int32_t nseries,
                         double tsamp, double zmax, double dz, int32_t numharm, double sigma,
                         fdas_cand *out_host, int64_t cap, int64_t *n_total, void *stream);

/* Un-normalised spectra A_k, k = 0..nsamp/2, as interleaved (re, im) float32
 * pairs [nseries][nsamp/2+1][2] into spec_dev (device), and, if norm_host is
 * not NULL, the normalisation of each series (float64 [nseries], host). */
fdas_status fdas_spectrum(fdas_plan p, const float *series_dev, int64_t nsamp, int32_t nseries,
                          float *spec_dev, double *norm_host, void *stream);

/* Search geometry for a series: lowest bin rlo, plane columns NR and rows NZ. */
fdas_status fdas_geometry(int64_t nsamp, double tsamp, double zmax, double dz,
                          const fdas_plan_opts *opts, int64_t *rlo, int64_t *nr, int32_t *nz);

/* Host FP64 helpers (no device work). fdas_threshold: T_H for H = harm.
 * fdas_sigma: Gaussian-equivalent significance of a sum of harm powers. */
double fdas_threshold(int32_t harm, double sigma);
double fdas_sigma(int32_t harm, double power);

/* Host FP64 unit-energy template taps of a trial at r = k0 + parity/2, drift
 * z: t_d = conj rho(parity/2 - d, z) / sqrt(E) for d = d0 .. d0 + ntaps - 1
 * (d0 = -m + parity, m = ceil(|z|/2) + K). re/im hold cap doubles each.
 * Returns FDAS_E_INVAL if cap is too small (*ntaps still set). */
fdas_status fdas_template_taps(double z, int32_t parity, int32_t K, double *re, double *im,
                               int32_t cap, int32_t *ntaps, int32_t *d0);

/* What a plan chose for its current template bank: overlap-save segment
 * length and the largest template half-width (the z rows are split into
 * groups, each segmenting the spectrum by its own widest template: a group
 * yields seg_len - 2 m valid bins per segment, m <= mseg), z rows, series per
 * plane chunk, the plane workspace in bytes, and,
 * for the last search, the number of drift blocks of the bounded harmonic
 * sums (0 if they were not used) and whether their maxima cover bin pairs. */
typedef struct {
    int32_t seg_len;
    int32_t mseg;
    int32_t nz;
    int32_t chunk_series;
    int64_t workspace_bytes;
    int32_t harm_blocks;
    int32_t harm_pair;
} fdas_plan_info;
fdas_status fdas_plan_get_info(fdas_plan p, fdas_plan_info *out);

/* Phase timing of a plan created with opts.profile != 0. HIP events are
 * recorded on the search stream around every kernel phase; ms[i] receives
 * the summed device milliseconds and launches[i] the number of timed
 * launches of phase i since the last reset (both arrays hold FDAS_NPHASES
 * entries, either may be NULL). Phases: 0 real FFT, 1 normalisation,
 * 2 power plane, 3 harmonic sums (with the maximising drift), 4 compaction,
 * 5 FP64 significance of the records, 6 copy-out,
 * 7 refinement, 8 dedispersion.
 * reset != 0 clears the totals after reading. */
#define FDAS_NPHASES 9
fdas_status fdas_profile_read(fdas_plan p, double *ms, int64_t *launches, int32_t reset);

/* ------------------------------------------------------------------ no allocation
 *
 * For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc. fdas_spectrum_noalloc
 * computes what fdas_spectrum returns on a plan with the default (median)
 * normalisation, without a plan: the un-normalised spectra A_k, k = 0..nsamp/2,
 * as interleaved (re, im) float32 pairs [nseries][nsamp/2+1][2] into spec_dev
 * (device, caller-owned), and, if norm_host is not NULL, each series' median
 * normalisation (float64 [nseries], host). It calls no allocating routine: its
 * FFT buffers, scales and median histograms live in a fixed device array of
 * FDAS_NOALLOC_SCRATCH_BYTES per GPU, kept until the process ends, so
 * nseries (nsamp/2) 8 bytes plus about 8 KiB per series must fit in it
 * (e.g. 12 series of 2^20 samples); larger requests return FDAS_E_INVAL.
 * Calls on one GPU share that array: calls that overlap on one GPU (other
 * streams or host threads) race; consecutive calls are independent.
 * Errors: FDAS_E_INVAL (NULL or misaligned pointer, odd nsamp or below 8,
 * nseries outside 1..65535, too large), FDAS_E_UNSUPPORTED (nsamp / 2 not a
 * product of powers of 2, 3 and 5), FDAS_E_DEVICE (a HIP call failed). */
#define FDAS_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
fdas_status fdas_spectrum_noalloc(const float *series_dev, int64_t nsamp, int32_t nseries,
                                  float *spec_dev, double *norm_host, void *stream);

/* Description of a status code (static storage). */
const char *fdas_status_string(fdas_status s);

/* Detail of the last failure on this plan ("" if none; static if p is NULL). */
const char *fdas_last_error(fdas_plan p);

#ifdef __cplusplus
}
#endif
#endif /* FDAS_H */
