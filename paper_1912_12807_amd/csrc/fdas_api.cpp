// C ABI and host runtime: plans, the FP64-built template bank, workspace
// management and the order in which the search kernels are enqueued.
//
// One search enqueues, on the caller's stream:
//   K1 real FFT of every series -> K2 median normalisation (or a fixed scale)
//   then per chunk of series (sized to the plane workspace):
//   K4 power plane -> K5 harmonic-sum maxima -> K6 ordered compaction -> argmax
// and finally copies the record count and the records to pinned host memory,
// where the FP64 significance and physical units are attached (the candidate
// list of the paper's Section 2, step 5).
#include "fdas_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

using namespace fdas;

namespace {

constexpr int64_t kDefaultCands = 1 << 20;

struct Geometry {
    int64_t nsamp = 0, half = 0, rlo = 0, NR = 0;
    int Z = 0, NZ = 0;
    double T = 0;
};

fdas_status geometry(int64_t nsamp, double tsamp, double zmax, double dz, double flo, Geometry &g) {
    if (nsamp < 8 || (nsamp & 1) || !(tsamp > 0) || !std::isfinite(tsamp) || !(dz > 0) ||
        !std::isfinite(dz) || !(zmax >= 0) || !std::isfinite(zmax) || !(flo >= 0) ||
        !std::isfinite(flo))
        return FDAS_E_INVAL;
    const double q = zmax / dz;
    const double Zr = std::round(q);
    if (std::fabs(q - Zr) > 1e-9 * std::max(1.0, std::fabs(q)) || Zr > 100000) return FDAS_E_INVAL;
    g.nsamp = nsamp;
    g.half = nsamp / 2;
    g.T = (double)nsamp * tsamp;
    g.rlo = std::max<int64_t>(1, (int64_t)std::ceil(flo * g.T));
    if (g.rlo >= g.half) return FDAS_E_INVAL;          // empty search band
    g.NR = nsamp - 2 * g.rlo;
    g.Z = (int)Zr;
    g.NZ = 2 * g.Z + 1;
    return FDAS_OK;
}

bool pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }
int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
int nstages_of(int numharm) {
    int s = 0;
    while ((1 << s) < numharm) ++s;
    return s + 1;
}
bool valid_numharm(int h) { return h == 1 || h == 2 || h == 4 || h == 8 || h == 16 || h == 32; }

}  // namespace

struct fdas_plan_s {
    int device = -1;
    int64_t max_nsamp = 0;
    int32_t max_series = 0;
    int32_t max_numharm = 1;
    fdas_plan_opts opts{};
    std::string last_error;
    bool sticky = false;

    // template bank
    double bank_zmax = -1, bank_dz = -1;
    int L = 0, mseg = 0, bankNZ = 0;
    float2 *d_bank = nullptr;
    size_t bank_bytes = 0;

    // workspace
    int64_t spitch = 0;
    float2 *d_spec = nullptr, *d_w0 = nullptr, *d_w1 = nullptr;
    float *d_scale = nullptr;
    double *d_norm = nullptr;
    float *d_thr = nullptr;
    int64_t *d_state = nullptr;
    float *d_plane = nullptr;
    int64_t plane_cap = 0;      // floats
    int chunk_series = 0;
    float *d_maxv = nullptr;
    int64_t maxv_cap = 0;       // floats
    int32_t *d_counts = nullptr;
    int64_t *d_offsets = nullptr;
    int64_t nblk_cap = 0;
    DevCand *d_rec = nullptr;
    int64_t rec_cap = 0;
    // drift-row block maxima for the bounded harmonic sums
    float *d_pyr = nullptr;
    int64_t pyr_cap = 0;        // floats
    int32_t *d_rb = nullptr;    // lo[nblk + 1] followed by of_row[NZ]
    int64_t rb_cap = 0;
    int rb_NZ = -1, rb_G = -1, rb_bz = -1, rb_nh = -1, rb_nblk = 0;
    int last_harm_blocks = 0, last_harm_pair = 0;   // what the last search's K5 used
    // pinned host staging
    int64_t *h_state = nullptr;
    float *h_small = nullptr;   // thresholds / fixed scales
    DevCand *h_rec = nullptr;
    int64_t h_rec_cap = 0;
    float *h_scale = nullptr;

    // phase timing (opts.profile)
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> ev_pending;
    double prof_ms[FDAS_NPHASES] = {0};
    int64_t prof_n[FDAS_NPHASES] = {0};

    hipEvent_t take_event() {
        if (!ev_pool.empty()) {
            hipEvent_t e = ev_pool.back();
            ev_pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return e;
    }
    hipEvent_t begin(hipStream_t st) {
        if (!opts.profile) return nullptr;
        hipEvent_t e = take_event();
        if (e) (void)hipEventRecord(e, st);
        return e;
    }
    void end(int phase, hipEvent_t a, hipStream_t st) {
        if (!a) return;
        hipEvent_t b = take_event();
        if (!b) return;
        (void)hipEventRecord(b, st);
        ev_pending.emplace_back(phase, a, b);
    }
    // after the stream has been synchronised
    void collect() {
        for (auto &t : ev_pending) {
            float ms = 0.f;
            if (hipEventElapsedTime(&ms, std::get<1>(t), std::get<2>(t)) == hipSuccess) {
                prof_ms[std::get<0>(t)] += ms;
                prof_n[std::get<0>(t)] += 1;
            } else {
                (void)hipGetLastError();
            }
            ev_pool.push_back(std::get<1>(t));
            ev_pool.push_back(std::get<2>(t));
        }
        ev_pending.clear();
    }

    fdas_status fail(fdas_status s, const std::string &msg) {
        last_error = msg;
        if (s == FDAS_E_DEVICE) sticky = true;
        return s;
    }
    fdas_status hip(hipError_t e, const char *what) {
        if (e == hipSuccess) return FDAS_OK;
        char buf[512];
        std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
        return fail(e == hipErrorOutOfMemory ? FDAS_E_NOMEM : FDAS_E_DEVICE, buf);
    }
};

#define TRY(expr)                                        \
    do {                                                 \
        fdas_status _s = (expr);                         \
        if (_s != FDAS_OK) return _s;                    \
    } while (0)
#define HIPTRY(p, expr) TRY((p)->hip((expr), #expr))

namespace {

template <typename T>
fdas_status dalloc(fdas_plan p, T **ptr, int64_t count, const char *what) {
    if (*ptr) {
        (void)hipFree(*ptr);
        *ptr = nullptr;
    }
    if (count <= 0) count = 1;
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, (size_t)count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return p->fail(FDAS_E_NOMEM, std::string("device allocation failed: ") + what);
    }
    *ptr = static_cast<T *>(q);
    return FDAS_OK;
}

template <typename T>
fdas_status halloc(fdas_plan p, T **ptr, int64_t count, const char *what) {
    if (*ptr) {
        (void)hipHostFree(*ptr);
        *ptr = nullptr;
    }
    if (count <= 0) count = 1;
    void *q = nullptr;
    hipError_t e = hipHostMalloc(&q, (size_t)count * sizeof(T), hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return p->fail(FDAS_E_NOMEM, std::string("pinned host allocation failed: ") + what);
    }
    *ptr = static_cast<T *>(q);
    return FDAS_OK;
}

int choose_L(int mseg, int requested) {
    if (requested) return (pow2(requested) && requested >= 512 && requested <= 4096 &&
                           requested - 2 * mseg >= 64) ? requested : 0;
    for (int L = 512; L <= 4096; L *= 2)
        if (L >= 16 * mseg) return L;
    return (4096 - 2 * mseg >= 1024) ? 4096 : 0;
}

// Build (or keep) the bank for (zmax, dz): [NZ][2][L] kernel spectra, FP64 -> float32.
fdas_status ensure_bank(fdas_plan p, double zmax, double dz) {
    if (p->d_bank && p->bank_zmax == zmax && p->bank_dz == dz) return FDAS_OK;
    const int Z = (int)std::round(zmax / dz);
    const int NZ = 2 * Z + 1;
    const int K = p->opts.K;
    const int mseg = half_width(Z * dz, K);
    const int L = choose_L(mseg, p->opts.seg_len);
    if (!L) return p->fail(FDAS_E_UNSUPPORTED, "zmax too large for the supported segment lengths");
    std::vector<float> host((size_t)NZ * 2 * L * 2);
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned w = 0; w < nth; ++w) {
        pool.emplace_back([&, w]() {
            for (int row = (int)w; row < 2 * NZ; row += (int)nth) {
                const int zi = row / 2, par = row % 2;
                kernel_spectrum((zi - Z) * dz, par, K, L, mseg, host.data() + (size_t)row * L * 2);
            }
        });
    }
    for (auto &t : pool) t.join();
    const size_t bytes = host.size() * sizeof(float);
    if (bytes > p->bank_bytes) {
        TRY(dalloc(p, &p->d_bank, (int64_t)(host.size() / 2), "template bank"));
        p->bank_bytes = bytes;
    }
    HIPTRY(p, hipMemcpy(p->d_bank, host.data(), bytes, hipMemcpyHostToDevice));
    p->bank_zmax = zmax;
    p->bank_dz = dz;
    p->L = L;
    p->mseg = mseg;
    p->bankNZ = NZ;
    return FDAS_OK;
}

fdas_status check_common(fdas_plan p, const void *dev, int64_t nsamp, int32_t nseries,
                         double tsamp, double zmax, double dz, Geometry &g) {
    if (!p) return FDAS_E_INVAL;
    if (p->sticky) return p->fail(FDAS_E_DEVICE, "plan is in a failed state: " + p->last_error);
    if (!dev || ((uintptr_t)dev & 7)) return p->fail(FDAS_E_INVAL, "device pointer NULL or not 8-byte aligned");
    if (nseries < 1 || nseries > p->max_series) return p->fail(FDAS_E_INVAL, "nseries out of range");
    if (nsamp > p->max_nsamp) return p->fail(FDAS_E_INVAL, "nsamp exceeds the plan's max_nsamp");
    fdas_status s = geometry(nsamp, tsamp, zmax, dz, p->opts.flo_hz, g);
    if (s != FDAS_OK) return p->fail(s, "invalid nsamp/tsamp/zmax/dz (odd nsamp, zmax not a multiple of dz, or empty band)");
    if (!pow2(nsamp)) return p->fail(FDAS_E_UNSUPPORTED, "nsamp must be a power of two");
    int dev_now = -1;
    if (hipGetDevice(&dev_now) != hipSuccess || dev_now != p->device)
        return p->fail(FDAS_E_INVAL, "current HIP device differs from the plan's device");
    return FDAS_OK;
}

// K1 + K2 for the batch; leaves spectra in d_spec and scales in d_scale.
fdas_status run_spectrum(fdas_plan p, const float *x, const Geometry &g, int nseries, hipStream_t st) {
    hipEvent_t e = p->begin(st);
    HIPTRY(p, launch_rfft(x, g.nsamp, nseries, p->d_w0, p->d_w1, p->d_spec, p->spitch, st));
    p->end(0, e, st);
    if (p->opts.norm == FDAS_NORM_MEDIAN) {
        e = p->begin(st);
        HIPTRY(p, launch_median_scale(p->d_spec, p->spitch, g.half, nseries, p->d_scale, p->d_norm, st));
        p->end(1, e, st);
    } else {
        const double nrm = (double)g.nsamp * p->opts.fixed_var;
        for (int b = 0; b < nseries; ++b) p->h_scale[b] = (float)std::sqrt(1.0 / nrm);
        HIPTRY(p, hipMemcpyAsync(p->d_scale, p->h_scale, nseries * sizeof(float), hipMemcpyHostToDevice, st));
    }
    return FDAS_OK;
}

CorrGeom corr_geom(fdas_plan p, const Geometry &g) {
    CorrGeom c;
    c.L = p->L;
    c.mseg = p->mseg;
    c.Lv = p->L - 2 * p->mseg;
    c.half = g.half;
    c.rlo = g.rlo;
    c.nseg = (int)((g.half - g.rlo + c.Lv - 1) / c.Lv);
    c.NZ = g.NZ;
    int G = 1;
    while (G < 8 && g.NZ >= 2 * G * 12) G *= 2;
    c.zgroups = G;
    return c;
}

int block_rows(fdas_plan p, int numharm) {
    if (p->opts.harm_block) return p->opts.harm_block;
    return numharm <= 8 ? 10 : numharm == 16 ? 8 : 6;
}

// Row-block tables for the bounded harmonic sums (cached per geometry):
// lo[nblk + 1], of_row[NZ], frange[nblk][numharm] in one device buffer.
fdas_status ensure_row_blocks(fdas_plan p, int NZ, int G, int bz, int numharm, RowBlocks &rb) {
    if (!(p->d_rb && p->rb_NZ == NZ && p->rb_G == G && p->rb_bz == bz && p->rb_nh == numharm)) {
        std::vector<int32_t> lo, of_row, fr;
        row_blocks(NZ, G, bz, lo, of_row);
        fraction_ranges(NZ, numharm, lo, of_row, fr);
        std::vector<int32_t> all(lo);
        all.insert(all.end(), of_row.begin(), of_row.end());
        all.insert(all.end(), fr.begin(), fr.end());
        const int64_t n = (int64_t)all.size();
        if (n > p->rb_cap) {
            TRY(dalloc(p, &p->d_rb, n, "row-block tables"));
            p->rb_cap = n;
        }
        HIPTRY(p, hipMemcpy(p->d_rb, all.data(), n * sizeof(int32_t), hipMemcpyHostToDevice));
        p->rb_NZ = NZ;
        p->rb_G = G;
        p->rb_bz = bz;
        p->rb_nh = numharm;
        p->rb_nblk = (int)lo.size() - 1;
    }
    rb.lo = p->d_rb;
    rb.of_row = p->d_rb + p->rb_nblk + 1;
    rb.frange = rb.of_row + NZ;
    rb.nblk = p->rb_nblk;
    rb.frange_nh = numharm;
    rb.pair = p->opts.harm_pair == 0;   // default: maxima per bin (pair); 1 selects per column
    return FDAS_OK;
}

// K5 + K6 + argmax for one chunk of planes.
fdas_status run_harm_chunk(fdas_plan p, const float *plane, int64_t pitch, int64_t sstride,
                           const Geometry &g, int numharm, int b0, int nb, hipStream_t st,
                           const float *pyr = nullptr, int64_t psstride = 0,
                           const RowBlocks *rb = nullptr) {
    const int NS = nstages_of(numharm);
    const int64_t mpitch = round_up(g.NR, 16);
    hipEvent_t e = p->begin(st);
    if (pyr) {
        HIPTRY(p, launch_harmsum_bounded(plane, pitch, sstride, pyr, psstride, *rb, g.NR, g.rlo, g.Z,
                                         numharm, nb, p->d_thr, p->d_maxv, mpitch, st));
    } else {
        const int order = p->opts.harm_order ? p->opts.harm_order : 1;
        HIPTRY(p, launch_harmsum(plane, pitch, sstride, g.NR, g.rlo, g.Z, numharm, nb, p->d_maxv, mpitch,
                                 order, st));
    }
    p->end(3, e, st);
    const int64_t nelem = (int64_t)nb * NS * mpitch;
    e = p->begin(st);
    HIPTRY(p, launch_compact(p->d_maxv, nelem, mpitch, NS, b0, p->d_thr, p->d_counts, p->d_offsets,
                             p->d_state, p->d_rec, p->rec_cap, st));
    p->end(4, e, st);
    e = p->begin(st);
    HIPTRY(p, launch_argmax(plane, pitch, sstride, g.rlo, g.Z, numharm, b0, p->d_rec, p->d_state,
                            p->rec_cap, st));
    p->end(5, e, st);
    return FDAS_OK;
}

fdas_status prepare_harm(fdas_plan p, const Geometry &g, int numharm, double sigma, hipStream_t st) {
    const int NS = nstages_of(numharm);
    for (int s = 0; s < NS; ++s) p->h_small[s] = (float)threshold(1 << s, sigma);
    HIPTRY(p, hipMemcpyAsync(p->d_thr, p->h_small, NS * sizeof(float), hipMemcpyHostToDevice, st));
    HIPTRY(p, hipMemsetAsync(p->d_state, 0, 2 * sizeof(int64_t), st));
    (void)g;
    return FDAS_OK;
}

fdas_status finish(fdas_plan p, const Geometry &g, int numharm, double dz, fdas_cand *out, int64_t cap,
                   int64_t *n_total, hipStream_t st, bool *need_regrow) {
    hipEvent_t e = p->begin(st);
    HIPTRY(p, hipMemcpyAsync(p->h_state, p->d_state, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    p->end(6, e, st);
    HIPTRY(p, hipStreamSynchronize(st));
    const int64_t total = p->h_state[0];
    *need_regrow = false;
    if (total > p->rec_cap && cap > p->rec_cap) {
        *need_regrow = true;
        return FDAS_OK;
    }
    const int64_t n = std::min<int64_t>(std::min<int64_t>(total, cap), p->rec_cap);
    if (n > 0) {
        if (n > p->h_rec_cap) {
            TRY(halloc(p, &p->h_rec, n, "candidate staging"));
            p->h_rec_cap = n;
        }
        e = p->begin(st);
        HIPTRY(p, hipMemcpyAsync(p->h_rec, p->d_rec, n * sizeof(DevCand), hipMemcpyDeviceToHost, st));
        p->end(6, e, st);
        HIPTRY(p, hipStreamSynchronize(st));
    }
    p->collect();
    for (int64_t i = 0; i < n; ++i) {
        const DevCand &d = p->h_rec[i];
        if (d.zq < -g.Z || d.zq > g.Z)
            return p->fail(FDAS_E_DEVICE, "internal error: candidate without a maximising drift");
        const int H = 1 << d.s;
        fdas_cand &c = out[i];
        c.series = d.b;
        c.harm = H;
        c.r_idx = (int64_t)d.c + 2 * g.rlo;
        c.z_idx = d.zq;
        c.power = d.power;
        c.sigma = sigma_of(H, (double)d.power);
        c.r_fund = (double)c.r_idx / (2.0 * H);
        c.z_fund = (double)d.zq * dz / H;
        c.f_hz = c.r_fund / g.T;
        c.fdot_hz_s = c.z_fund / (g.T * g.T);
    }
    *n_total = total;
    (void)numharm;
    return total > cap ? FDAS_E_TRUNC : FDAS_OK;
}

fdas_status grow_records(fdas_plan p, int64_t n) {
    TRY(dalloc(p, &p->d_rec, n, "candidate records"));
    p->rec_cap = n;
    return FDAS_OK;
}

}  // namespace

extern "C" {

void fdas_plan_opts_default(fdas_plan_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->flo_hz = 1.0;
    o->K = 16;
    o->norm = FDAS_NORM_MEDIAN;
    o->fixed_var = 1.0;
    o->max_workspace_bytes = 0;
    o->max_candidates = 0;
    o->seg_len = 0;
}

const char *fdas_status_string(fdas_status s) {
    switch (s) {
    case FDAS_OK: return "ok";
    case FDAS_E_INVAL: return "invalid argument";
    case FDAS_E_NOMEM: return "out of memory";
    case FDAS_E_DEVICE: return "device error";
    case FDAS_E_TRUNC: return "candidate list truncated";
    case FDAS_E_UNSUPPORTED: return "unsupported configuration";
    }
    return "unknown status";
}

const char *fdas_last_error(fdas_plan p) {
    if (!p) return "";
    return p->last_error.c_str();
}

fdas_status fdas_geometry(int64_t nsamp, double tsamp, double zmax, double dz,
                          const fdas_plan_opts *opts, int64_t *rlo, int64_t *nr, int32_t *nz) {
    fdas_plan_opts o;
    fdas_plan_opts_default(&o);
    if (opts) o = *opts;
    Geometry g;
    fdas_status s = geometry(nsamp, tsamp, zmax, dz, o.flo_hz, g);
    if (s != FDAS_OK) return s;
    if (rlo) *rlo = g.rlo;
    if (nr) *nr = g.NR;
    if (nz) *nz = g.NZ;
    return FDAS_OK;
}

void fdas_plan_destroy(fdas_plan p) {
    if (!p) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    if (p->device >= 0) (void)hipSetDevice(p->device);
    void *dev[] = {p->d_bank, p->d_spec, p->d_w0, p->d_w1, p->d_scale, p->d_norm, p->d_thr,
                   p->d_state, p->d_plane, p->d_maxv, p->d_counts, p->d_offsets, p->d_rec,
                   p->d_pyr, p->d_rb};
    for (void *q : dev)
        if (q) (void)hipFree(q);
    for (auto &t : p->ev_pending) {
        p->ev_pool.push_back(std::get<1>(t));
        p->ev_pool.push_back(std::get<2>(t));
    }
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    void *host[] = {p->h_state, p->h_small, p->h_rec, p->h_scale};
    for (void *q : host)
        if (q) (void)hipHostFree(q);
    if (cur >= 0) (void)hipSetDevice(cur);
    delete p;
}

fdas_status fdas_plan_create(fdas_plan *out, int64_t max_nsamp, int32_t max_series, double zmax,
                             double dz, int32_t numharm, const fdas_plan_opts *opts) {
    if (!out) return FDAS_E_INVAL;
    *out = nullptr;
    fdas_plan_opts o;
    fdas_plan_opts_default(&o);
    if (opts) o = *opts;
    for (int i = 0; i < 2; ++i)
        if (o.reserved[i]) return FDAS_E_INVAL;
    if (max_series < 1 || max_series > 65535 || !valid_numharm(numharm) || o.K < 1 || o.K > 1024 ||
        (o.norm != FDAS_NORM_MEDIAN && o.norm != FDAS_NORM_FIXED) ||
        (o.norm == FDAS_NORM_FIXED && !(o.fixed_var > 0)) || o.max_workspace_bytes < 0 ||
        o.max_candidates < 0 || o.harm_order < 0 || o.harm_order > 3 || o.harm_bound < 0 ||
        o.harm_bound > 1 || o.harm_block < 0 || o.harm_block > 64 || o.harm_pair < 0 ||
        o.harm_pair > 1)
        return FDAS_E_INVAL;
    Geometry g;
    if (geometry(max_nsamp, 1e-3, zmax, dz, 0.0, g) != FDAS_OK) return FDAS_E_INVAL;
    if (!pow2(max_nsamp)) return FDAS_E_UNSUPPORTED;
    if (o.seg_len && !choose_L(half_width(g.Z * dz, o.K), o.seg_len)) return FDAS_E_INVAL;

    fdas_plan p = new (std::nothrow) fdas_plan_s;
    if (!p) return FDAS_E_NOMEM;
    p->opts = o;
    p->max_nsamp = max_nsamp;
    p->max_series = max_series;
    p->max_numharm = numharm;
    auto bail = [&](fdas_status s) {
        fdas_plan_destroy(p);
        return s;
    };
    if (hipGetDevice(&p->device) != hipSuccess) {
        (void)hipGetLastError();
        return bail(FDAS_E_DEVICE);
    }
    fdas_status s = ensure_bank(p, zmax, dz);
    if (s != FDAS_OK) return bail(s);

    const int64_t half = max_nsamp / 2;
    p->spitch = round_up(half + 1, 2);
    if ((s = dalloc(p, &p->d_spec, (int64_t)max_series * p->spitch, "spectra")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_w0, (int64_t)max_series * half, "fft scratch")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_w1, (int64_t)max_series * half, "fft scratch")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_scale, max_series, "scales")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_norm, max_series, "norms")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_thr, 8, "thresholds")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_state, 2, "state")) != FDAS_OK) return bail(s);

    // plane workspace: as many series per chunk as the budget allows
    const int64_t pitch = round_up(max_nsamp, 64);        // >= NR of any search
    const int64_t per_series = (int64_t)p->bankNZ * pitch;   // floats
    int64_t budget = o.max_workspace_bytes;
    if (!budget) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            fr = (size_t)8 << 30;
        }
        budget = std::min<int64_t>((int64_t)64 << 30, (int64_t)(fr / 2));
    }
    int64_t chunk = std::min<int64_t>(max_series, budget / (per_series * 4));
    if (chunk < 1) return bail(FDAS_E_NOMEM);
    p->chunk_series = (int)chunk;
    p->plane_cap = chunk * per_series;
    if ((s = dalloc(p, &p->d_plane, p->plane_cap, "power plane")) != FDAS_OK) return bail(s);
    {
        // block maxima of every chunk series: at most NZ/bz + 8 blocks per series
        const int bz = block_rows(p, numharm);
        p->pyr_cap = chunk * (int64_t)(p->bankNZ / bz + 9) * (o.harm_pair == 0 ? pitch / 2 : pitch);
        if ((s = dalloc(p, &p->d_pyr, p->pyr_cap, "block maxima")) != FDAS_OK) return bail(s);
    }
    const int NS = nstages_of(numharm);
    p->maxv_cap = chunk * NS * round_up(max_nsamp, 16);
    if ((s = dalloc(p, &p->d_maxv, p->maxv_cap, "stage maxima")) != FDAS_OK) return bail(s);
    p->nblk_cap = compact_blocks(p->maxv_cap);
    if ((s = dalloc(p, &p->d_counts, p->nblk_cap, "compaction counts")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_offsets, p->nblk_cap, "compaction offsets")) != FDAS_OK) return bail(s);
    p->rec_cap = o.max_candidates ? o.max_candidates : kDefaultCands;
    if ((s = dalloc(p, &p->d_rec, p->rec_cap, "candidate records")) != FDAS_OK) return bail(s);
    if ((s = halloc(p, &p->h_state, 2, "state")) != FDAS_OK) return bail(s);
    if ((s = halloc(p, &p->h_small, 8, "thresholds")) != FDAS_OK) return bail(s);
    if ((s = halloc(p, &p->h_scale, max_series, "scales")) != FDAS_OK) return bail(s);
    p->h_rec_cap = 4096;
    if ((s = halloc(p, &p->h_rec, p->h_rec_cap, "candidate staging")) != FDAS_OK) return bail(s);
    *out = p;
    return FDAS_OK;
}

fdas_status fdas_search(fdas_plan p, const float *series_dev, int64_t nsamp, int32_t nseries,
                        double tsamp, double zmax, double dz, int32_t numharm, double sigma,
                        fdas_cand *out_host, int64_t cap, int64_t *n_total, void *stream) {
    Geometry g;
    TRY(check_common(p, series_dev, nsamp, nseries, tsamp, zmax, dz, g));
    if (!valid_numharm(numharm) || numharm > p->max_numharm)
        return p->fail(FDAS_E_INVAL, "numharm must be a power of two up to the plan's numharm");
    if (!(sigma > 0) || !std::isfinite(sigma)) return p->fail(FDAS_E_INVAL, "sigma must be finite and > 0");
    if (cap < 0 || (cap > 0 && !out_host) || !n_total) return p->fail(FDAS_E_INVAL, "bad output buffer");
    TRY(ensure_bank(p, zmax, dz));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const CorrGeom cg = corr_geom(p, g);
    const int64_t pitch = round_up(g.NR, 64);
    const int64_t sstride = (int64_t)g.NZ * pitch;
    if (sstride > p->plane_cap)
        return p->fail(FDAS_E_INVAL, "one series' plane exceeds the workspace; create the plan with this zmax");
    const int chunk = (int)std::min<int64_t>(p->chunk_series, p->plane_cap / sstride);
    // bounded harmonic sums need the block maxima of every chunk series
    // (K4 always writes them, so both harmonic-sum modes read the same plane)
    RowBlocks rb;
    TRY(ensure_row_blocks(p, g.NZ, cg.zgroups, block_rows(p, numharm), numharm, rb));
    const int64_t psstride = (int64_t)rb.nblk * (rb.pair ? pitch / 2 : pitch);
    float *pyr = (psstride * chunk <= p->pyr_cap) ? p->d_pyr : nullptr;
    const float *pyr_k5 = (p->opts.harm_bound || bounded_lds_bytes(rb.nblk, numharm) > kBoundLdsMax)
                              ? nullptr : pyr;
    p->last_harm_blocks = pyr_k5 ? rb.nblk : 0;
    p->last_harm_pair = rb.pair ? 1 : 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        TRY(run_spectrum(p, series_dev, g, nseries, st));
        TRY(prepare_harm(p, g, numharm, sigma, st));
        for (int b0 = 0; b0 < nseries; b0 += chunk) {
            const int nb = std::min(chunk, nseries - b0);
            hipEvent_t e = p->begin(st);
            HIPTRY(p, launch_corr_power(p->d_spec + (int64_t)b0 * p->spitch, p->spitch, p->d_scale + b0,
                                        p->d_bank, cg, nb, p->d_plane, pitch, sstride, pyr, psstride, rb, st));
            p->end(2, e, st);
            TRY(run_harm_chunk(p, p->d_plane, pitch, sstride, g, numharm, b0, nb, st, pyr_k5, psstride, &rb));
        }
        bool regrow = false;
        fdas_status s = finish(p, g, numharm, dz, out_host, cap, n_total, st, &regrow);
        if (!regrow) return s;
        TRY(grow_records(p, std::min<int64_t>(p->h_state[0], cap)));
    }
    return p->fail(FDAS_E_DEVICE, "internal error: candidate capacity did not converge");
}

fdas_status fdas_plane(fdas_plan p, const float *series_dev, int64_t nsamp, int32_t nseries,
                       double tsamp, double zmax, double dz, float *plane_dev, int64_t plane_elems,
                       void *stream) {
    Geometry g;
    TRY(check_common(p, series_dev, nsamp, nseries, tsamp, zmax, dz, g));
    if (!plane_dev || ((uintptr_t)plane_dev & 7) || plane_elems < (int64_t)nseries * g.NZ * g.NR)
        return p->fail(FDAS_E_INVAL, "plane buffer NULL, misaligned or too small");
    TRY(ensure_bank(p, zmax, dz));
    hipStream_t st = static_cast<hipStream_t>(stream);
    TRY(run_spectrum(p, series_dev, g, nseries, st));
    const CorrGeom cg = corr_geom(p, g);
    hipEvent_t e = p->begin(st);
    HIPTRY(p, launch_corr_power(p->d_spec, p->spitch, p->d_scale, p->d_bank, cg, nseries, plane_dev, g.NR,
                                (int64_t)g.NZ * g.NR, nullptr, 0, RowBlocks(), st));
    p->end(2, e, st);
    HIPTRY(p, hipStreamSynchronize(st));
    p->collect();
    return FDAS_OK;
}

fdas_status fdas_harmsum(fdas_plan p, const float *plane_dev, int64_t nsamp, int32_t nseries,
                         double tsamp, double zmax, double dz, int32_t numharm, double sigma,
                         fdas_cand *out_host, int64_t cap, int64_t *n_total, void *stream) {
    Geometry g;
    TRY(check_common(p, plane_dev, nsamp, nseries, tsamp, zmax, dz, g));
    if (!valid_numharm(numharm) || numharm > p->max_numharm)
        return p->fail(FDAS_E_INVAL, "numharm must be a power of two up to the plan's numharm");
    if (!(sigma > 0) || !std::isfinite(sigma)) return p->fail(FDAS_E_INVAL, "sigma must be finite and > 0");
    if (cap < 0 || (cap > 0 && !out_host) || !n_total) return p->fail(FDAS_E_INVAL, "bad output buffer");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t sstride = (int64_t)g.NZ * g.NR;
    const int NS = nstages_of(numharm);
    const int chunk = (int)std::max<int64_t>(1, std::min<int64_t>(p->max_series,
                                                 p->maxv_cap / (NS * round_up(g.NR, 16))));
    // block maxima of the caller's plane for the bounded sums (row blocks as a
    // single z group; results do not depend on the partition)
    RowBlocks rb;
    int64_t psstride = 0;
    int pchunk = chunk;
    if (!p->opts.harm_bound) {
        TRY(ensure_row_blocks(p, g.NZ, 1, block_rows(p, numharm), numharm, rb));
        psstride = (int64_t)rb.nblk * (rb.pair ? g.NR / 2 : g.NR);
        pchunk = (int)std::min<int64_t>(chunk, p->pyr_cap / std::max<int64_t>(1, psstride));
    }
    const bool bounded = !p->opts.harm_bound && pchunk >= 1 &&
                         bounded_lds_bytes(rb.nblk, numharm) <= kBoundLdsMax;
    const int step = bounded ? pchunk : chunk;
    for (int attempt = 0; attempt < 2; ++attempt) {
        TRY(prepare_harm(p, g, numharm, sigma, st));
        for (int b0 = 0; b0 < nseries; b0 += step) {
            const int nb = std::min(step, nseries - b0);
            const float *pl = plane_dev + (int64_t)b0 * sstride;
            if (bounded) {
                HIPTRY(p, launch_block_max(pl, g.NR, sstride, g.NR, rb, nb, p->d_pyr, psstride, st));
                TRY(run_harm_chunk(p, pl, g.NR, sstride, g, numharm, b0, nb, st, p->d_pyr, psstride, &rb));
            } else {
                TRY(run_harm_chunk(p, pl, g.NR, sstride, g, numharm, b0, nb, st));
            }
        }
        bool regrow = false;
        fdas_status s = finish(p, g, numharm, dz, out_host, cap, n_total, st, &regrow);
        if (!regrow) return s;
        TRY(grow_records(p, std::min<int64_t>(p->h_state[0], cap)));
    }
    return p->fail(FDAS_E_DEVICE, "internal error: candidate capacity did not converge");
}

fdas_status fdas_spectrum(fdas_plan p, const float *series_dev, int64_t nsamp, int32_t nseries,
                          float *spec_dev, double *norm_host, void *stream) {
    if (!p) return FDAS_E_INVAL;
    if (p->sticky) return p->fail(FDAS_E_DEVICE, "plan is in a failed state: " + p->last_error);
    if (!series_dev || ((uintptr_t)series_dev & 7) || !spec_dev || ((uintptr_t)spec_dev & 7))
        return p->fail(FDAS_E_INVAL, "device pointer NULL or not 8-byte aligned");
    if (nseries < 1 || nseries > p->max_series) return p->fail(FDAS_E_INVAL, "nseries out of range");
    if (nsamp < 8 || (nsamp & 1) || nsamp > p->max_nsamp)
        return p->fail(FDAS_E_INVAL, "nsamp odd, below 8 or above the plan's max_nsamp");
    if (!pow2(nsamp)) return p->fail(FDAS_E_UNSUPPORTED, "nsamp must be a power of two");
    Geometry g;
    g.nsamp = nsamp;
    g.half = nsamp / 2;
    hipStream_t st = static_cast<hipStream_t>(stream);
    TRY(run_spectrum(p, series_dev, g, nseries, st));
    HIPTRY(p, hipMemcpy2DAsync(spec_dev, (size_t)(g.half + 1) * sizeof(float2), p->d_spec,
                               (size_t)p->spitch * sizeof(float2), (size_t)(g.half + 1) * sizeof(float2),
                               (size_t)nseries, hipMemcpyDeviceToDevice, st));
    if (norm_host) {
        if (p->opts.norm == FDAS_NORM_MEDIAN) {
            HIPTRY(p, hipMemcpyAsync(norm_host, p->d_norm, nseries * sizeof(double), hipMemcpyDeviceToHost, st));
        } else {
            for (int b = 0; b < nseries; ++b) norm_host[b] = (double)nsamp * p->opts.fixed_var;
        }
    }
    HIPTRY(p, hipStreamSynchronize(st));
    p->collect();
    return FDAS_OK;
}

fdas_status fdas_plan_get_info(fdas_plan p, fdas_plan_info *out) {
    if (!p || !out) return FDAS_E_INVAL;
    out->seg_len = p->L;
    out->mseg = p->mseg;
    out->nz = p->bankNZ;
    out->chunk_series = p->chunk_series;
    out->workspace_bytes = p->plane_cap * (int64_t)sizeof(float);
    out->harm_blocks = p->last_harm_blocks;
    out->harm_pair = p->last_harm_pair;
    return FDAS_OK;
}

fdas_status fdas_profile_read(fdas_plan p, double *ms, int64_t *launches, int32_t reset) {
    if (!p) return FDAS_E_INVAL;
    for (int i = 0; i < FDAS_NPHASES; ++i) {
        if (ms) ms[i] = p->prof_ms[i];
        if (launches) launches[i] = p->prof_n[i];
        if (reset) {
            p->prof_ms[i] = 0;
            p->prof_n[i] = 0;
        }
    }
    return FDAS_OK;
}

}  // extern "C"
