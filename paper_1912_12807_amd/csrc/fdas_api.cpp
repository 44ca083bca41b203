// C ABI and host runtime: plans, the FP64-built template banks, workspace
// management, the autotuner, graph replay and the order in which the search
// kernels are enqueued.
//
// A search is a list of groups of series that share (nsamp, search band,
// zmax). Each group enqueues, on one stream:
//   K1 real FFT -> K2 median normalisation (or a fixed scale)
//   then per chunk of series (sized to the plane workspace):
//   K4 power plane + drift-block maxima -> K5 harmonic sums -> K6 ordered
//   compaction (with the drift argmax from the sums) -> significance.
// The record count and the records (with their FP64 significance) are then
// copied to pinned host memory, where physical units are attached (the
// candidate list of the paper's Section 2, step 5).
#include "fdas_internal.h"

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <list>
#include <map>
#include <memory>
#include <sstream>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

using namespace fdas;

namespace {

constexpr int64_t kDefaultCands = 1 << 20;
constexpr size_t kMaxBanks = 8;
constexpr size_t kMaxTables = 16;

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
bool run_parallel(int n, const std::function<void(int)> &fn) {
    std::atomic<bool> ok{true};
    auto share = [&](int w) {
        try {
            fn(w);
        } catch (...) {
            ok = false;
        }
    };
    std::vector<std::thread> pool;
    int w = 1;
    try {
        pool.reserve(n > 1 ? (size_t)n - 1 : 0);
        for (; w < n; ++w) pool.emplace_back(share, w);
    } catch (...) {
    }
    for (int v = w; v < n; ++v) share(v);
    if (n > 0) share(0);
    for (auto &t : pool) t.join();
    return ok;
}

int zgroups_of(int NZ) {
    int G = 1;
    while (G < 8 && NZ >= 2 * G * 12) G *= 2;
    return G;
}
// Drift rows per bound block. Above 8 harmonics, longer blocks are more often
// hot (a strong line enters many stage sums) and cost more when they are:
// 32 x 2^23 series with mains tones at numharm 16 took 83, 66, 68 and 99 ms of
// harmonic sums with 4, 6, 8 and 10 rows (46 ms at 6 with the code-pair
// bounds). Up to 8 harmonics, 128 x 2^18 series took 2.58, 2.34, 2.25, 2.43 and
// 2.47 ms with 6 to 10 rows.
int default_block_rows(int numharm) { return numharm <= 8 ? 8 : 6; }
// Block maxima per bin (both half-bin columns) or per column. Per column bounds
// are tighter at twice the memory; above 8 harmonics, where a strong line's
// half-bin neighbours enter many more stage sums, they win (e.g. 347 -> 227 ms
// on a batch of 32 x 2^23 series with mains tones at numharm 16).
bool maxima_per_bin(int harm_pair_opt, int numharm) {
    return harm_pair_opt == 2 || (harm_pair_opt == 0 && numharm <= 8);
}
constexpr int kMinBlockRows = 4;   // smallest block the autotuner tries (sizes the maxima buffer)

bool seg_len_ok(int L, int mseg) { return pow2(L) && L >= 512 && L <= 4096 && L - 2 * mseg >= 64; }

// Segment length for a half-width: the smallest L with L >= 16 mseg (>= 87.5 %
// of each segment valid), or the requested one if it leaves >= 64 valid bins.
int choose_L(int mseg, int requested) {
    if (requested) return seg_len_ok(requested, mseg) ? requested : 0;
    for (int L = 512; L <= 4096; L *= 2)
        if (L >= 16 * mseg) return L;
    return (4096 - 2 * mseg >= 1024) ? 4096 : 0;
}

// Tunable launch parameters of one group shape; none of them changes a
// result beyond FP32 rounding.
struct LaunchCfg {
    int L = 0;       // overlap-save segment length
    int bz = 0;      // drift rows per bound block
    int pair = 1;    // block maxima per bin (1) or per column (0)
};

struct Bank {
    double zmax = -1, dz = -1;
    int K = 0, L = 0, mseg = 0, NZ = 0;
    int G = 1;                                       // z groups of K4
    int32_t zb[kMaxZGroups + 1] = {};                // their row boundaries
    int gmseg[kMaxZGroups] = {};                     // and template half-widths
    float2 *d = nullptr;
    uint64_t used = 0;
};

struct RowTable {
    int NZ = -1, G = -1, bz = -1, nh = -1;
    int32_t zb[kMaxZGroups + 1] = {};
    int64_t ppitch = -1;
    int32_t *d = nullptr;
    int nblk = 0;
    uint64_t used = 0;
};

// One group of a search: series that share nsamp, band and zmax.
struct Group {
    Geometry g;
    double zmax = 0;
    int nb = 0;              // series in the group
    int vbase = 0;           // first virtual series id (position in the group-ordered batch)
    LaunchCfg cfg;
};

}  // namespace

struct fdas_plan_s {
    int device = -1;
    int64_t max_nsamp = 0;
    int32_t max_series = 0;
    int32_t max_numharm = 1;
    fdas_plan_opts opts{};
    std::string last_error;
    bool sticky = false;
    uint64_t tick = 0;
    uint64_t call_tick = 0;     // tick at the start of the current call
    int64_t n_alloc = 0;        // allocations made for the plan (the fail_alloc hook counts them)
    int min_bz = 1;             // smallest drift block the block-maxima buffer was sized for

    std::list<Bank> banks;      // list: entries keep their address while others are evicted
    std::list<RowTable> tables;
    std::map<std::tuple<int64_t, int, int>, LaunchCfg> tuned;   // (nsamp, zsteps, numharm)

    // workspace
    int64_t spitch = 0;
    float2 *d_spec = nullptr, *d_w0 = nullptr;
    float *d_scale = nullptr;
    double *d_norm = nullptr;
    uint8_t *d_med = nullptr;   // median-select scratch
    float *d_thr = nullptr;
    int64_t *d_state = nullptr;
    int64_t *d_offs = nullptr;  // ragged series offsets (complex units), group order
    float *d_plane = nullptr;
    int64_t plane_cap = 0;      // floats
    float *d_maxv = nullptr;
    int16_t *d_zarg = nullptr;  // maximising Zq of each stage maximum (maxv_cap entries)
    int64_t maxv_cap = 0;       // floats
    int32_t *d_counts = nullptr;
    int64_t *d_offsets = nullptr;
    int64_t nblk_cap = 0;
    DevCand *d_rec = nullptr;
    int64_t rec_cap = 0;
    bmax_t *d_pyr = nullptr;    // block maxima (half bits, rounded up)
    int64_t pyr_cap = 0;        // halves
    int last_harm_blocks = 0, last_harm_pair = 0;
    int last_L = 0, last_mseg = 0, last_NZ = 0;
    // pinned host staging
    int64_t *h_state = nullptr;
    float *h_small = nullptr;   // thresholds
    DevCand *h_rec = nullptr;
    int64_t h_rec_cap = 0;
    int64_t *h_offs = nullptr;
    // dedispersion: boxcar rows of two ranges, delay tables
    float *d_dd[2] = {nullptr, nullptr};
    int64_t dd_cap = 0;                 // floats per buffer
    int32_t *d_delays = nullptr, *h_delays = nullptr;
    int64_t delays_cap = 0;
    std::string dd_key;                     // description of the plan whose delay tables are on the device
    std::vector<int> dd_group, dd_span, dd_npad;
    int64_t dd_ntab = 0;
    // local normalisation: block tables per half-length and block-median scratch
    std::vector<std::pair<int64_t, std::pair<int32_t *, int>>> ltabs;
    float *d_lmed = nullptr;
    int64_t lmed_cap = 0;
    unsigned long long *d_csum = nullptr;   // per-channel sums and rounded means
    float *d_cpad = nullptr;
    int32_t cpad_cap = 0;
    // work lists of the merged bounded harmonic sums of a batch (and their staging)
    HarmItem *d_hitems = nullptr, *h_hitems = nullptr;
    int64_t hitems_cap = 0, h_hitems_cap = 0;
    int64_t *d_hstarts = nullptr, *h_hstarts = nullptr;
    int64_t hstarts_cap = 0, h_hstarts_cap = 0;
    // refinement points
    fdas_refine_point *d_rpts = nullptr, *h_rpts = nullptr;
    float *d_rpow = nullptr, *h_rpow = nullptr;
    int64_t rpts_cap = 0;

    // graph replay
    hipStream_t cap_st = nullptr;   // private stream that captures (never executes) the launches
    hipGraphExec_t graph = nullptr;
    hipGraph_t graph_def = nullptr;
    std::string graph_key;

    // phase timing (opts.profile)
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::tuple<int, hipEvent_t, hipEvent_t>> ev_pending;
    double prof_ms[FDAS_NPHASES] = {0};
    int64_t prof_n[FDAS_NPHASES] = {0};
    bool capturing = false;

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
        if (!opts.profile || capturing) return nullptr;
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

void drop_graph(fdas_plan p) {
    if (p->graph) (void)hipGraphExecDestroy(p->graph);
    if (p->graph_def) (void)hipGraphDestroy(p->graph_def);
    p->graph = nullptr;
    p->graph_def = nullptr;
    p->graph_key.clear();
}

// The allocation hook of the plan option fail_alloc: the fail_alloc-th
// allocation made for the plan fails as if memory were exhausted.
bool injected_failure(fdas_plan p) {
    ++p->n_alloc;
    return p->opts.fail_alloc > 0 && p->n_alloc == p->opts.fail_alloc;
}

// (Re)allocate *ptr for count elements. The old buffer is freed first; on
// failure *ptr is NULL. A captured graph holds buffer addresses, so any
// (re)allocation drops it (the next graph call captures again).
template <typename T>
fdas_status dalloc(fdas_plan p, T **ptr, int64_t count, const char *what) {
    drop_graph(p);
    if (*ptr) {
        (void)hipFree(*ptr);
        *ptr = nullptr;
    }
    if (count <= 0) count = 1;
    if (injected_failure(p)) return p->fail(FDAS_E_NOMEM, std::string("injected allocation failure: ") + what);
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
    drop_graph(p);
    if (*ptr) {
        (void)hipHostFree(*ptr);
        *ptr = nullptr;
    }
    if (count <= 0) count = 1;
    if (injected_failure(p)) return p->fail(FDAS_E_NOMEM, std::string("injected allocation failure: ") + what);
    void *q = nullptr;
    hipError_t e = hipHostMalloc(&q, (size_t)count * sizeof(T), hipHostMallocDefault);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return p->fail(FDAS_E_NOMEM, std::string("pinned host allocation failed: ") + what);
    }
    *ptr = static_cast<T *>(q);
    return FDAS_OK;
}

// Grow a buffer whose capacity is tracked in *cap: the capacity is 0 while the
// buffer is missing, so a failed allocation leaves the plan consistent (the
// next call allocates again instead of using a freed pointer).
template <typename T, typename C>
fdas_status grow(fdas_plan p, T **ptr, C *cap, int64_t count, const char *what, bool host = false) {
    *cap = 0;
    TRY(host ? halloc(p, ptr, count, what) : dalloc(p, ptr, count, what));
    *cap = (C)count;
    return FDAS_OK;
}

// Evict the least recently used entry of a cache if it is full and that entry
// was not used by the current call (earlier calls have completed on the device).
template <typename T>
void evict(fdas_plan p, std::list<T> &cache, size_t limit, void *(*mem)(T &)) {
    if (cache.size() < limit) return;
    auto it = std::min_element(cache.begin(), cache.end(),
                               [](const T &a, const T &b) { return a.used < b.used; });
    if (it->used >= p->call_tick) return;
    (void)hipFree(mem(*it));
    cache.erase(it);
    drop_graph(p);
}

// ---------------------------------------------------------------- template banks

// The bank for (zmax, dz, L): [NZ][2][L] kernel spectra, FP64 -> float32.
fdas_status get_bank(fdas_plan p, double zmax, double dz, int L, const Bank **out) {
    const int K = p->opts.K;
    for (auto &b : p->banks) {
        if (b.zmax == zmax && b.dz == dz && b.L == L && b.K == K) {
            b.used = ++p->tick;
            *out = &b;
            return FDAS_OK;
        }
    }
    const int Z = (int)std::round(zmax / dz);
    const int NZ = 2 * Z + 1;
    const int mseg = half_width(Z * dz, K);
    if (!seg_len_ok(L, mseg)) return p->fail(FDAS_E_UNSUPPORTED, "segment length too short for zmax");
    // each z group of K4 segments the spectrum by its own widest template, so
    // the kernel spectra of a row place the template at its group's half-width
    const int G = zgroups_of(NZ);
    int32_t zb[kMaxZGroups + 1];
    zgroup_bounds(NZ, dz, K, L, G, zb);
    int gm[kMaxZGroups];
    for (int i = 0; i < G; ++i)
        gm[i] = half_width(std::max(std::abs(zb[i] - Z), std::abs(zb[i + 1] - 1 - Z)) * dz, K);
    std::vector<int> msrow(NZ);
    for (int i = 0; i < G; ++i)
        for (int r = zb[i]; r < zb[i + 1]; ++r) msrow[r] = gm[i];
    std::vector<float> host((size_t)NZ * 2 * L * 2);
    const int nth = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const bool built = run_parallel(nth, [&](int w) {
        for (int row = w; row < 2 * NZ; row += nth) {
            const int zi = row / 2, par = row % 2;
            kernel_spectrum((zi - Z) * dz, par, K, L, msrow[zi], host.data() + (size_t)row * L * 2);
        }
    });
    if (!built) return p->fail(FDAS_E_NOMEM, "template bank: host computation failed");
    evict<Bank>(p, p->banks, kMaxBanks, [](Bank &b) -> void * { return b.d; });
    Bank b;
    b.zmax = zmax;
    b.dz = dz;
    b.K = K;
    b.L = L;
    b.mseg = mseg;
    b.NZ = NZ;
    b.G = G;
    for (int i = 0; i <= G; ++i) b.zb[i] = zb[i];
    for (int i = 0; i < G; ++i) b.gmseg[i] = gm[i];
    TRY(dalloc(p, &b.d, (int64_t)(host.size() / 2), "template bank"));
    if (hipMemcpy(b.d, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
        const hipError_t e = hipGetLastError();
        (void)hipFree(b.d);
        return p->hip(e == hipSuccess ? hipErrorUnknown : e, "template bank upload");
    }
    b.used = ++p->tick;
    p->banks.push_back(b);
    *out = &p->banks.back();
    return FDAS_OK;
}

// Row-block tables for the bounded harmonic sums, cached per geometry and
// maxima pitch: lo[nblk + 1], of_row[NZ], frange[nblk][numharm] and the bound
// test's gather table for code pairs [nblk][2 numharm + 2] in one device
// buffer.
fdas_status get_rows(fdas_plan p, int NZ, int G, const int32_t *zb, int bz, int numharm, bool pair,
                     int64_t ppitch, RowBlocks &rb) {
    RowTable *t = nullptr;
    for (auto &x : p->tables)
        if (x.NZ == NZ && x.G == G && std::equal(zb, zb + G + 1, x.zb) && x.bz == bz && x.nh == numharm &&
            x.ppitch == ppitch)
            t = &x;
    if (!t) {
        std::vector<int32_t> lo, of_row, fr, bo;
        row_blocks(zb, G, bz, lo, of_row);
        fraction_ranges(NZ, numharm, lo, of_row, fr);
        bound_offsets(numharm, fr, ppitch, bo);
        std::vector<int32_t> all(lo);
        all.insert(all.end(), of_row.begin(), of_row.end());
        all.insert(all.end(), fr.begin(), fr.end());
        all.insert(all.end(), bo.begin(), bo.end());
        evict<RowTable>(p, p->tables, kMaxTables, [](RowTable &r) -> void * { return r.d; });
        RowTable n;
        n.NZ = NZ;
        n.G = G;
        std::copy(zb, zb + G + 1, n.zb);
        n.bz = bz;
        n.nh = numharm;
        n.ppitch = ppitch;
        n.nblk = (int)lo.size() - 1;
        TRY(dalloc(p, &n.d, (int64_t)all.size(), "row-block tables"));
        if (hipMemcpy(n.d, all.data(), all.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
            const hipError_t e = hipGetLastError();
            (void)hipFree(n.d);
            return p->hip(e == hipSuccess ? hipErrorUnknown : e, "row-block table upload");
        }
        p->tables.push_back(n);
        t = &p->tables.back();
    }
    t->used = ++p->tick;
    rb.lo = t->d;
    rb.of_row = t->d + t->nblk + 1;
    rb.frange = rb.of_row + NZ;
    rb.nblk = t->nblk;
    rb.frange_nh = numharm;
    rb.table_ppitch = ppitch;
    rb.pair = pair;
    rb.ppitch = ppitch;
    return FDAS_OK;
}

LaunchCfg default_cfg(fdas_plan p, int Z, double dz, int numharm) {
    LaunchCfg c;
    c.L = choose_L(half_width(Z * dz, p->opts.K), p->opts.seg_len);
    c.bz = p->opts.harm_block ? p->opts.harm_block : default_block_rows(numharm);
    c.pair = maxima_per_bin(p->opts.harm_pair, numharm) ? 1 : 0;
    return c;
}

CorrGeom corr_geom(const Bank &bk, const Geometry &g) {
    CorrGeom c{};
    c.L = bk.L;
    c.mseg = bk.mseg;
    c.half = g.half;
    c.rlo = g.rlo;
    c.NZ = g.NZ;
    c.zgroups = bk.G;
    for (int i = 0; i <= bk.G; ++i) c.zb[i] = bk.zb[i];
    for (int i = 0; i < bk.G; ++i) {
        c.gmseg[i] = bk.gmseg[i];
        c.gLv[i] = bk.L - 2 * bk.gmseg[i];
        c.gnseg[i] = (int)((g.half - g.rlo + c.gLv[i] - 1) / c.gLv[i]);
    }
    return c;
}

// Block table of the local normalisation for spectra of `half` bins (cached), and
// block-median scratch for nb series. Allocates only outside graph capture.
fdas_status get_local(fdas_plan p, int64_t half, int nb, const int32_t **table, int *nblk) {
    for (auto &t : p->ltabs)
        if (t.first == half) {
            *table = t.second.first;
            *nblk = t.second.second;
            break;
        }
    if (!*table) {
        std::vector<int32_t> bs;
        for (int64_t b = 1; b < half;) {
            const int64_t e = std::min<int64_t>(half, b + std::min<int64_t>(200, 6 + b / 30));
            bs.push_back((int32_t)b);
            b = e;
        }
        bs.push_back((int32_t)half);
        int32_t *d = nullptr;
        TRY(dalloc(p, &d, (int64_t)bs.size(), "local-normalisation blocks"));
        if (hipMemcpy(d, bs.data(), bs.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
            const hipError_t e = hipGetLastError();
            (void)hipFree(d);
            return p->hip(e == hipSuccess ? hipErrorUnknown : e, "local-normalisation block upload");
        }
        p->ltabs.push_back({half, {d, (int)bs.size() - 1}});
        *table = d;
        *nblk = (int)bs.size() - 1;
    }
    if ((int64_t)*nblk * nb > p->lmed_cap) TRY(grow(p, &p->d_lmed, &p->lmed_cap, (int64_t)*nblk * nb, "block medians"));
    return FDAS_OK;
}

// ---------------------------------------------------------------- enqueue helpers

// K1 + K2 for nb series of nsamp samples (series b at x + b nsamp, or at
// x + 2 offs[b] floats); spectra, scales and norms go to batch slots v0...
fdas_status run_spectrum(fdas_plan p, const float *x, const int64_t *offs, int64_t nsamp, int nb, int v0,
                         hipStream_t st) {
    float2 *spec = p->d_spec + (int64_t)v0 * p->spitch;
    hipEvent_t e = p->begin(st);
    HIPTRY(p, launch_rfft(x, nsamp, nb, p->d_w0, spec, p->spitch, st, offs));
    p->end(0, e, st);
    if (p->opts.norm == FDAS_NORM_MEDIAN) {
        e = p->begin(st);
        HIPTRY(p, launch_median_scale(spec, p->spitch, nsamp / 2, nb, p->d_scale + v0, p->d_norm + v0, p->d_med,
                                      st));
        p->end(1, e, st);
    } else if (p->opts.norm == FDAS_NORM_LOCAL) {
        const int32_t *tab = nullptr;
        int nblk = 0;
        TRY(get_local(p, nsamp / 2, nb, &tab, &nblk));
        e = p->begin(st);
        HIPTRY(p, launch_local_norm(spec, p->spitch, nsamp / 2, nb, tab, nblk, p->d_lmed, p->d_scale + v0, st));
        p->end(1, e, st);
    } else {
        const float sc = (float)std::sqrt(1.0 / ((double)nsamp * p->opts.fixed_var));
        HIPTRY(p, launch_fill_scale(p->d_scale + v0, nb, sc, st));
    }
    return FDAS_OK;
}

// One K4/K5/K6 unit of a search: series b0 ... b0 + n - 1 of a group (batch
// slots vbase + b0 ...), with its regions of the plane, block-maxima and
// stage-maxima buffers.
struct WorkItem {
    const Geometry *g = nullptr;
    const Bank *bk = nullptr;
    CorrGeom cg{};
    RowBlocks rb;
    int vbase = 0, b0 = 0, n = 0;
    int64_t pitch = 0, sstride = 0, psstride = 0, mpitch = 0;
    bool with_pyr = false, bounded = false;
    int64_t plane_off = 0, pyr_off = 0, maxv_off = 0;   // elements into d_plane, d_pyr, d_maxv and d_zarg
};

// Layout of a group's series in the workspace (it, without series range or
// offsets) and *chunk, the most of them the workspace holds at once.
fdas_status group_item(fdas_plan p, const Geometry &g, const Bank &bk, const LaunchCfg &cfg, int numharm,
                       int vbase, WorkItem &it, int64_t *chunk) {
    it.g = &g;
    it.bk = &bk;
    it.cg = corr_geom(bk, g);
    it.vbase = vbase;
    it.pitch = round_up(g.NR, 64);
    it.sstride = (int64_t)g.NZ * it.pitch;
    TRY(get_rows(p, g.NZ, it.cg.zgroups, it.cg.zb, cfg.bz, numharm, cfg.pair != 0,
                 cfg.pair ? it.pitch / 2 : it.pitch, it.rb));
    it.psstride = (int64_t)it.rb.nblk * it.rb.ppitch;
    // K4 writes the block maxima whenever the buffer sized at plan creation
    // holds those of a chunk series. The exhaustive sums do not read them, but
    // every search then builds its plane with the same kernel instance, so that
    // bounded and exhaustive searches return bit-identical records. When they
    // do not fit, the plane is built without maxima (the chunk is then not
    // limited by their buffer) and every cell is summed.
    it.with_pyr = it.psstride <= kMaxPyrSeriesStride && it.psstride <= p->pyr_cap;
    it.bounded = it.with_pyr && !p->opts.harm_bound && bounded_table_bytes(it.rb.nblk, numharm) <= kBoundTableMax;
    it.mpitch = round_up(g.NR, 16);
    const int NS = nstages_of(numharm);
    int64_t c = std::min<int64_t>(p->plane_cap / it.sstride, p->maxv_cap / (NS * it.mpitch));
    if (it.with_pyr) c = std::min<int64_t>(c, p->pyr_cap / it.psstride);
    if (c < 1) return p->fail(FDAS_E_INVAL, "one series' plane exceeds the workspace");
    *chunk = c;
    p->last_harm_blocks = it.bounded ? it.rb.nblk : 0;
    p->last_harm_pair = it.rb.pair ? 1 : 0;
    p->last_L = bk.L;
    p->last_mseg = bk.mseg;
    p->last_NZ = g.NZ;
    return FDAS_OK;
}

fdas_status launch_item_k4(fdas_plan p, const WorkItem &it, hipStream_t st) {
    const int64_t v = it.vbase + it.b0;
    hipEvent_t e = p->begin(st);
    HIPTRY(p, launch_corr_power(p->d_spec + v * p->spitch, p->spitch, p->d_scale + v, it.bk->d, it.cg, it.n,
                                p->d_plane + it.plane_off, it.pitch, it.sstride,
                                it.with_pyr ? p->d_pyr + it.pyr_off : nullptr, it.psstride, it.rb, st));
    p->end(2, e, st);
    return FDAS_OK;
}

// K5 of one item in a launch of its own.
fdas_status launch_item_k5(fdas_plan p, const WorkItem &it, int numharm, hipStream_t st) {
    const Geometry &g = *it.g;
    hipEvent_t e = p->begin(st);
    if (it.bounded) {
        HIPTRY(p, launch_harmsum_bounded(p->d_plane + it.plane_off, it.pitch, it.sstride, p->d_pyr + it.pyr_off,
                                         it.psstride, it.rb, g.NR, g.rlo, g.Z, numharm, it.n, p->d_thr,
                                         p->d_maxv + it.maxv_off, p->d_zarg + it.maxv_off, it.mpitch, st));
    } else {
        const int order = p->opts.harm_order ? p->opts.harm_order : 1;
        HIPTRY(p, launch_harmsum(p->d_plane + it.plane_off, it.pitch, it.sstride, g.NR, g.rlo, g.Z, numharm, it.n,
                                 p->d_maxv + it.maxv_off, p->d_zarg + it.maxv_off, it.mpitch, order, st));
    }
    p->end(3, e, st);
    return FDAS_OK;
}

fdas_status launch_item_k6(fdas_plan p, const WorkItem &it, int numharm, hipStream_t st) {
    const int NS = nstages_of(numharm);
    hipEvent_t e = p->begin(st);
    HIPTRY(p, launch_compact(p->d_maxv + it.maxv_off, p->d_zarg + it.maxv_off, (int64_t)it.n * NS * it.mpitch,
                             it.mpitch, NS, it.vbase + it.b0, p->d_thr, p->d_counts, p->d_offsets, p->d_state,
                             p->d_rec, p->rec_cap, st));
    p->end(4, e, st);
    return FDAS_OK;
}

// K4 + K5 [+ K6] for the nb series of one group whose spectra are in batch
// slots vbase..., in chunks that the workspace holds. timing_only stops after
// K5 (autotuner).
fdas_status run_chunks(fdas_plan p, const Geometry &g, const Bank &bk, const LaunchCfg &cfg,
                       int numharm, int nb, int vbase, bool timing_only, hipStream_t st) {
    WorkItem it;
    int64_t chunk = 0;
    TRY(group_item(p, g, bk, cfg, numharm, vbase, it, &chunk));
    for (int b0 = 0; b0 < nb; b0 += (int)chunk) {
        it.b0 = b0;
        it.n = (int)std::min<int64_t>(chunk, nb - b0);
        TRY(launch_item_k4(p, it, st));
        TRY(launch_item_k5(p, it, numharm, st));
        if (!timing_only) TRY(launch_item_k6(p, it, numharm, st));
    }
    return FDAS_OK;
}

fdas_status upload_thresholds(fdas_plan p, int numharm, double sigma, hipStream_t st) {
    const int NS = nstages_of(numharm);
    for (int s = 0; s < NS; ++s) p->h_small[s] = (float)threshold(1 << s, sigma);
    HIPTRY(p, hipMemcpyAsync(p->d_thr, p->h_small, NS * sizeof(float), hipMemcpyHostToDevice, st));
    return FDAS_OK;
}

// ---------------------------------------------------------------- autotuner

// Launch parameters for a group: the plan's options, a tuned entry for the
// shape, or (autotune) the fastest candidate timed on the group's first series
// (K4 + K5 only; spectra of the sample are computed first).
fdas_status group_cfg(fdas_plan p, const Geometry &g, double zmax, double dz, int numharm, const float *x,
                      const int64_t *offs, int nb, int vbase, hipStream_t st, LaunchCfg *out) {
    const LaunchCfg base = default_cfg(p, g.Z, dz, numharm);
    if (!base.L) return p->fail(FDAS_E_UNSUPPORTED, "zmax too large for the supported segment lengths");
    *out = base;
    const int mseg = half_width(g.Z * dz, p->opts.K);
    const auto key = std::make_tuple(g.nsamp, g.Z, numharm);
    auto it = p->tuned.find(key);
    if (it != p->tuned.end() && seg_len_ok(it->second.L, mseg) && it->second.bz >= p->min_bz) {
        *out = it->second;
        return FDAS_OK;
    }
    if (!p->opts.autotune) return FDAS_OK;
    std::vector<int> Ls;
    for (int L = 512; L <= 4096; L *= 2)
        if (seg_len_ok(L, mseg) && L >= 4 * mseg && (p->opts.seg_len == 0 || L == p->opts.seg_len))
            Ls.push_back(L);
    if (Ls.empty()) Ls.push_back(base.L);
    std::vector<int> bzs;
    if (p->opts.harm_block) bzs = {p->opts.harm_block};
    else if (numharm <= 8) bzs = {6, 8, 10, 12, 16};
    else if (numharm == 16) bzs = {4, 6, 8, 10};
    else bzs = {4, 6, 8};
    // time on enough series to fill the chip as the real launch does (about
    // 2^31 plane cells), or on the whole group
    const int64_t cells = (int64_t)g.NZ * g.NR;
    const int sample = (int)std::min<int64_t>(nb, std::max<int64_t>(8, (((int64_t)1 << 31) + cells - 1) / cells));
    TRY(run_spectrum(p, x, offs, g.nsamp, sample, vbase, st));
    hipEvent_t a = p->take_event(), b = p->take_event();
    if (!a || !b) return p->fail(FDAS_E_DEVICE, "event creation failed");
    auto time_cfg = [&](const LaunchCfg &c, float *ms) -> fdas_status {
        const Bank *bk = nullptr;
        TRY(get_bank(p, zmax, dz, c.L, &bk));
        TRY(run_chunks(p, g, *bk, c, numharm, sample, vbase, true, st));   // warm
        HIPTRY(p, hipEventRecord(a, st));
        TRY(run_chunks(p, g, *bk, c, numharm, sample, vbase, true, st));
        HIPTRY(p, hipEventRecord(b, st));
        HIPTRY(p, hipEventSynchronize(b));
        HIPTRY(p, hipEventElapsedTime(ms, a, b));
        return FDAS_OK;
    };
    const int32_t was_profile = p->opts.profile;
    p->opts.profile = 0;
    LaunchCfg best = base;
    float best_ms = 3.0e38f;
    fdas_status s = FDAS_OK;
    // segment length first (default blocks), then block rows x granularity
    for (int L : Ls) {
        LaunchCfg c = base;
        c.L = L;
        float ms = 0;
        if ((s = time_cfg(c, &ms)) != FDAS_OK) break;
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    const LaunchCfg lbest = best;
    for (size_t i = 0; s == FDAS_OK && i < bzs.size(); ++i) {
        for (int pair : {1, 0}) {
            if ((p->opts.harm_pair == 1 && pair) || (p->opts.harm_pair == 2 && !pair)) continue;
            LaunchCfg c = lbest;
            c.bz = bzs[i];
            c.pair = pair;
            if (c.bz == lbest.bz && c.pair == lbest.pair) continue;
            float ms = 0;
            if ((s = time_cfg(c, &ms)) != FDAS_OK) break;
            if (ms < best_ms) {
                best_ms = ms;
                best = c;
            }
        }
    }
    p->opts.profile = was_profile;
    p->ev_pool.push_back(a);
    p->ev_pool.push_back(b);
    TRY(s);
    p->tuned[key] = best;
    *out = best;
    return FDAS_OK;
}

// ---------------------------------------------------------------- search driver

struct Batch {
    std::vector<Group> groups;
    std::vector<int> vmap;      // virtual id -> caller's series index
    std::vector<int> vgroup;    // virtual id -> group
    std::vector<double> vT;     // virtual id -> observation length (s)
};

// Copy the records of a finished search to the host, attach units, and write
// the first cap records in (series, harm, r_idx) order. need_regrow is set
// when the device buffer could not hold the records the output requires.
fdas_status finish(fdas_plan p, const Batch &B, double dz, bool sorted_on_device, fdas_cand *out,
                   int64_t cap, int64_t *n_total, hipStream_t st, bool *need_regrow) {
    hipEvent_t e = p->begin(st);
    HIPTRY(p, hipMemcpyAsync(p->h_state, p->d_state, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    p->end(6, e, st);
    HIPTRY(p, hipStreamSynchronize(st));
    const int64_t total = p->h_state[0];
    *need_regrow = false;
    const int64_t n = sorted_on_device ? std::min(total, cap) : total;
    if (n > p->rec_cap) {
        *need_regrow = true;
        p->collect();
        return FDAS_OK;
    }
    if (n > 0) {
        if (n > p->h_rec_cap) TRY(grow(p, &p->h_rec, &p->h_rec_cap, n, "candidate staging", true));
        e = p->begin(st);
        HIPTRY(p, hipMemcpyAsync(p->h_rec, p->d_rec, n * sizeof(DevCand), hipMemcpyDeviceToHost, st));
        p->end(6, e, st);
        HIPTRY(p, hipStreamSynchronize(st));
    }
    p->collect();
    // Two passes over host threads (long lists reach millions of records).
    // Device records are in (batch slot, stage, column) order and each slot
    // holds one caller series, so a stable counting sort by caller series
    // gives the (series, harm, r_idx) order: pass 1 checks the records and
    // counts each thread's records per series, the ranks follow series-major
    // then thread-major, and pass 2 writes each record (with units; the FP64
    // significance comes from the device) at its rank. Only ranks below cap
    // are written.
    const int64_t lim = std::min(n, cap);
    const int64_t per_thread = 16384;   // records per host thread (spawning costs tens of us)
    const int nth = (int)std::max<int64_t>(
        1, std::min<int64_t>(std::max(1u, std::min(16u, std::thread::hardware_concurrency())),
                             (n + per_thread - 1) / per_thread));
    auto over_threads = [&](const std::function<void(int, int64_t, int64_t)> &fn) {
        (void)run_parallel(nth, [&](int w) { fn(w, n * w / nth, n * (w + 1) / nth); });
    };
    int ns = 0;
    for (int v : B.vmap) ns = std::max(ns, v + 1);
    const size_t row = (size_t)ns + 8;   // per-thread counters, a cache line apart
    std::vector<int64_t> next(sorted_on_device ? 0 : (size_t)nth * row, 0);
    std::vector<char> bad((size_t)nth, 0);
    // a record's check: 0 valid, 1 unknown series or stage, 2 drift out of range
    auto check = [&](const DevCand &d) -> int {
        if (d.b < 0 || d.b >= (int)B.vmap.size() || d.s < 0 || d.s > 5) return 1;
        const Geometry &g = B.groups[B.vgroup[d.b]].g;
        return d.zq < -g.Z || d.zq > g.Z ? 2 : 0;
    };
    auto report = [&]() -> fdas_status {
        for (int w = 0; w < nth; ++w) {
            if (bad[w] == 1) return p->fail(FDAS_E_DEVICE, "internal error: candidate of an unknown series or stage");
            if (bad[w] == 2) return p->fail(FDAS_E_DEVICE, "internal error: candidate without a maximising drift");
        }
        return FDAS_OK;
    };
    // device order is the output order when sorted on the device: the checks
    // then run in the writing pass (one pass over the records instead of two)
    if (!sorted_on_device) {
        over_threads([&](int w, int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                const DevCand &d = p->h_rec[i];
                if (const int e = check(d)) {
                    bad[w] = (char)e;   // written only on failure: the flags share a cache line
                    return;
                }
                ++next[(size_t)w * row + B.vmap[d.b]];
            }
        });
        TRY(report());
        int64_t acc = 0;
        for (int v = 0; v < ns; ++v)
            for (int w = 0; w < nth; ++w) {
                int64_t &c = next[(size_t)w * row + v];
                const int64_t k = c;
                c = acc;
                acc += k;
            }
    }
    over_threads([&](int w, int64_t i0, int64_t i1) {
        int64_t *nx = sorted_on_device ? nullptr : next.data() + (size_t)w * row;
        for (int64_t i = i0; i < i1; ++i) {
            const DevCand &d = p->h_rec[i];
            if (sorted_on_device) {
                if (const int e = check(d)) {
                    bad[w] = (char)e;
                    return;
                }
            }
            const int64_t k = nx ? nx[B.vmap[d.b]]++ : i;
            if (k >= lim) continue;
            const Geometry &g = B.groups[B.vgroup[d.b]].g;
            const int H = 1 << d.s;
            const double T = B.vT[d.b];
            fdas_cand &c = out[k];
            c.series = B.vmap[d.b];
            c.harm = H;
            c.r_idx = (int64_t)d.c + 2 * g.rlo;
            c.z_idx = d.zq;
            c.power = d.power;
            c.sigma = d.sigma;
            c.r_fund = (double)c.r_idx / (2.0 * H);
            c.z_fund = (double)d.zq * dz / H;
            c.f_hz = c.r_fund / T;
            c.fdot_hz_s = c.z_fund / (T * T);
        }
    });
    TRY(report());
    *n_total = total;
    return total > cap ? FDAS_E_TRUNC : FDAS_OK;
}

// The work of a batch in waves. The items of a wave hold their own regions
// of the workspace together: their K4 launches run first, then one bounded
// K5 launch over the wave's bounded items (a work list), then their K6
// launches. A ragged batch of many small groups thus ends one partly idle K5
// tail per wave instead of one per group. A group of one search is split into
// chunks of the series the workspace holds, one wave each.
struct Wave {
    std::vector<WorkItem> items;
    int64_t plane = 0, pyr = 0, maxv = 0;   // elements of each buffer in use
    int list0 = 0, nlist = 0;               // work-list entries list0 ... (used when nlist > 1)
    int starts0 = 0;                        // its run starts (nlist + 1 entries)
    int64_t runs = 0;                       // tiles per XCD of the work-list launch
};

struct WavePlan {
    std::vector<Wave> waves;
    std::vector<HarmItem> list;
    std::vector<int64_t> starts;
};

// Items in batch order, each placed in the first wave with room in all three
// buffers. The records of a search of one group stay in series order: every
// full chunk fills one buffer too far to take another series, so each wave
// holds one chunk and the chunks run in order.
fdas_status plan_waves(fdas_plan p, const Batch &B, double dz, int numharm, WavePlan &W) {
    W = WavePlan();
    const int NS = nstages_of(numharm);
    for (const Group &G : B.groups) {
        const Bank *bk = nullptr;
        TRY(get_bank(p, G.zmax, dz, G.cfg.L, &bk));
        WorkItem it;
        int64_t chunk = 0;
        TRY(group_item(p, G.g, *bk, G.cfg, numharm, G.vbase, it, &chunk));
        for (int b0 = 0; b0 < G.nb; b0 += (int)chunk) {
            it.b0 = b0;
            it.n = (int)std::min<int64_t>(chunk, G.nb - b0);
            const int64_t pl = it.n * it.sstride, py = it.with_pyr ? it.n * it.psstride : 0;
            const int64_t mv = (int64_t)it.n * NS * it.mpitch;
            size_t w = 0;
            while (w < W.waves.size() && (W.waves[w].plane + pl > p->plane_cap || W.waves[w].pyr + py > p->pyr_cap ||
                                          W.waves[w].maxv + mv > p->maxv_cap))
                ++w;
            if (w == W.waves.size()) W.waves.emplace_back();
            Wave &X = W.waves[w];
            it.plane_off = X.plane;
            it.pyr_off = X.pyr;
            it.maxv_off = X.maxv;
            X.plane += pl;
            X.pyr += py;
            X.maxv += mv;
            X.items.push_back(it);
        }
    }
    // work lists: a wave's bounded items, those with the most drift blocks
    // (the costliest tiles) first
    for (Wave &X : W.waves) {
        std::vector<const WorkItem *> bi;
        for (const WorkItem &it : X.items)
            if (it.bounded) bi.push_back(&it);
        X.nlist = (int)bi.size();
        if (X.nlist < 2) continue;
        std::stable_sort(bi.begin(), bi.end(),
                         [](const WorkItem *a, const WorkItem *b) { return a->rb.nblk > b->rb.nblk; });
        X.list0 = (int)W.list.size();
        X.starts0 = (int)W.starts.size();
        for (const WorkItem *it : bi) {
            if (it->rb.frange_nh != numharm || it->rb.table_ppitch != it->rb.ppitch)
                return p->fail(FDAS_E_DEVICE, "internal error: row table of another numharm or pitch");
            HarmItem h{};
            h.plane = p->d_plane + it->plane_off;
            h.pitch = it->pitch;
            h.sstride = it->sstride;
            h.pyr = p->d_pyr + it->pyr_off;
            h.psstride = it->psstride;
            h.ppitch = it->rb.ppitch;
            h.blk_lo = it->rb.lo;
            h.frange = it->rb.frange;
            h.maxv = p->d_maxv + it->maxv_off;
            h.zarg = p->d_zarg + it->maxv_off;
            h.mpitch = it->mpitch;
            h.NR = it->g->NR;
            h.rlo = it->g->rlo;
            h.nblk = it->rb.nblk;
            h.Z = it->g->Z;
            h.pair = it->rb.pair ? 1 : 0;
            h.nseries = it->n;
            W.list.push_back(h);
        }
        W.starts.resize(W.starts.size() + X.nlist + 1);
        X.runs = harm_items_layout(W.list.data() + X.list0, X.nlist, numharm, W.starts.data() + X.starts0);
        if (X.runs < 1) return p->fail(FDAS_E_DEVICE, "internal error: invalid harmonic-sum work list");
    }
    return FDAS_OK;
}

// Copy the work lists to the device on st (grown first if needed, so before
// any capture).
fdas_status upload_lists(fdas_plan p, const WavePlan &W, hipStream_t st) {
    const int64_t ni = (int64_t)W.list.size(), ns = (int64_t)W.starts.size();
    if (!ni) return FDAS_OK;
    if (ni > p->hitems_cap) TRY(grow(p, &p->d_hitems, &p->hitems_cap, ni, "harmonic-sum work lists"));
    if (ni > p->h_hitems_cap) TRY(grow(p, &p->h_hitems, &p->h_hitems_cap, ni, "harmonic-sum work lists", true));
    if (ns > p->hstarts_cap) TRY(grow(p, &p->d_hstarts, &p->hstarts_cap, ns, "harmonic-sum work lists"));
    if (ns > p->h_hstarts_cap) TRY(grow(p, &p->h_hstarts, &p->h_hstarts_cap, ns, "harmonic-sum work lists", true));
    std::memcpy(p->h_hitems, W.list.data(), (size_t)ni * sizeof(HarmItem));
    std::memcpy(p->h_hstarts, W.starts.data(), (size_t)ns * sizeof(int64_t));
    HIPTRY(p, hipMemcpyAsync(p->d_hitems, p->h_hitems, (size_t)ni * sizeof(HarmItem), hipMemcpyHostToDevice, st));
    HIPTRY(p, hipMemcpyAsync(p->d_hstarts, p->h_hstarts, (size_t)ns * sizeof(int64_t), hipMemcpyHostToDevice, st));
    return FDAS_OK;
}

// Enqueue every group of a batch on st: the spectra of each length (groups of
// one length are adjacent in the batch: one K1 and one K2 launch per length),
// then the waves.
fdas_status enqueue_groups(fdas_plan p, const float *x, bool ragged, const Batch &B, const WavePlan &W,
                           int numharm, hipStream_t st) {
    HIPTRY(p, launch_zero_state(p->d_state, st));
    for (size_t i = 0; i < B.groups.size();) {
        size_t j = i;
        int nb = 0;
        while (j < B.groups.size() && B.groups[j].g.nsamp == B.groups[i].g.nsamp) nb += B.groups[j++].nb;
        const int v0 = B.groups[i].vbase;
        TRY(run_spectrum(p, x, ragged ? p->d_offs + v0 : nullptr, B.groups[i].g.nsamp, nb, v0, st));
        i = j;
    }
    for (const Wave &X : W.waves) {
        for (const WorkItem &it : X.items) TRY(launch_item_k4(p, it, st));
        if (X.nlist > 1) {
            hipEvent_t e = p->begin(st);
            HIPTRY(p, launch_harmsum_bounded_list(p->d_hitems + X.list0, p->d_hstarts + X.starts0, X.nlist, X.runs,
                                                  numharm, p->d_thr, st));
            p->end(3, e, st);
        }
        for (const WorkItem &it : X.items)
            if (!it.bounded || X.nlist < 2) TRY(launch_item_k5(p, it, numharm, st));
        for (const WorkItem &it : X.items) TRY(launch_item_k6(p, it, numharm, st));
    }
    // significance of every record of the call, in one launch
    hipEvent_t e = p->begin(st);
    HIPTRY(p, launch_cand_sigma(p->d_rec, p->d_state, p->rec_cap, st));
    p->end(5, e, st);
    return FDAS_OK;
}

// Run a prepared batch (thresholds and offsets already uploaded on st), eagerly
// or by replaying a captured graph, and collect the records; the device record
// buffer grows once if it was too small.
fdas_status run_batch(fdas_plan p, const float *x, bool ragged, const Batch &B, double dz, int numharm,
                      const std::string &key, fdas_cand *out, int64_t cap, int64_t *n_total, hipStream_t st) {
    const bool use_graph = p->opts.graph && !p->opts.profile;
    // every bank, row table and work list of the batch exists before any capture
    WavePlan W;
    TRY(plan_waves(p, B, dz, numharm, W));
    TRY(upload_lists(p, W, st));
    for (int attempt = 0; attempt < 2; ++attempt) {
        if (use_graph) {
            if (p->graph_key != key || !p->graph) {
                drop_graph(p);
                if (!p->cap_st) HIPTRY(p, hipStreamCreateWithFlags(&p->cap_st, hipStreamNonBlocking));
                if (p->opts.norm == FDAS_NORM_LOCAL) {
                    for (size_t i = 0; i < B.groups.size();) {
                        size_t j = i;
                        int nb = 0;
                        while (j < B.groups.size() && B.groups[j].g.nsamp == B.groups[i].g.nsamp)
                            nb += B.groups[j++].nb;
                        const int32_t *tab = nullptr;
                        int nblk = 0;
                        TRY(get_local(p, B.groups[i].g.nsamp / 2, nb, &tab, &nblk));
                        i = j;
                    }
                }
                HIPTRY(p, hipStreamBeginCapture(p->cap_st, hipStreamCaptureModeThreadLocal));
                p->capturing = true;
                const fdas_status s = enqueue_groups(p, x, ragged, B, W, numharm, p->cap_st);
                p->capturing = false;
                hipGraph_t gdef = nullptr;
                const hipError_t e = hipStreamEndCapture(p->cap_st, &gdef);
                if (s != FDAS_OK) {
                    if (gdef) (void)hipGraphDestroy(gdef);
                    return s;
                }
                HIPTRY(p, e);
                p->graph_def = gdef;
                HIPTRY(p, hipGraphInstantiate(&p->graph, gdef, nullptr, nullptr, 0));
                p->graph_key = key;
            }
            HIPTRY(p, hipGraphLaunch(p->graph, st));
        } else {
            TRY(enqueue_groups(p, x, ragged, B, W, numharm, st));
        }
        bool regrow = false;
        const fdas_status s = finish(p, B, dz, !ragged, out, cap, n_total, st, &regrow);
        if (!regrow) return s;
        const int64_t need = ragged ? p->h_state[0] : std::min<int64_t>(p->h_state[0], cap);
        TRY(grow(p, &p->d_rec, &p->rec_cap, need, "candidate records"));
    }
    return p->fail(FDAS_E_DEVICE, "internal error: candidate capacity did not converge");
}

fdas_status check_plan(fdas_plan p) {
    if (!p) return FDAS_E_INVAL;
    if (p->sticky) return p->fail(FDAS_E_DEVICE, "plan is in a failed state: " + p->last_error);
    int dev_now = -1;
    if (hipGetDevice(&dev_now) != hipSuccess || dev_now != p->device)
        return p->fail(FDAS_E_INVAL, "current HIP device differs from the plan's device");
    p->call_tick = p->tick + 1;
    return FDAS_OK;
}

fdas_status check_common(fdas_plan p, const void *dev, int64_t nsamp, int32_t nseries,
                         double tsamp, double zmax, double dz, Geometry &g) {
    TRY(check_plan(p));
    if (!dev || ((uintptr_t)dev & 7)) return p->fail(FDAS_E_INVAL, "device pointer NULL or not 8-byte aligned");
    if (nseries < 1 || nseries > p->max_series) return p->fail(FDAS_E_INVAL, "nseries out of range");
    if (nsamp > p->max_nsamp) return p->fail(FDAS_E_INVAL, "nsamp exceeds the plan's max_nsamp");
    fdas_status s = geometry(nsamp, tsamp, zmax, dz, p->opts.flo_hz, g);
    if (s != FDAS_OK) return p->fail(s, "invalid nsamp/tsamp/zmax/dz (odd nsamp, zmax not a multiple of dz, or empty band)");
    if (!fft_length_supported(nsamp)) return p->fail(FDAS_E_UNSUPPORTED, "nsamp / 2 must be a product of powers of 2, 3 and 5 (at most 2^26)");
    return FDAS_OK;
}

fdas_status check_search(fdas_plan p, int32_t numharm, double sigma, fdas_cand *out, int64_t cap,
                         int64_t *n_total) {
    if (!valid_numharm(numharm) || numharm > p->max_numharm)
        return p->fail(FDAS_E_INVAL, "numharm must be a power of two up to the plan's numharm");
    if (!(sigma > 0) || !std::isfinite(sigma)) return p->fail(FDAS_E_INVAL, "sigma must be finite and > 0");
    if (cap < 0 || (cap > 0 && !out) || !n_total) return p->fail(FDAS_E_INVAL, "bad output buffer");
    return FDAS_OK;
}

// One series' plane must fit the workspace.
fdas_status check_fits(fdas_plan p, const Geometry &g) {
    const int64_t sstride = (int64_t)g.NZ * round_up(g.NR, 64);
    if (sstride > p->plane_cap)
        return p->fail(FDAS_E_INVAL, "one series' plane exceeds the workspace; create the plan with this zmax");
    return FDAS_OK;
}

void key_group(std::ostringstream &k, const Group &G) {
    k << '|' << G.g.nsamp << ',' << G.g.rlo << ',' << G.g.Z << ',' << G.nb << ',' << G.cfg.L << ','
      << G.cfg.bz << ',' << G.cfg.pair;
}

}  // namespace

// entry-point error handler: records the message on the plan (if any)
static fdas_status plan_entry_error(fdas_plan p, fdas_status s, const char *msg) { return p ? p->fail(s, msg) : s; }

extern "C" {

void fdas_plan_opts_default(fdas_plan_opts *o) {
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->flo_hz = 1.0;
    o->K = 16;
    o->norm = FDAS_NORM_MEDIAN;
    o->fixed_var = 1.0;
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
    drop_graph(p);
    if (p->cap_st) (void)hipStreamDestroy(p->cap_st);
    for (auto &b : p->banks) (void)hipFree(b.d);
    for (auto &t : p->tables) (void)hipFree(t.d);
    for (auto &t : p->ltabs) (void)hipFree(t.second.first);
    void *dev[] = {p->d_spec, p->d_w0, p->d_scale, p->d_norm, p->d_med, p->d_thr, p->d_state, p->d_offs,
                   p->d_plane, p->d_maxv, p->d_zarg, p->d_counts, p->d_offsets, p->d_rec, p->d_pyr, p->d_rpts, p->d_rpow, p->d_dd[0], p->d_dd[1], p->d_delays, p->d_csum, p->d_cpad, p->d_lmed,
                   p->d_hitems, p->d_hstarts};
    for (void *q : dev)
        if (q) (void)hipFree(q);
    for (auto &t : p->ev_pending) {
        p->ev_pool.push_back(std::get<1>(t));
        p->ev_pool.push_back(std::get<2>(t));
    }
    for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
    void *host[] = {p->h_state, p->h_small, p->h_rec, p->h_offs, p->h_rpts, p->h_rpow, p->h_delays,
                    p->h_hitems, p->h_hstarts};
    for (void *q : host)
        if (q) (void)hipHostFree(q);
    if (cur >= 0) (void)hipSetDevice(cur);
    delete p;
}

fdas_status fdas_plan_create(fdas_plan *out, int64_t max_nsamp, int32_t max_series, double zmax,
                             double dz, int32_t numharm, const fdas_plan_opts *opts) {
    FDAS_ENTRY_TRY
    if (!out) return FDAS_E_INVAL;
    *out = nullptr;
    fdas_plan_opts o;
    fdas_plan_opts_default(&o);
    if (opts) o = *opts;
    for (int i = 0; i < 3; ++i)
        if (o.reserved[i]) return FDAS_E_INVAL;
    if (o.fail_alloc < 0) return FDAS_E_INVAL;
    if (max_series < 1 || max_series > 65535 || !valid_numharm(numharm) || o.K < 1 || o.K > 1024 ||
        (o.norm != FDAS_NORM_MEDIAN && o.norm != FDAS_NORM_FIXED && o.norm != FDAS_NORM_LOCAL) ||
        (o.norm == FDAS_NORM_FIXED && !(o.fixed_var > 0)) || o.max_workspace_bytes < 0 ||
        o.max_candidates < 0 || o.harm_order < 0 || o.harm_order > 3 || o.harm_bound < 0 ||
        o.harm_bound > 1 || o.harm_block < 0 || o.harm_block > 64 || o.harm_pair < 0 || o.harm_pair > 2 ||
        o.autotune < 0 || o.autotune > 1 || o.graph < 0 || o.graph > 1)
        return FDAS_E_INVAL;
    Geometry g;
    if (geometry(max_nsamp, 1e-3, zmax, dz, 0.0, g) != FDAS_OK) return FDAS_E_INVAL;
    const int mseg = half_width(g.Z * dz, o.K);
    if (!choose_L(mseg, o.seg_len)) return o.seg_len ? FDAS_E_INVAL : FDAS_E_UNSUPPORTED;

    // the guard destroys a half-built plan on every early return and on a host
    // exception caught at the ABI boundary
    std::unique_ptr<fdas_plan_s, void (*)(fdas_plan)> guard(new (std::nothrow) fdas_plan_s, fdas_plan_destroy);
    fdas_plan p = guard.get();
    if (!p) return FDAS_E_NOMEM;
    p->opts = o;
    p->max_nsamp = max_nsamp;
    p->max_series = max_series;
    p->max_numharm = numharm;
    auto bail = [](fdas_status s) { return s; };
    if (hipGetDevice(&p->device) != hipSuccess) {
        (void)hipGetLastError();
        return bail(FDAS_E_DEVICE);
    }
    const Bank *bk = nullptr;
    fdas_status s = get_bank(p, g.Z * dz, dz, default_cfg(p, g.Z, dz, numharm).L, &bk);
    if (s != FDAS_OK) return bail(s);

    const int64_t half = max_nsamp / 2;
    p->spitch = round_up(half + 1, 2);
    if ((s = dalloc(p, &p->d_spec, (int64_t)max_series * p->spitch, "spectra")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_w0, (int64_t)max_series * half, "fft scratch")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_scale, max_series, "scales")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_norm, max_series, "norms")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_med, (int64_t)median_scratch_bytes(max_series), "median scratch")) != FDAS_OK)
        return bail(s);
    if ((s = dalloc(p, &p->d_thr, 8, "thresholds")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_state, 2, "state")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_offs, max_series, "series offsets")) != FDAS_OK) return bail(s);

    // plane workspace: as many series per chunk as the budget allows
    const int64_t pitch = round_up(max_nsamp, 64);           // >= NR of any search
    const int64_t per_series = (int64_t)g.NZ * pitch;        // floats
    int64_t budget = o.max_workspace_bytes;
    if (!budget) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
            (void)hipGetLastError();
            fr = (size_t)8 << 30;
        }
        budget = std::min<int64_t>((int64_t)64 << 30, (int64_t)(fr / 2));
    }
    const int64_t chunk = std::min<int64_t>(max_series, budget / (per_series * 4));
    if (chunk < 1) return bail(FDAS_E_NOMEM);
    p->plane_cap = chunk * per_series;
    if ((s = dalloc(p, &p->d_plane, p->plane_cap, "power plane")) != FDAS_OK) return bail(s);
    // block maxima of every chunk series: blocks of >= kMinBlockRows rows
    // (NZ / bz + 8 blocks at most, z groups cut blocks), 16 bits per column
    const int bzmin = o.harm_block ? o.harm_block : kMinBlockRows;
    p->min_bz = bzmin;
    p->pyr_cap = chunk * (int64_t)(g.NZ / bzmin + 9) * pitch;
    if ((s = dalloc(p, &p->d_pyr, p->pyr_cap, "block maxima")) != FDAS_OK) return bail(s);
    const int NS = nstages_of(numharm);
    p->maxv_cap = chunk * NS * round_up(max_nsamp, 16);
    if ((s = dalloc(p, &p->d_maxv, p->maxv_cap, "stage maxima")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_zarg, p->maxv_cap, "stage maxima drift indices")) != FDAS_OK) return bail(s);
    p->nblk_cap = compact_blocks(p->maxv_cap);
    if ((s = dalloc(p, &p->d_counts, p->nblk_cap, "compaction counts")) != FDAS_OK) return bail(s);
    if ((s = dalloc(p, &p->d_offsets, p->nblk_cap, "compaction offsets")) != FDAS_OK) return bail(s);
    p->rec_cap = o.max_candidates ? o.max_candidates : kDefaultCands;
    if ((s = dalloc(p, &p->d_rec, p->rec_cap, "candidate records")) != FDAS_OK) return bail(s);
    if ((s = halloc(p, &p->h_state, 2, "state")) != FDAS_OK) return bail(s);
    if ((s = halloc(p, &p->h_small, 8, "thresholds")) != FDAS_OK) return bail(s);
    if ((s = halloc(p, &p->h_offs, max_series, "series offsets")) != FDAS_OK) return bail(s);
    p->h_rec_cap = 4096;
    if ((s = halloc(p, &p->h_rec, p->h_rec_cap, "candidate staging")) != FDAS_OK) return bail(s);
    *out = guard.release();
    return FDAS_OK;
    FDAS_ENTRY_CATCH(plan_entry_error, nullptr)
}

fdas_status fdas_search(fdas_plan p, const float *series_dev, int64_t nsamp, int32_t nseries,
                        double tsamp, double zmax, double dz, int32_t numharm, double sigma,
                        fdas_cand *out_host, int64_t cap, int64_t *n_total, void *stream) {
    FDAS_ENTRY_TRY
    Geometry g;
    TRY(check_common(p, series_dev, nsamp, nseries, tsamp, zmax, dz, g));
    TRY(check_search(p, numharm, sigma, out_host, cap, n_total));
    TRY(check_fits(p, g));
    hipStream_t st = static_cast<hipStream_t>(stream);
    Batch B;
    B.groups.resize(1);
    Group &G = B.groups[0];
    G.g = g;
    G.zmax = g.Z * dz;
    G.nb = nseries;
    G.vbase = 0;
    B.vmap.resize(nseries);
    for (int i = 0; i < nseries; ++i) B.vmap[i] = i;
    B.vgroup.assign(nseries, 0);
    B.vT.assign(nseries, g.T);
    TRY(upload_thresholds(p, numharm, sigma, st));
    TRY(group_cfg(p, g, G.zmax, dz, numharm, series_dev, nullptr, nseries, 0, st, &G.cfg));
    std::ostringstream key;
    key << "h " << (const void *)series_dev << ' ' << dz << ' ' << numharm << ' ' << p->rec_cap;
    key_group(key, G);
    return run_batch(p, series_dev, false, B, dz, numharm, key.str(), out_host, cap, n_total, st);
    FDAS_ENTRY_CATCH(plan_entry_error, p)
}

fdas_status fdas_search_ragged(fdas_plan p, const float *series_dev, const int64_t *offsets,
                               const int64_t *nsamp, const double *tsamp, const double *zmax,
                               int32_t nseries, double dz, int32_t numharm, double sigma,
                               fdas_cand *out_host, int64_t cap, int64_t *n_total, void *stream) {
    FDAS_ENTRY_TRY
    TRY(check_plan(p));
    if (!series_dev || ((uintptr_t)series_dev & 7) || !offsets || !nsamp || !tsamp || !zmax)
        return p->fail(FDAS_E_INVAL, "NULL or misaligned argument");
    if (nseries < 1 || nseries > p->max_series) return p->fail(FDAS_E_INVAL, "nseries out of range");
    TRY(check_search(p, numharm, sigma, out_host, cap, n_total));
    // group series by (nsamp, band, zmax)
    std::map<std::tuple<int64_t, int64_t, int>, int> gid;
    Batch B;
    std::vector<std::vector<int>> members;
    std::vector<Geometry> geo(nseries);
    for (int i = 0; i < nseries; ++i) {
        Geometry &g = geo[i];
        if (offsets[i] < 0 || (offsets[i] & 1)) return p->fail(FDAS_E_INVAL, "series offset negative or odd");
        if (nsamp[i] > p->max_nsamp) return p->fail(FDAS_E_INVAL, "nsamp exceeds the plan's max_nsamp");
        fdas_status s = geometry(nsamp[i], tsamp[i], zmax[i], dz, p->opts.flo_hz, g);
        if (s != FDAS_OK) return p->fail(s, "invalid nsamp/tsamp/zmax/dz of a series");
        if (!fft_length_supported(nsamp[i])) return p->fail(FDAS_E_UNSUPPORTED, "nsamp / 2 must be a product of powers of 2, 3 and 5 (at most 2^26)");
        TRY(check_fits(p, g));
        const auto key = std::make_tuple(g.nsamp, g.rlo, g.Z);
        auto it = gid.find(key);
        if (it == gid.end()) {
            it = gid.emplace(key, (int)B.groups.size()).first;
            Group G;
            G.g = g;
            G.zmax = g.Z * dz;
            B.groups.push_back(G);
            members.emplace_back();
        }
        members[it->second].push_back(i);
    }
    // batch order: groups by (nsamp, band, zmax), so that groups of one length
    // are adjacent; series in caller order inside a group
    {
        std::vector<Group> sorted;
        std::vector<std::vector<int>> smembers;
        for (const auto &kv : gid) {
            sorted.push_back(B.groups[kv.second]);
            smembers.push_back(std::move(members[kv.second]));
        }
        B.groups.swap(sorted);
        members.swap(smembers);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (size_t gi = 0; gi < B.groups.size(); ++gi) {
        Group &G = B.groups[gi];
        G.vbase = (int)B.vmap.size();
        G.nb = (int)members[gi].size();
        for (int i : members[gi]) {
            p->h_offs[B.vmap.size()] = offsets[i] / 2;   // complex-sample units
            B.vmap.push_back(i);
            B.vgroup.push_back((int)gi);
            B.vT.push_back(geo[i].T);
        }
    }
    TRY(upload_thresholds(p, numharm, sigma, st));
    HIPTRY(p, hipMemcpyAsync(p->d_offs, p->h_offs, nseries * sizeof(int64_t), hipMemcpyHostToDevice, st));
    for (auto &G : B.groups)
        TRY(group_cfg(p, G.g, G.zmax, dz, numharm, series_dev, p->d_offs + G.vbase, G.nb, G.vbase, st, &G.cfg));
    // graph key: every value the enqueued launches depend on (offsets are
    // read from device memory, uploaded every call)
    std::ostringstream key;
    key << "r " << (const void *)series_dev << ' ' << nseries << ' ' << dz << ' ' << numharm << ' '
        << p->rec_cap;
    for (const auto &G : B.groups) key_group(key, G);
    return run_batch(p, series_dev, true, B, dz, numharm, key.str(), out_host, cap, n_total, st);
    FDAS_ENTRY_CATCH(plan_entry_error, p)
}

fdas_status fdas_dedisperse(fdas_plan p, const uint8_t *fil_dev, int64_t nsamp, int32_t nchan, double tsamp,
                            double f0_mhz, double df_mhz, const fdas_dm_range *ranges, int32_t nranges,
                            float *out_dev, int64_t out_elems, void *stream) {
    FDAS_ENTRY_TRY
    TRY(check_plan(p));
    if (!fil_dev || !out_dev || ((uintptr_t)out_dev & 3) || !ranges || nranges < 1 || nsamp < 1 || nchan < 1 ||
        nchan > 65535 || !(tsamp > 0) || !std::isfinite(tsamp) || !std::isfinite(f0_mhz) || !std::isfinite(df_mhz))
        return p->fail(FDAS_E_INVAL, "bad filterbank description or buffers");
    const double flast = f0_mhz + (nchan - 1) * df_mhz;
    if (!(f0_mhz > 0) || !(flast > 0)) return p->fail(FDAS_E_INVAL, "channel frequencies must be positive");
    const double fhi = std::max(f0_mhz, flast);
    int64_t need = 0, rows_max = 0;
    for (int r = 0; r < nranges; ++r) {
        const fdas_dm_range &R = ranges[r];
        if (R.ndm < 1 || R.downsamp < 1 || nsamp % R.downsamp || !(R.dm_start >= 0) || !(R.dm_step >= 0) ||
            !std::isfinite(R.dm_start) || !std::isfinite(R.dm_step))
            return p->fail(FDAS_E_INVAL, "DM range: ndm >= 1, downsamp >= 1 dividing nsamp, DMs >= 0");
        if ((double)nchan * R.downsamp * 255.0 >= 16777216.0 || nsamp > (int64_t)65535 * 4096)
            return p->fail(FDAS_E_UNSUPPORTED, "sums beyond 2^24 (nchan D 255) or more than 2^28 samples");
        need += (int64_t)R.ndm * (nsamp / R.downsamp);
        rows_max = std::max<int64_t>(rows_max, nsamp / R.downsamp);
    }
    if (need > out_elems) return p->fail(FDAS_E_INVAL, "output buffer too small for the DM plan");
    // delay tables depend only on the description: keep them on the device between calls
    std::string key;
    {
        std::ostringstream k;
        k.precision(17);
        k << nsamp << ' ' << nchan << ' ' << tsamp << ' ' << f0_mhz << ' ' << df_mhz;
        for (int r = 0; r < nranges; ++r)
            k << '|' << ranges[r].dm_start << ',' << ranges[r].dm_step << ',' << ranges[r].ndm << ','
              << ranges[r].downsamp;
        key = k.str();
    }
    const bool have_tables = (key == p->dd_key);
    if (!have_tables) {
        p->dd_key.clear();
        // delays, FP64, in the order of the formula: K DM (f^-2 - fhi^-2) / (D tsamp) + 1/2, floor;
        // per range a table [nchan][ndm_pad] (ndm_pad a multiple of the DM group, entries
        // past ndm repeating the last DM) and the group size / staged channels that fit LDS
        std::vector<int> group(nranges), span(nranges), npad(nranges);
        std::vector<std::vector<int32_t>> tab(nranges);
        int64_t ntab = 0;
        for (int r = 0; r < nranges; ++r) {
            const fdas_dm_range &R = ranges[r];
            std::vector<int32_t> d((size_t)R.ndm * nchan);      // [dm][c]
            for (int i = 0; i < R.ndm; ++i) {
                const double dm = R.dm_start + i * R.dm_step;
                for (int c = 0; c < nchan; ++c) {
                    const double f = f0_mhz + c * df_mhz;
                    const double x =
                        4.148808e3 * dm * (1.0 / (f * f) - 1.0 / (fhi * fhi)) / ((double)R.downsamp * tsamp) + 0.5;
                    const double v = std::floor(x);
                    if (!(v <= 2e9)) return p->fail(FDAS_E_INVAL, "dispersion delay beyond 2^31 samples");
                    d[(size_t)i * nchan + c] = (int32_t)v;
                }
            }
            for (int G = 16; G >= 1; G /= 2) {
                int sp = 0;
                for (int i0 = 0; i0 < R.ndm; i0 += G)
                    for (int c = 0; c < nchan; ++c)
                        sp = std::max(sp, d[(size_t)std::min(i0 + G - 1, R.ndm - 1) * nchan + c] -
                                              d[(size_t)i0 * nchan + c]);
                if (dedisperse_width(sp) || G == 1) {
                    group[r] = G;
                    span[r] = sp;
                    break;
                }
            }
            const int G = group[r];
            npad[r] = (R.ndm + G - 1) / G * G;
            tab[r].resize((size_t)nchan * npad[r]);
            for (int c = 0; c < nchan; ++c)
                for (int i = 0; i < npad[r]; ++i)
                    tab[r][(size_t)c * npad[r] + i] = d[(size_t)std::min(i, R.ndm - 1) * nchan + c];
            ntab += (int64_t)nchan * npad[r];
        }
        if (ntab > p->delays_cap) {
            int64_t hcap = 0;
            TRY(grow(p, &p->d_delays, &p->delays_cap, ntab, "delay tables"));
            p->delays_cap = 0;
            TRY(grow(p, &p->h_delays, &hcap, ntab, "delay tables", true));
            p->delays_cap = ntab;
        }
        {
            int64_t o = 0;
            for (int r = 0; r < nranges; ++r) {
                std::memcpy(p->h_delays + o, tab[r].data(), tab[r].size() * sizeof(int32_t));
                o += (int64_t)tab[r].size();
            }
        }
        p->dd_group = group;
        p->dd_span = span;
        p->dd_npad = npad;
        p->dd_ntab = ntab;
    }
    const std::vector<int> &group = p->dd_group, &span = p->dd_span, &npad = p->dd_npad;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (rows_max * nchan > p->dd_cap) {
        TRY(grow(p, &p->d_dd[0], &p->dd_cap, rows_max * nchan, "dedispersion rows"));
        p->dd_cap = 0;
        TRY(dalloc(p, &p->d_dd[1], rows_max * nchan, "dedispersion rows"));
        p->dd_cap = rows_max * nchan;
    }
    if (nchan > p->cpad_cap) {
        TRY(grow(p, &p->d_csum, &p->cpad_cap, nchan, "channel sums"));
        p->cpad_cap = 0;
        TRY(dalloc(p, &p->d_cpad, nchan, "channel means"));
        p->cpad_cap = nchan;
    }
    if (!have_tables) {
        HIPTRY(p, hipMemcpyAsync(p->d_delays, p->h_delays, p->dd_ntab * sizeof(int32_t), hipMemcpyHostToDevice,
                                 st));
        p->dd_key = key;
    }
    hipEvent_t e = p->begin(st);
    HIPTRY(p, launch_zero_sums(p->d_csum, nchan, st));
    // boxcar rows of a range come from the previous range's rows when its factor
    // divides this one (the same rows when equal), otherwise from the file; the
    // first pass over the file also totals each channel for the padding mean
    int64_t o_out = 0, o_del = 0;
    int ybuf = -1, prevD = 0;
    for (int r = 0; r < nranges; ++r) {
        const fdas_dm_range &R = ranges[r];
        const int64_t n = nsamp / R.downsamp;
        int nb = ybuf;
        if (prevD != R.downsamp) {
            nb = ybuf < 0 ? 0 : (ybuf ^ 1);
            if (prevD && R.downsamp % prevD == 0) {
                HIPTRY(p, launch_downsample_rows(p->d_dd[ybuf], nsamp / prevD, n, R.downsamp / prevD, nchan,
                                                 p->d_dd[nb], n, st));
            } else {
                HIPTRY(p, launch_fil_downsample(fil_dev, nsamp, nchan, R.downsamp, p->d_dd[nb], n,
                                                ybuf < 0 ? p->d_csum : nullptr, st));
            }
        }
        HIPTRY(p, launch_channel_pad(p->d_csum, nsamp, R.downsamp, nchan, p->d_cpad, st));
        HIPTRY(p, launch_dedisperse(p->d_dd[nb], n, n, nchan, p->d_cpad, p->d_delays + o_del, R.ndm,
                                    npad[r], group[r], span[r], out_dev + o_out, n, st));
        o_out += (int64_t)R.ndm * n;
        o_del += (int64_t)nchan * npad[r];
        ybuf = nb;
        prevD = R.downsamp;
    }
    p->end(8, e, st);
    HIPTRY(p, hipStreamSynchronize(st));
    p->collect();
    return FDAS_OK;
    FDAS_ENTRY_CATCH(plan_entry_error, p)
}

fdas_status fdas_refine_window(double r0, double z0, double dz, int32_t K, int64_t *k0, int32_t *m) {
    if (!k0 || !m || !std::isfinite(r0) || !std::isfinite(z0) || !(dz > 0) || !std::isfinite(dz) || K < 0 ||
        K > 1024 || std::fabs(r0) > 9e15)
        return FDAS_E_INVAL;
    const double mm = std::ceil((std::fabs(z0) + 2.0 * dz) / 2.0) + K + 1;
    if (mm > kRefineMaxM) return FDAS_E_INVAL;
    *k0 = (int64_t)std::floor(r0 + 0.5);
    *m = (int32_t)mm;
    return FDAS_OK;
}

static fdas_status check_refine_args(const float *spec, int64_t spitch, int64_t nbins, int32_t nseries,
                                     const fdas_refine_point *pts, int64_t n, int32_t max_m) {
    if (!spec || ((uintptr_t)spec & 7) || !pts || ((uintptr_t)pts & 7) || nbins < 2 || spitch < nbins ||
        nseries < 1 || n < 0 || n > 0x7fffffffLL || max_m < 0 || max_m > kRefineMaxM)
        return FDAS_E_INVAL;
    return FDAS_OK;
}

fdas_status fdas_refine_eval(const float *spec_dev, int64_t spitch, int64_t nbins, int32_t nseries,
                             const float *scale_dev, const fdas_refine_point *pts_dev, int64_t n,
                             int32_t max_m, float *power_dev, float *dpdr_dev, float *dpdz_dev,
                             void *stream) {
    TRY(check_refine_args(spec_dev, spitch, nbins, nseries, pts_dev, n, max_m));
    if (!power_dev) return FDAS_E_INVAL;
    if (n == 0) return FDAS_OK;
    const hipError_t e = launch_refine_eval(reinterpret_cast<const float2 *>(spec_dev), spitch, nbins, nseries,
                                            scale_dev, pts_dev, n, max_m, power_dev, dpdr_dev, dpdz_dev,
                                            static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FDAS_OK : FDAS_E_DEVICE;
}

fdas_status fdas_refine_grad(const float *spec_dev, int64_t spitch, int64_t nbins, int32_t nseries,
                             const float *scale_dev, const fdas_refine_point *pts_dev, int64_t n,
                             int32_t max_m, const float *grad_power_dev, float *grad_r_dev,
                             float *grad_z_dev, float *grad_spec_dev, void *stream) {
    TRY(check_refine_args(spec_dev, spitch, nbins, nseries, pts_dev, n, max_m));
    if (!grad_power_dev || ((uintptr_t)grad_spec_dev & 7)) return FDAS_E_INVAL;
    if (n == 0) return FDAS_OK;
    const hipError_t e = launch_refine_grad(reinterpret_cast<const float2 *>(spec_dev), spitch, nbins, nseries,
                                            scale_dev, pts_dev, n, max_m, grad_power_dev, grad_r_dev, grad_z_dev,
                                            grad_spec_dev, static_cast<hipStream_t>(stream));
    return e == hipSuccess ? FDAS_OK : FDAS_E_DEVICE;
}

fdas_status fdas_refine(fdas_plan p, const float *series_dev, int64_t nsamp, int32_t nseries, double dz,
                        int32_t iters, fdas_refine_point *pts_host, float *power_host, int64_t n,
                        void *stream) {
    FDAS_ENTRY_TRY
    TRY(check_plan(p));
    if (!series_dev || ((uintptr_t)series_dev & 7)) return p->fail(FDAS_E_INVAL, "series pointer NULL or misaligned");
    if (nseries < 1 || nseries > p->max_series) return p->fail(FDAS_E_INVAL, "nseries out of range");
    if (nsamp < 8 || (nsamp & 1) || nsamp > p->max_nsamp)
        return p->fail(FDAS_E_INVAL, "nsamp odd, below 8 or above the plan's max_nsamp");
    if (!fft_length_supported(nsamp)) return p->fail(FDAS_E_UNSUPPORTED, "nsamp / 2 must be a product of powers of 2, 3 and 5 (at most 2^26)");
    if (!(dz > 0) || !std::isfinite(dz) || iters < 0 || iters > 10000 || n < 0 || n > 0x7fffffffLL ||
        (n > 0 && (!pts_host || !power_host)))
        return p->fail(FDAS_E_INVAL, "bad dz, iters or point arrays");
    if (n == 0) return FDAS_OK;
    int32_t max_m = 0;
    for (int64_t i = 0; i < n; ++i) {
        fdas_refine_point &q = pts_host[i];
        if (q.series < 0 || q.series >= nseries || !std::isfinite(q.r) || !std::isfinite(q.z) ||
            std::fabs(q.z) + 2.0 * dz > 8192.0 || q.r < 0.0 || q.r > (double)(nsamp / 2))
            return p->fail(FDAS_E_INVAL, "refinement start out of range (series, r in 0..nsamp/2, |z|)");
        if (fdas_refine_window(q.r, q.z, dz, p->opts.K, &q.k0, &q.m) != FDAS_OK)
            return p->fail(FDAS_E_INVAL, "refinement window too wide for this drift");
        max_m = std::max(max_m, q.m);
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n > p->rpts_cap) {
        TRY(grow(p, &p->d_rpts, &p->rpts_cap, n, "refinement points"));
        p->rpts_cap = 0;
        TRY(dalloc(p, &p->d_rpow, n, "refinement powers"));
        TRY(halloc(p, &p->h_rpts, n, "refinement points"));
        TRY(halloc(p, &p->h_rpow, n, "refinement powers"));
        p->rpts_cap = n;
    }
    std::memcpy(p->h_rpts, pts_host, (size_t)n * sizeof(fdas_refine_point));
    TRY(run_spectrum(p, series_dev, nullptr, nsamp, nseries, 0, st));
    HIPTRY(p, hipMemcpyAsync(p->d_rpts, p->h_rpts, n * sizeof(fdas_refine_point), hipMemcpyHostToDevice, st));
    hipEvent_t e = p->begin(st);
    HIPTRY(p, launch_refine_ascent(p->d_spec, p->spitch, nsamp / 2, nseries, p->d_scale, p->d_rpts, n, max_m, dz,
                                   iters, p->d_rpow, st));
    p->end(7, e, st);
    HIPTRY(p, hipMemcpyAsync(p->h_rpts, p->d_rpts, n * sizeof(fdas_refine_point), hipMemcpyDeviceToHost, st));
    HIPTRY(p, hipMemcpyAsync(p->h_rpow, p->d_rpow, n * sizeof(float), hipMemcpyDeviceToHost, st));
    HIPTRY(p, hipStreamSynchronize(st));
    p->collect();
    std::memcpy(pts_host, p->h_rpts, (size_t)n * sizeof(fdas_refine_point));
    std::memcpy(power_host, p->h_rpow, (size_t)n * sizeof(float));
    return FDAS_OK;
    FDAS_ENTRY_CATCH(plan_entry_error, p)
}

fdas_status fdas_plane(fdas_plan p, const float *series_dev, int64_t nsamp, int32_t nseries,
                       double tsamp, double zmax, double dz, float *plane_dev, int64_t plane_elems,
                       void *stream) {
    FDAS_ENTRY_TRY
    Geometry g;
    TRY(check_common(p, series_dev, nsamp, nseries, tsamp, zmax, dz, g));
    if (!plane_dev || ((uintptr_t)plane_dev & 7) || plane_elems < (int64_t)nseries * g.NZ * g.NR)
        return p->fail(FDAS_E_INVAL, "plane buffer NULL, misaligned or too small");
    const LaunchCfg c = default_cfg(p, g.Z, dz, 1);
    if (!c.L) return p->fail(FDAS_E_UNSUPPORTED, "zmax too large for the supported segment lengths");
    const Bank *bk = nullptr;
    TRY(get_bank(p, g.Z * dz, dz, c.L, &bk));
    hipStream_t st = static_cast<hipStream_t>(stream);
    TRY(run_spectrum(p, series_dev, nullptr, g.nsamp, nseries, 0, st));
    const CorrGeom cg = corr_geom(*bk, g);
    hipEvent_t e = p->begin(st);
    HIPTRY(p, launch_corr_power(p->d_spec, p->spitch, p->d_scale, bk->d, cg, nseries, plane_dev, g.NR,
                                (int64_t)g.NZ * g.NR, nullptr, 0, RowBlocks(), st));
    p->end(2, e, st);
    HIPTRY(p, hipStreamSynchronize(st));
    p->collect();
    return FDAS_OK;
    FDAS_ENTRY_CATCH(plan_entry_error, p)
}

fdas_status fdas_harmsum(fdas_plan p, const float *plane_dev, int64_t nsamp, int32_t nseries,
                         double tsamp, double zmax, double dz, int32_t numharm, double sigma,
                         fdas_cand *out_host, int64_t cap, int64_t *n_total, void *stream) {
    FDAS_ENTRY_TRY
    Geometry g;
    TRY(check_common(p, plane_dev, nsamp, nseries, tsamp, zmax, dz, g));
    TRY(check_search(p, numharm, sigma, out_host, cap, n_total));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t sstride = (int64_t)g.NZ * g.NR;
    const int NS = nstages_of(numharm);
    const int64_t mpitch = round_up(g.NR, 16);
    // block maxima of the caller's plane for the bounded sums (row blocks as a
    // single z group; results do not depend on the partition)
    RowBlocks rb;
    // maxima rows padded like the search's (a multiple of 32 halves)
    const bool mpair = maxima_per_bin(p->opts.harm_pair, numharm);
    const int32_t whole[2] = {0, g.NZ};
    TRY(get_rows(p, g.NZ, 1, whole, p->opts.harm_block ? p->opts.harm_block : default_block_rows(numharm),
                 numharm, mpair, mpair ? round_up(g.NR, 64) / 2 : round_up(g.NR, 64), rb));
    const int64_t psstride = (int64_t)rb.nblk * rb.ppitch;
    int64_t chunk = std::min<int64_t>(p->max_series, p->maxv_cap / (NS * mpitch));
    const bool bounded = !p->opts.harm_bound && bounded_table_bytes(rb.nblk, numharm) <= kBoundTableMax &&
                         psstride <= kMaxPyrSeriesStride && p->pyr_cap >= psstride;
    if (bounded) chunk = std::min<int64_t>(chunk, p->pyr_cap / psstride);
    if (chunk < 1) return p->fail(FDAS_E_INVAL, "one series exceeds the workspace");
    Batch B;
    B.groups.resize(1);
    B.groups[0].g = g;
    B.vmap.resize(nseries);
    for (int i = 0; i < nseries; ++i) B.vmap[i] = i;
    B.vgroup.assign(nseries, 0);
    B.vT.assign(nseries, g.T);
    for (int attempt = 0; attempt < 2; ++attempt) {
        TRY(upload_thresholds(p, numharm, sigma, st));
        HIPTRY(p, launch_zero_state(p->d_state, st));
        for (int b0 = 0; b0 < nseries; b0 += (int)chunk) {
            const int nb = (int)std::min<int64_t>(chunk, nseries - b0);
            const float *pl = plane_dev + (int64_t)b0 * sstride;
            hipEvent_t e = p->begin(st);
            if (bounded) {
                HIPTRY(p, launch_block_max(pl, g.NR, sstride, g.NR, rb, nb, p->d_pyr, psstride, st));
                HIPTRY(p, launch_harmsum_bounded(pl, g.NR, sstride, p->d_pyr, psstride, rb, g.NR, g.rlo, g.Z,
                                                 numharm, nb, p->d_thr, p->d_maxv, p->d_zarg, mpitch, st));
            } else {
                const int order = p->opts.harm_order ? p->opts.harm_order : 1;
                HIPTRY(p, launch_harmsum(pl, g.NR, sstride, g.NR, g.rlo, g.Z, numharm, nb, p->d_maxv, p->d_zarg,
                                         mpitch, order, st));
            }
            p->end(3, e, st);
            e = p->begin(st);
            HIPTRY(p, launch_compact(p->d_maxv, p->d_zarg, (int64_t)nb * NS * mpitch, mpitch, NS, b0, p->d_thr,
                                     p->d_counts, p->d_offsets, p->d_state, p->d_rec, p->rec_cap, st));
            p->end(4, e, st);
        }
        hipEvent_t e = p->begin(st);
        HIPTRY(p, launch_cand_sigma(p->d_rec, p->d_state, p->rec_cap, st));
        p->end(5, e, st);
        bool regrow = false;
        const fdas_status s = finish(p, B, dz, true, out_host, cap, n_total, st, &regrow);
        if (!regrow) return s;
        TRY(grow(p, &p->d_rec, &p->rec_cap, std::min<int64_t>(p->h_state[0], cap), "candidate records"));
    }
    return p->fail(FDAS_E_DEVICE, "internal error: candidate capacity did not converge");
    FDAS_ENTRY_CATCH(plan_entry_error, p)
}

fdas_status fdas_spectrum(fdas_plan p, const float *series_dev, int64_t nsamp, int32_t nseries,
                          float *spec_dev, double *norm_host, void *stream) {
    FDAS_ENTRY_TRY
    TRY(check_plan(p));
    if (!series_dev || ((uintptr_t)series_dev & 7) || !spec_dev || ((uintptr_t)spec_dev & 7))
        return p->fail(FDAS_E_INVAL, "device pointer NULL or not 8-byte aligned");
    if (nseries < 1 || nseries > p->max_series) return p->fail(FDAS_E_INVAL, "nseries out of range");
    if (nsamp < 8 || (nsamp & 1) || nsamp > p->max_nsamp)
        return p->fail(FDAS_E_INVAL, "nsamp odd, below 8 or above the plan's max_nsamp");
    if (!fft_length_supported(nsamp)) return p->fail(FDAS_E_UNSUPPORTED, "nsamp / 2 must be a product of powers of 2, 3 and 5 (at most 2^26)");
    Geometry g;
    g.nsamp = nsamp;
    g.half = nsamp / 2;
    hipStream_t st = static_cast<hipStream_t>(stream);
    TRY(run_spectrum(p, series_dev, nullptr, g.nsamp, nseries, 0, st));
    HIPTRY(p, hipMemcpy2DAsync(spec_dev, (size_t)(g.half + 1) * sizeof(float2), p->d_spec,
                               (size_t)p->spitch * sizeof(float2), (size_t)(g.half + 1) * sizeof(float2),
                               (size_t)nseries, hipMemcpyDeviceToDevice, st));
    if (norm_host) {
        if (p->opts.norm == FDAS_NORM_MEDIAN) {
            HIPTRY(p, hipMemcpyAsync(norm_host, p->d_norm, nseries * sizeof(double), hipMemcpyDeviceToHost, st));
        } else if (p->opts.norm == FDAS_NORM_LOCAL) {
            for (int b = 0; b < nseries; ++b) norm_host[b] = NAN;
        } else {
            for (int b = 0; b < nseries; ++b) norm_host[b] = (double)nsamp * p->opts.fixed_var;
        }
    }
    HIPTRY(p, hipStreamSynchronize(st));
    p->collect();
    return FDAS_OK;
    FDAS_ENTRY_CATCH(plan_entry_error, p)
}

fdas_status fdas_plan_get_info(fdas_plan p, fdas_plan_info *out) {
    if (!p || !out) return FDAS_E_INVAL;
    const Bank *first = p->banks.empty() ? nullptr : &p->banks.front();
    out->seg_len = p->last_L ? p->last_L : (first ? first->L : 0);
    out->mseg = p->last_L ? p->last_mseg : (first ? first->mseg : 0);
    out->nz = p->last_L ? p->last_NZ : (first ? first->NZ : 0);
    const int64_t per = (first ? first->NZ : 1) * round_up(p->max_nsamp, 64);
    out->chunk_series = (int32_t)std::min<int64_t>(p->max_series, p->plane_cap / per);
    out->workspace_bytes = p->plane_cap * (int64_t)sizeof(float);
    out->harm_blocks = p->last_harm_blocks;
    out->harm_pair = p->last_harm_pair;
    return FDAS_OK;
}

fdas_status fdas_tuning_export(fdas_plan p, char *buf, int64_t cap, int64_t *len) {
    FDAS_ENTRY_TRY
    if (!p || !len || cap < 0 || (cap > 0 && !buf)) return FDAS_E_INVAL;
    std::ostringstream os;
    for (auto &kv : p->tuned)
        os << std::get<0>(kv.first) << ' ' << std::get<1>(kv.first) << ' ' << std::get<2>(kv.first) << ' '
           << kv.second.L << ' ' << kv.second.bz << ' ' << (kv.second.pair ? 0 : 1) << '\n';
    const std::string s = os.str();
    *len = (int64_t)s.size();
    if (cap > 0) {
        const int64_t n = std::min<int64_t>(cap - 1, (int64_t)s.size());
        std::memcpy(buf, s.data(), (size_t)n);
        buf[n] = 0;
    }
    return (cap == 0 || cap > (int64_t)s.size()) ? FDAS_OK : FDAS_E_TRUNC;
    FDAS_ENTRY_CATCH(plan_entry_error, p)
}

fdas_status fdas_tuning_import(fdas_plan p, const char *text) {
    FDAS_ENTRY_TRY
    if (!p || !text) return FDAS_E_INVAL;
    std::istringstream is(text);
    std::string line;
    std::vector<std::pair<std::tuple<int64_t, int, int>, LaunchCfg>> add;
    while (std::getline(is, line)) {
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        std::istringstream ls(line);
        int64_t n = 0;
        int Z = -1, nh = 0, L = 0, bz = 0, harm_pair = -1;
        std::string rest;
        if (!(ls >> n >> Z >> nh >> L >> bz >> harm_pair) || (ls >> rest) || n < 8 || (n & 1) || Z < 0 ||
            !valid_numharm(nh) || !pow2(L) || L < 512 || L > 4096 || bz < 1 || bz > 64 ||
            (harm_pair != 0 && harm_pair != 1))
            return p->fail(FDAS_E_INVAL, "malformed tuning line: " + line);
        if (bz < p->min_bz)
            return p->fail(FDAS_E_INVAL, "tuning line with fewer drift rows per block than the plan's block-maxima "
                                         "buffer allows (" + std::to_string(p->min_bz) + "): " + line);
        LaunchCfg c;
        c.L = L;
        c.bz = bz;
        c.pair = harm_pair ? 0 : 1;
        add.emplace_back(std::make_tuple(n, Z, nh), c);
    }
    for (auto &kv : add) p->tuned[kv.first] = kv.second;
    drop_graph(p);
    return FDAS_OK;
    FDAS_ENTRY_CATCH(plan_entry_error, p)
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
