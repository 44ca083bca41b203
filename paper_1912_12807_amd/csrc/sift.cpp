// Host sifting of candidate lists (the paper's Section 2, step 5: the search
// results are sifted before folding). Candidate lists are small (KB-MB) and
// already on the host when a search returns, so this runs on the host:
//
//   order      sigma descending, then series, harm, r_idx ascending;
//   duplicates walking that order, a candidate whose fundamental frequency lies
//              within tol / min(T_a, T_b) Hz of an already kept candidate joins
//              the first such kept candidate, otherwise it is kept;
//   harmonics  walking the kept candidates in order, B is dropped when a
//              stronger surviving A has |f_B - rho f_A| <= rho tol / min(T_A, T_B)
//              with rho = n or 1/n, 2 <= n <= max_ratio.
// T = r_fund / f_hz is each candidate's observation length. Kept candidates sit
// in frequency-ordered maps, so each test looks only at the frequencies within
// the widest tolerance.
#include "fdas_internal.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <vector>

extern "C" fdas_status fdas_sift(const fdas_cand *c, int64_t n, double tol_bins, int32_t max_ratio,
                                 fdas_sifted *out, int64_t cap, int64_t *n_out) {
    FDAS_ENTRY_TRY
    if (n < 0 || (n > 0 && !c) || !(tol_bins >= 0) || !std::isfinite(tol_bins) || max_ratio < 1 ||
        max_ratio > 1024 || cap < 0 || (cap > 0 && !out) || !n_out)
        return FDAS_E_INVAL;
    double tmin = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        if (!(c[i].f_hz > 0) || !(c[i].r_fund > 0) || !std::isfinite(c[i].sigma))
            return FDAS_E_INVAL;
        tmin = std::min(tmin, c[i].r_fund / c[i].f_hz);
    }
    std::vector<int64_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
        if (c[a].sigma != c[b].sigma) return c[a].sigma > c[b].sigma;
        if (c[a].series != c[b].series) return c[a].series < c[b].series;
        if (c[a].harm != c[b].harm) return c[a].harm < c[b].harm;
        return c[a].r_idx < c[b].r_idx;
    });
    auto T = [&](int64_t i) { return c[i].r_fund / c[i].f_hz; };
    const double wmax = n ? tol_bins / tmin : 0.0;     // widest tolerance of any pair
    // duplicates
    std::vector<int64_t> kept;                          // kept, in order
    std::vector<int32_t> hits, lo, hi;
    std::multimap<double, int64_t> byf;                 // f -> position in kept
    for (int64_t i : order) {
        const double f = c[i].f_hz, Ti = T(i);
        int64_t home = -1;
        for (auto it = byf.lower_bound(f - wmax * (1 + 1e-12)); it != byf.end() && it->first <= f + wmax * (1 + 1e-12);
             ++it) {
            const int64_t j = kept[it->second];
            if (std::fabs(f - c[j].f_hz) <= tol_bins / std::min(Ti, T(j)) && (home < 0 || it->second < home))
                home = it->second;
        }
        if (home < 0) {
            byf.emplace(f, (int64_t)kept.size());
            kept.push_back(i);
            hits.push_back(1);
            lo.push_back(c[i].series);
            hi.push_back(c[i].series);
        } else {
            hits[home] += 1;
            lo[home] = std::min(lo[home], c[i].series);
            hi[home] = std::max(hi[home], c[i].series);
        }
    }
    // harmonics of stronger survivors
    std::vector<int64_t> alive;
    std::multimap<double, int64_t> alive_f;             // f -> kept position
    for (int64_t k = 0; k < (int64_t)kept.size(); ++k) {
        const int64_t b = kept[k];
        const double fb = c[b].f_hz, Tb = T(b);
        bool harmonic = false;
        for (int m = 2; m <= max_ratio && !harmonic; ++m) {
            for (int dir = 0; dir < 2 && !harmonic; ++dir) {
                // rho = m (f_A near f_B / m) or 1/m (f_A near m f_B)
                const double rho = dir == 0 ? (double)m / 1.0 : 1.0 / (double)m;
                const double centre = fb / rho;
                const double half = wmax * (1 + 1e-12) + 1e-300;
                for (auto it = alive_f.lower_bound(centre - half); it != alive_f.end() && it->first <= centre + half;
                     ++it) {
                    const int64_t a = kept[it->second];
                    const double tol = tol_bins / std::min(T(a), Tb);
                    if (std::fabs(fb - rho * c[a].f_hz) <= rho * tol) {
                        harmonic = true;
                        break;
                    }
                }
            }
        }
        if (!harmonic) {
            alive.push_back(k);
            alive_f.emplace(fb, k);
        }
    }
    *n_out = (int64_t)alive.size();
    const int64_t m = std::min<int64_t>(cap, (int64_t)alive.size());
    for (int64_t i = 0; i < m; ++i) {
        const int64_t k = alive[i];
        out[i].index = kept[k];
        out[i].hits = hits[k];
        out[i].series_lo = lo[k];
        out[i].series_hi = hi[k];
        out[i].reserved = 0;
    }
    return cap >= (int64_t)alive.size() ? FDAS_OK : FDAS_E_TRUNC;
    FDAS_ENTRY_CATCH(fdas::status_only, nullptr)
}
