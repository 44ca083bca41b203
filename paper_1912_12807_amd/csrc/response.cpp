// Host FP64 response of a linearly drifting sinusoid and the overlap-save
// template bank built from it.
//
// rho(q, z) = int_0^1 exp(2 pi i [q u + z (u^2 - u)/2]) du is the Fourier
// response, at offset q = r - k bins, of a sinusoid whose frequency drifts by
// z bins over the observation (r at mid-observation). Completing the square
// gives, for z > 0,
//   rho = exp(-i pi (q - z/2)^2 / z) / sqrt(2 z) * [F(Ye) - F(Ys)],
//   Y(e,s) = (q +- z/2) sqrt(2/z),  F(x) = C(x) + i S(x) = int_0^x exp(i pi t^2/2) dt,
// with rho(q, -z) = conj rho(-q, z) and rho(q, 0) = exp(i pi q) sinc(q).
//
// F is evaluated here by two published methods: composite Gauss-Legendre
// quadrature of its integral for |x| <= 4, and the asymptotic expansion in the
// auxiliary functions f, g of Abramowitz & Stegun 7.3.9-7.3.10 / 7.3.27-7.3.28
// above. Below |z| = 1e-3 the closed form loses digits, and rho is taken by
// Gauss-Legendre quadrature of its own defining integral.
#include "fdas_internal.h"

#include <cmath>
#include <complex>
#include <mutex>
#include <vector>

namespace fdas {

using cd = std::complex<double>;
static constexpr double kPi = 3.14159265358979323846264338327950288;

// ---------------------------------------------------------------- Gauss-Legendre nodes

struct GaussLegendre {
    std::vector<double> x, w;   // nodes/weights on [-1, 1]
    explicit GaussLegendre(int n) : x(n), w(n) {
        // Newton iteration on P_n from the Chebyshev-like initial guesses.
        for (int i = 0; i < (n + 1) / 2; ++i) {
            double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
            double dp = 0.0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= n; ++k) {
                    double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (z * p1 - p0) / (z * z - 1.0);
                double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) break;
            }
            {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= n; ++k) {
                    double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (z * p1 - p0) / (z * z - 1.0);
            }
            x[i] = -z;
            x[n - 1 - i] = z;
            w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

static const GaussLegendre &gl16() {
    static const GaussLegendre g(16);
    return g;
}

const GaussLegendre16 &gauss_legendre16() {
    static const GaussLegendre16 t = [] {
        GaussLegendre16 r;
        const GaussLegendre &g = gl16();
        for (int i = 0; i < 16; ++i) {
            r.x[i] = g.x[i];
            r.w[i] = g.w[i];
        }
        return r;
    }();
    return t;
}

// ---------------------------------------------------------------- Fresnel integral F(x)

// int_a^b exp(i pi t^2 / 2) dt by composite 16-point Gauss-Legendre, panels <= 0.25 wide.
static cd fresnel_quad(double a, double b) {
    const GaussLegendre &g = gl16();
    double len = b - a;
    int npan = (int)std::ceil(std::fabs(len) / 0.25);
    if (npan < 1) npan = 1;
    double h = len / npan;
    cd acc(0.0, 0.0);
    for (int p = 0; p < npan; ++p) {
        double a0 = a + p * h;
        cd s(0.0, 0.0);
        for (size_t i = 0; i < g.x.size(); ++i) {
            double t = a0 + 0.5 * h * (g.x[i] + 1.0);
            double ph = 0.5 * kPi * t * t;
            s += g.w[i] * cd(std::cos(ph), std::sin(ph));
        }
        acc += 0.5 * h * s;
    }
    return acc;
}

// F(x) for x >= 4 by the asymptotic expansion (A&S 7.3.9, 7.3.10, 7.3.27, 7.3.28):
// C = 1/2 + f sin(pi x^2/2) - g cos(pi x^2/2), S = 1/2 - f cos(pi x^2/2) - g sin(pi x^2/2),
// f ~ (1/(pi x)) sum_m (-1)^m (4m-1)!! / (pi x^2)^(2m),
// g ~ (1/(pi^2 x^3)) sum_m (-1)^m (4m+1)!! / (pi x^2)^(2m).
static cd fresnel_asym(double x) {
    double y = kPi * x * x;
    double y2 = y * y;
    double fs = 1.0, gs = 1.0;
    double tf = 1.0, tg = 1.0;
    for (int m = 1; m < 60; ++m) {
        double ntf = -tf * (4.0 * m - 3.0) * (4.0 * m - 1.0) / y2;   // (4m-1)!!/y^(2m)
        double ntg = -tg * (4.0 * m - 1.0) * (4.0 * m + 1.0) / y2;   // (4m+1)!!/y^(2m)
        if (std::fabs(ntf) > std::fabs(tf) || std::fabs(ntg) > std::fabs(tg)) break;
        tf = ntf;
        tg = ntg;
        fs += tf;
        gs += tg;
        if (std::fabs(tf) < 1e-18 && std::fabs(tg) < 1e-18) break;
    }
    double f = fs / (kPi * x);
    double g = gs / (kPi * kPi * x * x * x);
    double ph = 0.5 * y;
    double s = std::sin(ph), c = std::cos(ph);
    return cd(0.5 + f * s - g * c, 0.5 - f * c - g * s);
}

cd fresnel(double x) {
    double ax = std::fabs(x);
    cd v = (ax <= 4.0) ? fresnel_quad(0.0, ax) : fresnel_asym(ax);
    return x < 0 ? -v : v;
}

// ---------------------------------------------------------------- response rho(q, z)

static cd rho_quad(double q, double z) {
    const GaussLegendre &g = gl16();
    int npan = (int)std::ceil(kPi * (std::fabs(q) + std::fabs(z) / 2.0 + 1.0)) + 4;
    double h = 1.0 / npan;
    cd acc(0.0, 0.0);
    for (int p = 0; p < npan; ++p) {
        double a0 = p * h;
        cd s(0.0, 0.0);
        for (size_t i = 0; i < g.x.size(); ++i) {
            double u = a0 + 0.5 * h * (g.x[i] + 1.0);
            double ph = 2.0 * kPi * (q * u + z * (u * u - u) * 0.5);
            s += g.w[i] * cd(std::cos(ph), std::sin(ph));
        }
        acc += 0.5 * h * s;
    }
    return acc;
}

cd response(double q, double z) {
    if (z == 0.0) {
        if (q == 0.0) return cd(1.0, 0.0);
        // exp(i pi q) sin(pi q) / (pi q); sin(pi q) with exact reduction of q mod 2
        double r = std::fmod(q, 2.0);
        double s = std::sin(kPi * r);
        double c = std::cos(kPi * r);
        double sinc = s / (kPi * q);
        return cd(c * sinc, s * sinc);
    }
    if (z < 0.0) return std::conj(response(-q, -z));
    if (z < 1e-3) return rho_quad(q, z);
    double sc = std::sqrt(2.0 / z);
    double ye = (q + 0.5 * z) * sc;
    double ys = (q - 0.5 * z) * sc;
    cd d = fresnel(ye) - fresnel(ys);
    double a = q - 0.5 * z;
    double ph = -kPi * a * a / z;
    return cd(std::cos(ph), std::sin(ph)) * d / std::sqrt(2.0 * z);
}

int half_width(double z, int K) { return (int)std::ceil(std::fabs(z) / 2.0) + K; }

void unit_taps(double z, int parity, int K, std::vector<cd> &taps, int &d0) {
    int m = half_width(z, K);
    d0 = -m + parity;
    int n = m - d0 + 1;
    taps.resize(n);
    double e = 0.0;
    for (int i = 0; i < n; ++i) {
        int d = d0 + i;
        cd t = std::conj(response(0.5 * parity - d, z));
        taps[i] = t;
        e += std::norm(t);
    }
    double s = 1.0 / std::sqrt(e);
    for (auto &t : taps) t *= s;
}

// Spectrum of the circular correlation kernel for one (z, parity):
// T[f] = (1/L) sum_j g[j] exp(+2 pi i f j / L), g[mseg + d] = unit tap at offset d.
// Correlating a length-L segment s with g through a forward FFT of s, a
// product with T and an unnormalised inverse FFT yields
// c[i] = sum_d s[i + mseg + d] t_d for i < L - 2 mseg.
void kernel_spectrum(double z, int parity, int K, int L, int mseg, float *out_interleaved) {
    std::vector<cd> taps;
    int d0;
    unit_taps(z, parity, K, taps, d0);
    std::vector<cd> tw(L);
    for (int n = 0; n < L; ++n) {
        double a = 2.0 * kPi * (double)n / (double)L;
        tw[n] = cd(std::cos(a), std::sin(a));
    }
    const double inv_l = 1.0 / (double)L;
    for (int f = 0; f < L; ++f) {
        cd acc(0.0, 0.0);
        for (size_t i = 0; i < taps.size(); ++i) {
            long j = (long)mseg + d0 + (long)i;
            long idx = ((long)f * j) & (long)(L - 1);   // L is a power of two
            acc += taps[i] * tw[idx];
        }
        acc *= inv_l;
        out_interleaved[2 * f] = (float)acc.real();
        out_interleaved[2 * f + 1] = (float)acc.imag();
    }
}

}  // namespace fdas

extern "C" fdas_status fdas_template_taps(double z, int32_t parity, int32_t K, double *re,
                                          double *im, int32_t cap, int32_t *ntaps, int32_t *d0) {
    FDAS_ENTRY_TRY
    if (!ntaps || !d0 || (parity != 0 && parity != 1) || K < 0 || !std::isfinite(z))
        return FDAS_E_INVAL;
    std::vector<fdas::cd> taps;
    int dd0;
    fdas::unit_taps(z, parity, K, taps, dd0);
    *ntaps = (int32_t)taps.size();
    *d0 = dd0;
    if (!re || !im || cap < (int32_t)taps.size()) return FDAS_E_INVAL;
    for (size_t i = 0; i < taps.size(); ++i) {
        re[i] = taps[i].real();
        im[i] = taps[i].imag();
    }
    return FDAS_OK;
    FDAS_ENTRY_CATCH(fdas::status_only, nullptr)
}
