// K7/K8: candidate refinement at fractional (r, z), forward and backward.
//
// Objective of a point with window (k0, M) on normalised spectrum a_k = s A_k:
//   c(r, z) = sum_{k=k0-M}^{k0+M} a_k conj rho(r - k, z),   P = |c|^2,
//   rho(q, z) = int_0^1 exp(2 pi i theta(u)) du,  theta = q u + z (u^2 - u)/2,
// with a_k = 0 outside bins 1..nbins-1. Swapping the tap sum and the integral,
//   c = int_0^1 V(u) du,  V(u) = sum_j a_j exp(-2 pi i theta_j(u)),
//   theta_j(u) = theta_0(u) - j u   (tap j is bin k0 - M + j, q_j = r - k0 + M - j),
// and the derivatives follow under the integral:
//   dc/dr = int -2 pi i u V(u) du,  dc/dz = int -pi i (u^2 - u) V(u) du.
// The integral is taken by composite 16-point Gauss-Legendre quadrature, one
// panel per turn of the fastest phase (M + |r - k0| + |z|/2 + 1 panels). At a
// node, V is a polynomial in T = exp(2 pi i u): blocks of 16 taps are summed by
// Horner's rule in FP32 and multiplied by the block's phasor
// exp(-2 pi i (theta_0 - 16 b u)), whose phase is reduced in FP64 (the r ~ 1e6
// bins and large z of long series keep their fractional turns exact); the node
// sums accumulate in FP64. One wave evaluates one point; the lanes split the
// quadrature nodes.
//
// The ascent kernel iterates (r, z) += (eta_r dP/dr, eta_z dP/dz) / P, clamped
// to |r - r0| <= 1, |z - z0| <= 2 dz, inside the wave.
#include "fdas_internal.h"

namespace fdas {

static constexpr int kRefineWaves = 1;     // one wave per workgroup (window in LDS)
static constexpr double kTwoPi = 6.283185307179586476925286766559;
static constexpr double kPiD = 3.1415926535897932384626433832795;

struct RefineEval {
    double cr, ci;      // c
    double rr, ri;      // int u V du
    double zr, zi;      // int (u^2 - u) V du
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// exp(-2 pi i x) for x given in turns, reduced in FP64 and evaluated in FP32.
__device__ __forceinline__ float2 turns_neg(double x) {
    const double f = x - rint(x);
    float s, c;
    sincospif(-2.0f * (float)f, &s, &c);
    return make_float2(c, s);
}

// Window a_j = s A[k0 - M + j], j < taps (zero outside bins 1..nbins-1), padded
// with zeros to a multiple of 16.
__device__ void load_window(float2 *win, const float2 *row, float scale, int64_t nbins, int64_t k0, int M,
                            int taps16) {
    for (int j = threadIdx.x; j < taps16; j += 64) {
        const int64_t k = k0 - M + j;
        float2 v = make_float2(0.f, 0.f);
        if (j <= 2 * M && k >= 1 && k < nbins) {
            const float2 a = row[k];
            v = make_float2(a.x * scale, a.y * scale);
        }
        win[j] = v;
    }
    __syncthreads();
}

// Lane l always handles Gauss-Legendre node l mod 16 of a panel (64 lanes, 16
// nodes per panel): its node and weight, selected without dynamic indexing.
struct LaneNode {
    double x, w;
};
__device__ __forceinline__ LaneNode lane_node(const GaussLegendre16 &gl) {
    const int lg = threadIdx.x & 15;
    LaneNode n{0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        n.x = (k == lg) ? gl.x[k] : n.x;
        n.w = (k == lg) ? gl.w[k] : n.w;
    }
    return n;
}

__device__ RefineEval eval_point(const float2 *win, int M, int taps16, int64_t k0, double r, double z,
                                 const LaneNode &nd) {
    const double dk = r - (double)k0;
    const double q0 = dk + (double)M;
    const double zh = 0.5 * z;
    const int npan = (int)ceil((double)M + fabs(dk) + 0.5 * fabs(z) + 1.0);
    const double h = 1.0 / npan;
    const int nodes = 16 * npan;
    const int nblk = taps16 / 16;
    double ac_r = 0, ac_i = 0, ar_r = 0, ar_i = 0, az_r = 0, az_i = 0;
    for (int i = threadIdx.x; i < nodes; i += 64) {
        const int p = i >> 4;
        const double u = h * ((double)p + 0.5 * (nd.x + 1.0));
        const double w = 0.5 * h * nd.w;
        const double th0 = u * (q0 + zh * (u - 1.0));
        float ts, tc;
        sincospif(2.0f * (float)u, &ts, &tc);
        const float2 T = make_float2(tc, ts);
        float vr = 0.f, vi = 0.f;
        for (int b = 0; b < nblk; ++b) {
            const float2 *a = win + 16 * b;
            float hr = a[15].x, hi = a[15].y;
#pragma unroll
            for (int t = 14; t >= 0; --t) {
                const float nr = fmaf(hr, T.x, fmaf(-hi, T.y, a[t].x));
                const float ni = fmaf(hr, T.y, fmaf(hi, T.x, a[t].y));
                hr = nr;
                hi = ni;
            }
            const float2 B = turns_neg(th0 - 16.0 * b * u);
            vr = fmaf(B.x, hr, fmaf(-B.y, hi, vr));
            vi = fmaf(B.x, hi, fmaf(B.y, hr, vi));
        }
        const double wv_r = w * (double)vr, wv_i = w * (double)vi;
        const double uu = u * u - u;
        ac_r += wv_r;
        ac_i += wv_i;
        ar_r = fma(u, wv_r, ar_r);
        ar_i = fma(u, wv_i, ar_i);
        az_r = fma(uu, wv_r, az_r);
        az_i = fma(uu, wv_i, az_i);
    }
    RefineEval e;
    e.cr = wave_sum(ac_r);
    e.ci = wave_sum(ac_i);
    e.rr = wave_sum(ar_r);
    e.ri = wave_sum(ar_i);
    e.zr = wave_sum(az_r);
    e.zi = wave_sum(az_i);
    return e;
}

// P, dP/dr, dP/dz from the quadrature sums:
// dc/dr = -2 pi i int u V, dc/dz = -pi i int (u^2 - u) V, dP/dx = 2 Re(conj(c) dc/dx).
__device__ __forceinline__ void power_grad(const RefineEval &e, double &P, double &gr, double &gz) {
    P = e.cr * e.cr + e.ci * e.ci;
    // -i (x + i y) = y - i x
    const double drr = kTwoPi * e.ri, dri = -kTwoPi * e.rr;
    const double dzr = kPiD * e.zi, dzi = -kPiD * e.zr;
    gr = 2.0 * (e.cr * drr + e.ci * dri);
    gz = 2.0 * (e.cr * dzr + e.ci * dzi);
}

__device__ __forceinline__ bool point_ok(const fdas_refine_point &pt, int nseries, int max_m) {
    return pt.series >= 0 && pt.series < nseries && pt.m >= 0 && pt.m <= max_m && isfinite(pt.r) &&
           isfinite(pt.z) && fabs(pt.r - (double)pt.k0) <= 64.0 && fabs(pt.z) <= 8192.0;
}

__global__ __launch_bounds__(64) void k_refine_eval(const float2 *__restrict__ spec, int64_t spitch, int64_t nbins,
                                                    int nseries, const float *__restrict__ scale,
                                                    const fdas_refine_point *__restrict__ pts, int64_t n,
                                                    int max_m, GaussLegendre16 gl, float *__restrict__ power,
                                                    float *__restrict__ dpdr, float *__restrict__ dpdz) {
    extern __shared__ float2 win[];
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    const fdas_refine_point pt = pts[i];
    if (!point_ok(pt, nseries, max_m)) {
        if (threadIdx.x == 0) {
            power[i] = __builtin_nanf("");
            if (dpdr) dpdr[i] = __builtin_nanf("");
            if (dpdz) dpdz[i] = __builtin_nanf("");
        }
        return;
    }
    const int taps16 = (2 * pt.m + 1 + 15) & ~15;
    load_window(win, spec + (int64_t)pt.series * spitch, scale ? scale[pt.series] : 1.0f, nbins, pt.k0, pt.m,
                taps16);
    const RefineEval e = eval_point(win, pt.m, taps16, pt.k0, pt.r, pt.z, lane_node(gl));
    double P, gr, gz;
    power_grad(e, P, gr, gz);
    if (threadIdx.x == 0) {
        power[i] = (float)P;
        if (dpdr) dpdr[i] = (float)gr;
        if (dpdz) dpdz[i] = (float)gz;
    }
}

// Gradients: grad_r = g dP/dr, grad_z = g dP/dz and, if grad_spec is set,
// d(g P)/d A_k (as d/dRe + i d/dIm) = 2 g s c rho(r - k, z) added to grad_spec
// for every window bin in 1..nbins-1.
__global__ __launch_bounds__(64) void k_refine_grad(const float2 *__restrict__ spec, int64_t spitch, int64_t nbins,
                                                    int nseries, const float *__restrict__ scale,
                                                    const fdas_refine_point *__restrict__ pts, int64_t n,
                                                    int max_m, GaussLegendre16 gl,
                                                    const float *__restrict__ grad_power,
                                                    float *__restrict__ grad_r, float *__restrict__ grad_z,
                                                    float *__restrict__ grad_spec) {
    extern __shared__ float2 win[];
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    const fdas_refine_point pt = pts[i];
    if (!point_ok(pt, nseries, max_m)) {
        if (threadIdx.x == 0) {
            if (grad_r) grad_r[i] = __builtin_nanf("");
            if (grad_z) grad_z[i] = __builtin_nanf("");
        }
        return;
    }
    const float s = scale ? scale[pt.series] : 1.0f;
    const int taps16 = (2 * pt.m + 1 + 15) & ~15;
    const LaneNode ln = lane_node(gl);
    __shared__ double s_gx[16], s_gw[16];
    if (threadIdx.x < 16) {
        s_gx[threadIdx.x] = ln.x;
        s_gw[threadIdx.x] = ln.w;
    }
    load_window(win, spec + (int64_t)pt.series * spitch, s, nbins, pt.k0, pt.m, taps16);
    const RefineEval e = eval_point(win, pt.m, taps16, pt.k0, pt.r, pt.z, ln);
    double P, gr, gz;
    power_grad(e, P, gr, gz);
    const double g = (double)grad_power[i];
    if (threadIdx.x == 0) {
        if (grad_r) grad_r[i] = (float)(g * gr);
        if (grad_z) grad_z[i] = (float)(g * gz);
    }
    if (!grad_spec || g == 0.0) return;
    // rho_j = sum_n w_n exp(2 pi i theta_0(u_n)) exp(-2 pi i j u_n); lanes over taps
    const double dk = pt.r - (double)pt.k0;
    const double q0 = dk + (double)pt.m;
    const double zh = 0.5 * pt.z;
    const int npan = (int)ceil((double)pt.m + fabs(dk) + 0.5 * fabs(pt.z) + 1.0);
    const double h = 1.0 / npan;
    const int nodes = 16 * npan;
    const int taps = 2 * pt.m + 1;
    float *gs = grad_spec + 2 * (int64_t)pt.series * spitch;
    for (int j0 = 0; j0 < taps; j0 += 64) {
        const int j = j0 + (int)threadIdx.x;
        double rr = 0.0, ri = 0.0;
        for (int nd = 0; nd < nodes; ++nd) {
            const int p = nd >> 4, gi = nd & 15;
            const double u = h * ((double)p + 0.5 * (s_gx[gi] + 1.0));
            const double w = 0.5 * h * s_gw[gi];
            // exp(+2 pi i (theta_0 - j u)) = conj of turns_neg
            const float2 E = turns_neg(u * (q0 + zh * (u - 1.0)) - (double)j * u);
            rr = fma(w, (double)E.x, rr);
            ri = fma(w, -(double)E.y, ri);
        }
        const int64_t k = pt.k0 - pt.m + j;
        if (j < taps && k >= 1 && k < nbins) {
            // 2 g s c rho_j
            const double f = 2.0 * g * (double)s;
            atomicAdd(gs + 2 * k, (float)(f * (e.cr * rr - e.ci * ri)));
            atomicAdd(gs + 2 * k + 1, (float)(f * (e.cr * ri + e.ci * rr)));
        }
    }
}

// Ascent: iters steps from each point's (r, z) (the window stays at its k0, m),
// then the point's final (r, z) and power are written back.
__global__ __launch_bounds__(64) void k_refine_ascent(const float2 *__restrict__ spec, int64_t spitch,
                                                      int64_t nbins, int nseries, const float *__restrict__ scale,
                                                      fdas_refine_point *__restrict__ pts, int64_t n, int max_m,
                                                      GaussLegendre16 gl, double dz, int iters,
                                                      float *__restrict__ power) {
    extern __shared__ float2 win[];
    const int64_t i = blockIdx.x;
    if (i >= n) return;
    const fdas_refine_point pt = pts[i];
    if (!point_ok(pt, nseries, max_m)) {
        if (threadIdx.x == 0) power[i] = __builtin_nanf("");
        return;
    }
    const int taps16 = (2 * pt.m + 1 + 15) & ~15;
    load_window(win, spec + (int64_t)pt.series * spitch, scale ? scale[pt.series] : 1.0f, nbins, pt.k0, pt.m,
                taps16);
    const double eta_r = 3.0 / (2.0 * kPiD * kPiD), eta_z = 90.0 / (kPiD * kPiD);
    const LaneNode ln = lane_node(gl);
    double r = pt.r, z = pt.z;
    for (int it = 0; it < iters; ++it) {
        const RefineEval e = eval_point(win, pt.m, taps16, pt.k0, r, z, ln);
        double P, gr, gz;
        power_grad(e, P, gr, gz);
        if (!(P > 0.0)) break;
        r = fmin(fmax(r + eta_r * gr / P, pt.r - 1.0), pt.r + 1.0);
        z = fmin(fmax(z + eta_z * gz / P, pt.z - 2.0 * dz), pt.z + 2.0 * dz);
    }
    const RefineEval e = eval_point(win, pt.m, taps16, pt.k0, r, z, ln);
    double P, gr, gz;
    power_grad(e, P, gr, gz);
    if (threadIdx.x == 0) {
        pts[i].r = r;
        pts[i].z = z;
        power[i] = (float)P;
    }
}

static size_t window_bytes(int max_m) { return (size_t)((2 * max_m + 1 + 15) & ~15) * sizeof(float2); }

hipError_t launch_refine_eval(const float2 *spec, int64_t spitch, int64_t nbins, int nseries, const float *scale,
                              const fdas_refine_point *pts, int64_t n, int max_m, float *power, float *dpdr,
                              float *dpdz, hipStream_t st) {
    if (n < 1 || n > 0x7fffffffLL || max_m < 0 || max_m > kRefineMaxM) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_refine_eval, dim3((unsigned)n), dim3(64 * kRefineWaves), window_bytes(max_m), st, spec,
                       spitch, nbins, nseries, scale, pts, n, max_m, gauss_legendre16(), power, dpdr, dpdz);
    return hipGetLastError();
}

hipError_t launch_refine_grad(const float2 *spec, int64_t spitch, int64_t nbins, int nseries, const float *scale,
                              const fdas_refine_point *pts, int64_t n, int max_m, const float *grad_power,
                              float *grad_r, float *grad_z, float *grad_spec, hipStream_t st) {
    if (n < 1 || n > 0x7fffffffLL || max_m < 0 || max_m > kRefineMaxM) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_refine_grad, dim3((unsigned)n), dim3(64 * kRefineWaves), window_bytes(max_m), st, spec,
                       spitch, nbins, nseries, scale, pts, n, max_m, gauss_legendre16(), grad_power, grad_r, grad_z,
                       grad_spec);
    return hipGetLastError();
}

hipError_t launch_refine_ascent(const float2 *spec, int64_t spitch, int64_t nbins, int nseries, const float *scale,
                                fdas_refine_point *pts, int64_t n, int max_m, double dz, int iters, float *power,
                                hipStream_t st) {
    if (n < 1 || n > 0x7fffffffLL || max_m < 0 || max_m > kRefineMaxM || iters < 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_refine_ascent, dim3((unsigned)n), dim3(64 * kRefineWaves), window_bytes(max_m), st, spec,
                       spitch, nbins, nseries, scale, pts, n, max_m, gauss_legendre16(), dz, iters, power);
    return hipGetLastError();
}

}  // namespace fdas
