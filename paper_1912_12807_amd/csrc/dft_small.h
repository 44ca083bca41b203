// Register-resident complex helpers and small DFTs (radix 2 to 32, 3 and 5) for the
// FFT kernels. DIR = -1 computes X_k = sum_n v_n exp(-2 pi i n k / R),
// DIR = +1 the unnormalised inverse. Complex values are float2 (x = re, y = im).
#pragma once

#include <hip/hip_runtime.h>

namespace fdas {

// IEEE half bits of a half >= x for x >= 0: the nearest half, stepped up once
// when it lies below x (+inf above the largest finite half; NaN stays NaN), and
// never a subnormal (positive x below the smallest normal half gives that
// half), so the bound holds whether or not subnormals are flushed. Block
// maxima stored this way still bound every power of their block.
__device__ __forceinline__ uint16_t bound_half(float x) {
    const _Float16 h = (_Float16)x;                 // round to nearest even
    uint16_t u = __builtin_bit_cast(uint16_t, h);
    if ((float)h < x) ++u;                          // next half up (finite, non-negative)
    if (u < 0x0400u && x > 0.0f) u = 0x0400u;       // smallest normal half, 2^-14
    return u;
}
__device__ __forceinline__ float half_bits_to_float(uint16_t u) {
    return (float)__builtin_bit_cast(_Float16, u);
}

// 8-bit code of an upper bound of x >= 0: code c stands for
// (1 + (c mod 32) / 32) 2^(c / 32), i.e. 1 to 252 with five mantissa bits
// (the float whose bits are c << 18 above those of 1.0). x <= 1 gives 0 (1.0);
// above 1 the code is the float's top five mantissa bits, stepped up once
// when a lower bit is set, so code_value(bound_code(x)) >= x for x <= 252;
// larger values, +inf and NaN saturate at 255 (252). A bound built from such
// values still exceeds any threshold below 252 wherever the exact value does.
__device__ __forceinline__ uint32_t bound_code(float x) {
    // ceil((bits(x) - bits(1.0)) / 2^18), clamped to 0..255: negative (x < 1)
    // gives 0, +inf and NaN land far above 255
    const int32_t c = (int32_t)(__float_as_uint(x) - 0x3f7c0001u) >> 18;
    return (uint32_t)(c < 0 ? 0 : c > 255 ? 255 : c);
}
__device__ __forceinline__ float code_value(uint32_t c) { return __uint_as_float((c << 18) + 0x3f800000u); }
constexpr float kCodeMax = 252.0f;   // code_value(255)

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// Complex products with the fused multiply-adds written out, so that every
// kernel instance rounds them the same way whatever the compiler's contraction
// choices around them (results do not depend on launch options).
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(__fmaf_rn(a.x, b.x, -__fmul_rn(a.y, b.y)), __fmaf_rn(a.x, b.y, __fmul_rn(a.y, b.x)));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
    return make_float2(__fmaf_rn(a.x, b.x, __fmul_rn(a.y, b.y)), __fmaf_rn(a.y, b.x, -__fmul_rn(a.x, b.y)));
}
// a * (DIR i): DIR = +1 -> i a, DIR = -1 -> -i a
template <int DIR>
__device__ __forceinline__ float2 cmul_i(float2 a) {
    return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// twiddle with DIR applied to a twiddle stored for DIR = +1
template <int DIR>
__device__ __forceinline__ float2 ctw(float2 a, float2 w) {
    return DIR > 0 ? cmul(a, w) : cmulc(a, w);
}

template <int DIR>
__device__ __forceinline__ void dft2(float2 &a, float2 &b) {
    float2 t = a;
    a = cadd(t, b);
    b = csub(t, b);
}

// in-place 4-point DFT of (a0, a1, a2, a3)
template <int DIR>
__device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3) {
    float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
    float2 t2 = cadd(a1, a3), t3 = cmul_i<DIR>(csub(a1, a3));
    a0 = cadd(t0, t2);
    a2 = csub(t0, t2);
    a1 = cadd(t1, t3);
    a3 = csub(t1, t3);
}

// in-place 3-point DFT: with w = exp(DIR 2 pi i / 3) = -1/2 + DIR i sqrt(3)/2,
// X1 = a0 - (a1 + a2)/2 + DIR i sqrt(3)/2 (a1 - a2), X2 the conjugate combination
template <int DIR>
__device__ __forceinline__ void dft3(float2 *v) {
    constexpr float s = 0.86602540378443864676f * DIR;   // sin(2 pi / 3), signed
    const float2 t = cadd(v[1], v[2]);
    const float2 d = csub(v[1], v[2]);
    const float2 m = make_float2(__fmaf_rn(-0.5f, t.x, v[0].x), __fmaf_rn(-0.5f, t.y, v[0].y));
    const float2 r = make_float2(-s * d.y, s * d.x);       // DIR i sqrt(3)/2 (a1 - a2)
    v[0] = cadd(v[0], t);
    v[1] = cadd(m, r);
    v[2] = csub(m, r);
}

// in-place 5-point DFT: with c_k = cos(2 pi k / 5), s_k = DIR sin(2 pi k / 5),
// b1 = a1 + a4, b2 = a2 + a3, d1 = a1 - a4, d2 = a2 - a3:
// X1,4 = a0 + c1 b1 + c2 b2 +- i (s1 d1 + s2 d2), X2,3 = a0 + c2 b1 + c1 b2 +- i (s2 d1 - s1 d2)
template <int DIR>
__device__ __forceinline__ void dft5(float2 *v) {
    constexpr float c1 = 0.30901699437494742410f, c2 = -0.80901699437494742410f;
    constexpr float s1 = 0.95105651629515357212f * DIR, s2 = 0.58778525229247312917f * DIR;
    const float2 b1 = cadd(v[1], v[4]), b2 = cadd(v[2], v[3]);
    const float2 d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
    const float2 a0 = v[0];
    const float2 p1 = make_float2(__fmaf_rn(c2, b2.x, __fmaf_rn(c1, b1.x, a0.x)),
                                  __fmaf_rn(c2, b2.y, __fmaf_rn(c1, b1.y, a0.y)));
    const float2 p2 = make_float2(__fmaf_rn(c1, b2.x, __fmaf_rn(c2, b1.x, a0.x)),
                                  __fmaf_rn(c1, b2.y, __fmaf_rn(c2, b1.y, a0.y)));
    const float2 q1 = make_float2(__fmaf_rn(s2, d2.x, __fmul_rn(s1, d1.x)), __fmaf_rn(s2, d2.y, __fmul_rn(s1, d1.y)));
    const float2 q2 = make_float2(__fmaf_rn(-s1, d2.x, __fmul_rn(s2, d1.x)), __fmaf_rn(-s1, d2.y, __fmul_rn(s2, d1.y)));
    v[0] = cadd(a0, cadd(b1, b2));
    v[1] = make_float2(p1.x - q1.y, p1.y + q1.x);       // p1 + i q1
    v[4] = make_float2(p1.x + q1.y, p1.y - q1.x);       // p1 - i q1
    v[2] = make_float2(p2.x - q2.y, p2.y + q2.x);
    v[3] = make_float2(p2.x + q2.y, p2.y - q2.x);
}

// in-place 8-point DFT of v[0..7] (natural order in and out)
template <int DIR>
__device__ __forceinline__ void dft8(float2 *v) {
    constexpr float h = 0.70710678118654752440f;
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<DIR>(e0, e1, e2, e3);
    dft4<DIR>(o0, o1, o2, o3);
    // w8^k = exp(DIR 2 pi i k / 8)
    float2 w1 = make_float2(h * (o1.x - DIR * o1.y), h * (o1.y + DIR * o1.x));
    float2 w2 = cmul_i<DIR>(o2);
    float2 w3 = make_float2(h * (-o3.x - DIR * o3.y), h * (DIR * o3.x - o3.y));
    v[0] = cadd(e0, o0);
    v[4] = csub(e0, o0);
    v[1] = cadd(e1, w1);
    v[5] = csub(e1, w1);
    v[2] = cadd(e2, w2);
    v[6] = csub(e2, w2);
    v[3] = cadd(e3, w3);
    v[7] = csub(e3, w3);
}

// a * exp(DIR 2 pi i K / 32) for a compile-time K in [0, 16)
template <int K, int DIR>
__device__ __forceinline__ float2 rot32(float2 a) {
    if constexpr (K == 0) {
        return a;
    } else if constexpr (K == 8) {
        return cmul_i<DIR>(a);
    } else {
        // cos(m pi / 16), m = 0..8
        constexpr float T[9] = {1.0f,
                                0.980785280403230449126f,
                                0.923879532511286756128f,
                                0.831469612302545237079f,
                                0.707106781186547524401f,
                                0.555570233019602224743f,
                                0.382683432365089771728f,
                                0.195090322016128267848f,
                                0.0f};
        constexpr float c = K <= 8 ? T[K] : -T[16 - K];
        constexpr float s = K <= 8 ? T[8 - K] : T[K - 8];
        return cmul(a, make_float2(c, DIR * s));
    }
}

// radix-2 combination of the half-length DFTs e (even inputs) and o (odd):
// v[k] = e[k] + w^k o[k], v[k + H] = e[k] - w^k o[k], w = exp(DIR 2 pi i / (2 H))
template <int H, int DIR, int K = 0>
__device__ __forceinline__ void combine2(float2 *v, const float2 *e, const float2 *o) {
    if constexpr (K < H) {
        const float2 t = rot32<K * (16 / H), DIR>(o[K]);
        v[K] = cadd(e[K], t);
        v[K + H] = csub(e[K], t);
        combine2<H, DIR, K + 1>(v, e, o);
    }
}

// in-place 16- and 32-point DFTs (natural order in and out): even/odd split
// into two half-length DFTs and one radix-2 combination
template <int DIR>
__device__ __forceinline__ void dft16(float2 *v) {
    float2 e[8], o[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        e[i] = v[2 * i];
        o[i] = v[2 * i + 1];
    }
    dft8<DIR>(e);
    dft8<DIR>(o);
    combine2<8, DIR>(v, e, o);
}

template <int DIR>
__device__ __forceinline__ void dft32(float2 *v) {
    float2 e[16], o[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        e[i] = v[2 * i];
        o[i] = v[2 * i + 1];
    }
    dft16<DIR>(e);
    dft16<DIR>(o);
    combine2<16, DIR>(v, e, o);
}

template <int R, int DIR>
__device__ __forceinline__ void dft_r(float2 *v) {
    if constexpr (R == 2) {
        dft2<DIR>(v[0], v[1]);
    } else if constexpr (R == 3) {
        dft3<DIR>(v);
    } else if constexpr (R == 5) {
        dft5<DIR>(v);
    } else if constexpr (R == 4) {
        dft4<DIR>(v[0], v[1], v[2], v[3]);
    } else if constexpr (R == 8) {
        dft8<DIR>(v);
    } else if constexpr (R == 16) {
        dft16<DIR>(v);
    } else {
        static_assert(R == 32, "radix 2, 3, 4, 5, 8, 16 or 32");
        dft32<DIR>(v);
    }
}

// exp(i pi x) for x exactly representable (x = 2 k / n with integers k, n)
__device__ __forceinline__ float2 expipi(float x) {
    float s, c;
    sincospif(x, &s, &c);
    return make_float2(c, s);
}

}  // namespace fdas
