// Device helpers of libsf: the random stream and the binary32 decision
// contract (the arithmetic that decides which texel a sample reads).
//
// Everything here is compiled with FP contraction off; where the contract
// specifies a fused multiply-add it is written as __builtin_fmaf, so each
// decision is a fixed sequence of IEEE binary32 operations.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sf_internal.hpp"

#pragma clang fp contract(off)

namespace sfk {

enum { NEAREST = 0, LINEAR = 1, BSPLINE3 = 2, KEYS3 = 3, GAUSS_FRS = 4, GAUSS_FIS = 5, BSPLINE3_FIS = 6, EWA = 7,
       MITCHELL = 8 };
enum { BEFORE = 0, AFTER = 1, STOCH = 2, SPLIT = 3 };

// ---------------------------------------------------------------- random stream
// 4-D PCG hash (Jarzynski & Olano, "Hash Functions for GPU Rendering",
// JCGT 9(3) 2020): an LCG step on each word, a cross-multiplying mix, a
// 16-bit xorshift and a second mix, all modulo 2^32.
__device__ __forceinline__ uint4 pcg4d(uint4 v)
{
    v.x = v.x * 1664525u + 1013904223u;
    v.y = v.y * 1664525u + 1013904223u;
    v.z = v.z * 1664525u + 1013904223u;
    v.w = v.w * 1664525u + 1013904223u;
    v.x += v.y * v.w;
    v.y += v.z * v.x;
    v.z += v.x * v.y;
    v.w += v.y * v.z;
    v.x ^= v.x >> 16;
    v.y ^= v.y >> 16;
    v.z ^= v.z >> 16;
    v.w ^= v.w >> 16;
    v.x += v.y * v.w;
    v.y += v.z * v.x;
    v.z += v.x * v.y;
    v.w += v.y * v.z;
    return v;
}

// The same hash for a key whose words 0, 1 and 3 stay fixed while word 2
// (the step index) advances: the parts that depend only on the fixed words
// are computed once per (query, sample).  Returns the first three words.
struct StepHash {
    uint32_t x2;      // word 0 after the first mix and the xorshift
    uint32_t y0, w0;  // words 1 and 3 after the LCG step
    uint32_t x1;      // word 0 after the first mix
    __device__ __forceinline__ void init(uint32_t q, uint32_t s, uint32_t seed)
    {
        uint32_t x0 = q * 1664525u + 1013904223u;
        y0 = s * 1664525u + 1013904223u;
        w0 = seed * 1664525u + 1013904223u;
        x1 = x0 + y0 * w0;
        x2 = x1 ^ (x1 >> 16);
    }
    __device__ __forceinline__ uint3 at(uint32_t k) const
    {
        uint32_t z0 = k * 1664525u + 1013904223u;
        uint32_t y1 = y0 + z0 * x1;
        uint32_t z1 = z0 + x1 * y1;
        uint32_t w1 = w0 + y1 * z1;
        uint32_t y2 = y1 ^ (y1 >> 16);
        uint32_t z2 = z1 ^ (z1 >> 16);
        uint32_t w2 = w1 ^ (w1 >> 16);
        uint32_t x3 = x2 + y2 * w2;
        uint32_t y3 = y2 + z2 * x3;
        uint32_t z3 = z2 + x3 * y3;
        return make_uint3(x3, y3, z3);
    }
};

// 24-bit uniform in [0, 1), exact in binary32.
__device__ __forceinline__ float u24(uint32_t w) { return (float)(w >> 8) * 0x1p-24f; }

// ----------------------------------------------------------- decision contract
// Running sums of the cubic B-spline weights on taps i0-1..i0+2 for the
// fraction t (Suppl. S.2 eq. cubic-bspline, factored):
//   C0 = ((s*s)*s)/6, s = 1 - t;  C1 = C0 + (2/3 - t^2 (1 - t/2));
//   C2 = 1 - ((t*t)*t)/6.
struct Thr3 {
    float c0, c1, c2;
};
__device__ __forceinline__ Thr3 bspline_thresholds(float t)
{
    const float k6 = 1.0f / 6.0f, k23 = 2.0f / 3.0f;
    float s = 1.0f - t;
    float w0 = ((s * s) * s) * k6;
    float t2 = t * t;
    float half = __builtin_fmaf(-0.5f, t, 1.0f);
    float w1 = __builtin_fmaf(-t2, half, k23);
    float w3 = (t2 * t) * k6;
    Thr3 c;
    c.c0 = w0;
    c.c1 = w0 + w1;
    c.c2 = 1.0f - w3;
    return c;
}

// The cubic B-spline thresholds times 2^24.  Every operand of the binary32
// contract is scaled by a power of two, so each rounded result is exactly
// 2^24 times the unscaled one, and [u >= C] == [(float)(w >> 8) >= 2^24 C]
// for u = (w >> 8) 2^-24: the same decisions without converting the word
// into [0, 1).
__device__ __forceinline__ Thr3 bspline_thresholds_2p24(float t)
{
    const float k6 = (1.0f / 6.0f) * 16777216.0f, k23 = (2.0f / 3.0f) * 16777216.0f;
    const float s = 1.0f - t;
    const float t2 = t * t;
    const float w0 = ((s * s) * s) * k6;
    const float half = __builtin_fmaf(-8388608.0f, t, 16777216.0f);
    const float w1 = __builtin_fmaf(-t2, half, k23);
    const float w3 = (t2 * t) * k6;
    Thr3 c;
    c.c0 = w0;
    c.c1 = w0 + w1;
    c.c2 = 16777216.0f - w3;
    return c;
}

// The word's 24-bit lattice index as a float (exact).
__device__ __forceinline__ float u24i(uint32_t w) { return (float)(w >> 8); }

// Tap offset relative to i0 picked by uniform u (ties advance).
template <int F>
__device__ __forceinline__ int pick_off(float t, float u)
{
    if constexpr (F == BSPLINE3) {
        Thr3 c = bspline_thresholds(t);
        return -1 + (u >= c.c0) + (u >= c.c1) + (u >= c.c2);
    } else if constexpr (F == LINEAR) {
        return (u >= 1.0f - t) ? 1 : 0;
    } else {
        return (t >= 0.5f) ? 1 : 0;
    }
}

// pick_off on the lattice index ui = w >> 8 of the uniform's word, against
// thresholds scaled by 2^24 (identical decisions, one multiply fewer per axis).
template <int F>
__device__ __forceinline__ int pick_off_2p24(float t, float ui)
{
    if constexpr (F == BSPLINE3) {
        const Thr3 c = bspline_thresholds_2p24(t);
        return -1 + (ui >= c.c0) + (ui >= c.c1) + (ui >= c.c2);
    } else if constexpr (F == LINEAR) {
        return ui >= __builtin_fmaf(-16777216.0f, t, 16777216.0f) ? 1 : 0;
    } else {
        return (t >= 0.5f) ? 1 : 0;
    }
}

// Pick and re-derive the uniform inside the picked bin (uniform sample reuse).
template <int F>
__device__ __forceinline__ int pick_off_reuse(float t, float &u)
{
    const float top = 0x1.fffffep-1f;
    if constexpr (F == BSPLINE3) {
        Thr3 c = bspline_thresholds(t);
        int j = (u >= c.c0) + (u >= c.c1) + (u >= c.c2);
        float lo = j == 0 ? 0.0f : (j == 1 ? c.c0 : (j == 2 ? c.c1 : c.c2));
        float hi = j == 0 ? c.c0 : (j == 1 ? c.c1 : (j == 2 ? c.c2 : 1.0f));
        float r = (u - lo) / (hi - lo);
        u = r > top ? top : r;
        return j - 1;
    } else if constexpr (F == LINEAR) {
        float c0 = 1.0f - t;
        int j = u >= c0;
        float lo = j ? c0 : 0.0f, hi = j ? 1.0f : c0;
        float r = (u - lo) / (hi - lo);
        u = r > top ? top : r;
        return j;
    } else {
        return (t >= 0.5f) ? 1 : 0;
    }
}

// ---------------------------------------------------------------- Gaussian / FIS contract
// The Gaussian samplers decide texels through ln, exp, cos and sin.  These
// are fixed sequences of correctly rounded binary32 operations (+ - * /,
// sqrt, fma, floor, frexp, ldexp), so the decisions are reproducible bit for
// bit on any IEEE machine; their accuracy (a few ulp) is checked against
// libm on the CPU.
constexpr float LN2_HI = 0x1.62e4p-1f;    // ln 2 to 17 bits: n * LN2_HI exact for |n| < 128
constexpr float LN2_LO = 1.42860677e-6f;  // ln 2 - LN2_HI

// ln x, x in (0, 1]: x = m 2^e, m in [sqrt(1/2), sqrt(2)); ln m = 2 atanh(s),
// s = (m-1)/(m+1), series 2s(1 + z/3 + z^2/5 + z^3/7 + z^4/9), z = s^2;
// e ln 2 added in two parts (Cody & Waite).
__device__ __forceinline__ float lnc(float x)
{
    int e;
    float m = __builtin_frexpf(x, &e);
    if (m < 0.70710678f) {
        m = m * 2.0f;
        e = e - 1;
    }
    const float s = (m - 1.0f) / (m + 1.0f);
    const float z = s * s;
    float p = __builtin_fmaf(z, 1.0f / 9.0f, 1.0f / 7.0f);
    p = __builtin_fmaf(z, p, 1.0f / 5.0f);
    p = __builtin_fmaf(z, p, 1.0f / 3.0f);
    p = __builtin_fmaf(z, p, 1.0f);
    const float r = (2.0f * s) * p;
    const float fe = (float)e;
    return __builtin_fmaf(fe, LN2_HI, __builtin_fmaf(fe, LN2_LO, r));
}

// log2 x for positive normal x: the same reduction and series, then
// e + ln(m) log2(e); -inf below 2^-126 (and for NaN), +inf for +inf.
__device__ __forceinline__ float log2c(float x)
{
    if (!(x >= 0x1p-126f))
        return -__builtin_inff();
    if (x == __builtin_inff())
        return x;
    int e;
    float m = __builtin_frexpf(x, &e);
    if (m < 0.70710678f) {
        m = m * 2.0f;
        e = e - 1;
    }
    const float s = (m - 1.0f) / (m + 1.0f);
    const float z = s * s;
    float p = __builtin_fmaf(z, 1.0f / 9.0f, 1.0f / 7.0f);
    p = __builtin_fmaf(z, p, 1.0f / 5.0f);
    p = __builtin_fmaf(z, p, 1.0f / 3.0f);
    p = __builtin_fmaf(z, p, 1.0f);
    const float r = (2.0f * s) * p;
    return __builtin_fmaf(r, 1.44269504f, (float)e);
}

// e^x, x in [-80, 0] (0 below): n = floor(x log2 e + 1/2), r = x - n ln 2
// (two parts), Taylor polynomial of e^r to r^7, scaled by 2^n.
__device__ __forceinline__ float expc(float x)
{
    if (!(x >= -80.0f))
        return 0.0f;
    const float n = __builtin_floorf(__builtin_fmaf(x, 1.44269504f, 0.5f));
    float r = __builtin_fmaf(-n, LN2_HI, x);
    r = __builtin_fmaf(-n, LN2_LO, r);
    float p = __builtin_fmaf(r, 1.0f / 5040.0f, 1.0f / 720.0f);
    p = __builtin_fmaf(r, p, 1.0f / 120.0f);
    p = __builtin_fmaf(r, p, 1.0f / 24.0f);
    p = __builtin_fmaf(r, p, 1.0f / 6.0f);
    p = __builtin_fmaf(r, p, 0.5f);
    p = __builtin_fmaf(r, p, 1.0f);
    p = __builtin_fmaf(r, p, 1.0f);
    return __builtin_ldexpf(p, (int)n);
}

// cos and sin of 2 pi v, v in [0, 1): quadrant from 4v (exact), the rest
// folded to x in [0, pi/4]; Taylor to x^9 (sin) and x^10 (cos).
__device__ __forceinline__ void sincos2pi(float v, float &c, float &s)
{
    const float a = 4.0f * v;
    const float qf = __builtin_floorf(a);
    const float f = a - qf;
    const int q = (int)qf & 3;
    const bool fold = f > 0.5f;
    const float h = fold ? 1.0f - f : f;
    const float x = h * 1.57079637f;
    const float z = x * x;
    float sp = __builtin_fmaf(z, 1.0f / 362880.0f, -1.0f / 5040.0f);
    sp = __builtin_fmaf(z, sp, 1.0f / 120.0f);
    sp = __builtin_fmaf(z, sp, -1.0f / 6.0f);
    sp = __builtin_fmaf(z, sp, 1.0f);
    const float sn = x * sp;
    float cp = __builtin_fmaf(z, -1.0f / 3628800.0f, 1.0f / 40320.0f);
    cp = __builtin_fmaf(z, cp, -1.0f / 720.0f);
    cp = __builtin_fmaf(z, cp, 1.0f / 24.0f);
    cp = __builtin_fmaf(z, cp, -0.5f);
    const float cs = __builtin_fmaf(z, cp, 1.0f);
    const float c0 = fold ? sn : cs, s0 = fold ? cs : sn;
    c = q == 0 ? c0 : (q == 1 ? -s0 : (q == 2 ? -c0 : s0));
    s = q == 0 ? s0 : (q == 1 ? c0 : (q == 2 ? -s0 : -c0));
}

// Discrete Gaussian on taps i0-1..i0+2 (FRS, Sec. 4.1): weights
// exp(min a - a_k), a_k = (d d) h, d = (k-1) - t, h = 1/(2 sigma^2); running
// sums divided by their total.  Returns the tap offset (-1..2) for u.
__device__ __forceinline__ int gauss_frs_pick(float t, float h, float u)
{
    float a[4], g[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float d = (float)(k - 1) - t;
        a[k] = (d * d) * h;
    }
    const float amin = __builtin_fminf(__builtin_fminf(a[0], a[1]), __builtin_fminf(a[2], a[3]));
#pragma unroll
    for (int k = 0; k < 4; ++k)
        g[k] = expc(amin - a[k]);
    const float s1 = g[0] + g[1], s2 = s1 + g[2], W = s2 + g[3];
    return -1 + (u >= g[0] / W) + (u >= s1 / W) + (u >= s2 / W);
}

// Gaussian FIS: Box-Muller radius sigma sqrt(-2 ln(1 - u0)), angle 2 pi u1,
// then the nearest texel: offset floor((t + 1/2) + d) per axis.
__device__ __forceinline__ void gauss_fis_pick(float tx, float ty, float sigma, float u0, float u1, int &ox,
                                               int &oy)
{
    const float r = sigma * __builtin_sqrtf(-2.0f * lnc(1.0f - u0));
    float c, s;
    sincos2pi(u1, c, s);
    ox = (int)__builtin_floorf((tx + 0.5f) + r * c);
    oy = (int)__builtin_floorf((ty + 0.5f) + r * s);
}

// Cubic B-spline by FIS: the nearest texel after the offset
// xi1 + xi2 + xi3 - 3/2; with S = a + b + c (24-bit words) = 2^24 q + r the
// offset is q - 1 + [r 2^-24 >= 1 - t].
__device__ __forceinline__ int bspline_fis_pick(float t, uint32_t a, uint32_t b, uint32_t c)
{
    const uint32_t S = (a >> 8) + (b >> 8) + (c >> 8);
    const float r = (float)(S & 0xffffffu) * 0x1p-24f;
    return (int)(S >> 24) - 1 + (r >= 1.0f - t);
}

// Interpolating Keys cubic (S.2's K3, a = -1/2) on taps i0-1..i0+2, split
// into its positive pair (p1, p2) and negative pair (-m0, -m3), factored:
// m0 = t s^2/2, m3 = s t^2/2, p1 = 1 - 5t^2/2 + 3t^3/2, p2 likewise in s = 1-t.
struct KeysAxis {
    float m0, m3, Pm, p1, p2, Pp;
};
__device__ __forceinline__ KeysAxis keys_axis(float t)
{
    KeysAxis k;
    const float s = 1.0f - t;
    k.m0 = (0.5f * t) * (s * s);
    k.m3 = (0.5f * s) * (t * t);
    k.Pm = k.m0 + k.m3;
    k.p1 = __builtin_fmaf(t * t, __builtin_fmaf(1.5f, t, -2.5f), 1.0f);
    k.p2 = __builtin_fmaf(s * s, __builtin_fmaf(1.5f, s, -2.5f), 1.0f);
    k.Pp = k.p1 + k.p2;
    return k;
}

// Mitchell-Netravali cubic (B = C = 1/3) on taps i0-1..i0+2, factored
// binary32 weights, s = 1-t: w0 = ((s s) fma(-7, t, 1))/18 (positive for
// t < 1/7), w1 = fma(t t, fma(7/6, t, -2), 8/9), w2 likewise in s,
// w3 = ((t t) fma(7, t, -6))/18 (positive for t > 6/7).  Positivisation
// sorts each tap into the positive or negative set by the sign of its
// binary32 weight; P+ and P- sum |w| in tap order.
struct PnAxis {
    float w[4], Pp, Pm;
};
__device__ __forceinline__ PnAxis mitchell_axis(float t)
{
    const float K18 = 1.0f / 18.0f, K76 = 7.0f / 6.0f, K89 = 8.0f / 9.0f;
    PnAxis a;
    const float s = 1.0f - t;
    a.w[0] = ((s * s) * __builtin_fmaf(-7.0f, t, 1.0f)) * K18;
    a.w[1] = __builtin_fmaf(t * t, __builtin_fmaf(K76, t, -2.0f), K89);
    a.w[2] = __builtin_fmaf(s * s, __builtin_fmaf(K76, s, -2.0f), K89);
    a.w[3] = ((t * t) * __builtin_fmaf(7.0f, t, -6.0f)) * K18;
    a.Pp = 0.0f;
    a.Pm = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        a.Pp = a.w[k] > 0.0f ? a.Pp + a.w[k] : a.Pp;
        a.Pm = a.w[k] < 0.0f ? a.Pm + (-a.w[k]) : a.Pm;
    }
    return a;
}

// Tap (0..3) of the positive (pos) or negative set: the first whose running
// sum c of |w| (tap order) satisfies u P < c, else the set's last tap.
__device__ __forceinline__ int pn_pick(const PnAxis &a, bool pos, float u)
{
    const float uP = u * (pos ? a.Pp : a.Pm);
    float c = 0.0f;
    int pick = -1;
    bool done = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float m = pos ? a.w[k] : -a.w[k];
        if (m > 0.0f && !done) {
            c = c + m;
            pick = k;
            done = uP < c;
        }
    }
    return pick;
}

// Weights of the taps (value path, binary32), same tap order as pick_off.
template <int F>
__device__ __forceinline__ void axis_weights(float t, float w[4])
{
    if constexpr (F == BSPLINE3) {
        const float k6 = 1.0f / 6.0f, k23 = 2.0f / 3.0f;
        float s = 1.0f - t;
        float t2 = t * t, s2 = s * s;
        w[0] = (s2 * s) * k6;
        w[1] = __builtin_fmaf(-t2, __builtin_fmaf(-0.5f, t, 1.0f), k23);
        w[2] = __builtin_fmaf(-s2, __builtin_fmaf(-0.5f, s, 1.0f), k23);
        w[3] = (t2 * t) * k6;
    } else if constexpr (F == LINEAR) {
        w[0] = 1.0f - t;
        w[1] = t;
    } else if constexpr (F == KEYS3) {
        const KeysAxis k = keys_axis(t);
        w[0] = -k.m0;
        w[1] = k.p1;
        w[2] = k.p2;
        w[3] = -k.m3;
    } else if constexpr (F == MITCHELL) {
        const PnAxis a = mitchell_axis(t);
        w[0] = a.w[0];
        w[1] = a.w[1];
        w[2] = a.w[2];
        w[3] = a.w[3];
    } else {
        w[0] = 1.0f;
    }
}

// Compensated summation in binary32 (contraction is off in every source and
// nothing reassociates): the running sum s is the plain binary32 sum, and the
// exact rounding error of every addition, found by Knuth's TwoSum (six
// operations, no branch, any signs), is accumulated in c.  s + c is then as
// accurate as a sum in twice the working precision: within
// u |sum| + gamma_{n-1}^2 sum |x_i| of the exact sum, u = 2^-24,
// gamma_k = k u / (1 - k u) (Ogita, Rump and Oishi, "Accurate sum and dot
// product", SIAM J. Sci. Comput. 26(6), 2005, algorithm Sum2).  Adding an
// exact zero changes neither s nor c, so a sum that skips zero terms is
// bit-identical to one that adds them.
struct CompSum {
    float s, c;
    __device__ __forceinline__ void init()
    {
        s = 0.0f;
        c = 0.0f;
    }
    __device__ __forceinline__ void add(float x)
    {
        const float t = s + x;
        const float bp = t - s;
        const float e = (s - (t - bp)) + (x - bp);
        s = t;
        c = c + e;
    }
    __device__ __forceinline__ float value() const { return s + c; }
};

// A product of positive factors kept as an unevaluated binary32 pair
// hi + lo: each multiplication keeps its rounding error through one fma (the
// error-free product of Dekker, as in Ogita, Rump and Oishi), so the pair
// carries about 44 significant bits and the relative error after n factors
// is O(n u^2) on top of what the factors bring in.  A factor is passed as a
// pair too: a transmittance close to 1 is best known as 1 - a with a
// accurate to a few ulp of a (not of 1), and mul_one_minus splits it
// exactly (Dekker's Fast2Sum, |1| >= |a|); a factor far from 1 is best known
// directly and is passed as (f, 0).  Multiplying by exactly 1 changes nothing.
struct PairProduct {
    float hi, lo;
    __device__ __forceinline__ void init()
    {
        hi = 1.0f;
        lo = 0.0f;
    }
    __device__ __forceinline__ void mul(float fh, float fl)
    {
        const float p = hi * fh;
        float e = __builtin_fmaf(hi, fh, -p);
        e = __builtin_fmaf(hi, fl, e);
        e = __builtin_fmaf(lo, fh, e);
        const float s = p + e;
        lo = e - (s - p);
        hi = s;
    }
    __device__ __forceinline__ void mul_one_minus(float a)
    {
        const float fh = 1.0f - a;
        mul(fh, (1.0f - fh) - a);
    }
    __device__ __forceinline__ float value() const { return hi + lo; }
};

// e = e^(-x) and m = 1 - e^(-x), each with a small relative error: e on the
// transcendental unit (2^(-x log2 e)); m for |x| < 1/4 by the degree-7 Taylor
// polynomial (first omitted term below 2e-9 of the value), otherwise as
// 1 - e, whose 1-ulp error stays below 4 ulp of the difference there
// (e <= 0.78 for x >= 1/4).
__device__ __forceinline__ void exp_neg_pair(float x, float &e, float &m)
{
    float p = __builtin_fmaf(x, 1.0f / 5040.0f, -1.0f / 720.0f);
    p = __builtin_fmaf(x, p, 1.0f / 120.0f);
    p = __builtin_fmaf(x, p, -1.0f / 24.0f);
    p = __builtin_fmaf(x, p, 1.0f / 6.0f);
    p = __builtin_fmaf(x, p, -0.5f);
    p = __builtin_fmaf(x, p, 1.0f);
    e = __builtin_amdgcn_exp2f(x * -1.44269504088896341f);
    m = __builtin_fabsf(x) < 0.25f ? x * p : 1.0f - e;
}

template <int F>
struct Taps {
    static constexpr int n = (F == BSPLINE3 || F == KEYS3 || F == GAUSS_FRS || F == MITCHELL) ? 4 : (F == LINEAR ? 2 : 1);
    static constexpr int first = (F == BSPLINE3 || F == KEYS3 || F == GAUSS_FRS || F == MITCHELL) ? -1 : 0;
};

// Workgroups are dispatched round-robin over the 8 XCDs of the chip; map the
// hardware block index to a logical one so that consecutive logical blocks
// (neighbouring tiles of the query stream) land on the same XCD and share
// its L2.  nb_pad must be a multiple of 8; logical indices >= the real block
// count are idle.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nb_pad)
{
    return (b & 7u) * (nb_pad >> 3) + (b >> 3);
}

// ------------------------------------------------------------ ray geometry
// Per-ray constants of the step contract: dt = (t1-t0)/S; raster origin
// A = fma(o - wmin, scale, -0.5), direction B = d*scale, entry E = fma(t0, B, A),
// step G = dt*B; step k sits at fma(k + 1/2, G, E).
struct RayGeom {
    float E[3], G[3], dt;
};

// 0: march; 1: empty segment (T = 1); 2: invalid input (T = NaN).
__device__ __forceinline__ int ray_setup_dev(const float *wmin, const float *scale, const float *r8, int steps,
                                             RayGeom &g)
{
    const float4 a = *reinterpret_cast<const float4 *>(r8);
    const float4 b = *reinterpret_cast<const float4 *>(r8 + 4);
    const float r[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
    bool fin = true;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        fin &= __builtin_isfinite(r[k]);
    if (!fin)
        return 2;
    if (!(r[7] > r[6]))
        return 1;
    g.dt = (r[7] - r[6]) / (float)steps;
    bool ok = true;
    const float last = (float)(steps - 1) + 0.5f;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float A = __builtin_fmaf(r[k] - wmin[k], scale[k], -0.5f);
        const float B = r[3 + k] * scale[k];
        g.E[k] = __builtin_fmaf(r[6], B, A);
        g.G[k] = g.dt * B;
        const float pa = __builtin_fmaf(0.5f, g.G[k], g.E[k]);
        const float pb = __builtin_fmaf(last, g.G[k], g.E[k]);
        ok &= (__builtin_fabsf(pa) <= 4194304.0f) & (__builtin_fabsf(pb) <= 4194304.0f);
    }
    return ok ? 0 : 2;
}

// ----------------------------------------------------------------- shading
// GGX + Lambert times the cosine for the fixed directions folded into g
// (the texel supplies albedo RGB and the roughness parameter A).
// With G1(c) = 2c / (c + sqrt(a^2 + (1 - a^2) c^2)) the specular term
// D G1(no) G1(ni) F / (4 no ni) is a^2 (F/pi) / ((no + s_o)(ni + s_i) d^2):
// one reciprocal.  Shaded values decide nothing, so the hardware reciprocal
// and square root (about 1 ulp each) serve; the result is within a few ulp.
__device__ __forceinline__ float3 shade_ggx_dev(const GgxConst &g, float4 c)
{
    const float r = __builtin_fmaf(g.r_scale, c.w, g.r_bias);
    const float a = r * r;
    const float a2 = a * a;
    const float d = __builtin_fmaf(g.nh2, a2 - 1.0f, 1.0f);
    const float om = 1.0f - a2;
    const float so = __builtin_amdgcn_sqrtf(__builtin_fmaf(om, g.no2, a2));
    const float si = __builtin_amdgcn_sqrtf(__builtin_fmaf(om, g.ni2, a2));
    const float den = ((g.no + so) * (g.ni + si)) * (d * d);
    const float spec = (a2 * g.spec_c) * __builtin_amdgcn_rcpf(den);
    return make_float3(__builtin_fmaf(g.kd[0], c.x, g.ks[0] * spec), __builtin_fmaf(g.kd[1], c.y, g.ks[1] * spec),
                       __builtin_fmaf(g.kd[2], c.z, g.ks[2] * spec));
}

// a b - c d within about 1.5 ulp (Kahan's algorithm: the rounding error of
// c d, recovered by an fma, is added back).
__device__ __forceinline__ float diff_prod(float a, float b, float c, float d)
{
    const float w = c * d;
    const float e = __builtin_fmaf(-c, d, w);
    const float f = __builtin_fmaf(a, b, -w);
    return f + e;
}

// Normal-mapped GGX + Lambert of a grey material (albedo 1/2): the texel's
// RGB encodes the tangent-space normal m = 2 rgb - 1 (renormalised; z for
// m = 0), A the roughness parameter; h, wo, wi come in the tangent frame, so
// each cosine is one dot product with m.  Cosines are clamped at 0 and the
// masking factors taken as G1(c)/c = 2/(c + sqrt(a^2 + (1 - a^2) c^2)), so
// the result is continuous (0 where the normal faces away from the light).
__device__ __forceinline__ float3 shade_ggx_normal_dev(const GgxConst &g, float4 c)
{
    float mx = __builtin_fmaf(2.0f, c.x, -1.0f), my = __builtin_fmaf(2.0f, c.y, -1.0f),
          mz = __builtin_fmaf(2.0f, c.z, -1.0f);
    const float ml2 = mx * mx + my * my + mz * mz;
    float inv = 1.0f;
    if (ml2 > 0.0f) {
        inv = 1.0f / __builtin_sqrtf(ml2);
    } else {
        mx = 0.0f, my = 0.0f, mz = 1.0f;
    }
    const float no = __builtin_fmaxf((mx * g.to[0] + my * g.to[1] + mz * g.to[2]) * inv, 0.0f);
    const float ni = __builtin_fmaxf((mx * g.ti[0] + my * g.ti[1] + mz * g.ti[2]) * inv, 0.0f);
    const float r = __builtin_fmaf(g.r_scale, c.w, g.r_bias);
    const float a = r * r;
    const float a2 = a * a;
    // 1 - (n.h)^2 (1 - alpha^2) cancels near the peak of a glossy lobe; it is
    // formed as sin^2 + cos^2 alpha^2 of the angle between m and h, the sine
    // from the cross product, two non-negative terms.  h comes as a binary32
    // pair th + thl (a direction rounded to binary32 moves a glossy lobe's
    // value by ~1e-5), and each cross-product component keeps the rounding of
    // its products (Kahan's a b - c d), where they cancel near the peak.
    const float nh = (mx * g.th[0] + my * g.th[1] + mz * g.th[2]) + (mx * g.thl[0] + my * g.thl[1] + mz * g.thl[2]);
    const float cx = diff_prod(my, g.th[2], mz, g.th[1]) + (my * g.thl[2] - mz * g.thl[1]);
    const float cy = diff_prod(mz, g.th[0], mx, g.th[2]) + (mz * g.thl[0] - mx * g.thl[2]);
    const float cz = diff_prod(mx, g.th[1], my, g.th[0]) + (mx * g.thl[1] - my * g.thl[0]);
    const float il2 = 1.0f / ml2;
    // 1 - c2 = s2 + (1 - |h|^2): the tangent frame of a binary32 normal is
    // orthonormal only to ~1e-8, so |h|^2 differs from 1 by that much, which
    // is not negligible beside s2 + c2 alpha^2 at a sharp lobe's peak
    const float c2 = (nh * nh) * il2, s2 = ((cx * cx + cy * cy) + cz * cz) * il2;
    const float dd = (s2 + g.th_defect) + c2 * a2;
    const float D = a2 / (dd * dd);   // times 1/pi below
    const float om = 1.0f - a2;
    const float go = 2.0f / (no + __builtin_sqrtf(__builtin_fmaf(om, no * no, a2)));   // G1(no)/no
    const float gi = 2.0f / (ni + __builtin_sqrtf(__builtin_fmaf(om, ni * ni, a2)));
    const float spec = (D * go * gi * g.F) * (1.0f / (4.0f * 3.14159265f));
    return make_float3(ni * __builtin_fmaf(g.rad[0], spec, g.kdn[0]), ni * __builtin_fmaf(g.rad[1], spec, g.kdn[1]),
                       ni * __builtin_fmaf(g.rad[2], spec, g.kdn[2]));
}

__device__ __forceinline__ float half_bits_to_float(uint16_t h)
{
    return (float)__builtin_bit_cast(_Float16, h);
}

}  // namespace sfk
