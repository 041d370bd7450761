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

enum { NEAREST = 0, LINEAR = 1, BSPLINE3 = 2, KEYS3 = 3 };
enum { BEFORE = 0, AFTER = 1, STOCH = 2 };

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
    } else {
        w[0] = 1.0f;
    }
}

// The same weights in binary64 from the binary32 fraction: they sum to one
// within ~1e-16, which the long products of the exact-after comparator need.
template <int F>
__device__ __forceinline__ void axis_weights64(float tf, double w[4])
{
    const double t = (double)tf;
    if constexpr (F == BSPLINE3) {
        const double s = 1.0 - t, t2 = t * t, s2 = s * s;
        w[0] = (s2 * s) * (1.0 / 6.0);
        w[1] = 2.0 / 3.0 - t2 * (1.0 - 0.5 * t);
        w[2] = 2.0 / 3.0 - s2 * (1.0 - 0.5 * s);
        w[3] = (t2 * t) * (1.0 / 6.0);
    } else if constexpr (F == LINEAR) {
        w[0] = 1.0 - t;
        w[1] = t;
    } else {
        w[0] = 1.0;
    }
}

template <int F>
struct Taps {
    static constexpr int n = (F == BSPLINE3 || F == KEYS3) ? 4 : (F == LINEAR ? 2 : 1);
    static constexpr int first = (F == BSPLINE3 || F == KEYS3) ? -1 : 0;
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
__device__ __forceinline__ float3 shade_ggx_dev(const GgxConst &g, float4 c)
{
    const float r = __builtin_fmaf(g.r_scale, c.w, g.r_bias);
    const float a = r * r;
    const float a2 = a * a;
    const float d = __builtin_fmaf(g.nh2, a2 - 1.0f, 1.0f);
    const float om = 1.0f - a2;
    const float go = (2.0f * g.no) / (g.no + __builtin_sqrtf(__builtin_fmaf(om, g.no2, a2)));
    const float gi = (2.0f * g.ni) / (g.ni + __builtin_sqrtf(__builtin_fmaf(om, g.ni2, a2)));
    const float spec = (a2 * go * gi * g.spec_k) / (d * d);
    return make_float3(__builtin_fmaf(g.kd[0], c.x, g.ks[0] * spec), __builtin_fmaf(g.kd[1], c.y, g.ks[1] * spec),
                       __builtin_fmaf(g.kd[2], c.z, g.ks[2] * spec));
}

__device__ __forceinline__ float half_bits_to_float(uint16_t h)
{
    return (float)__builtin_bit_cast(_Float16, h);
}

}  // namespace sfk
