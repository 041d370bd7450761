// 2-D texture access helpers shared by the plain, anisotropic and
// compressed-texture kernels: coordinate wrap, raster position, MIP level
// choice, texel fetch, GGX shading and output store.
#pragma once
#include "sf_device.hpp"
#include "sf_internal.hpp"

#pragma clang fp contract(off)

namespace sfk {

__device__ __forceinline__ float wrap_coord(int wrap, float u)
{
    return wrap == SF_WRAP_REPEAT ? u - __builtin_floorf(u) : __builtin_fminf(__builtin_fmaxf(u, 0.0f), 1.0f);
}

// Taps lie in [-2, n+1]: one conditional add or subtract wraps them.
__device__ __forceinline__ int wrap_tap(int wrap, int i, int n)
{
    if (wrap == SF_WRAP_REPEAT) {
        int r = i < 0 ? i + n : (i >= n ? i - n : i);
        return n == 1 ? 0 : r;
    }
    return min(max(i, 0), n - 1);
}

// Any tap index (the FIS Gaussian reaches 25 texels past the point).
__device__ __forceinline__ int wrap_any(int wrap, int i, int n)
{
    if (wrap == SF_WRAP_REPEAT) {
        const int r = i % n;
        return r < 0 ? r + n : r;
    }
    return min(max(i, 0), n - 1);
}

__device__ __forceinline__ void raster(float u, int n, int &i0, float &t)
{
    float p = __builtin_fmaf(u, (float)n, -0.5f);
    float f = __builtin_floorf(p);
    i0 = (int)f;
    t = p - f;
}

__device__ __forceinline__ void levels_of(const Tex2DArgs &tx, float lam, int &l0, int &l1, float &f)
{
    if (tx.mip == SF_MIP_NONE) {
        l0 = l1 = 0;
        f = 0.0f;
        return;
    }
    float lc = __builtin_fminf(__builtin_fmaxf(lam, 0.0f), (float)(tx.levels - 1));
    float fl = __builtin_floorf(lc);
    float fr = lc - fl;
    int a = (int)fl;
    if (tx.mip == SF_MIP_NEAREST) {
        a += fr >= 0.5f;
        a = min(a, tx.levels - 1);
        l0 = l1 = a;
        f = 0.0f;
        return;
    }
    l0 = a;
    l1 = min(a + 1, tx.levels - 1);
    f = fr;
}

// DCT basis c_k(x) = alpha(k) cos((2x+1) k pi / 16) for k = 1, 2 from the
// symmetries of the cosine: |c_1| takes four values mirrored about x = 3.5
// with the sign of x < 4; |c_2| is a for x in {0, 3, 4, 7} and b otherwise,
// negative for x in 2..5.
__device__ __forceinline__ float dct_c1(int x)
{
    const int m = min(x, 7 - x);
    const float v = m == 0 ? 0.49039262533187866f
                           : (m == 1 ? 0.41573479771614075f : (m == 2 ? 0.27778512239456177f : 0.09754516184329987f));
    return x < 4 ? v : -v;
}

__device__ __forceinline__ float dct_c2(int x)
{
    const float v = ((x + 1) >> 1) & 1 ? 0.19134171307086945f : 0.4619397521018982f;
    return ((x + 2) >> 2) & 1 ? -v : v;
}

constexpr float DCT_C0 = 0.3535533845424652f;

// One channel of a DCT block word at block position (x, y).
__device__ __forceinline__ float dct_channel(uint32_t wd, float R, float c1x, float c2x, float c1y, float c2y)
{
    const float q = R * (1.0f / 15.0f);
    float v = (float)(wd & 127u) * ((8.0f / 127.0f) * (DCT_C0 * DCT_C0));
    v = __builtin_fmaf((float)((int)((wd >> 7) & 31u) - 15) * q, c1x * DCT_C0, v);    // (1,0)
    v = __builtin_fmaf((float)((int)((wd >> 12) & 31u) - 15) * q, DCT_C0 * c1y, v);   // (0,1)
    v = __builtin_fmaf((float)((int)((wd >> 17) & 31u) - 15) * q, DCT_C0 * c2y, v);   // (0,2)
    v = __builtin_fmaf((float)((int)((wd >> 22) & 31u) - 15) * q, c1x * c1y, v);      // (1,1)
    v = __builtin_fmaf((float)((int)(wd >> 27) - 15) * q, c2x * DCT_C0, v);           // (2,0)
    return __builtin_fminf(__builtin_fmaxf(v, 0.0f), 1.0f);
}

// Texel (x, y) of level l, the texture's levels read from `base` (its own
// base pointer, or a copy of its bytes at the same offsets).
__device__ __forceinline__ float4 texel(const Tex2DArgs &tx, const uint8_t *base, int l, int x, int y)
{
    int wl = max(1, tx.w >> l);
    int64_t idx = (int64_t)y * wl + x;
    const uint8_t *lv = base + tx.off[l];
    if (tx.fmt == SF_DCT8) {
        const int bw = (wl + 7) >> 3;
        const uint4 b = reinterpret_cast<const uint4 *>(lv)[(int64_t)(y >> 3) * bw + (x >> 3)];
        const float4 R = reinterpret_cast<const float4 *>(tx.dct_range)[l];
        const int xi = x & 7, yi = y & 7;
        const float c1x = dct_c1(xi), c2x = dct_c2(xi), c1y = dct_c1(yi), c2y = dct_c2(yi);
        return make_float4(dct_channel(b.x, R.x, c1x, c2x, c1y, c2y), dct_channel(b.y, R.y, c1x, c2x, c1y, c2y),
                           dct_channel(b.z, R.z, c1x, c2x, c1y, c2y), dct_channel(b.w, R.w, c1x, c2x, c1y, c2y));
    }
    if (tx.fmt == SF_RGBA32F)
        return reinterpret_cast<const float4 *>(lv)[idx];
    uint32_t px = reinterpret_cast<const uint32_t *>(lv)[idx];
    const float k = 1.0f / 255.0f;
    return make_float4((float)(px & 0xffu) * k, (float)((px >> 8) & 0xffu) * k, (float)((px >> 16) & 0xffu) * k,
                       (float)(px >> 24) * k);
}

__device__ __forceinline__ float4 texel(const Tex2DArgs &tx, int l, int x, int y) { return texel(tx, tx.base, l, x, y); }

template <int SHADE>
__device__ __forceinline__ float4 shade(const GgxConst &g, float4 c)
{
    if constexpr (SHADE == SF_SHADE_GGX) {
        float3 v = shade_ggx_dev(g, c);
        return make_float4(v.x, v.y, v.z, 0.0f);
    } else if constexpr (SHADE == SF_SHADE_GGX_NORMAL) {
        float3 v = shade_ggx_normal_dev(g, c);
        return make_float4(v.x, v.y, v.z, 0.0f);
    } else {
        return c;
    }
}

template <int SHADE>
__device__ __forceinline__ void store(float *out, int64_t q, float4 v)
{
    if constexpr (SHADE != SF_SHADE_NONE) {
        out[3 * q] = v.x;
        out[3 * q + 1] = v.y;
        out[3 * q + 2] = v.z;
    } else {
        reinterpret_cast<float4 *>(out)[q] = v;
    }
}

__device__ __forceinline__ bool query_ok(const Tex2DArgs &tx, float3 q)
{
    bool ok = __builtin_isfinite(q.x) & __builtin_isfinite(q.y);
    return ok & (tx.mip == SF_MIP_NONE || __builtin_isfinite(q.z));
}

__device__ __forceinline__ float4 add4(float4 a, float4 b) { return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }

// The reconstruction filter alone on level l at the wrapped coordinate
// (uu, vv): sum_i w_i t_i with binary32 weights, as the deterministic kernels
// (the split-filtering estimator shades this once per sample).
template <int F>
__device__ __forceinline__ float4 recon_level(const Tex2DArgs &tx, float uu, float vv, int l)
{
    constexpr int NT = Taps<F>::n;
    constexpr int F0 = Taps<F>::first;
    const int wl = max(1, tx.w >> l), hl = max(1, tx.h >> l);
    int ix, iy;
    float fx, fy, wx[4], wy[4];
    raster(uu, wl, ix, fx);
    raster(vv, hl, iy, fy);
    if constexpr (F == NEAREST) {
        ix += fx >= 0.5f;
        iy += fy >= 0.5f;
    }
    axis_weights<F>(fx, wx);
    axis_weights<F>(fy, wy);
    float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int b = 0; b < NT; ++b) {
        const int y = wrap_tap(tx.wrap, iy + F0 + b, hl);
#pragma unroll
        for (int a = 0; a < NT; ++a) {
            const float wgt = wx[a] * wy[b];
            const float4 t = texel(tx, l, wrap_tap(tx.wrap, ix + F0 + a, wl), y);
            sum.x = __builtin_fmaf(wgt, t.x, sum.x);
            sum.y = __builtin_fmaf(wgt, t.y, sum.y);
            sum.z = __builtin_fmaf(wgt, t.z, sum.z);
            sum.w = __builtin_fmaf(wgt, t.w, sum.w);
        }
    }
    return sum;
}

}  // namespace sfk
