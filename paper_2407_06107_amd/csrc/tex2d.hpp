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

__device__ __forceinline__ float4 texel(const Tex2DArgs &tx, int l, int x, int y)
{
    int wl = max(1, tx.w >> l);
    int64_t idx = (int64_t)y * wl + x;
    const uint8_t *lv = tx.base + tx.off[l];
    if (tx.fmt == SF_RGBA32F)
        return reinterpret_cast<const float4 *>(lv)[idx];
    uint32_t px = reinterpret_cast<const uint32_t *>(lv)[idx];
    const float k = 1.0f / 255.0f;
    return make_float4((float)(px & 0xffu) * k, (float)((px >> 8) & 0xffu) * k, (float)((px >> 16) & 0xffu) * k,
                       (float)(px >> 24) * k);
}

template <int SHADE>
__device__ __forceinline__ float4 shade(const GgxConst &g, float4 c)
{
    if constexpr (SHADE == SF_SHADE_GGX) {
        float3 v = shade_ggx_dev(g, c);
        return make_float4(v.x, v.y, v.z, 0.0f);
    } else {
        return c;
    }
}

template <int SHADE>
__device__ __forceinline__ void store(float *out, int64_t q, float4 v)
{
    if constexpr (SHADE == SF_SHADE_GGX) {
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

}  // namespace sfk
