// Anisotropic minification by screen-space jitter (Sec. 4.2.1; the level of
// detail of Suppl. S.4.3; Sec. 5 "Anisotropic filtering and minification").
//
// A query is a pixel: uv and its screen derivatives.  Stochastic mode: each
// sample jitters uv over the pixel's parallelogram, reads ONE level chosen
// from the footprint's minor axis (anisotropy limited to amax) with a
// uniform level jitter, and ONE texel of it (FRS tent / B-spline / nearest,
// or the FIS Gaussian).  Samples of a query are spread over G lanes and
// reduced by a butterfly, as in the plain 2-D kernel.  The deterministic
// comparators average N probes along the major axis, each filtered on two
// levels (the anisotropic filter of texture hardware when the filter is the
// tent, before or after shading).
#include "sf_device.hpp"
#include "sf_internal.hpp"
#include "tex2d.hpp"

#pragma clang fp contract(off)

namespace sfk {

struct AnisoLod {
    float lam;
    bool major_y;
    int nprobe;
};

// Footprint axes in level-0 texels, x-axis (W du/dx, H dv/dx) and y-axis
// (W du/dy, H dv/dy); the shorter is the minor axis, lengthened to
// major/amax beyond the anisotropy limit; lambda = log2(minor).
__device__ __forceinline__ AnisoLod aniso_lod(int W, int H, float d0, float d1, float d2, float d3, int amax)
{
    const float ax = (float)W * d0, ay = (float)H * d1;
    const float bx = (float)W * d2, by = (float)H * d3;
    const float la2 = ax * ax + ay * ay, lb2 = bx * bx + by * by;
    const bool swap = la2 > lb2;
    float lmin = __builtin_sqrtf(swap ? lb2 : la2);
    const float lmax = __builtin_sqrtf(swap ? la2 : lb2);
    const float A = (float)amax;
    if (lmin > 0.0f && lmin * A < lmax) {
        const float scale = lmax / (lmin * A);
        lmin = lmin * scale;
    }
    AnisoLod r;
    r.major_y = !swap;
    if (lmin > 0.0f) {
        const float k = __builtin_ceilf(lmax / lmin);
        r.nprobe = k < 1.0f ? 1 : (!(k <= A) ? amax : (int)k);
    } else {
        r.nprobe = lmax > 0.0f ? amax : 1;
    }
    r.lam = log2c(lmin);
    return r;
}

// Usable query: six finite values, and finite extreme jittered coordinates
// |u| + |du/dx| + |du/dy| (and for v).
__device__ __forceinline__ bool aniso_finite(const float *q)
{
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 6; ++k)
        ok &= __builtin_isfinite(q[k]);
    const float eu = (__builtin_fabsf(q[0]) + __builtin_fabsf(q[2])) + __builtin_fabsf(q[4]);
    const float ev = (__builtin_fabsf(q[1]) + __builtin_fabsf(q[3])) + __builtin_fabsf(q[5]);
    return ok & __builtin_isfinite(eu) & __builtin_isfinite(ev);
}

template <int F, int SHADE>
__global__ __launch_bounds__(256) void k_aniso_stoch(AnisoCall c, int log_g)
{
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int G = 1 << log_g;
    const int64_t q = gid >> log_g;
    const int lane = (int)(gid & (G - 1));
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    const bool active = q < c.n;
    if (active) {
        float qq[6];
#pragma unroll
        for (int k = 0; k < 6; ++k)
            qq[k] = c.q[6 * q + k];
        if (!aniso_finite(qq)) {
            const float nan = __builtin_nanf("");
            acc = make_float4(nan, nan, nan, nan);
            if (c.taps)
                for (int s = lane; s < c.spp; s += G)
                    for (int k = 0; k < 3; ++k)
                        c.taps[(q * c.spp + s) * 3 + k] = SF_TAP_NONE;
        } else {
            const AnisoLod lod = aniso_lod(c.tex.w, c.tex.h, qq[2], qq[3], qq[4], qq[5], c.amax);
            const float lmaxf = (float)(c.tex.levels - 1);
            for (int s = lane; s < c.spp; s += G) {
                const uint4 w0 = pcg4d(make_uint4((uint32_t)q, (uint32_t)s, 0u, c.seed));
                const uint4 w1 = pcg4d(make_uint4((uint32_t)q, (uint32_t)s, 1u, c.seed));
                const float jx = u24(w0.x) - 0.5f, jy = u24(w0.y) - 0.5f;
                const float u = __builtin_fmaf(jy, qq[4], __builtin_fmaf(jx, qq[2], qq[0]));
                const float v = __builtin_fmaf(jy, qq[5], __builtin_fmaf(jx, qq[3], qq[1]));
                float lj = lod.lam + (u24(w0.z) - 0.5f);
                lj = __builtin_fminf(__builtin_fmaxf(lj, 0.0f), lmaxf);
                const int l = (int)__builtin_floorf(lj + 0.5f);
                const int wl = max(1, c.tex.w >> l), hl = max(1, c.tex.h >> l);
                int ix, iy;
                float tx, ty;
                raster(wrap_coord(c.tex.wrap, u), wl, ix, tx);
                raster(wrap_coord(c.tex.wrap, v), hl, iy, ty);
                int ox, oy;
                if constexpr (F == GAUSS_FIS) {
                    gauss_fis_pick(tx, ty, c.sigma, u24(w1.x), u24(w1.y), ox, oy);
                } else {
                    ox = pick_off_2p24<F>(tx, u24i(w1.x));
                    oy = pick_off_2p24<F>(ty, u24i(w1.y));
                }
                const int x = wrap_any(c.tex.wrap, ix + ox, wl), y = wrap_any(c.tex.wrap, iy + oy, hl);
                if (c.taps) {
                    int32_t *tp = c.taps + (q * c.spp + s) * 3;
                    tp[0] = l;
                    tp[1] = x;
                    tp[2] = y;
                }
                acc = add4(acc, shade<SHADE>(c.g, texel(c.tex, l, x, y)));
            }
        }
    }
    for (int m = G >> 1; m >= 1; m >>= 1) {
        acc.x += __shfl_xor(acc.x, m);
        acc.y += __shfl_xor(acc.y, m);
        acc.z += __shfl_xor(acc.z, m);
        acc.w += __shfl_xor(acc.w, m);
    }
    if (active && lane == 0) {
        const float inv = 1.0f / (float)c.spp;
        store<SHADE>(c.out, q, make_float4(acc.x * inv, acc.y * inv, acc.z * inv, acc.w * inv));
    }
}

// Probe comparators (binary32 weights as the plain deterministic kernel,
// binary64 sums over up to 64 probes x 2 levels x 16 taps).
template <int F, int SHADE, int MODE>
__global__ __launch_bounds__(256) void k_aniso_det(AnisoCall c)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= c.n)
        return;
    float qq[6];
#pragma unroll
    for (int k = 0; k < 6; ++k)
        qq[k] = c.q[6 * q + k];
    if (!aniso_finite(qq)) {
        const float nan = __builtin_nanf("");
        store<SHADE>(c.out, q, make_float4(nan, nan, nan, nan));
        return;
    }
    const AnisoLod lod = aniso_lod(c.tex.w, c.tex.h, qq[2], qq[3], qq[4], qq[5], c.amax);
    int l0, l1;
    float f;
    Tex2DArgs tx2 = c.tex;
    tx2.mip = SF_MIP_LINEAR;
    levels_of(tx2, lod.lam, l0, l1, f);
    const float mu = lod.major_y ? qq[4] : qq[2], mv = lod.major_y ? qq[5] : qq[3];
    constexpr int NT = Taps<F>::n;
    constexpr int F0 = Taps<F>::first;
    const double wp = 1.0 / (double)lod.nprobe;
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < lod.nprobe; ++k) {
        const float o = ((float)k + 0.5f) / (float)lod.nprobe - 0.5f;
        const float uu = wrap_coord(c.tex.wrap, __builtin_fmaf(o, mu, qq[0]));
        const float vv = wrap_coord(c.tex.wrap, __builtin_fmaf(o, mv, qq[1]));
        for (int li = 0; li < 2; ++li) {
            const double pl = li == 0 ? 1.0 - (double)f : (double)f;
            if (pl == 0.0)
                continue;
            const int l = li == 0 ? l0 : l1;
            const int wl = max(1, c.tex.w >> l), hl = max(1, c.tex.h >> l);
            int ix, iy;
            float tx, ty;
            raster(uu, wl, ix, tx);
            raster(vv, hl, iy, ty);
            if constexpr (F == NEAREST) {
                ix += tx >= 0.5f;
                iy += ty >= 0.5f;
            }
            double wx[4], wy[4];
            axis_weights64<F>(tx, wx);
            axis_weights64<F>(ty, wy);
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                const int y = wrap_tap(c.tex.wrap, iy + F0 + b, hl);
#pragma unroll
                for (int a = 0; a < NT; ++a) {
                    const double wgt = wp * pl * wx[a] * wy[b];
                    const float4 t = texel(c.tex, l, wrap_tap(c.tex.wrap, ix + F0 + a, wl), y);
                    const float4 val = MODE == BEFORE ? t : shade<SHADE>(c.g, t);
                    sum[0] += wgt * (double)val.x;
                    sum[1] += wgt * (double)val.y;
                    sum[2] += wgt * (double)val.z;
                    sum[3] += wgt * (double)val.w;
                }
            }
        }
    }
    const float4 r = make_float4((float)sum[0], (float)sum[1], (float)sum[2], (float)sum[3]);
    store<SHADE>(c.out, q, MODE == BEFORE ? shade<SHADE>(c.g, r) : r);
}

template <int F, int SHADE>
static void launch_a2(const AnisoCall &c, hipStream_t s)
{
    if (c.mode == STOCH) {
        int G = 1;
        while (G * 2 <= c.spp && G * 2 <= 64)
            G *= 2;
        const int64_t threads = c.n * G;
        k_aniso_stoch<F, SHADE><<<dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s>>>(c, __builtin_ctz(G));
    } else if constexpr (F != GAUSS_FIS) {
        const dim3 grid((uint32_t)((c.n + 255) / 256)), block(256);
        if (c.mode == BEFORE)
            k_aniso_det<F, SHADE, BEFORE><<<grid, block, 0, s>>>(c);
        else
            k_aniso_det<F, SHADE, AFTER><<<grid, block, 0, s>>>(c);
    }
}

template <int F>
static void launch_a1(const AnisoCall &c, hipStream_t s)
{
    if (c.shade == SF_SHADE_GGX)
        launch_a2<F, SF_SHADE_GGX>(c, s);
    else
        launch_a2<F, SF_SHADE_NONE>(c, s);
}

hipError_t launch_aniso(const AnisoCall &c, hipStream_t s)
{
    switch (c.filter) {
    case NEAREST:
        launch_a1<NEAREST>(c, s);
        break;
    case LINEAR:
        launch_a1<LINEAR>(c, s);
        break;
    case GAUSS_FIS:
        launch_a1<GAUSS_FIS>(c, s);
        break;
    default:
        launch_a1<BSPLINE3>(c, s);
        break;
    }
    return hipGetLastError();
}

}  // namespace sfk
