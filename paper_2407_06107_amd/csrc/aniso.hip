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

// Split filtering over the pixel (Sec. 3 eq. split-filtering-shading,
// estimated as in Sec. 4): per sample the jitter and the jittered level of
// the stochastic mode (key words 0, 1, 2) sample the low-pass filter; the
// reconstruction filter is evaluated on that level and shaded once.
template <int F, int SHADE>
__global__ __launch_bounds__(256) void k_aniso_split(AnisoCall c, int log_g)
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
                const float jx = u24(w0.x) - 0.5f, jy = u24(w0.y) - 0.5f;
                const float u = __builtin_fmaf(jy, qq[4], __builtin_fmaf(jx, qq[2], qq[0]));
                const float v = __builtin_fmaf(jy, qq[5], __builtin_fmaf(jx, qq[3], qq[1]));
                float lj = lod.lam + (u24(w0.z) - 0.5f);
                lj = __builtin_fminf(__builtin_fmaxf(lj, 0.0f), lmaxf);
                const int l = (int)__builtin_floorf(lj + 0.5f);
                if (c.taps) {
                    int32_t *tp = c.taps + (q * c.spp + s) * 3;
                    tp[0] = l;
                    tp[1] = SF_TAP_NONE;
                    tp[2] = SF_TAP_NONE;
                }
                const float4 r = recon_level<F>(c.tex, wrap_coord(c.tex.wrap, u), wrap_coord(c.tex.wrap, v), l);
                acc = add4(acc, shade<SHADE>(c.g, r));
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

// ---------------------------------------------------------------- EWA
// Elliptically weighted average and its stochastic form (Sec. 4.1: a level
// from the ellipse's extent, then one texel by weighted reservoir sampling
// over all EWA weights; Suppl. S.4, the EWA kernel).  The footprint ellipse
// of the derivatives, regularised by one texel (the +1 of A and C), is
// scanned over its bounding box row by row; weights e^(-2 r^2) - e^(-2) come
// from a 128-entry table built per block in LDS.  All decisions are binary32
// in the order written below (no contraction), so picks are reproducible
// bit for bit.
constexpr int EWA_LUT = 128;

struct EwaFrame {
    float lod;
    float a0, a1, b0, b1;  // axes after the anisotropy limit, texture units
};

// Longer axis first (lengths in level-0 texels); the shorter lengthened to
// longer/amax beyond the limit, a zero shorter axis counting as longer/amax;
// lod = max(0, log2(shorter)).
__device__ __forceinline__ EwaFrame ewa_frame(int W, int H, const float *q, int amax)
{
    float a0 = q[2], a1 = q[3], b0 = q[4], b1 = q[5];
    const float ax = (float)W * a0, ay = (float)H * a1, bx = (float)W * b0, by = (float)H * b1;
    float la2 = ax * ax + ay * ay, lb2 = bx * bx + by * by;
    if (la2 < lb2) {
        float x = a0, y = a1, l = la2;
        a0 = b0, a1 = b1, la2 = lb2;
        b0 = x, b1 = y, lb2 = l;
    }
    const float la = __builtin_sqrtf(la2);
    float lb = __builtin_sqrtf(lb2);
    const float A = (float)amax;
    if (lb > 0.0f && lb * A < la) {
        const float scale = la / (lb * A);
        b0 = b0 * scale;
        b1 = b1 * scale;
        lb = lb * scale;
    } else if (lb == 0.0f) {
        lb = la / A;
    }
    EwaFrame e;
    e.a0 = a0, e.a1 = a1, e.b0 = b0, e.b1 = b1;
    e.lod = __builtin_fmaxf(0.0f, log2c(lb));
    return e;
}

struct EwaLevel {
    float s, t, A, B, C;
    int s0, s1, t0, t1;
};

// Ellipse coefficients and bounding box at level l (W_l x H_l texels) for
// the wrapped coordinate (u, v).
__device__ __forceinline__ EwaLevel ewa_level(int wl, int hl, float u, float v, const EwaFrame &e)
{
    EwaLevel r;
    r.s = u * (float)wl - 0.5f;
    r.t = v * (float)hl - 0.5f;
    const float d00 = e.a0 * (float)wl, d01 = e.a1 * (float)hl;
    const float d10 = e.b0 * (float)wl, d11 = e.b1 * (float)hl;
    float A = d01 * d01 + d11 * d11 + 1.0f;
    float B = -2.0f * (d00 * d01 + d10 * d11);
    float C = d00 * d00 + d10 * d10 + 1.0f;
    const float invF = 1.0f / (A * C - B * B * 0.25f);
    A = A * invF;
    B = B * invF;
    C = C * invF;
    const float det = -B * B + 4.0f * A * C;
    const float invDet = 1.0f / det;
    const float uS = __builtin_sqrtf(__builtin_fmaxf(0.0f, det * C));
    const float vS = __builtin_sqrtf(__builtin_fmaxf(0.0f, A * det));
    r.s0 = (int)__builtin_ceilf(r.s - 2.0f * invDet * uS);
    r.s1 = (int)__builtin_floorf(r.s + 2.0f * invDet * uS);
    r.t0 = (int)__builtin_ceilf(r.t - 2.0f * invDet * vS);
    r.t1 = (int)__builtin_floorf(r.t + 2.0f * invDet * vS);
    r.A = A, r.B = B, r.C = C;
    return r;
}

// Weight of cell (is, it): 0 outside the ellipse (r^2 >= 1).
__device__ __forceinline__ float ewa_weight(const EwaLevel &v, const float *lut, int is, int it)
{
    const float ss = (float)is - v.s, tt = (float)it - v.t;
    const float r2 = v.A * (ss * ss) + v.B * ss * tt + v.C * (tt * tt);
    if (!(r2 < 1.0f))
        return 0.0f;
    const int idx = max(0, min((int)(r2 * (float)EWA_LUT), EWA_LUT - 1));
    return lut[idx];
}

// Table of e^(-2 r^2) - e^(-2), r^2 = i/127, with the contract exp; the
// block's first 128 threads fill it.
__device__ __forceinline__ void ewa_fill_lut(float *lut)
{
    if (threadIdx.x < EWA_LUT) {
        const float r2 = (float)threadIdx.x / 127.0f;
        lut[threadIdx.x] = expc(-2.0f * r2) - expc(-2.0f);
    }
    __syncthreads();
}

// Stochastic EWA: per sample, key (query, sample, 0, seed); word 3 picks
// level floor(lod) + [u >= 1 - f], word 0 drives the one-uniform reservoir
// (the uniform is reused after each step: u/p on a pick, (u-p)/(1-p)
// otherwise).  Samples of a query spread over G lanes.
template <int SHADE>
__global__ __launch_bounds__(256) void k_ewa_stoch(AnisoCall c, int log_g)
{
    __shared__ float lut[EWA_LUT];
    ewa_fill_lut(lut);
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
        const int L1 = c.tex.levels - 1;
        if (!aniso_finite(qq)) {
            const float nan = __builtin_nanf("");
            acc = make_float4(nan, nan, nan, nan);
            if (c.taps)
                for (int s = lane; s < c.spp; s += G)
                    for (int k = 0; k < 3; ++k)
                        c.taps[(q * c.spp + s) * 3 + k] = SF_TAP_NONE;
        } else {
            const EwaFrame e = ewa_frame(c.tex.w, c.tex.h, qq, c.amax);
            const float lmax = (float)L1;
            if (e.lod > lmax) {
                // wider than the texture: the last (1 x 1) level
                const float4 t = shade<SHADE>(c.g, texel(c.tex, L1, 0, 0));
                for (int s = lane; s < c.spp; s += G) {
                    if (c.taps) {
                        int32_t *tp = c.taps + (q * c.spp + s) * 3;
                        tp[0] = L1;
                        tp[1] = 0;
                        tp[2] = 0;
                    }
                    acc = add4(acc, t);
                }
            } else {
                const float uu = wrap_coord(c.tex.wrap, qq[0]), vv = wrap_coord(c.tex.wrap, qq[1]);
                const float lc = __builtin_fminf(e.lod, lmax);
                const float fl = __builtin_floorf(lc);
                const float th = 1.0f - (lc - fl);
                for (int s = lane; s < c.spp; s += G) {
                    const uint4 w = pcg4d(make_uint4((uint32_t)q, (uint32_t)s, 0u, c.seed));
                    const int l = min((int)fl + (u24(w.w) >= th ? 1 : 0), L1);
                    const int wl = max(1, c.tex.w >> l), hl = max(1, c.tex.h >> l);
                    const EwaLevel v = ewa_level(wl, hl, uu, vv, e);
                    float u = u24(w.x), sum = 0.0f;
                    int px = 0, py = 0;
                    bool found = false;
                    for (int it = v.t0; it <= v.t1; ++it)
                        for (int is = v.s0; is <= v.s1; ++is) {
                            const float wt = ewa_weight(v, lut, is, it);
                            if (!(wt > 0.0f))
                                continue;
                            sum += wt;
                            const float p = wt / sum;
                            const bool take = u < p;
                            px = take ? is : px;
                            py = take ? it : py;
                            found |= take;
                            u = (take ? u : u - p) / (take ? p : 1.0f - p);
                        }
                    const int x = wrap_any(c.tex.wrap, px, wl), y = wrap_any(c.tex.wrap, py, hl);
                    if (c.taps) {
                        int32_t *tp = c.taps + (q * c.spp + s) * 3;
                        tp[0] = found ? l : SF_TAP_NONE;
                        tp[1] = found ? x : SF_TAP_NONE;
                        tp[2] = found ? y : SF_TAP_NONE;
                    }
                    if (found)
                        acc = add4(acc, shade<SHADE>(c.g, texel(c.tex, l, x, y)));
                }
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

// Deterministic EWA on levels floor(lod), floor(lod)+1 (weights 1-f, f),
// each normalised by its weight total; binary64 sums.
template <int SHADE, int MODE>
__global__ __launch_bounds__(256) void k_ewa_det(AnisoCall c)
{
    __shared__ float lut[EWA_LUT];
    ewa_fill_lut(lut);
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
    const int L1 = c.tex.levels - 1;
    const EwaFrame e = ewa_frame(c.tex.w, c.tex.h, qq, c.amax);
    const float lmax = (float)L1;
    if (e.lod > lmax) {
        store<SHADE>(c.out, q, shade<SHADE>(c.g, texel(c.tex, L1, 0, 0)));
        return;
    }
    const float uu = wrap_coord(c.tex.wrap, qq[0]), vv = wrap_coord(c.tex.wrap, qq[1]);
    const float lc = __builtin_fminf(e.lod, lmax);
    const float fl = __builtin_floorf(lc);
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    for (int li = 0; li < 2; ++li) {
        const double pl = li == 0 ? 1.0 - (double)(lc - fl) : (double)(lc - fl);
        if (pl == 0.0)
            continue;
        const int l = min((int)fl + li, L1);
        const int wl = max(1, c.tex.w >> l), hl = max(1, c.tex.h >> l);
        const EwaLevel v = ewa_level(wl, hl, uu, vv, e);
        double part[4] = {0.0, 0.0, 0.0, 0.0}, W = 0.0;
        for (int it = v.t0; it <= v.t1; ++it) {
            const int y = wrap_any(c.tex.wrap, it, hl);
            for (int is = v.s0; is <= v.s1; ++is) {
                const float wt = ewa_weight(v, lut, is, it);
                if (!(wt > 0.0f))
                    continue;
                const float4 t = texel(c.tex, l, wrap_any(c.tex.wrap, is, wl), y);
                const float4 val = MODE == BEFORE ? t : shade<SHADE>(c.g, t);
                const double wd = (double)wt;
                W += wd;
                part[0] += wd * (double)val.x;
                part[1] += wd * (double)val.y;
                part[2] += wd * (double)val.z;
                part[3] += wd * (double)val.w;
            }
        }
        if (W > 0.0)
            for (int k = 0; k < 4; ++k)
                sum[k] += pl * part[k] / W;
    }
    const float4 r = make_float4((float)sum[0], (float)sum[1], (float)sum[2], (float)sum[3]);
    store<SHADE>(c.out, q, MODE == BEFORE ? shade<SHADE>(c.g, r) : r);
}

template <int SHADE>
static void launch_ewa(const AnisoCall &c, hipStream_t s)
{
    if (c.mode == STOCH) {
        const int G = lane_group(c.n, c.spp);
        const int64_t threads = c.n * G;
        k_ewa_stoch<SHADE><<<dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s>>>(c, __builtin_ctz(G));
    } else {
        const dim3 grid((uint32_t)((c.n + 255) / 256)), block(256);
        if (c.mode == BEFORE)
            k_ewa_det<SHADE, BEFORE><<<grid, block, 0, s>>>(c);
        else
            k_ewa_det<SHADE, AFTER><<<grid, block, 0, s>>>(c);
    }
}

template <int F, int SHADE>
static void launch_a2(const AnisoCall &c, hipStream_t s)
{
    if constexpr (F <= KEYS3 || F == MITCHELL) {
        if (c.mode == SPLIT) {
            const int G = lane_group(c.n, c.spp);
            const int64_t threads = c.n * G;
            k_aniso_split<F, SHADE><<<dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s>>>(c, __builtin_ctz(G));
            return;
        }
    }
    if constexpr (F == KEYS3 || F == MITCHELL)
        return;   // the positivised cubics take the split mode only here
    else if (c.mode == STOCH) {
        const int G = lane_group(c.n, c.spp);
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
    else if (c.shade == SF_SHADE_GGX_NORMAL)
        launch_a2<F, SF_SHADE_GGX_NORMAL>(c, s);
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
    case KEYS3:
        launch_a1<KEYS3>(c, s);
        break;
    case MITCHELL:
        launch_a1<MITCHELL>(c, s);
        break;
    case EWA:
        if (c.shade == SF_SHADE_GGX)
            launch_ewa<SF_SHADE_GGX>(c, s);
        else if (c.shade == SF_SHADE_GGX_NORMAL)
            launch_ewa<SF_SHADE_GGX_NORMAL>(c, s);
        else
            launch_ewa<SF_SHADE_NONE>(c, s);
        break;
    default:
        launch_a1<BSPLINE3>(c, s);
        break;
    }
    return hipGetLastError();
}

}  // namespace sfk
