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
// compensated binary32 sums over up to 64 probes x 2 levels x 16 taps).
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
    // binary32 weights, compensated sums (up to 64 probes x 2 levels x 16 taps)
    const float wp = 1.0f / (float)lod.nprobe;
    CompSum sum[4];
    for (int k = 0; k < 4; ++k)
        sum[k].init();
    for (int k = 0; k < lod.nprobe; ++k) {
        const float o = ((float)k + 0.5f) / (float)lod.nprobe - 0.5f;
        const float uu = wrap_coord(c.tex.wrap, __builtin_fmaf(o, mu, qq[0]));
        const float vv = wrap_coord(c.tex.wrap, __builtin_fmaf(o, mv, qq[1]));
        for (int li = 0; li < 2; ++li) {
            const float pl = li == 0 ? 1.0f - f : f;
            if (pl == 0.0f)
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
            float wx[4], wy[4];
            axis_weights<F>(tx, wx);
            axis_weights<F>(ty, wy);
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                const int y = wrap_tap(c.tex.wrap, iy + F0 + b, hl);
#pragma unroll
                for (int a = 0; a < NT; ++a) {
                    const float wgt = ((wp * pl) * wx[a]) * wy[b];
                    const float4 t = texel(c.tex, l, wrap_tap(c.tex.wrap, ix + F0 + a, wl), y);
                    const float4 val = MODE == BEFORE ? t : shade<SHADE>(c.g, t);
                    sum[0].add(wgt * val.x);
                    sum[1].add(wgt * val.y);
                    sum[2].add(wgt * val.z);
                    sum[3].add(wgt * val.w);
                }
            }
        }
    }
    const float4 r = make_float4(sum[0].value(), sum[1].value(), sum[2].value(), sum[3].value());
    store<SHADE>(c.out, q, MODE == BEFORE ? shade<SHADE>(c.g, r) : r);
}

// ---------------------------------------------------------------- EWA
// Elliptically weighted average and its stochastic form (Sec. 4.1: a level
// from the ellipse's extent, then one texel drawn from all the EWA weights).
// The footprint Jacobian J (columns d(s,t)/dx, d(s,t)/dy in level-0 texels)
// gives the footprint covariance S = J J^T (Greene and Heckbert's EWA); the
// minor axis (J's smaller singular value) is lengthened to major/amax beyond
// the anisotropy limit by adding to S a multiple of the projector on the
// minor eigenvector; lod = max(0, log2(minor)).  At a level, V = S_l + I
// (one texel of reconstruction), a texel at offset d has radius
// r^2 = d^T V^-1 d and weight e^(-2 r^2) - e^(-2) (contract exp) for
// r^2 < 1, and the ellipse's bounding box has half-extents sqrt(V_ss),
// sqrt(V_tt).  The stochastic form takes the first cell in scan order (rows,
// then columns) whose running weight sum exceeds u W (Sec. 2.2, sampling
// arrays): one pass for W, one for the pick.  All decisions are binary32 in
// the order written below (no contraction), so picks are reproducible bit
// for bit.
struct EwaFrame {
    float lod;
    float vss, vtt, vst, det;  // S after the anisotropy limit, and det S
};

__device__ __forceinline__ EwaFrame ewa_frame(int W, int H, const float *q, int amax)
{
    EwaFrame e;
    const float jsx = (float)W * q[2], jtx = (float)H * q[3];
    const float jsy = (float)W * q[4], jty = (float)H * q[5];
    const float m = __builtin_fmaxf(__builtin_fmaxf(__builtin_fabsf(jsx), __builtin_fabsf(jtx)),
                                    __builtin_fmaxf(__builtin_fabsf(jsy), __builtin_fabsf(jty)));
    if (!(m < 0x1p40f)) {
        // the major axis is at least m texels, so the minor at least
        // 2^40/amax: beyond the last level of any pyramid
        e.lod = __builtin_inff();
        e.vss = e.vtt = e.vst = e.det = 0.0f;
        return e;
    }
    float vss = jsx * jsx + jsy * jsy;
    float vtt = jtx * jtx + jty * jty;
    float vst = jsx * jtx + jsy * jty;
    const float dj = jsx * jty - jtx * jsy;
    float det = dj * dj;
    const float half = (vss - vtt) * 0.5f, mean = (vss + vtt) * 0.5f;
    const float lp = mean + __builtin_sqrtf(half * half + vst * vst);   // larger eigenvalue
    const float s1 = __builtin_sqrtf(lp);
    float minor = lp > 0.0f ? __builtin_fabsf(dj) / s1 : 0.0f;
    if (minor * (float)amax < s1) {
        const float lm = det / lp;   // smaller eigenvalue
        minor = s1 / (float)amax;
        const float k = lp > lm ? (minor * minor - lm) / (lp - lm) : 1.0f;
        vss = vss + k * (lp - vss);
        vtt = vtt + k * (lp - vtt);
        vst = vst - k * vst;
        det = lp * (minor * minor);
    }
    e.vss = vss, e.vtt = vtt, e.vst = vst, e.det = det;
    e.lod = minor > 0.0f ? __builtin_fmaxf(0.0f, log2c(minor)) : 0.0f;
    return e;
}

struct EwaLevel {
    float s, t, qss, qtt, q2st;
    int s0, s1, t0, t1;
};

// V^-1 and the bounding box at level l (wl x hl texels of a W x H texture)
// for the wrapped coordinate (u, v).
__device__ __forceinline__ EwaLevel ewa_level(int W, int H, int wl, int hl, float u, float v, const EwaFrame &e)
{
    EwaLevel r;
    const float fs = (float)wl / (float)W, ft = (float)hl / (float)H;
    const float lss = e.vss * (fs * fs), ltt = e.vtt * (ft * ft), lst = e.vst * (fs * ft);
    const float ldet = e.det * ((fs * fs) * (ft * ft));
    const float a = lss + 1.0f, c = ltt + 1.0f;
    const float D = ((ldet + lss) + ltt) + 1.0f;   // det V, non-negative terms
    r.qss = c / D;
    r.qtt = a / D;
    r.q2st = -(2.0f * lst) / D;
    const float ex = __builtin_sqrtf(a), ey = __builtin_sqrtf(c);
    r.s = u * (float)wl - 0.5f;
    r.t = v * (float)hl - 0.5f;
    r.s0 = (int)__builtin_ceilf(r.s - ex);
    r.s1 = (int)__builtin_floorf(r.s + ex);
    r.t0 = (int)__builtin_ceilf(r.t - ey);
    r.t1 = (int)__builtin_floorf(r.t + ey);
    return r;
}

// Weight of cell (is, it): 0 outside the ellipse (r^2 >= 1).  e2 = e^(-2)
// by the contract exp.
__device__ __forceinline__ float ewa_weight(const EwaLevel &v, float e2, int is, int it)
{
    const float ds = (float)is - v.s, dt = (float)it - v.t;
    const float r2 = (v.qss * (ds * ds) + v.qtt * (dt * dt)) + v.q2st * (ds * dt);
    return r2 < 1.0f ? expc(-2.0f * r2) - e2 : 0.0f;
}

// Stochastic EWA: per sample, key (query, sample, 0, seed); word 3 picks
// level floor(lod) + [u >= 1 - f], word 0 is the uniform of the inverse-CDF
// pick.  Samples of a query spread over G lanes.
template <int SHADE>
__global__ __launch_bounds__(256) void k_ewa_stoch(AnisoCall c, int log_g)
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
                const float fl = __builtin_floorf(e.lod);
                const float th = 1.0f - (e.lod - fl);
                const float e2 = expc(-2.0f);
                for (int s = lane; s < c.spp; s += G) {
                    const uint4 w = pcg4d(make_uint4((uint32_t)q, (uint32_t)s, 0u, c.seed));
                    const int l = min((int)fl + (u24(w.w) >= th ? 1 : 0), L1);
                    const int wl = max(1, c.tex.w >> l), hl = max(1, c.tex.h >> l);
                    const EwaLevel v = ewa_level(c.tex.w, c.tex.h, wl, hl, uu, vv, e);
                    float W = 0.0f;
                    for (int it = v.t0; it <= v.t1; ++it)
                        for (int is = v.s0; is <= v.s1; ++is) {
                            const float wt = ewa_weight(v, e2, is, it);
                            W = wt > 0.0f ? W + wt : W;
                        }
                    const float thr = u24(w.x) * W;
                    const bool found = W > 0.0f;
                    float S = 0.0f;
                    int px = 0, py = 0;
                    bool done = !found;
                    for (int it = v.t0; it <= v.t1 && !done; ++it)
                        for (int is = v.s0; is <= v.s1 && !done; ++is) {
                            const float wt = ewa_weight(v, e2, is, it);
                            if (!(wt > 0.0f))
                                continue;
                            S = S + wt;
                            px = is;   // the last positive cell if u W rounds up to W
                            py = it;
                            done = S > thr;
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
// each normalised by its weight total; binary32 weights, compensated sums.
template <int SHADE, int MODE>
__global__ __launch_bounds__(256) void k_ewa_det(AnisoCall c)
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
    const int L1 = c.tex.levels - 1;
    const EwaFrame e = ewa_frame(c.tex.w, c.tex.h, qq, c.amax);
    const float lmax = (float)L1;
    if (e.lod > lmax) {
        store<SHADE>(c.out, q, shade<SHADE>(c.g, texel(c.tex, L1, 0, 0)));
        return;
    }
    const float uu = wrap_coord(c.tex.wrap, qq[0]), vv = wrap_coord(c.tex.wrap, qq[1]);
    const float fl = __builtin_floorf(e.lod);
    const float e2 = expc(-2.0f);
    float sum[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int li = 0; li < 2; ++li) {
        const float pl = li == 0 ? 1.0f - (e.lod - fl) : e.lod - fl;
        if (pl == 0.0f)
            continue;
        const int l = min((int)fl + li, L1);
        const int wl = max(1, c.tex.w >> l), hl = max(1, c.tex.h >> l);
        const EwaLevel v = ewa_level(c.tex.w, c.tex.h, wl, hl, uu, vv, e);
        CompSum part[4], W;
        W.init();
        for (int k = 0; k < 4; ++k)
            part[k].init();
        for (int it = v.t0; it <= v.t1; ++it) {
            const int y = wrap_any(c.tex.wrap, it, hl);
            for (int is = v.s0; is <= v.s1; ++is) {
                const float wt = ewa_weight(v, e2, is, it);
                if (!(wt > 0.0f))
                    continue;
                const float4 t = texel(c.tex, l, wrap_any(c.tex.wrap, is, wl), y);
                const float4 val = MODE == BEFORE ? t : shade<SHADE>(c.g, t);
                W.add(wt);
                part[0].add(wt * val.x);
                part[1].add(wt * val.y);
                part[2].add(wt * val.z);
                part[3].add(wt * val.w);
            }
        }
        const float Wv = W.value();
        if (Wv > 0.0f)
            for (int k = 0; k < 4; ++k)
                sum[k] += pl * (part[k].value() / Wv);
    }
    const float4 r = make_float4(sum[0], sum[1], sum[2], sum[3]);
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
