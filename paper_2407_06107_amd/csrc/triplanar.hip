// Triplanar mapping (Sec. 5 "Triplanar mapping").  A surface point is
// textured from three planar projections blended by b_i = n_i^4 / sum n^4.
// The blend is a weighted mean, so one plane picked with probability b_i
// per sample estimates it (eq. stochastic-sum): with a stochastic filter on
// the picked plane a sample costs ONE texel fetch (one decode for SF_DCT8
// textures) instead of 3 x 4 (trilinear) or 3 x 16 (bicubic) per level.
// Samples of a query are spread over G lanes as in the plain 2-D kernel.
#include "sf_device.hpp"
#include "sf_internal.hpp"
#include "tex2d.hpp"

#pragma clang fp contract(off)

namespace sfk {

__device__ __forceinline__ void tri_uv(const float *p, int plane, float scale, float &u, float &v)
{
    const float a = plane == 0 ? p[1] : p[0];
    const float b = plane == 2 ? p[1] : p[2];
    u = a * scale;
    v = b * scale;
}

// One texel per sample on one plane: level pick (u_l), raster, per-axis
// inverse-CDF picks on the 24-bit lattice indices ix_u, iy_u of the x and y
// uniforms, fetch, shade.
template <int F, int SHADE>
__device__ __forceinline__ float4 stoch_point(const TriplanarCall &c, float u, float v, float lam, float ux,
                                              float uy, float ul, int32_t *tap3)
{
    int l0, l1;
    float f;
    levels_of(c.tex, lam, l0, l1, f);
    const int l = ul >= 1.0f - f ? l1 : l0;
    const int wl = max(1, c.tex.w >> l), hl = max(1, c.tex.h >> l);
    int ix, iy;
    float tx, ty;
    raster(wrap_coord(c.tex.wrap, u), wl, ix, tx);
    raster(wrap_coord(c.tex.wrap, v), hl, iy, ty);
    const int x = wrap_tap(c.tex.wrap, ix + pick_off_2p24<F>(tx, ux), wl);
    const int y = wrap_tap(c.tex.wrap, iy + pick_off_2p24<F>(ty, uy), hl);
    if (tap3) {
        tap3[0] = l;
        tap3[1] = x;
        tap3[2] = y;
    }
    return shade<SHADE>(c.g, texel(c.tex, l, x, y));
}

// All taps of the filter on the level pair of lambda, weighted by `wgt`:
// texels (before) or shaded texels (after) added into sum.
template <int F, int SHADE, int MODE>
__device__ __forceinline__ void det_point(const TriplanarCall &c, float u, float v, float lam, float wgt, float4 &sum)
{
    int l0, l1;
    float f;
    levels_of(c.tex, lam, l0, l1, f);
    const float uu = wrap_coord(c.tex.wrap, u), vv = wrap_coord(c.tex.wrap, v);
    constexpr int NT = Taps<F>::n;
    constexpr int F0 = Taps<F>::first;
    for (int li = 0; li < 2; ++li) {
        const float pl = li == 0 ? 1.0f - f : f;
        if (pl == 0.0f)
            continue;
        const int l = li == 0 ? l0 : l1;
        const int wl = max(1, c.tex.w >> l), hl = max(1, c.tex.h >> l);
        int ix, iy;
        float tx, ty, wx[4], wy[4];
        raster(uu, wl, ix, tx);
        raster(vv, hl, iy, ty);
        if constexpr (F == NEAREST) {
            ix += tx >= 0.5f;
            iy += ty >= 0.5f;
        }
        axis_weights<F>(tx, wx);
        axis_weights<F>(ty, wy);
#pragma unroll
        for (int b = 0; b < NT; ++b) {
            const int y = wrap_tap(c.tex.wrap, iy + F0 + b, hl);
#pragma unroll
            for (int a = 0; a < NT; ++a) {
                const float w = (wgt * pl) * (wx[a] * wy[b]);
                const float4 t = texel(c.tex, l, wrap_tap(c.tex.wrap, ix + F0 + a, wl), y);
                const float4 val = MODE == BEFORE ? t : shade<SHADE>(c.g, t);
                sum.x = __builtin_fmaf(w, val.x, sum.x);
                sum.y = __builtin_fmaf(w, val.y, sum.y);
                sum.z = __builtin_fmaf(w, val.z, sum.z);
                sum.w = __builtin_fmaf(w, val.w, sum.w);
            }
        }
    }
}

// Usable query: finite point, normal and lambda, and finite projected
// coordinates p_k * scale.
__device__ __forceinline__ bool tri_finite(const float *q, float scale)
{
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 7; ++k)
        ok &= __builtin_isfinite(q[k]);
#pragma unroll
    for (int k = 0; k < 3; ++k)
        ok &= __builtin_isfinite(q[k] * scale);
    return ok;
}

__device__ __forceinline__ void tri_weights(const float *nrm, float w[3], float &W)
{
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const float a = nrm[i] * nrm[i];
        w[i] = a * a;
    }
    W = (w[0] + w[1]) + w[2];
}

// Sampled forms: plane_mode 1 (any filter mode) or a stochastic filter.
template <int F, int SHADE, int MODE>
__global__ __launch_bounds__(256) void k_tri_sampled(TriplanarCall c, int log_g)
{
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int G = 1 << log_g;
    const int64_t q = gid >> log_g;
    const int lane = (int)(gid & (G - 1));
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    const bool active = q < c.n;
    if (active) {
        float qq[8];
        const float4 a0 = reinterpret_cast<const float4 *>(c.q)[2 * q];
        const float4 a1 = reinterpret_cast<const float4 *>(c.q)[2 * q + 1];
        qq[0] = a0.x, qq[1] = a0.y, qq[2] = a0.z, qq[3] = a0.w, qq[4] = a1.x, qq[5] = a1.y, qq[6] = a1.z;
        if (!tri_finite(qq, c.scale)) {
            const float nan = __builtin_nanf("");
            acc = make_float4(nan, nan, nan, nan);
            if (c.taps)
                for (int s = lane; s < c.spp; s += G)
                    for (int k = 0; k < 4; ++k)
                        c.taps[(q * c.spp + s) * 4 + k] = SF_TAP_NONE;
        } else {
            float w[3], W;
            tri_weights(qq + 3, w, W);
            const float C0 = w[0] / W, C1 = (w[0] + w[1]) / W;
            for (int s = lane; s < c.spp; s += G) {
                const uint4 wd = pcg4d(make_uint4((uint32_t)q, (uint32_t)s, 0u, c.seed));
                // x and y as 24-bit lattice indices (thresholds scaled by 2^24), plane and level as uniforms
                const float ux = u24i(wd.x), uy = u24i(wd.y), up = u24(wd.z), ul = u24(wd.w);
                if (c.plane_mode == 0) {
                    // MODE == STOCH here: all three planes with the sample's uniforms
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        float u, v;
                        tri_uv(qq, j, c.scale, u, v);
                        const float4 val = stoch_point<F, SHADE>(c, u, v, qq[6], ux, uy, ul, nullptr);
                        const float b = w[j] / W;
                        acc.x = __builtin_fmaf(b, val.x, acc.x);
                        acc.y = __builtin_fmaf(b, val.y, acc.y);
                        acc.z = __builtin_fmaf(b, val.z, acc.z);
                        acc.w = __builtin_fmaf(b, val.w, acc.w);
                    }
                    continue;
                }
                const int j = (up >= C0) + (up >= C1);
                float u, v;
                tri_uv(qq, j, c.scale, u, v);
                int32_t *tp = c.taps ? c.taps + (q * c.spp + s) * 4 : nullptr;
                if (tp)
                    tp[0] = j;
                if constexpr (MODE == STOCH) {
                    acc = add4(acc, stoch_point<F, SHADE>(c, u, v, qq[6], ux, uy, ul, tp ? tp + 1 : nullptr));
                } else {
                    float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
                    det_point<F, SHADE, MODE>(c, u, v, qq[6], 1.0f, sum);
                    acc = add4(acc, MODE == BEFORE ? shade<SHADE>(c.g, sum) : sum);
                    if (tp)
                        tp[1] = tp[2] = tp[3] = SF_TAP_NONE;
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

// Fully deterministic blend: sum_j b_j filter_j.
template <int F, int SHADE, int MODE>
__global__ __launch_bounds__(256) void k_tri_det(TriplanarCall c)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= c.n)
        return;
    float qq[8];
    const float4 a0 = reinterpret_cast<const float4 *>(c.q)[2 * q];
    const float4 a1 = reinterpret_cast<const float4 *>(c.q)[2 * q + 1];
    qq[0] = a0.x, qq[1] = a0.y, qq[2] = a0.z, qq[3] = a0.w, qq[4] = a1.x, qq[5] = a1.y, qq[6] = a1.z;
    if (!tri_finite(qq, c.scale)) {
        const float nan = __builtin_nanf("");
        store<SHADE>(c.out, q, make_float4(nan, nan, nan, nan));
        return;
    }
    float w[3], W;
    tri_weights(qq + 3, w, W);
    float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        float u, v;
        tri_uv(qq, j, c.scale, u, v);
        det_point<F, SHADE, MODE>(c, u, v, qq[6], w[j] / W, sum);
    }
    store<SHADE>(c.out, q, MODE == BEFORE ? shade<SHADE>(c.g, sum) : sum);
}

template <int F, int SHADE, int MODE>
static void launch_t3(const TriplanarCall &c, hipStream_t s)
{
    if (c.plane_mode == 0 && MODE != STOCH) {
        k_tri_det<F, SHADE, MODE><<<dim3((uint32_t)((c.n + 255) / 256)), dim3(256), 0, s>>>(c);
        return;
    }
    const int G = lane_group(c.n, c.spp);
    const int64_t threads = c.n * G;
    k_tri_sampled<F, SHADE, MODE><<<dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s>>>(c, __builtin_ctz(G));
}

template <int F, int SHADE>
static void launch_t2(const TriplanarCall &c, hipStream_t s)
{
    if (c.mode == STOCH)
        launch_t3<F, SHADE, STOCH>(c, s);
    else if (c.mode == BEFORE)
        launch_t3<F, SHADE, BEFORE>(c, s);
    else
        launch_t3<F, SHADE, AFTER>(c, s);
}

template <int F>
static void launch_t1(const TriplanarCall &c, hipStream_t s)
{
    if (c.shade == SF_SHADE_GGX)
        launch_t2<F, SF_SHADE_GGX>(c, s);
    else
        launch_t2<F, SF_SHADE_NONE>(c, s);
}

hipError_t launch_triplanar(const TriplanarCall &c, hipStream_t s)
{
    switch (c.filter) {
    case NEAREST:
        launch_t1<NEAREST>(c, s);
        break;
    case LINEAR:
        launch_t1<LINEAR>(c, s);
        break;
    default:
        launch_t1<BSPLINE3>(c, s);
        break;
    }
    return hipGetLastError();
}

}  // namespace sfk
