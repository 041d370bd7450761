// 2-D path of libsf: filtered, shaded texture lookups.
//
// Stochastic mode (Sec. 2.2 eq. stochastic-sum, Sec. 4.1 FRS): each sample
// picks one MIP level (Sec. 4.2.1) and one texel per axis by inverse CDF and
// shades that single texel; a query's samples are spread over a group of G
// lanes (G a power of two dividing the wavefront) and summed with a
// butterfly over those lanes.  Deterministic modes (Sec. 3,
// eqs. filter-before-shading / filtering-after-shading) visit every tap.
#include <algorithm>

#include "sf_device.hpp"
#include "sf_internal.hpp"
#include "tex2d.hpp"

#pragma clang fp contract(off)

namespace sfk {

// One thread's share of the stochastic lookups: lane `gid % G` of query
// `gid / G`, texels read from `base` (the texture in global memory, or the
// workgroup's LDS copy of it, at the same offsets).
template <int F, int SHADE, int VAR>
__device__ __forceinline__ void filter2d_stoch_thread(const Filter2DCall &c, const uint8_t *base, int log_g,
                                                      int64_t gid)
{
    const int G = 1 << log_g;
    const int64_t q = gid >> log_g;
    const int lane = (int)(gid & (G - 1));
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    const bool active = q < c.n;
    if (active) {
        float3 qq = make_float3(c.q[3 * q], c.q[3 * q + 1], c.q[3 * q + 2]);
        if (!query_ok(c.tex, qq)) {
            float nan = __builtin_nanf("");
            acc = make_float4(nan, nan, nan, nan);
            if (c.taps) {
                constexpr int TW = (F == KEYS3 || F == MITCHELL) ? 5 : 3;
                for (int s = lane; s < c.spp; s += G)
                    for (int k = 0; k < TW; ++k)
                        c.taps[(q * c.spp + s) * TW + k] = SF_TAP_NONE;
            }
        } else {
            const float uu = wrap_coord(c.tex.wrap, qq.x), vv = wrap_coord(c.tex.wrap, qq.y);
            int l0, l1;
            float f;
            levels_of(c.tex, qq.z, l0, l1, f);
            const float cl = 1.0f - f;
            const float h = 0.5f / (c.sigma * c.sigma);   // discrete Gaussian: 1/(2 sigma^2)
            for (int s = lane; s < c.spp; s += G) {
                uint4 w = pcg4d(make_uint4((uint32_t)q, (uint32_t)s, 0u, c.seed));
                int l = u24(w.w) >= cl ? l1 : l0;
                int wl = max(1, c.tex.w >> l), hl = max(1, c.tex.h >> l);
                int ix, iy;
                float tx, ty;
                raster(uu, wl, ix, tx);
                raster(vv, hl, iy, ty);
                if constexpr (F == KEYS3 || F == MITCHELL) {
                    // positivisation (Sec. 2.2): one tap from the positive and
                    // one from the negative product weights, W+ f(t+) - W- f(t-)
                    const uint4 w2 = pcg4d(make_uint4((uint32_t)q, (uint32_t)s, 1u, c.seed));
                    int ox, oy, nx, ny;
                    float A, B, Cn, Dn;
                    if constexpr (F == KEYS3) {
                        const KeysAxis kx = keys_axis(tx), ky = keys_axis(ty);
                        A = kx.Pp * ky.Pp, B = kx.Pm * ky.Pm, Cn = kx.Pp * ky.Pm, Dn = kx.Pm * ky.Pp;
                        if (u24(w.z) * (A + B) < A) {
                            ox = u24(w.x) * kx.Pp < kx.p1 ? 0 : 1;
                            oy = u24(w.y) * ky.Pp < ky.p1 ? 0 : 1;
                        } else {
                            ox = u24(w.x) * kx.Pm < kx.m0 ? -1 : 2;
                            oy = u24(w.y) * ky.Pm < ky.m0 ? -1 : 2;
                        }
                        if (u24(w2.z) * (Cn + Dn) < Cn) {
                            nx = u24(w2.x) * kx.Pp < kx.p1 ? 0 : 1;
                            ny = u24(w2.y) * ky.Pm < ky.m0 ? -1 : 2;
                        } else {
                            nx = u24(w2.x) * kx.Pm < kx.m0 ? -1 : 2;
                            ny = u24(w2.y) * ky.Pp < ky.p1 ? 0 : 1;
                        }
                    } else {
                        // Mitchell-Netravali: the sets follow the taps' signs
                        const PnAxis ax = mitchell_axis(tx), ay = mitchell_axis(ty);
                        A = ax.Pp * ay.Pp, B = ax.Pm * ay.Pm, Cn = ax.Pp * ay.Pm, Dn = ax.Pm * ay.Pp;
                        const bool pp = u24(w.z) * (A + B) < A;
                        ox = pn_pick(ax, pp, u24(w.x)) - 1;
                        oy = pn_pick(ay, pp, u24(w.y)) - 1;
                        const bool xpos = u24(w2.z) * (Cn + Dn) < Cn;
                        nx = pn_pick(ax, xpos, u24(w2.x)) - 1;
                        ny = pn_pick(ay, !xpos, u24(w2.y)) - 1;
                    }
                    const bool has_neg = (Cn + Dn) > 0.0f;
                    const int xp = wrap_tap(c.tex.wrap, ix + ox, wl), yp = wrap_tap(c.tex.wrap, iy + oy, hl);
                    const int xn = wrap_tap(c.tex.wrap, ix + nx, wl), yn = wrap_tap(c.tex.wrap, iy + ny, hl);
                    if (c.taps) {
                        int32_t *tp = c.taps + (q * c.spp + s) * 5;
                        tp[0] = l;
                        tp[1] = xp;
                        tp[2] = yp;
                        tp[3] = has_neg ? xn : SF_TAP_NONE;
                        tp[4] = has_neg ? yn : SF_TAP_NONE;
                    }
                    const float Wp = A + B, Wm = Cn + Dn;
                    const float4 vp = shade<SHADE>(c.g, texel(c.tex, base, l, xp, yp));
                    float4 vn = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (has_neg)
                        vn = shade<SHADE>(c.g, texel(c.tex, base, l, xn, yn));
                    acc.x += Wp * vp.x - Wm * vn.x;
                    acc.y += Wp * vp.y - Wm * vn.y;
                    acc.z += Wp * vp.z - Wm * vn.z;
                    acc.w += Wp * vp.w - Wm * vn.w;
                    continue;
                }
                int ox, oy;
                if constexpr (F == GAUSS_FRS) {
                    ox = gauss_frs_pick(tx, h, u24(w.x));
                    oy = gauss_frs_pick(ty, h, u24(w.y));
                } else if constexpr (F == GAUSS_FIS) {
                    gauss_fis_pick(tx, ty, c.sigma, u24(w.x), u24(w.y), ox, oy);
                } else if constexpr (F == BSPLINE3_FIS) {
                    // three uniforms per axis: words 0..2 of the key with step 0 (x), step 1 (y)
                    const uint4 w2 = pcg4d(make_uint4((uint32_t)q, (uint32_t)s, 1u, c.seed));
                    ox = bspline_fis_pick(tx, w.x, w.y, w.z);
                    oy = bspline_fis_pick(ty, w2.x, w2.y, w2.z);
                } else if constexpr (VAR == 0) {
                    ox = pick_off_2p24<F>(tx, u24i(w.x));
                    oy = pick_off_2p24<F>(ty, u24i(w.y));
                } else {
                    float u = u24(w.x);
                    ox = pick_off_reuse<F>(tx, u);
                    oy = pick_off_reuse<F>(ty, u);
                }
                int x, y;
                if constexpr (F == GAUSS_FIS) {
                    x = wrap_any(c.tex.wrap, ix + ox, wl);
                    y = wrap_any(c.tex.wrap, iy + oy, hl);
                } else {
                    x = wrap_tap(c.tex.wrap, ix + ox, wl);
                    y = wrap_tap(c.tex.wrap, iy + oy, hl);
                }
                if (c.taps) {
                    int32_t *tp = c.taps + (q * c.spp + s) * 3;
                    tp[0] = l;
                    tp[1] = x;
                    tp[2] = y;
                }
                acc = add4(acc, shade<SHADE>(c.g, texel(c.tex, base, l, x, y)));
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

// LDS: the workgroup first copies the texture's c.lds_bytes (every level, at
// the same offsets) into LDS and then walks the lookups in tiles of 256
// threads (tile t by workgroup t mod the grid size), its texel reads LDS
// reads.  Otherwise one tile per workgroup, texels from global memory.
template <int F, int SHADE, int VAR, bool LDS>
__global__ __launch_bounds__(256) void k_filter2d_stoch(Filter2DCall c, int log_g)
{
    if constexpr (LDS) {
        extern __shared__ uint4 lds_tex[];
        const int nw16 = c.lds_bytes >> 4;
        const uint4 *src16 = reinterpret_cast<const uint4 *>(c.tex.base);
        for (int k = threadIdx.x; k < nw16; k += 256)
            lds_tex[k] = src16[k];
        const int nw4 = c.lds_bytes >> 2;   // a tail of 4-byte words (RGBA8)
        const uint32_t *src4 = reinterpret_cast<const uint32_t *>(c.tex.base);
        uint32_t *dst4 = reinterpret_cast<uint32_t *>(lds_tex);
        for (int k = 4 * nw16 + (int)threadIdx.x; k < nw4; k += 256)
            dst4[k] = src4[k];
        __syncthreads();
        const uint8_t *lds_base = reinterpret_cast<const uint8_t *>(lds_tex);
        const int64_t total = c.n << log_g;
        for (int64_t t0 = (int64_t)blockIdx.x * 256; t0 < total; t0 += (int64_t)gridDim.x * 256)
            filter2d_stoch_thread<F, SHADE, VAR>(c, lds_base, log_g, t0 + threadIdx.x);
    } else {
        filter2d_stoch_thread<F, SHADE, VAR>(c, c.tex.base, log_g, (int64_t)blockIdx.x * 256 + threadIdx.x);
    }
}

// Split filtering (Sec. 3 eq. split-filtering-shading, estimated as in
// Sec. 4): per sample the stochastic level of the key's word 3 (the low-pass
// filter over levels, sampled), then shade(sum_i w_i t_i) of that level (the
// reconstruction filter, evaluated before shading).
template <int F, int SHADE>
__global__ __launch_bounds__(256) void k_filter2d_split(Filter2DCall c, int log_g)
{
    const int64_t gid = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int G = 1 << log_g;
    const int64_t q = gid >> log_g;
    const int lane = (int)(gid & (G - 1));
    float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
    const bool active = q < c.n;
    if (active) {
        float3 qq = make_float3(c.q[3 * q], c.q[3 * q + 1], c.q[3 * q + 2]);
        if (!query_ok(c.tex, qq)) {
            float nan = __builtin_nanf("");
            acc = make_float4(nan, nan, nan, nan);
            if (c.taps)
                for (int s = lane; s < c.spp; s += G)
                    for (int k = 0; k < 3; ++k)
                        c.taps[(q * c.spp + s) * 3 + k] = SF_TAP_NONE;
        } else {
            const float uu = wrap_coord(c.tex.wrap, qq.x), vv = wrap_coord(c.tex.wrap, qq.y);
            int l0, l1;
            float f;
            levels_of(c.tex, qq.z, l0, l1, f);
            const float cl = 1.0f - f;
            for (int s = lane; s < c.spp; s += G) {
                const uint4 w = pcg4d(make_uint4((uint32_t)q, (uint32_t)s, 0u, c.seed));
                const int l = u24(w.w) >= cl ? l1 : l0;
                if (c.taps) {
                    int32_t *tp = c.taps + (q * c.spp + s) * 3;
                    tp[0] = l;
                    tp[1] = SF_TAP_NONE;
                    tp[2] = SF_TAP_NONE;
                }
                acc = add4(acc, shade<SHADE>(c.g, recon_level<F>(c.tex, uu, vv, l)));
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

template <int F, int SHADE, int MODE>
__global__ __launch_bounds__(256) void k_filter2d_det(Filter2DCall c)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= c.n)
        return;
    float3 qq = make_float3(c.q[3 * q], c.q[3 * q + 1], c.q[3 * q + 2]);
    if (!query_ok(c.tex, qq)) {
        float nan = __builtin_nanf("");
        store<SHADE>(c.out, q, make_float4(nan, nan, nan, nan));
        return;
    }
    const float uu = wrap_coord(c.tex.wrap, qq.x), vv = wrap_coord(c.tex.wrap, qq.y);
    int l0, l1;
    float f;
    levels_of(c.tex, qq.z, l0, l1, f);
    constexpr int NT = Taps<F>::n;
    constexpr int F0 = Taps<F>::first;
    float4 sum = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int li = 0; li < 2; ++li) {
        const float pl = li == 0 ? 1.0f - f : f;
        if (pl == 0.0f)
            continue;
        const int l = li == 0 ? l0 : l1;
        int wl = max(1, c.tex.w >> l), hl = max(1, c.tex.h >> l);
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
                const float wgt = pl * wx[a] * wy[b];
                float4 t = texel(c.tex, l, wrap_tap(c.tex.wrap, ix + F0 + a, wl), y);
                float4 v = MODE == BEFORE ? t : shade<SHADE>(c.g, t);
                sum.x = __builtin_fmaf(wgt, v.x, sum.x);
                sum.y = __builtin_fmaf(wgt, v.y, sum.y);
                sum.z = __builtin_fmaf(wgt, v.z, sum.z);
                sum.w = __builtin_fmaf(wgt, v.w, sum.w);
            }
        }
    }
    store<SHADE>(c.out, q, MODE == BEFORE ? shade<SHADE>(c.g, sum) : sum);
}

// Deterministic Gaussian comparators, binary32 weights and compensated sums
// (the FIS window has up to 60 x 60 taps): the discrete Gaussian's
// normalised e^(-d^2 h) on the 4x4 window, or the FIS Gaussian's cell masses
// Phi((k + 1/2 - t)/sigma) - Phi((k - 1/2 - t)/sigma) on offsets -R..R+1,
// R = ceil(7 sigma) + 1, each mass taken from the tail on its own side of the
// lookup point (erfc of a positive argument), so that no mass is the small
// difference of two values near 1.
__device__ __forceinline__ void gauss4(float t, float h, float w[4])
{
    float W = 0.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float d = (float)(k - 1) - t;
        w[k] = expf(-((d * d) * h));
        W += w[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        w[k] /= W;
}

__device__ __forceinline__ float gauss_cell(float r2, float t, int k)
{
    const float a = ((float)k - 0.5f - t) / r2, b = ((float)k + 0.5f - t) / r2;
    // right of the point: 0.5 (erfc(a) - erfc(b)); left: 0.5 (erfc(-b) - erfc(-a))
    return a >= 0.0f ? 0.5f * (erfcf(a) - erfcf(b))
                     : (b <= 0.0f ? 0.5f * (erfcf(-b) - erfcf(-a)) : 1.0f - 0.5f * (erfcf(-a) + erfcf(b)));
}

template <int F, int SHADE, int MODE>
__global__ __launch_bounds__(256) void k_filter2d_gauss_det(Filter2DCall c)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= c.n)
        return;
    float3 qq = make_float3(c.q[3 * q], c.q[3 * q + 1], c.q[3 * q + 2]);
    if (!query_ok(c.tex, qq)) {
        float nan = __builtin_nanf("");
        store<SHADE>(c.out, q, make_float4(nan, nan, nan, nan));
        return;
    }
    const float uu = wrap_coord(c.tex.wrap, qq.x), vv = wrap_coord(c.tex.wrap, qq.y);
    int l0, l1;
    float f;
    levels_of(c.tex, qq.z, l0, l1, f);
    const float sig = c.sigma;
    const float h = 0.5f / (sig * sig), r2 = 1.41421356f * sig;
    const int R = (int)ceilf(7.0f * sig) + 1;
    const int first = F == GAUSS_FRS ? -1 : -R;
    const int ntap = F == GAUSS_FRS ? 4 : 2 * R + 2;
    CompSum sum[4];
    for (int k = 0; k < 4; ++k)
        sum[k].init();
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
        float gx[4], gy[4];
        if constexpr (F == GAUSS_FRS) {
            gauss4(tx, h, gx);
            gauss4(ty, h, gy);
        }
        for (int b = 0; b < ntap; ++b) {
            const float wy = F == GAUSS_FRS ? gy[b & 3] : gauss_cell(r2, ty, first + b);
            const int y = wrap_any(c.tex.wrap, iy + first + b, hl);
            for (int a = 0; a < ntap; ++a) {
                const float wx = F == GAUSS_FRS ? gx[a & 3] : gauss_cell(r2, tx, first + a);
                const float wgt = (pl * wx) * wy;
                const float4 t = texel(c.tex, l, wrap_any(c.tex.wrap, ix + first + a, wl), y);
                const float4 v = MODE == BEFORE ? t : shade<SHADE>(c.g, t);
                sum[0].add(wgt * v.x);
                sum[1].add(wgt * v.y);
                sum[2].add(wgt * v.z);
                sum[3].add(wgt * v.w);
            }
        }
    }
    const float4 r = make_float4(sum[0].value(), sum[1].value(), sum[2].value(), sum[3].value());
    store<SHADE>(c.out, q, MODE == BEFORE ? shade<SHADE>(c.g, r) : r);
}

// Workgroups of 256 lanes of kernel K with `smem` bytes of dynamic LDS
// resident on the current device at once, at least 1.
template <typename K>
static int64_t resident_blocks_smem(K kernel, int smem)
{
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, smem) != hipSuccess)
        return 512;
    return std::max<int64_t>(1, (int64_t)std::max(per_cu, 1) * std::max(ncu, 1));
}

template <int F, int SHADE>
static void launch_f2(const Filter2DCall &c, hipStream_t s)
{
    if constexpr (F <= KEYS3 || F == MITCHELL) {
        if (c.mode == SPLIT) {
            const int G = lane_group(c.n, c.spp);
            const int64_t threads = c.n * G;
            k_filter2d_split<F, SHADE>
                <<<dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s>>>(c, __builtin_ctz(G));
            return;
        }
    }
    if (c.mode == STOCH) {
        const int G = lane_group(c.n, c.spp);
        int log_g = __builtin_ctz(G);
        int64_t threads = c.n * G;
        dim3 grid((uint32_t)((threads + 255) / 256)), block(256);
        if constexpr (F <= BSPLINE3) {
            // resident workgroups at the largest staged texture (64 KiB)
            static const int64_t resident =
                resident_blocks_smem(k_filter2d_stoch<F, SHADE, 0, true>, kMaxLdsTexture);
            // Staging pays while every workgroup has one tile: with more
            // tiles than resident workgroups, the two workgroups per CU that
            // 64 KiB of LDS allows hide less latency than the full occupancy
            // of the global-memory kernel, whose texel reads hit the caches
            // (measured: 1 Mi queries x 16 samples 0.18 ms staged, 0.088 ms
            // from global memory; 4096 queries 7.9 us staged, 8.5 us).
            if (c.lds_bytes > 0 && (int64_t)grid.x <= resident) {
                const dim3 g2 = grid;
                if (c.variant)
                    k_filter2d_stoch<F, SHADE, 1, true><<<g2, block, (size_t)c.lds_bytes, s>>>(c, log_g);
                else
                    k_filter2d_stoch<F, SHADE, 0, true><<<g2, block, (size_t)c.lds_bytes, s>>>(c, log_g);
                return;
            }
            if (c.variant) {
                k_filter2d_stoch<F, SHADE, 1, false><<<grid, block, 0, s>>>(c, log_g);
                return;
            }
        }
        k_filter2d_stoch<F, SHADE, 0, false><<<grid, block, 0, s>>>(c, log_g);
    } else {
        dim3 grid((uint32_t)((c.n + 255) / 256)), block(256);
        if constexpr (F == GAUSS_FRS || F == GAUSS_FIS) {
            if (c.mode == BEFORE)
                k_filter2d_gauss_det<F, SHADE, BEFORE><<<grid, block, 0, s>>>(c);
            else
                k_filter2d_gauss_det<F, SHADE, AFTER><<<grid, block, 0, s>>>(c);
        } else {
            // the B-spline FIS realises the cubic B-spline itself
            constexpr int FD = F == BSPLINE3_FIS ? BSPLINE3 : F;
            if (c.mode == BEFORE)
                k_filter2d_det<FD, SHADE, BEFORE><<<grid, block, 0, s>>>(c);
            else
                k_filter2d_det<FD, SHADE, AFTER><<<grid, block, 0, s>>>(c);
        }
    }
}

template <int F>
static void launch_f1(const Filter2DCall &c, hipStream_t s)
{
    if (c.shade == SF_SHADE_GGX)
        launch_f2<F, SF_SHADE_GGX>(c, s);
    else if (c.shade == SF_SHADE_GGX_NORMAL)
        launch_f2<F, SF_SHADE_GGX_NORMAL>(c, s);
    else
        launch_f2<F, SF_SHADE_NONE>(c, s);
}

hipError_t launch_filter2d(const Filter2DCall &c, hipStream_t s)
{
    switch (c.filter) {
    case NEAREST:
        launch_f1<NEAREST>(c, s);
        break;
    case LINEAR:
        launch_f1<LINEAR>(c, s);
        break;
    case KEYS3:
        launch_f1<KEYS3>(c, s);
        break;
    case MITCHELL:
        launch_f1<MITCHELL>(c, s);
        break;
    case GAUSS_FRS:
        launch_f1<GAUSS_FRS>(c, s);
        break;
    case GAUSS_FIS:
        launch_f1<GAUSS_FIS>(c, s);
        break;
    case BSPLINE3_FIS:
        launch_f1<BSPLINE3_FIS>(c, s);
        break;
    default:
        launch_f1<BSPLINE3>(c, s);
        break;
    }
    return hipGetLastError();
}

}  // namespace sfk
