// 3-D paths of libsf: transmittance ray marching through a density grid
// (Sec. 5 "Offline rendering": density lookups with trilinear / tricubic
// filters and their stochastic one-lookup forms), emission ray marching
// through a temperature grid (Sec. 5 "Filtering nonlinear physical
// properties") and filtered point lookups.
//
// One lane marches one ray.  The stochastic kernel is the hot path: per step
// it forms the raster position, hashes (ray, sample, step, seed), picks one
// tap per axis by inverse CDF on the separable weights (Sec. 4.1 FRS) and
// gathers ONE voxel; the optical depth is a compensated binary32 sum.
#include "volume_dev.hpp"

#pragma clang fp contract(off)

namespace sfk {

// Black-body emission (Sec. 5, "Filtering nonlinear physical properties"):
// spectral radiance in W sr^-1 m^-2 nm^-1 at 700, 546.1 and 435.8 nm of a
// temperature T in kelvin, B = A_l / (e^x - 1) with x = c2 / (lambda T).
// e^x is evaluated as exp2(K_l / T) on the transcendental unit; below
// x = 1/2 a degree-7 Taylor polynomial of e^x - 1 replaces the subtraction.
// T <= 0 emits nothing, NaN stays NaN.  Binary32 values (not decisions):
// the relative error is about (x + 3) ulp.
struct PlanckConst {
    static constexpr double h = 6.62607015e-34, c = 299792458.0, k = 1.380649e-23;
    static constexpr double A(double nm)
    {
        return 2.0 * h * c * c / (nm * 1e-9 * nm * 1e-9 * nm * 1e-9 * nm * 1e-9 * nm * 1e-9) * 1e-9;
    }
    static constexpr double K(double nm) { return h * c / (nm * 1e-9 * k) * 1.4426950408889634074; }
};

__device__ __forceinline__ float planck_band(float r, float A, float K)
{
    const float y = K * r;   // x log2(e)
    float em1;
    if (y < 0.72134752f) {
        const float x = y * 0.69314718f;
        float p = __builtin_fmaf(x, 1.0f / 5040.0f, 1.0f / 720.0f);
        p = __builtin_fmaf(x, p, 1.0f / 120.0f);
        p = __builtin_fmaf(x, p, 1.0f / 24.0f);
        p = __builtin_fmaf(x, p, 1.0f / 6.0f);
        p = __builtin_fmaf(x, p, 0.5f);
        p = __builtin_fmaf(x, p, 1.0f);
        em1 = x * p;
    } else {
        em1 = __builtin_amdgcn_exp2f(y) - 1.0f;   // +inf beyond y = 128: B = 0
    }
    return A * __builtin_amdgcn_rcpf(em1);
}

__device__ __forceinline__ void planck3(float T, float B[3])
{
    constexpr float A0 = (float)PlanckConst::A(700.0), A1 = (float)PlanckConst::A(546.1),
                    A2 = (float)PlanckConst::A(435.8);
    constexpr float K0 = (float)PlanckConst::K(700.0), K1 = (float)PlanckConst::K(546.1),
                    K2 = (float)PlanckConst::K(435.8);
    float r = __builtin_amdgcn_rcpf(T);
    r = __builtin_fmaf(__builtin_fmaf(-T, r, 1.0f), r, r);   // one Newton step
    const bool cold = T <= 0.0f;
    B[0] = cold ? 0.0f : planck_band(r, A0, K0);
    B[1] = cold ? 0.0f : planck_band(r, A1, K1);
    B[2] = cold ? 0.0f : planck_band(r, A2, K2);
}

// ---------------------------------------------------------------- ray march
template <int F, bool HALF, int VAR, bool DBG, bool OCC, bool P2>
__global__ __launch_bounds__(256) void k_ray_stoch(RaymarchCall c, uint32_t nb_pad)
{
    static_assert(!(DBG && OCC), "the tap dump records every step, so it never skips bricks");
    const int64_t i = (int64_t)xcd_block(blockIdx.x, nb_pad) * 256 + threadIdx.x;
    if (i >= c.n)
        return;
    RayGeom g;
    int st = ray_setup_dev(c.vol.wmin, c.vol.scale, c.rays + 8 * i, c.steps, g);
    if (st != 0) {
        c.T[i] = st == 1 ? 1.0f : __builtin_nanf("");
        if constexpr (DBG) {
            int64_t per = (int64_t)3 * c.spp * c.steps;
            for (int64_t k = 0; k < per; ++k)
                c.taps[per * i + k] = SF_TAP_NONE;
        }
        return;
    }
    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(c.vol.base), 0,
                                                                  (int)c.vol.bytes, kBufferFlags);
    // optical depth and the mean over samples as compensated binary32 sums:
    // tau within 2u tau of its exact value, so T = e^(-dt tau) within about
    // (2 tau + 3) u relative of the exact transmittance of the picked voxels
    __amdgpu_buffer_rsrc_t rm;
    if constexpr (OCC)
        rm = occ_rsrc(c.vol);
    CompSum Tsum;
    Tsum.init();
    for (int s = 0; s < c.spp; ++s) {
        StepHash h;
        h.init((uint32_t)i, (uint32_t)s, c.seed);
        CompSum tau;
        tau.init();
        // software pipeline: a step's voxel is added one step later, so its
        // load overlaps the next step's arithmetic
        uint32_t pend = 0;
        float kh = 0.5f;
        if constexpr (OCC) {
            // With the brick mask, the brick word of step k + 1 is loaded
            // during step k as well, ahead of step k's voxel, and every step
            // loads a voxel (a step in an empty brick loads past the grid's
            // end and adds the 0.0 it reads, which leaves the compensated
            // sum unchanged): every pass then finds the same two loads in
            // flight in the same order, and a step waits only for loads
            // issued one step earlier.  Two steps per pass, so that the
            // state of step k + 1 is formed in place of step k - 1's.
            constexpr uint32_t kOut = HALF ? 0xfffffffeu : 0xfffffffcu;
            struct At {
                float p[3];
                int i0[3];
                uint32_t word, bit;   // brick word and bit index
            };
            auto step = [&](int k, const At &cur, At &nxt) {
                const bool empty = __builtin_amdgcn_ubfe(cur.word, cur.bit, 1u) != 0u;
                kh += 1.0f;
                step_pos(g, kh, nxt.p, nxt.i0);
                nxt.word = brick_word(rm, c.vol, nxt.i0, nxt.bit);
                tau.add(bits_value<HALF>(pend));   // step k - 1
                uint32_t off = kOut;
                if (!empty) {
                    float t[3];
                    int o[3];
                    step_frac(cur.p, cur.i0, t);
                    pick3<F, VAR>(t, h.at((uint32_t)k), o);
                    off = voxel_offset_or_outside<HALF, P2>(c.vol, cur.i0[0] + o[0], cur.i0[1] + o[1],
                                                             cur.i0[2] + o[2]);
                }
                pend = voxel_bits<HALF>(rs, off);  // step k
            };
            At a, b;
            step_pos(g, kh, a.p, a.i0);
            a.word = brick_word(rm, c.vol, a.i0, a.bit);
            // a first load of zero behind the first brick word (its offset
            // depends on the brick index so that it is not moved ahead)
            __builtin_amdgcn_sched_barrier(0);
            pend = voxel_bits<HALF>(rs, kOut | (a.bit >> 31));
            int k = 0;
            for (; k + 1 < c.steps; k += 2) {
                step(k, a, b);
                step(k + 1, b, a);
            }
            if (k < c.steps)
                step(k, a, b);
            tau.add(bits_value<HALF>(pend));
            Tsum.add(expf(-(g.dt * tau.value())));
            continue;
        }
        for (int k = 0; k < c.steps; ++k, kh += 1.0f) {
            int i0[3], o[3];
            float p[3], t[3];
            step_pos(g, kh, p, i0);
            step_frac(p, i0, t);
            pick3<F, VAR>(t, h.at((uint32_t)k), o);
            int x = i0[0] + o[0], y = i0[1] + o[1], z = i0[2] + o[2];
            if constexpr (DBG) {
                int32_t *tp = c.taps + (((int64_t)i * c.spp + s) * c.steps + k) * 3;
                tp[0] = x;
                tp[1] = y;
                tp[2] = z;
            }
            const uint32_t off = voxel_offset_or_outside<HALF, P2>(c.vol, x, y, z);
            tau.add(bits_value<HALF>(pend));     // step k-1
            pend = voxel_bits<HALF>(rs, off);    // step k (0 outside the grid)
        }
        tau.add(bits_value<HALF>(pend));
        Tsum.add(expf(-(g.dt * tau.value())));
    }
    c.T[i] = Tsum.value() / (float)c.spp;
}

// Deterministic comparators: all taps of the separable footprint per step.
// BEFORE: exp(-dt sum_k sum_i w_i sigma_i); AFTER: prod_k sum_i w_i e^{-dt sigma_i}.
// Binary32 throughout.  The AFTER product's factors are multiplied as
// binary32 pairs, and a step's factor f_k enters in the form that is known
// to a few ulp of itself: f_k = sum_i w_i e^{-dt sigma_i} when it is below
// 1/2, else 1 - a_k with a_k = sum_i w_i (1 - e^{-dt sigma_i}) (a factor
// close to 1 formed directly would carry the rounding of the binary32
// weights, which sum to 1 +- 3e-7, into every one of 256 factors).  Both
// modes then stay within about 20 u tau of the exact transmittance,
// tau = -ln T, u = 2^-24.
template <int F, bool HALF, int MODE, bool OCC>
__global__ __launch_bounds__(256) void k_ray_det(RaymarchCall c, uint32_t nb_pad)
{
    const int64_t i = (int64_t)xcd_block(blockIdx.x, nb_pad) * 256 + threadIdx.x;
    if (i >= c.n)
        return;
    RayGeom g;
    int st = ray_setup_dev(c.vol.wmin, c.vol.scale, c.rays + 8 * i, c.steps, g);
    if (st != 0) {
        c.T[i] = st == 1 ? 1.0f : __builtin_nanf("");
        return;
    }
    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(c.vol.base), 0,
                                                                  (int)c.vol.bytes, kBufferFlags);
    __amdgpu_buffer_rsrc_t rm;
    if constexpr (OCC)
        rm = occ_rsrc(c.vol);
    constexpr int NT = Taps<F>::n;
    constexpr int F0 = Taps<F>::first;
    const float dt = g.dt;
    CompSum tau;
    tau.init();
    PairProduct Tp;
    Tp.init();
    float kh = 0.5f;
    for (int k = 0; k < c.steps; ++k, kh += 1.0f) {
        int i0[3];
        float t[3];
        float wx[4], wy[4], wz[4];
        step_coords(g, kh, i0, t);
        if constexpr (OCC) {
            if (brick_empty_clamped(rm, c.vol, i0))
                continue;   // every tap is zero: before adds 0, after multiplies by 1 - 0
        }
        if constexpr (F == NEAREST) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                i0[a] += t[a] >= 0.5f;
        }
        axis_weights<F>(t[0], wx);
        axis_weights<F>(t[1], wy);
        axis_weights<F>(t[2], wz);
        // BEFORE: acc = sum_i w_i sigma_i.  AFTER: acc = a_k, accf = f_k.
        float acc = 0.0f, accf = 0.0f;
        // one x row of taps (NT voxels) into the sums, in tap order
        auto add_row = [&](const float *sg, int by, int cz) {
            float row = 0.0f, rowf = 0.0f;
#pragma unroll
            for (int ax = 0; ax < NT; ++ax) {
                if constexpr (MODE == BEFORE) {
                    row = __builtin_fmaf(wx[ax], sg[ax], row);
                } else {
                    float e, m;
                    exp_neg_pair(sg[ax] * dt, e, m);
                    row = __builtin_fmaf(wx[ax], m, row);
                    rowf = __builtin_fmaf(wx[ax], e, rowf);
                }
            }
            const float wyz = wy[by] * wz[cz];
            acc = __builtin_fmaf(wyz, row, acc);
            if constexpr (MODE != BEFORE)
                accf = __builtin_fmaf(wyz, rowf, accf);
        };
        // Binary16 tricubic steps whose 4x4x4 taps lie inside the grid (with
        // two voxels to spare past the row in x) read each row of four
        // voxels with one 12-byte load at the 4-byte boundary at or below it
        // and take the voxels by a funnel shift; other steps load tap by tap.
        // The values, and so the sums, are the same either way.
        bool rows = false;
        if constexpr (HALF && NT == 4)
            rows = rows4_inside(c.vol, i0);
        if (rows) {
            const uint32_t nx = (uint32_t)c.vol.nx, ny = (uint32_t)c.vol.ny;
            const uint32_t e0 = ((uint32_t)(i0[2] - 1) * ny + (uint32_t)(i0[1] - 1)) * nx + (uint32_t)(i0[0] - 1);
#pragma unroll
            for (int cz = 0; cz < NT; ++cz) {
#pragma unroll
                for (int by = 0; by < NT; ++by) {
                    float sg[4];
                    voxel_row4_half(rs, e0 + ((uint32_t)cz * ny + (uint32_t)by) * nx, sg);
                    add_row(sg, by, cz);
                }
            }
        } else {
#pragma unroll
            for (int cz = 0; cz < NT; ++cz) {
#pragma unroll
                for (int by = 0; by < NT; ++by) {
                    float sg[NT];
#pragma unroll
                    for (int ax = 0; ax < NT; ++ax)
                        sg[ax] = voxel<HALF>(rs, c.vol, i0[0] + F0 + ax, i0[1] + F0 + by, i0[2] + F0 + cz);
                    add_row(sg, by, cz);
                }
            }
        }
        if constexpr (MODE == BEFORE) {
            tau.add(acc);
        } else {
            if (accf < 0.5f)
                Tp.mul(accf, 0.0f);
            else
                Tp.mul_one_minus(acc);
        }
    }
    c.T[i] = MODE == BEFORE ? expf(-(dt * tau.value())) : Tp.value();
}

// ------------------------------------------------------------ emission march
// An emitting, non-absorbing medium of temperatures: a ray gathers
// dt * sum_k E_k at three wavelengths, E_k the step's emission.  Stochastic:
// E_k = B(T) of the one voxel the step picks (keys, picks and the occupancy
// skip as in the transmittance march; empty bricks emit nothing).  The sums
// are compensated binary32 sums of positive terms.
// Gaussian footprint perpendicular to the ray (Sec. 5: filtering after
// shading under minification): the plane's basis by the branchless
// construction of Duff et al., "Building an Orthonormal Basis, Revisited"
// (JCGT 6(1), 2017), scaled to raster axes A, B; per step the key
// (ray, sample | 2^31, step, seed) gives u0, u1 and Box-Muller with the
// contract ln and cos/sin moves p to fma(g2, B, fma(g1, A, p)).
struct PerpFrame {
    float A[3], B[3];
};

__device__ __forceinline__ PerpFrame perp_frame(const float *r8, const float *scale, float sigma)
{
    const float dx = r8[3], dy = r8[4], dz = r8[5];
    const float sg = __builtin_copysignf(1.0f, dz);
    const float a = -1.0f / (sg + dz);
    const float b = (dx * dy) * a;
    const float e1[3] = {1.0f + ((sg * dx) * dx) * a, sg * b, -sg * dx};
    const float e2[3] = {b, sg + (dy * dy) * a, -dy};
    PerpFrame f;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        f.A[i] = (sigma * e1[i]) * scale[i];
        f.B[i] = (sigma * e2[i]) * scale[i];
    }
    return f;
}

// The samples of a ray are spread over G = 2^log_g adjacent lanes (a
// power of two up to 64, inside one wave) and their sums reduced by a
// butterfly, so small images with many samples still fill the chip.
template <int F, bool HALF, int VAR, bool DBG, bool OCC, bool P2, bool JIT = false>
__global__ __launch_bounds__(256) void k_emit_stoch(RaymarchCall c, uint32_t nb_pad, int log_g)
{
    const int64_t gid = (int64_t)xcd_block(blockIdx.x, nb_pad) * 256 + threadIdx.x;
    const int G = 1 << log_g;
    const int64_t i = gid >> log_g;
    const int lane = (int)(gid & (G - 1));
    if (i >= c.n)
        return;   // the whole group of lanes shares i
    RayGeom g;
    int st = ray_setup_dev(c.vol.wmin, c.vol.scale, c.rays + 8 * i, c.steps, g);
    if (st != 0) {
        const float v = st == 1 ? 0.0f : __builtin_nanf("");
        if (lane == 0) {
            c.T[3 * i] = v;
            c.T[3 * i + 1] = v;
            c.T[3 * i + 2] = v;
        }
        if constexpr (DBG) {
            const int64_t per = (int64_t)3 * c.steps;
            for (int s = lane; s < c.spp; s += G)
                for (int64_t k = 0; k < per; ++k)
                    c.taps[((int64_t)i * c.spp + s) * per + k] = SF_TAP_NONE;
        }
        return;
    }
    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(c.vol.base), 0,
                                                                  (int)c.vol.bytes, kBufferFlags);
    __amdgpu_buffer_rsrc_t rm;
    if constexpr (OCC)
        rm = occ_rsrc(c.vol);
    CompSum acc[3];
    acc[0].init();
    acc[1].init();
    acc[2].init();
    PerpFrame pf;
    if constexpr (JIT)
        pf = perp_frame(c.rays + 8 * i, c.vol.scale, c.footprint);
    for (int s = lane; s < c.spp; s += G) {
        StepHash h, hj;
        h.init((uint32_t)i, (uint32_t)s, c.seed);
        if constexpr (JIT)
            hj.init((uint32_t)i, (uint32_t)s | 0x80000000u, c.seed);
        uint32_t pend = 0;
        float kh = 0.5f;
        for (int k = 0; k < c.steps; ++k, kh += 1.0f) {
            int i0[3], o[3];
            float t[3];
            if constexpr (JIT) {
                const uint3 wj = hj.at((uint32_t)k);
                const float rr = __builtin_sqrtf(-2.0f * lnc(1.0f - u24(wj.x)));
                float cs, sn;
                sincos2pi(u24(wj.y), cs, sn);
                const float g1 = rr * cs, g2 = rr * sn;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    float p = __builtin_fmaf(kh, g.G[a], g.E[a]);
                    p = __builtin_fmaf(g2, pf.B[a], __builtin_fmaf(g1, pf.A[a], p));
                    const float fl = __builtin_floorf(p);
                    i0[a] = (int)fl;
                    t[a] = p - fl;
                }
            } else {
                step_coords(g, kh, i0, t);
            }
            if constexpr (OCC) {
                if (brick_empty(rm, c.vol, i0))
                    continue;
            }
            pick3<F, VAR>(t, h.at((uint32_t)k), o);
            int x = i0[0] + o[0], y = i0[1] + o[1], z = i0[2] + o[2];
            if constexpr (DBG) {
                int32_t *tp = c.taps + (((int64_t)i * c.spp + s) * c.steps + k) * 3;
                tp[0] = x;
                tp[1] = y;
                tp[2] = z;
            }
            const uint32_t off = voxel_offset_or_outside<HALF, P2>(c.vol, x, y, z);
            float B[3];
            planck3(bits_value<HALF>(pend), B);    // step k-1
            acc[0].add(B[0]);
            acc[1].add(B[1]);
            acc[2].add(B[2]);
            pend = voxel_bits<HALF>(rs, off);      // step k (0 outside the grid)
        }
        float B[3];
        planck3(bits_value<HALF>(pend), B);
        acc[0].add(B[0]);
        acc[1].add(B[1]);
        acc[2].add(B[2]);
    }
    // the lanes' sums (at most 64, positive) meet in a butterfly
    float e[3] = {acc[0].value(), acc[1].value(), acc[2].value()};
    for (int m = G >> 1; m >= 1; m >>= 1) {
        e[0] += __shfl_xor(e[0], m);
        e[1] += __shfl_xor(e[1], m);
        e[2] += __shfl_xor(e[2], m);
    }
    if (lane == 0) {
        const float sc = g.dt / (float)c.spp;
        c.T[3 * i] = e[0] * sc;
        c.T[3 * i + 1] = e[1] * sc;
        c.T[3 * i + 2] = e[2] * sc;
    }
}

// Deterministic emission: E_k = B(sum_i w_i T_i) before shading,
// sum_i w_i B(T_i) after; binary32 weights and per-step sums of positive
// terms, steps summed with compensation.
template <int F, bool HALF, int MODE, bool OCC>
__global__ __launch_bounds__(256) void k_emit_det(RaymarchCall c, uint32_t nb_pad)
{
    const int64_t i = (int64_t)xcd_block(blockIdx.x, nb_pad) * 256 + threadIdx.x;
    if (i >= c.n)
        return;
    RayGeom g;
    int st = ray_setup_dev(c.vol.wmin, c.vol.scale, c.rays + 8 * i, c.steps, g);
    if (st != 0) {
        const float v = st == 1 ? 0.0f : __builtin_nanf("");
        c.T[3 * i] = v;
        c.T[3 * i + 1] = v;
        c.T[3 * i + 2] = v;
        return;
    }
    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(c.vol.base), 0,
                                                                  (int)c.vol.bytes, kBufferFlags);
    __amdgpu_buffer_rsrc_t rm;
    if constexpr (OCC)
        rm = occ_rsrc(c.vol);
    constexpr int NT = Taps<F>::n;
    constexpr int F0 = Taps<F>::first;
    CompSum acc[3];
    acc[0].init();
    acc[1].init();
    acc[2].init();
    float kh = 0.5f;
    for (int k = 0; k < c.steps; ++k, kh += 1.0f) {
        int i0[3];
        float t[3];
        float wx[4], wy[4], wz[4];
        step_coords(g, kh, i0, t);
        if constexpr (OCC) {
            if (brick_empty_clamped(rm, c.vol, i0))
                continue;   // every tap is 0 K: no emission either way
        }
        if constexpr (F == NEAREST) {
#pragma unroll
            for (int a = 0; a < 3; ++a)
                i0[a] += t[a] >= 0.5f;
        }
        axis_weights<F>(t[0], wx);
        axis_weights<F>(t[1], wy);
        axis_weights<F>(t[2], wz);
        float e[3] = {0.0f, 0.0f, 0.0f};
        // one x row of temperatures into the sums, in tap order
        auto add_row = [&](const float *Tr, int by, int cz) {
            const float wyz = wy[by] * wz[cz];
#pragma unroll
            for (int ax = 0; ax < NT; ++ax) {
                const float T = Tr[ax];
                const float w = wx[ax] * wyz;
                if constexpr (MODE == BEFORE) {
                    e[0] = __builtin_fmaf(w, T, e[0]);
                } else {
                    float B[3];
                    planck3(T, B);
                    e[0] = __builtin_fmaf(w, B[0], e[0]);
                    e[1] = __builtin_fmaf(w, B[1], e[1]);
                    e[2] = __builtin_fmaf(w, B[2], e[2]);
                }
            }
        };
        // rows of four binary16 voxels by one load where every tap is inside
        // the grid, as in the transmittance comparators
        bool rows = false;
        if constexpr (HALF && NT == 4)
            rows = rows4_inside(c.vol, i0);
        if (rows) {
            const uint32_t nx = (uint32_t)c.vol.nx, ny = (uint32_t)c.vol.ny;
            const uint32_t e0 = ((uint32_t)(i0[2] - 1) * ny + (uint32_t)(i0[1] - 1)) * nx + (uint32_t)(i0[0] - 1);
#pragma unroll
            for (int cz = 0; cz < NT; ++cz) {
#pragma unroll
                for (int by = 0; by < NT; ++by) {
                    float Tr[4];
                    voxel_row4_half(rs, e0 + ((uint32_t)cz * ny + (uint32_t)by) * nx, Tr);
                    add_row(Tr, by, cz);
                }
            }
        } else {
#pragma unroll
            for (int cz = 0; cz < NT; ++cz) {
#pragma unroll
                for (int by = 0; by < NT; ++by) {
                    float Tr[NT];
#pragma unroll
                    for (int ax = 0; ax < NT; ++ax)
                        Tr[ax] = voxel<HALF>(rs, c.vol, i0[0] + F0 + ax, i0[1] + F0 + by, i0[2] + F0 + cz);
                    add_row(Tr, by, cz);
                }
            }
        }
        if constexpr (MODE == BEFORE) {
            float B[3];
            planck3(e[0], B);
            acc[0].add(B[0]);
            acc[1].add(B[1]);
            acc[2].add(B[2]);
        } else {
            acc[0].add(e[0]);
            acc[1].add(e[1]);
            acc[2].add(e[2]);
        }
    }
    c.T[3 * i] = acc[0].value() * g.dt;
    c.T[3 * i + 1] = acc[1].value() * g.dt;
    c.T[3 * i + 2] = acc[2].value() * g.dt;
}

// ------------------------------------------------------------- point lookups
// Point lookups shaded by black-body emission: out is n x 3.
template <int F, bool HALF>
__device__ void filter3d_planck(const Filter3DCall &c, int64_t i, int i0[3], const float t[3],
                                __amdgpu_buffer_rsrc_t rs)
{
    CompSum acc[3];
    acc[0].init();
    acc[1].init();
    acc[2].init();
    if (c.mode == STOCH) {
        for (int s = 0; s < c.spp; ++s) {
            uint4 w4 = pcg4d(make_uint4((uint32_t)i, (uint32_t)s, 0u, c.seed));
            uint3 w = make_uint3(w4.x, w4.y, w4.z);
            int o[3];
            if (c.variant == 0)
                pick3<F, 0>(t, w, o);
            else
                pick3<F, 1>(t, w, o);
            int tx = i0[0] + o[0], ty = i0[1] + o[1], tz = i0[2] + o[2];
            if (c.taps) {
                int32_t *tp = c.taps + ((int64_t)i * c.spp + s) * 3;
                tp[0] = tx;
                tp[1] = ty;
                tp[2] = tz;
            }
            float B[3];
            planck3(voxel<HALF>(rs, c.vol, tx, ty, tz), B);
            for (int k = 0; k < 3; ++k)
                acc[k].add(B[k]);
        }
        for (int k = 0; k < 3; ++k)
            c.out[3 * i + k] = acc[k].value() / (float)c.spp;
        return;
    }
    constexpr int NT = Taps<F>::n;
    constexpr int F0 = Taps<F>::first;
    if constexpr (F == NEAREST) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
            i0[a] += t[a] >= 0.5f;
    }
    float wx[4], wy[4], wz[4];
    axis_weights<F>(t[0], wx);
    axis_weights<F>(t[1], wy);
    axis_weights<F>(t[2], wz);
    // binary32 weights; the weighted terms are summed with compensation
    // (before: signed temperatures are allowed, so no positivity is assumed)
    for (int cz = 0; cz < NT; ++cz)
        for (int by = 0; by < NT; ++by)
            for (int ax = 0; ax < NT; ++ax) {
                const float wgt = (wx[ax] * wy[by]) * wz[cz];
                const float T = voxel<HALF>(rs, c.vol, i0[0] + F0 + ax, i0[1] + F0 + by, i0[2] + F0 + cz);
                if (c.mode == BEFORE) {
                    acc[0].add(wgt * T);
                } else {
                    float B[3];
                    planck3(T, B);
                    for (int k = 0; k < 3; ++k)
                        acc[k].add(wgt * B[k]);
                }
            }
    float B[3];
    if (c.mode == BEFORE)
        planck3(acc[0].value(), B);
    for (int k = 0; k < 3; ++k)
        c.out[3 * i + k] = c.mode == BEFORE ? B[k] : acc[k].value();
}

template <int F, bool HALF>
__global__ __launch_bounds__(256) void k_filter3d(Filter3DCall c)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= c.n)
        return;
    float x[3] = {c.pos[3 * i], c.pos[3 * i + 1], c.pos[3 * i + 2]};
    bool ok = __builtin_isfinite(x[0]) & __builtin_isfinite(x[1]) & __builtin_isfinite(x[2]);
    float p[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        p[a] = __builtin_fmaf(x[a] - c.vol.wmin[a], c.vol.scale[a], -0.5f);
        ok &= __builtin_fabsf(p[a]) <= 4194304.0f;
    }
    if (!ok) {
        const int ch = c.shade == SF_SHADE_PLANCK ? 3 : 1;
        for (int k = 0; k < ch; ++k)
            c.out[ch * i + k] = __builtin_nanf("");
        if (c.taps && c.mode == STOCH)
            for (int k = 0; k < 3 * c.spp; ++k)
                c.taps[(int64_t)3 * c.spp * i + k] = SF_TAP_NONE;
        return;
    }
    int i0[3];
    float t[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float fl = __builtin_floorf(p[a]);
        i0[a] = (int)fl;
        t[a] = p[a] - fl;
    }
    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(c.vol.base), 0,
                                                                  (int)c.vol.bytes, kBufferFlags);
    const bool trans = c.shade == SF_SHADE_TRANSMITTANCE;
    if (c.shade == SF_SHADE_PLANCK) {
        filter3d_planck<F, HALF>(c, i, i0, t, rs);
        return;
    }
    if (c.mode == STOCH) {
        CompSum acc;
        acc.init();
        for (int s = 0; s < c.spp; ++s) {
            uint4 w4 = pcg4d(make_uint4((uint32_t)i, (uint32_t)s, 0u, c.seed));
            uint3 w = make_uint3(w4.x, w4.y, w4.z);
            int o[3];
            if (c.variant == 0)
                pick3<F, 0>(t, w, o);
            else
                pick3<F, 1>(t, w, o);
            int tx = i0[0] + o[0], ty = i0[1] + o[1], tz = i0[2] + o[2];
            if (c.taps) {
                int32_t *tp = c.taps + ((int64_t)i * c.spp + s) * 3;
                tp[0] = tx;
                tp[1] = ty;
                tp[2] = tz;
            }
            float sg = voxel<HALF>(rs, c.vol, tx, ty, tz);
            acc.add(trans ? expf(-(sg * c.ds)) : sg);
        }
        c.out[i] = acc.value() / (float)c.spp;
        return;
    }
    constexpr int NT = Taps<F>::n;
    constexpr int F0 = Taps<F>::first;
    if constexpr (F == NEAREST) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
            i0[a] += t[a] >= 0.5f;
    }
    float wx[4], wy[4], wz[4];
    axis_weights<F>(t[0], wx);
    axis_weights<F>(t[1], wy);
    axis_weights<F>(t[2], wz);
    // binary32 weights, compensated sum (densities may be signed here)
    CompSum sum;
    sum.init();
    for (int cz = 0; cz < NT; ++cz)
        for (int by = 0; by < NT; ++by)
            for (int ax = 0; ax < NT; ++ax) {
                const float wgt = (wx[ax] * wy[by]) * wz[cz];
                const float sg = voxel<HALF>(rs, c.vol, i0[0] + F0 + ax, i0[1] + F0 + by, i0[2] + F0 + cz);
                const float v = (c.mode == BEFORE || !trans) ? sg : expf(-(sg * c.ds));
                sum.add(wgt * v);
            }
    float r = sum.value();
    if (c.mode == BEFORE && trans)
        r = expf(-(r * c.ds));
    c.out[i] = r;
}

// ---------------------------------------------------------- occupancy bricks
// One lane per bit of the mask (OccLayout): a padding bit is 0; a brick's
// bit is 1 when its box grown by 2 voxels on every side holds only zeros (a
// NaN counts as non-zero), the scan stopping at the first other voxel.  A
// wave's 64 bits are gathered with a ballot and written as two words.
template <bool HALF>
__global__ __launch_bounds__(256) void k_build_occ(VolArgs v, uint32_t *occ, int64_t words)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t bits = (int64_t)v.occ_sx * v.occ_sy * v.nbz;
    bool empty = false;
    if (b < bits) {
        const int bx = (int)(b % v.occ_sx), by = (int)((b / v.occ_sx) % v.occ_sy);
        const int bz = (int)(b / ((int64_t)v.occ_sx * v.occ_sy));
        if (bx < v.nbx && by < v.nby) {
            const int B = 1 << v.occ_log2;
            const int x0 = max(bx * B - 2, 0), x1 = min(bx * B + B + 2, v.nx);
            const int y0 = max(by * B - 2, 0), y1 = min(by * B + B + 2, v.ny);
            const int z0 = max(bz * B - 2, 0), z1 = min(bz * B + B + 2, v.nz);
            empty = true;
            for (int z = z0; z < z1 && empty; ++z)
                for (int y = y0; y < y1 && empty; ++y) {
                    const int64_t row = ((int64_t)z * v.ny + y) * v.nx;
                    for (int x = x0; x < x1; ++x) {
                        float val;
                        if constexpr (HALF)
                            val = half_bits_to_float(static_cast<const uint16_t *>(v.base)[row + x]);
                        else
                            val = static_cast<const float *>(v.base)[row + x];
                        empty &= val == 0.0f;
                    }
                }
        }
    }
    const uint64_t m = __ballot(empty);
    if ((threadIdx.x & 63) == 0) {
        const int64_t w0 = b >> 5;   // b is a multiple of 64 here
        if (w0 < words)
            occ[w0] = (uint32_t)m;
        if (w0 + 1 < words)
            occ[w0 + 1] = (uint32_t)(m >> 32);
    }
}

hipError_t launch_build_occupancy(const VolArgs &v, uint32_t *occ, hipStream_t s)
{
    const int64_t words = v.occ_bytes / 4;
    dim3 grid((uint32_t)((words * 32 + 255) / 256)), block(256);
    if (v.fmt == SF_R16F)
        k_build_occ<true><<<grid, block, 0, s>>>(v, occ, words);
    else
        k_build_occ<false><<<grid, block, 0, s>>>(v, occ, words);
    return hipGetLastError();
}

// ---------------------------------------------------------------- launchers
static uint32_t blocks_for(int64_t n) { return (uint32_t)((n + 255) / 256); }

template <int F, bool HALF, bool OCC, bool P2>
static void launch_ray_fo(const RaymarchCall &c, dim3 grid, hipStream_t s, uint32_t nb_pad)
{
    dim3 block(256);
    if (c.mode == STOCH) {
        if (c.variant)
            k_ray_stoch<F, HALF, 1, false, OCC, P2><<<grid, block, 0, s>>>(c, nb_pad);
        else
            k_ray_stoch<F, HALF, 0, false, OCC, P2><<<grid, block, 0, s>>>(c, nb_pad);
    } else if (c.mode == BEFORE) {
        k_ray_det<F, HALF, BEFORE, OCC><<<grid, block, 0, s>>>(c, nb_pad);
    } else {
        k_ray_det<F, HALF, AFTER, OCC><<<grid, block, 0, s>>>(c, nb_pad);
    }
}

template <int F, bool HALF>
static hipError_t launch_ray_f(const RaymarchCall &c, hipStream_t s)
{
    uint32_t nb = blocks_for(c.n);
    uint32_t nb_pad = (nb + 7u) & ~7u;
    dim3 grid(nb_pad), block(256);
    const bool p2 = c.vol.lx >= 0;
    if (c.mode == STOCH && c.taps) {
        // the tap dump records every step, so it never skips empty bricks
        if (c.variant)
            k_ray_stoch<F, HALF, 1, true, false, false><<<grid, block, 0, s>>>(c, nb_pad);
        else
            k_ray_stoch<F, HALF, 0, true, false, false><<<grid, block, 0, s>>>(c, nb_pad);
    } else if (c.vol.occ) {
        if (p2)
            launch_ray_fo<F, HALF, true, true>(c, grid, s, nb_pad);
        else
            launch_ray_fo<F, HALF, true, false>(c, grid, s, nb_pad);
    } else {
        if (p2)
            launch_ray_fo<F, HALF, false, true>(c, grid, s, nb_pad);
        else
            launch_ray_fo<F, HALF, false, false>(c, grid, s, nb_pad);
    }
    return hipGetLastError();
}

template <int F, bool HALF, int VAR, bool DBG, bool OCC, bool P2>
static void launch_emit_stoch(const RaymarchCall &c, hipStream_t s)
{
    const int G = lane_group(c.n, c.spp);
    const uint32_t nb = blocks_for(c.n * G);
    const uint32_t nb_pad = (nb + 7u) & ~7u;
    const int lg = __builtin_ctz(G);
    if (c.footprint > 0.0f)
        k_emit_stoch<F, HALF, VAR, DBG, OCC, P2, true><<<dim3(nb_pad), dim3(256), 0, s>>>(c, nb_pad, lg);
    else
        k_emit_stoch<F, HALF, VAR, DBG, OCC, P2, false><<<dim3(nb_pad), dim3(256), 0, s>>>(c, nb_pad, lg);
}

template <int F, bool HALF, bool OCC, bool P2>
static void launch_emit_fo(const RaymarchCall &c, dim3 grid, hipStream_t s, uint32_t nb_pad)
{
    dim3 block(256);
    if (c.mode == STOCH) {
        if (c.variant)
            launch_emit_stoch<F, HALF, 1, false, OCC, P2>(c, s);
        else
            launch_emit_stoch<F, HALF, 0, false, OCC, P2>(c, s);
    } else if (c.mode == BEFORE) {
        k_emit_det<F, HALF, BEFORE, OCC><<<grid, block, 0, s>>>(c, nb_pad);
    } else {
        k_emit_det<F, HALF, AFTER, OCC><<<grid, block, 0, s>>>(c, nb_pad);
    }
}

template <int F, bool HALF>
static hipError_t launch_emit_f(const RaymarchCall &c, hipStream_t s)
{
    uint32_t nb = blocks_for(c.n);
    uint32_t nb_pad = (nb + 7u) & ~7u;
    dim3 grid(nb_pad);
    const bool p2 = c.vol.lx >= 0;
    if (c.mode == STOCH && c.taps) {
        if (c.variant)
            launch_emit_stoch<F, HALF, 1, true, false, false>(c, s);
        else
            launch_emit_stoch<F, HALF, 0, true, false, false>(c, s);
    } else if (c.vol.occ) {
        if (p2)
            launch_emit_fo<F, HALF, true, true>(c, grid, s, nb_pad);
        else
            launch_emit_fo<F, HALF, true, false>(c, grid, s, nb_pad);
    } else {
        if (p2)
            launch_emit_fo<F, HALF, false, true>(c, grid, s, nb_pad);
        else
            launch_emit_fo<F, HALF, false, false>(c, grid, s, nb_pad);
    }
    return hipGetLastError();
}

hipError_t launch_emission(const RaymarchCall &c, hipStream_t s)
{
    const bool half = c.vol.fmt == SF_R16F;
    switch (c.filter) {
    case NEAREST:
        return half ? launch_emit_f<NEAREST, true>(c, s) : launch_emit_f<NEAREST, false>(c, s);
    case LINEAR:
        return half ? launch_emit_f<LINEAR, true>(c, s) : launch_emit_f<LINEAR, false>(c, s);
    default:
        return half ? launch_emit_f<BSPLINE3, true>(c, s) : launch_emit_f<BSPLINE3, false>(c, s);
    }
}

hipError_t launch_raymarch(const RaymarchCall &c, hipStream_t s)
{
    const bool half = c.vol.fmt == SF_R16F;
    switch (c.filter) {
    case NEAREST:
        return half ? launch_ray_f<NEAREST, true>(c, s) : launch_ray_f<NEAREST, false>(c, s);
    case LINEAR:
        return half ? launch_ray_f<LINEAR, true>(c, s) : launch_ray_f<LINEAR, false>(c, s);
    default:
        return half ? launch_ray_f<BSPLINE3, true>(c, s) : launch_ray_f<BSPLINE3, false>(c, s);
    }
}

hipError_t launch_filter3d(const Filter3DCall &c, hipStream_t s)
{
    dim3 grid(blocks_for(c.n)), block(256);
    const bool half = c.vol.fmt == SF_R16F;
    switch (c.filter) {
    case NEAREST:
        if (half)
            k_filter3d<NEAREST, true><<<grid, block, 0, s>>>(c);
        else
            k_filter3d<NEAREST, false><<<grid, block, 0, s>>>(c);
        break;
    case LINEAR:
        if (half)
            k_filter3d<LINEAR, true><<<grid, block, 0, s>>>(c);
        else
            k_filter3d<LINEAR, false><<<grid, block, 0, s>>>(c);
        break;
    default:
        if (half)
            k_filter3d<BSPLINE3, true><<<grid, block, 0, s>>>(c);
        else
            k_filter3d<BSPLINE3, false><<<grid, block, 0, s>>>(c);
        break;
    }
    return hipGetLastError();
}

}  // namespace sfk
