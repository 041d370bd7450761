// Benchmark-only library libsf_bench.so (not part of libsf: nothing in
// include/ declares it, and no product path loads it).
//
// The gather-only twin of the stochastic tricubic ray march: the ceiling the
// memory system sets for that kernel's access pattern.  It is the timed
// kernel (k_ray_stoch for the cubic B-spline, binary16 grid, independent
// uniforms, occupancy mask, power-of-two addressing) with the random pick
// taken out: the same ray setup, XCD block mapping, per-step raster position,
// brick words loaded a step ahead, pipelined binary16 voxel load (one per
// step, past the grid's end in an empty brick) and result write; the tap of step k on axis a is
// i0 - 1 + ((k >> 2a) & 3), which walks all 64 taps of the 4 x 4 x 4 range
// the B-spline pick draws from (so the gathers spread over the same cache
// footprint), and the densities are added in a plain binary32 sum.
// t(twin) / t(real kernel) on the same launch is the fraction of this gather
// ceiling the real kernel reaches.
#include "volume_dev.hpp"

#pragma clang fp contract(off)

namespace sfk {

__global__ __launch_bounds__(256) void k_ray_gather_twin(RaymarchCall c, uint32_t nb_pad)
{
    const int64_t i = (int64_t)xcd_block(blockIdx.x, nb_pad) * 256 + threadIdx.x;
    if (i >= c.n)
        return;
    RayGeom g;
    const int st = ray_setup_dev(c.vol.wmin, c.vol.scale, c.rays + 8 * i, c.steps, g);
    if (st != 0) {
        c.T[i] = st == 1 ? 1.0f : __builtin_nanf("");
        return;
    }
    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(c.vol.base), 0,
                                                                  (int)c.vol.bytes, kBufferFlags);
    const __amdgpu_buffer_rsrc_t rm = occ_rsrc(c.vol);
    constexpr uint32_t kOut = 0xfffffffeu;
    struct At {
        float p[3];
        int i0[3];
        uint32_t word, bit;
    };
    float tau = 0.0f;
    uint32_t pend;
    float kh = 0.5f;
    auto step = [&](int k, const At &cur, At &nxt) {
        const bool empty = __builtin_amdgcn_ubfe(cur.word, cur.bit, 1u) != 0u;
        kh += 1.0f;
        step_pos(g, kh, nxt.p, nxt.i0);
        nxt.word = brick_word(rm, c.vol, nxt.i0, nxt.bit);
        tau += bits_value<true>(pend);     // step k - 1
        uint32_t off = kOut;
        if (!empty)
            off = voxel_offset_or_outside<true, true>(c.vol, cur.i0[0] + (k & 3) - 1, cur.i0[1] + ((k >> 2) & 3) - 1,
                                                      cur.i0[2] + ((k >> 4) & 3) - 1);
        pend = voxel_bits<true>(rs, off);  // step k
    };
    At a, b;
    step_pos(g, kh, a.p, a.i0);
    a.word = brick_word(rm, c.vol, a.i0, a.bit);
    __builtin_amdgcn_sched_barrier(0);
    pend = voxel_bits<true>(rs, kOut | (a.bit >> 31));
    int k = 0;
    for (; k + 1 < c.steps; k += 2) {
        step(k, a, b);
        step(k + 1, b, a);
    }
    if (k < c.steps)
        step(k, a, b);
    tau += bits_value<true>(pend);
    c.T[i] = expf(-(g.dt * tau));
}

}  // namespace sfk

// Launch over n rays of `steps` steps through a binary16 grid with power-of-
// two x and y sides and an occupancy mask (the benchmark's configuration).
// grid: device pointer to nz*ny*nx binary16 densities; occ: the mask that
// sf_build_occupancy wrote for bricks of 2^brick_log2; rays: n x 8 floats,
// 16-byte aligned; T: n floats.  Returns 0, or -1 for arguments outside that
// configuration, or the HIP error of the launch.
extern "C" int sfb_gather_twin(const void *grid, int32_t nx, int32_t ny, int32_t nz, const float *wmin,
                               const float *scale, const uint32_t *occ, int32_t brick_log2, const float *rays,
                               int64_t n, int32_t steps, float *T, void *stream)
{
    const bool p2 = nx > 0 && ny > 0 && (nx & (nx - 1)) == 0 && (ny & (ny - 1)) == 0;
    const uint64_t bytes = (uint64_t)nx * ny * nz * 2;
    if (!grid || !occ || !rays || !T || !wmin || !scale || !p2 || nz < 1 || bytes > 0xffffffffULL || n < 1 ||
        n > 0x7fffffffLL || steps < 1 || brick_log2 < 1 || brick_log2 > 6 ||
        (reinterpret_cast<uintptr_t>(rays) & 15) != 0)
        return -1;
    sfk::RaymarchCall c{};
    c.vol.base = grid;
    c.vol.nx = nx;
    c.vol.ny = ny;
    c.vol.nz = nz;
    c.vol.fmt = SF_R16F;
    c.vol.bytes = (uint32_t)bytes;
    for (int k = 0; k < 3; ++k) {
        c.vol.wmin[k] = wmin[k];
        c.vol.scale[k] = scale[k];
    }
    const sfk::OccLayout o = sfk::occ_layout(nx, ny, nz, brick_log2);
    if (o.bits > sfk::kMaxOccBits || (int64_t)o.sy * (o.nbz + 1) >= (1LL << 23))
        return -1;
    c.vol.occ = occ;
    c.vol.occ_log2 = brick_log2;
    c.vol.nbx = o.nbx;
    c.vol.nby = o.nby;
    c.vol.nbz = o.nbz;
    c.vol.occ_sx = o.sx;
    c.vol.occ_sy = o.sy;
    c.vol.occ_bytes = (uint32_t)(o.words * 4);
    c.vol.lx = __builtin_ctz((unsigned)nx);
    c.vol.ly = __builtin_ctz((unsigned)ny);
    c.rays = rays;
    c.n = n;
    c.steps = steps;
    c.spp = 1;
    c.T = T;
    const uint32_t nb = (uint32_t)((n + 255) / 256), nb_pad = (nb + 7u) & ~7u;
    sfk::k_ray_gather_twin<<<dim3(nb_pad), dim3(256), 0, (hipStream_t)stream>>>(c, nb_pad);
    return (int)hipGetLastError();
}
