// Device helpers of the 3-D paths, shared by the ray-march kernels of libsf
// and by the benchmark's gather-only copy of the stochastic march: voxel
// addressing through a raw buffer resource, the per-step raster position,
// the brick occupancy test and the per-axis tap picks.
#pragma once
#include "sf_device.hpp"
#include "sf_internal.hpp"

#pragma clang fp contract(off)

namespace sfk {

constexpr uint32_t kBufferFlags = 0x00020000u;  // raw buffer, 32-bit data format

// Byte offset of voxel (x, y, z) and whether it lies in the grid.  A tap
// outside the grid gets offset 0 (always valid) and its value is discarded.
// P2: nx and ny are powers of two, so the index is built with shifts.
template <bool HALF, bool P2>
__device__ __forceinline__ uint32_t voxel_offset(const VolArgs &v, int x, int y, int z, bool &ok)
{
    ok = ((uint32_t)x < (uint32_t)v.nx) & ((uint32_t)y < (uint32_t)v.ny) & ((uint32_t)z < (uint32_t)v.nz);
    uint32_t idx;
    if constexpr (P2)
        idx = ((((uint32_t)z << v.ly) | (uint32_t)y) << v.lx) | (uint32_t)x;
    else
        idx = __umul24(__umul24((uint32_t)z, (uint32_t)v.ny) + (uint32_t)y, (uint32_t)v.nx) + (uint32_t)x;
    return ok ? idx * (HALF ? 2u : 4u) : 0u;
}

template <bool HALF>
__device__ __forceinline__ uint32_t voxel_bits(__amdgpu_buffer_rsrc_t rs, uint32_t off)
{
    if constexpr (HALF)
        return __builtin_amdgcn_raw_buffer_load_b16(rs, off, 0, 0);
    else
        return __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
}

template <bool HALF>
__device__ __forceinline__ float bits_value(uint32_t b)
{
    if constexpr (HALF)
        return half_bits_to_float((uint16_t)b);
    else
        return __builtin_bit_cast(float, b);
}

template <bool HALF>
__device__ __forceinline__ float voxel_load(__amdgpu_buffer_rsrc_t rs, uint32_t off)
{
    return bits_value<HALF>(voxel_bits<HALF>(rs, off));
}

// Whether the 4x4x4 taps around raster cell i0 (offsets -1..2 per axis) lie
// inside the grid with two voxels to spare past each x row, so that
// voxel_row4_half may read every row.
__device__ __forceinline__ bool rows4_inside(const VolArgs &v, const int i0[3])
{
    return i0[0] - 1 >= 0 && i0[0] + 4 < v.nx && i0[1] - 1 >= 0 && i0[1] + 2 < v.ny && i0[2] - 1 >= 0 &&
           i0[2] + 2 < v.nz;
}

// The four binary16 voxels e..e+3 (e a voxel index; a row of the grid that
// extends at least two voxels past e+3) read with one 12-byte load at the
// 4-byte boundary at or below voxel e and a funnel shift.
__device__ __forceinline__ void voxel_row4_half(__amdgpu_buffer_rsrc_t rs, uint32_t e, float sg[4])
{
    typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
    const u32x3 w = __builtin_bit_cast(u32x3, __builtin_amdgcn_raw_buffer_load_b96(rs, (2u * e) & ~3u, 0, 0));
    const uint32_t sh = (e & 1u) * 16u;   // the row starts in the high half of its first word
    const uint32_t d0 = __builtin_amdgcn_alignbit(w.y, w.x, sh);
    const uint32_t d1 = __builtin_amdgcn_alignbit(w.z, w.y, sh);
    sg[0] = half_bits_to_float((uint16_t)d0);
    sg[1] = half_bits_to_float((uint16_t)(d0 >> 16));
    sg[2] = half_bits_to_float((uint16_t)d1);
    sg[3] = half_bits_to_float((uint16_t)(d1 >> 16));
}

// One voxel; zero outside the grid.
template <bool HALF>
__device__ __forceinline__ float voxel(__amdgpu_buffer_rsrc_t rs, const VolArgs &v, int x, int y, int z)
{
    bool ok;
    const uint32_t off = voxel_offset<HALF, false>(v, x, y, z, ok);
    const float val = voxel_load<HALF>(rs, off);
    return ok ? val : 0.0f;
}

__device__ __forceinline__ void step_coords(const RayGeom &g, float kh, int i0[3], float t[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        float p = __builtin_fmaf(kh, g.G[a], g.E[a]);
        float fl = __builtin_floorf(p);
        i0[a] = (int)fl;
        t[a] = p - fl;
    }
}

// True unless the lookup point's brick is known to be empty: a tap of any
// filter lies within [i0-1, i0+2] per axis, inside the brick's 2-voxel
// dilation, so a clear bit means every tap reads zero.  The brick
// coordinates are clamped to the grid's bricks, which is exact as well: for
// i0 < 0 the taps inside the grid lie in [0, 1], and for i0 at or beyond the
// last brick's end they lie in {n-1} (or nowhere), both within the dilation
// of the nearest brick; so no step whose taps can read a non-zero voxel is
// skipped, and the index always lies inside the mask.  The bit is extracted
// with the hardware's offset-mod-32 field extract.
// P2: nx and ny are powers of two, so are the brick counts along x and y
// (nx >> occ_log2, or 1 below one brick) and the index is built with shifts.
// clamp(x, 0, hi) for a wave-uniform hi in one instruction (the compiler
// forms v_med3_i32 only for compile-time bounds)
__device__ __forceinline__ int clamp0_uniform(int x, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(x), "s"(hi));
    return r;
}

template <bool P2 = false>
__device__ __forceinline__ bool brick_occupied(const VolArgs &v, const int i0[3])
{
    const uint32_t bx = (uint32_t)clamp0_uniform(i0[0] >> v.occ_log2, v.nbx - 1);
    const uint32_t by = (uint32_t)clamp0_uniform(i0[1] >> v.occ_log2, v.nby - 1);
    const uint32_t bz = (uint32_t)clamp0_uniform(i0[2] >> v.occ_log2, v.nbz - 1);
    uint32_t b;
    if constexpr (P2) {
        const int lbx = max(v.lx - v.occ_log2, 0), lby = max(v.ly - v.occ_log2, 0);
        b = (((bz << lby) | by) << lbx) | bx;
    } else {
        b = __umul24(__umul24(bz, (uint32_t)v.nby) + by, (uint32_t)v.nbx) + bx;
    }
    return __builtin_amdgcn_ubfe(v.occ[b >> 5], b, 1u) != 0u;
}

// The loaded bits, or 0 (the value 0.0) for a tap outside the grid.  The
// empty asm pins the select to the loaded 32-bit word, ahead of the
// conversion, so that the compiler does not move it past the conversion.
__device__ __forceinline__ uint32_t masked_bits(uint32_t b, bool ok)
{
    uint32_t r = ok ? b : 0u;
    asm volatile("" : "+v"(r));
    return r;
}

template <int F, int VAR>
__device__ __forceinline__ void pick3(const float t[3], uint3 w, int o[3])
{
    if constexpr (VAR == 0) {
        o[0] = pick_off_2p24<F>(t[0], u24i(w.x));
        o[1] = pick_off_2p24<F>(t[1], u24i(w.y));
        o[2] = pick_off_2p24<F>(t[2], u24i(w.z));
    } else {
        float u = u24(w.x);
        o[0] = pick_off_reuse<F>(t[0], u);
        o[1] = pick_off_reuse<F>(t[1], u);
        o[2] = pick_off_reuse<F>(t[2], u);
    }
}

}  // namespace sfk
