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

// floor(p) as an integer in one instruction (a conversion that rounds toward
// -inf); exact for the raster positions the ray setup admits (|p| < 2^22).
__device__ __forceinline__ int floor_to_int(float p)
{
    int r;
    asm("v_cvt_flr_i32_f32 %0, %1" : "=v"(r) : "v"(p));
    return r;
}

// Raster position p of the step at kh = k + 1/2 and its cell i0 = floor(p).
__device__ __forceinline__ void step_pos(const RayGeom &g, float kh, float p[3], int i0[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        p[a] = __builtin_fmaf(kh, g.G[a], g.E[a]);
        i0[a] = floor_to_int(p[a]);
    }
}

// The fractions t = p - i0: exact, and equal to p - floor(p) (i0 converts
// back to binary32 exactly).
__device__ __forceinline__ void step_frac(const float p[3], const int i0[3], float t[3])
{
#pragma unroll
    for (int a = 0; a < 3; ++a)
        t[a] = p[a] - (float)i0[a];
}

__device__ __forceinline__ void step_coords(const RayGeom &g, float kh, int i0[3], float t[3])
{
    float p[3];
    step_pos(g, kh, p, i0);
    step_frac(p, i0, t);
}

// Byte offset of voxel (x, y, z), or for a tap outside the grid an offset at
// or past the end of every grid (a grid holds less than 2^32 bytes, a
// multiple of its voxel size), where the raw buffer load reads 0, the value
// +0.0: no select on the loaded value is needed.
template <bool HALF, bool P2>
__device__ __forceinline__ uint32_t voxel_offset_or_outside(const VolArgs &v, int x, int y, int z)
{
    const bool ok = ((uint32_t)x < (uint32_t)v.nx) & ((uint32_t)y < (uint32_t)v.ny) & ((uint32_t)z < (uint32_t)v.nz);
    uint32_t idx;
    if constexpr (P2)
        idx = ((((uint32_t)z << v.ly) | (uint32_t)y) << v.lx) | (uint32_t)x;
    else
        idx = __umul24(__umul24((uint32_t)z, (uint32_t)v.ny) + (uint32_t)y, (uint32_t)v.nx) + (uint32_t)x;
    return ok ? idx * (HALF ? 2u : 4u) : (HALF ? 0xfffffffeu : 0xfffffffcu);
}

// The brick mask (OccLayout) as a raw buffer: loads past its end read 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t occ_rsrc(const VolArgs &v)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(v.occ), 0, (int)v.occ_bytes, kBufferFlags);
}

// The mask word that holds the bit of the lookup point's brick, and the
// bit's index b (bit b & 31 of the word).  A 1 bit means the brick is
// provably empty, so that a step there can be skipped exactly: a tap of any
// filter lies within [i0-1, i0+2] per axis, inside the 2-voxel dilation of
// i0's brick.  Brick coordinates are arithmetic shifts of i0, and the bit
// index is formed without clamps:
// - a point whose brick coordinates all lie in [-1, nb] (every point of the
//   grid's raster box, i0 >= -1) reads its own brick's bit, or a 0: a
//   coordinate of -1 in x or y lands on the padding bit that ends the
//   previous row or the padding row that ends the previous plane, -1 in z
//   gives a negative index (a word offset past the end, read as 0), nb in x
//   or y lands on padding and nb in z on padding or past the end;
// - a point with a brick coordinate below -1 or above nb has i0 <= -3 or
//   i0 >= n + 2 on that axis (bricks of at least 2 voxels), so all of its
//   taps lie outside the grid and read zero whatever the bit says.
// The 24-bit multiplies are exact for coordinates in [-1, nb]: nbz*sy and sx
// stay below 2^23, and the mask holds at most 2^30 bits.
__device__ __forceinline__ uint32_t brick_word(__amdgpu_buffer_rsrc_t rm, const VolArgs &v, const int i0[3],
                                               uint32_t &b)
{
    const int bx = i0[0] >> v.occ_log2, by = i0[1] >> v.occ_log2, bz = i0[2] >> v.occ_log2;
    b = (uint32_t)(__mul24(__mul24(bz, v.occ_sy) + by, v.occ_sx) + bx);
    return __builtin_amdgcn_raw_buffer_load_b32(rm, (b >> 3) & ~3u, 0, 0);
}

// True when the lookup point's brick is provably empty (brick_word's bit).
__device__ __forceinline__ bool brick_empty(__amdgpu_buffer_rsrc_t rm, const VolArgs &v, const int i0[3])
{
    uint32_t b;
    const uint32_t w = brick_word(rm, v, i0, b);
    return __builtin_amdgcn_ubfe(w, b, 1u) != 0u;
}

// clamp(x, 0, hi) for a wave-uniform hi in one instruction (the compiler
// forms v_med3_i32 only for compile-time bounds)
__device__ __forceinline__ int clamp0_uniform(int x, int hi)
{
    int r;
    asm("v_med3_i32 %0, %1, 0, %2" : "=v"(r) : "v"(x), "s"(hi));
    return r;
}

// brick_empty with the brick coordinates clamped to the grid's bricks, for
// the comparators: a point just outside the grid (i0 = -1, or at or past the
// last brick's end) tests the nearest brick, whose 2-voxel dilation holds
// every tap of such a point that lies inside the grid, so it too may be
// skipped exactly (the comparators' steps at the grid's faces read their
// taps one by one, so skipping them matters there).
__device__ __forceinline__ bool brick_empty_clamped(__amdgpu_buffer_rsrc_t rm, const VolArgs &v, const int i0[3])
{
    const int bx = clamp0_uniform(i0[0] >> v.occ_log2, v.nbx - 1);
    const int by = clamp0_uniform(i0[1] >> v.occ_log2, v.nby - 1);
    const int bz = clamp0_uniform(i0[2] >> v.occ_log2, v.nbz - 1);
    const uint32_t b = (uint32_t)(__mul24(__mul24(bz, v.occ_sy) + by, v.occ_sx) + bx);
    const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(rm, (b >> 3) & ~3u, 0, 0);
    return __builtin_amdgcn_ubfe(w, b, 1u) != 0u;
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
