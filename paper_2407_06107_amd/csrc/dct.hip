// DCT texture compressor (Sec. 5 "Texture compression"): 8x8 blocks, the
// six lowest-frequency coefficients per channel in one 32-bit word.  The
// decoder is part of the texel fetch (tex2d.hpp), so every 2-D filter reads
// SF_DCT8 textures.
//
// Two passes over all levels at once, one thread per block: the first
// takes each channel's largest |AC| per level (wavefront max, then one
// atomic max per wavefront and channel on the float's bits, valid for
// non-negative values); the second recomputes the coefficients and writes
// the codes.  Every coefficient is one fixed chain of binary32 fused
// multiply-adds, so the codes are reproducible bit for bit.
#include "sf_device.hpp"
#include "sf_internal.hpp"
#include "tex2d.hpp"

#pragma clang fp contract(off)

namespace sfk {

__device__ __forceinline__ float dct_basis(int k, int x) { return k == 0 ? DCT_C0 : (k == 1 ? dct_c1(x) : dct_c2(x)); }

// Level and block of a global block index.
__device__ __forceinline__ int level_of(const DctEncodeCall &c, int64_t b)
{
    int l = 0;
    while (l + 1 < c.levels && b >= c.first_block[l + 1])
        ++l;
    return l;
}

// Six coefficients, zigzag order (0,0) (1,0) (0,1) (0,2) (1,1) (2,0), of the
// four channels of block (bx, by) of an RGBA8 level.
__device__ void block_coeffs(const uint8_t *lv, int wl, int hl, int bx, int by, float C[4][6])
{
    float R[4][3][8];
#pragma unroll
    for (int y = 0; y < 8; ++y) {
        const int yy = min(by * 8 + y, hl - 1);
        float v[4][8];
#pragma unroll
        for (int x = 0; x < 8; ++x) {
            const int xx = min(bx * 8 + x, wl - 1);
            const uint32_t px = reinterpret_cast<const uint32_t *>(lv)[(int64_t)yy * wl + xx];
#pragma unroll
            for (int ch = 0; ch < 4; ++ch)
                v[ch][x] = (float)((px >> (8 * ch)) & 0xffu) / 255.0f;
        }
#pragma unroll
        for (int ch = 0; ch < 4; ++ch)
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                float acc = 0.0f;
#pragma unroll
                for (int x = 0; x < 8; ++x)
                    acc = __builtin_fmaf(dct_basis(u, x), v[ch][x], acc);
                R[ch][u][y] = acc;
            }
    }
    constexpr int U[6] = {0, 1, 0, 0, 1, 2}, V[6] = {0, 0, 1, 2, 1, 0};
#pragma unroll
    for (int ch = 0; ch < 4; ++ch)
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            float acc = 0.0f;
#pragma unroll
            for (int y = 0; y < 8; ++y)
                acc = __builtin_fmaf(dct_basis(V[k], y), R[ch][U[k]][y], acc);
            C[ch][k] = acc;
        }
}

__global__ __launch_bounds__(256) void k_dct_zero(float *range, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        range[i] = 0.0f;
}

__global__ __launch_bounds__(256) void k_dct_range(DctEncodeCall c)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool active = b < c.first_block[c.levels];
    const int l = active ? level_of(c, b) : c.levels;      // inactive lanes: a level no lane has
    float m[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (active) {
        const int wl = max(1, c.w >> l), hl = max(1, c.h >> l), bw = (wl + 7) >> 3;
        const int64_t j = b - c.first_block[l];
        float C[4][6];
        block_coeffs(c.src + c.src_off[l], wl, hl, (int)(j % bw), (int)(j / bw), C);
#pragma unroll
        for (int ch = 0; ch < 4; ++ch)
#pragma unroll
            for (int k = 1; k < 6; ++k)
                m[ch] = __builtin_fmaxf(m[ch], __builtin_fabsf(C[ch][k]));
    }
    const int l0 = __builtin_amdgcn_readfirstlane(l);
    if (__all(l == l0)) {
        if (l0 >= c.levels)
            return;
#pragma unroll
        for (int ch = 0; ch < 4; ++ch)
            for (int s = 32; s >= 1; s >>= 1)
                m[ch] = __builtin_fmaxf(m[ch], __shfl_xor(m[ch], s));
        if ((threadIdx.x & 63) == 0)
#pragma unroll
            for (int ch = 0; ch < 4; ++ch)
                atomicMax(reinterpret_cast<unsigned int *>(c.range) + 4 * l0 + ch, __float_as_uint(m[ch]));
    } else if (active) {
#pragma unroll
        for (int ch = 0; ch < 4; ++ch)
            atomicMax(reinterpret_cast<unsigned int *>(c.range) + 4 * l + ch, __float_as_uint(m[ch]));
    }
}

__global__ __launch_bounds__(256) void k_dct_codes(DctEncodeCall c)
{
    const int64_t b = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (b >= c.first_block[c.levels])
        return;
    const int l = level_of(c, b);
    const int wl = max(1, c.w >> l), hl = max(1, c.h >> l), bw = (wl + 7) >> 3;
    const int64_t j = b - c.first_block[l];
    float C[4][6];
    block_coeffs(c.src + c.src_off[l], wl, hl, (int)(j % bw), (int)(j / bw), C);
    uint32_t word[4];
#pragma unroll
    for (int ch = 0; ch < 4; ++ch) {
        const float R = c.range[4 * l + ch];
        const float sc = R > 0.0f ? 15.0f / R : 0.0f;
        const int dc = min(max((int)__builtin_floorf(C[ch][0] * 15.875f + 0.5f), 0), 127);
        uint32_t wd = (uint32_t)dc;
#pragma unroll
        for (int k = 1; k < 6; ++k) {
            int a = 15;
            if (R > 0.0f)
                a = min(max((int)__builtin_floorf(C[ch][k] * sc + 0.5f), -15), 15) + 15;
            wd |= (uint32_t)a << (7 + 5 * (k - 1));
        }
        word[ch] = wd;
    }
    reinterpret_cast<uint4 *>(c.dst + c.dst_off[l])[j] = make_uint4(word[0], word[1], word[2], word[3]);
}

hipError_t launch_dct_encode(const DctEncodeCall &c, hipStream_t s)
{
    const int64_t nb = c.first_block[c.levels];
    k_dct_zero<<<dim3((uint32_t)((4 * c.levels + 255) / 256)), dim3(256), 0, s>>>(c.range, 4 * c.levels);
    const dim3 grid((uint32_t)((nb + 255) / 256)), block(256);
    k_dct_range<<<grid, block, 0, s>>>(c);
    k_dct_codes<<<grid, block, 0, s>>>(c);
    return hipGetLastError();
}

}  // namespace sfk
