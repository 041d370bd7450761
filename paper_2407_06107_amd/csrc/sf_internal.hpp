// Internal interfaces of libsf: kernel argument blocks (passed by value as
// kernel arguments) and the host-side launchers behind the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sf.h"

namespace sfk {

// Host-side shading constants derived once per call from sf_ggx: with fixed
// directions the half vector, the cosines and the Fresnel term do not depend
// on the texel, only the roughness does.
struct GgxConst {
    float nh2, no, no2, ni, ni2;
    float spec_c;          // F / pi
    float kd[3], ks[3];    // radiance * (n.wi) / pi, radiance * (n.wi)
    float r_bias, r_scale;
    // normal-mapped shading: h, wo, wi in the tangent frame (e1, e2, n) of
    // the surface normal, Fresnel, radiance and the grey diffuse term
    float to[3], ti[3];
    float th[3], thl[3];   // h as a binary32 pair: th + thl
    float th_defect;       // 1 - |h|^2 in the (nearly orthonormal) frame
    float F;
    float rad[3], kdn[3];  // radiance, radiance * (1/2) / pi
};

struct Tex2DArgs {
    const uint8_t *base;
    int32_t w, h, levels, fmt, wrap, mip;
    int64_t off[SF_MAX_LEVELS];
    const float *dct_range;  // SF_DCT8 only
};

struct VolArgs {
    const void *base;
    int32_t nx, ny, nz, fmt;
    uint32_t bytes;          // size of the grid in bytes (< 2^32)
    float wmin[3], scale[3];
    const uint32_t *occ;     // brick mask (see OccLayout) or null
    int32_t occ_log2, nbx, nby, nbz;
    int32_t occ_sx, occ_sy;  // the mask's row length and rows per plane, in bricks
    uint32_t occ_bytes;      // size of the mask in bytes
    int32_t lx, ly;          // log2(nx), log2(ny) when both are powers of two, else -1
};

// Layout of the brick mask: one bit per brick, 1 when every voxel within 2
// voxels of the brick is zero (the brick is provably empty), else 0, in
// planes of sy = nby + 1 rows of sx = nbx + 1 bits: every row ends in a
// padding bit and every plane in a padding row, all 0.  Brick (bx, by, bz)
// is bit b = (bz*sy + by)*sx + bx, bit (b & 31) of 32-bit word b >> 5; the
// bits past the last brick in the last word are 0.  At most kMaxOccBits bits.
struct OccLayout {
    int32_t nbx, nby, nbz, sx, sy;
    int64_t bits, words;
};

constexpr int64_t kMaxOccBits = 1LL << 30;

inline OccLayout occ_layout(int32_t nx, int32_t ny, int32_t nz, int32_t log2b)
{
    OccLayout o;
    const int32_t B = 1 << log2b;
    o.nbx = (nx + B - 1) / B;
    o.nby = (ny + B - 1) / B;
    o.nbz = (nz + B - 1) / B;
    o.sx = o.nbx + 1;
    o.sy = o.nby + 1;
    o.bits = (int64_t)o.sx * o.sy * o.nbz;
    o.words = (o.bits + 31) / 32;
    return o;
}

struct Filter2DCall {
    Tex2DArgs tex;
    const float *q;
    int64_t n;
    int32_t filter, mode, spp, variant, shade;
    uint32_t seed;
    float sigma;
    GgxConst g;
    float *out;
    int32_t *taps;
    int32_t lds_bytes;  // > 0: the stochastic kernel stages the texture's first lds_bytes bytes in LDS
};

// Largest texture (all levels, from the base pointer) that the stochastic
// 2-D kernel stages in LDS.
constexpr int kMaxLdsTexture = 65536;

struct AnisoCall {
    Tex2DArgs tex;
    const float *q;  // n x {u, v, du/dx, dv/dx, du/dy, dv/dy}
    int64_t n;
    int32_t filter, mode, spp, shade, amax;
    uint32_t seed;
    float sigma;
    GgxConst g;
    float *out;
    int32_t *taps;
};

struct DctEncodeCall {
    const uint8_t *src;
    int64_t src_off[SF_MAX_LEVELS];
    uint8_t *dst;
    int64_t dst_off[SF_MAX_LEVELS];
    float *range;
    int32_t w, h, levels;
    int64_t first_block[SF_MAX_LEVELS + 1];  // prefix sums of the levels' block counts
};

struct TriplanarCall {
    Tex2DArgs tex;
    const float *q;  // n x {p, n, lambda, unused}
    int64_t n;
    int32_t filter, mode, spp, shade, plane_mode;
    uint32_t seed;
    float scale;
    GgxConst g;
    float *out;
    int32_t *taps;
};

struct Filter3DCall {
    VolArgs vol;
    const float *pos;
    int64_t n;
    int32_t filter, mode, spp, variant, shade;
    uint32_t seed;
    float ds;
    float *out;
    int32_t *taps;
};

struct RaymarchCall {
    VolArgs vol;
    const float *rays;
    int64_t n;
    int32_t steps, filter, mode, spp, variant;
    uint32_t seed;
    float *T;        // transmittance (n), or emission (n x 3)
    int32_t *taps;
    float footprint; // emission: perpendicular Gaussian, world units (0: none)
};

struct LatentArgs {
    const void *latents;
    const float *scales;
    int32_t dims, res[3], C, fmt, block_log2;
    float wmin[3], scale[3];
    __host__ __device__ int32_t nb(int a) const { return (res[a] + (1 << block_log2) - 1) >> block_log2; }
    __host__ __device__ int64_t nblocks() const { return (int64_t)nb(0) * nb(1) * nb(2); }
    // block of lattice point (x, y, z)
    __host__ __device__ int32_t block_at(int x, int y, int z) const
    {
        return ((z >> block_log2) * nb(1) + (y >> block_log2)) * nb(0) + (x >> block_log2);
    }
};

struct MlpArgs {
    const void *params;   // packed BF16: W1, b1, W2, b2, W3, b3
    int32_t in_dim, out_dim;
};

struct NeuralCall {
    LatentArgs lat;
    MlpArgs mlp;
    const float *q;
    const float *rays;
    int64_t n;
    int32_t steps, filter, mode, spp, shade;
    uint32_t seed;
    GgxConst g;
    float *out;
    float *T;
    int32_t *taps;
};

struct TrainCall {
    float *latents, *params, *m_lat, *v_lat, *m_par, *v_par;
    const int32_t *idx;
    const float *targets;
    int64_t batch, n_lattice;
    int32_t C, O;
    float lr_latent, lr_mlp, bc1, bc2;
    float inv_bc1, inv_bc2;   // 1 / bc1, 1 / bc2 (binary32 of the exact reciprocals)
    float *loss_out, *grad_params, *grad_latents;
};

// Launchers return hipSuccess or the launch error; arguments are validated.
hipError_t launch_filter2d(const Filter2DCall &c, hipStream_t s);
hipError_t launch_aniso(const AnisoCall &c, hipStream_t s);
hipError_t launch_dct_encode(const DctEncodeCall &c, hipStream_t s);
hipError_t launch_triplanar(const TriplanarCall &c, hipStream_t s);
hipError_t launch_filter3d(const Filter3DCall &c, hipStream_t s);
// Lanes per query for kernels that spread a query's samples over adjacent
// lanes: the largest power of two up to min(spp, 64) that keeps the grid
// within 2^31 work-items.
inline int lane_group(int64_t n, int spp)
{
    int G = 1;
    while (G * 2 <= spp && G * 2 <= 64 && n * (G * 2) <= (int64_t(1) << 31))
        G *= 2;
    return G;
}

hipError_t launch_raymarch(const RaymarchCall &c, hipStream_t s);
hipError_t launch_emission(const RaymarchCall &c, hipStream_t s);
hipError_t launch_build_occupancy(const VolArgs &v, uint32_t *occ, hipStream_t s);
hipError_t launch_to_bf16(const float *in, int64_t n, uint16_t *out, hipStream_t s);
hipError_t launch_quant_fp8(const float *lat, const LatentArgs &g, uint8_t *codes, float *scales, hipStream_t s);
hipError_t launch_train(const TrainCall &t, float *workspace, int nparts, int64_t chunk, hipStream_t s);
// BF16 matrix-core training: per-wavefront partial gradients into
// `partials`, then launch_train_reduce (fixed-order sum and Adam).
hipError_t launch_train_mfma(const TrainCall &t, float *partials, int nparts, int64_t chunk, hipStream_t s);
hipError_t launch_train_reduce(const TrainCall &t, float *workspace, int nparts, hipStream_t s);
int train_nparams(int C, int O);
int train_reduce_chunks(int nparts);
hipError_t launch_neural2d(const NeuralCall &c, hipStream_t s);
hipError_t launch_neural_ray(const NeuralCall &c, hipStream_t s);
hipError_t launch_decode_lattice(const NeuralCall &c, const int64_t *idx, hipStream_t s);
hipError_t launch_error_stats(const float *est, const double *ref, int64_t count, int32_t ch, double *out,
                              double *partials, int32_t nblocks, hipStream_t s);

}  // namespace sfk
