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
    float spec_k;          // F / (4 (n.wo)(n.wi) pi)
    float kd[3], ks[3];    // radiance * (n.wi) / pi, radiance * (n.wi)
    float r_bias, r_scale;
};

struct Tex2DArgs {
    const uint8_t *base;
    int32_t w, h, levels, fmt, wrap, mip;
    int64_t off[SF_MAX_LEVELS];
};

struct VolArgs {
    const void *base;
    int32_t nx, ny, nz, fmt;
    uint32_t bytes;          // size of the grid in bytes (< 2^31)
    float wmin[3], scale[3];
    const uint32_t *occ;     // brick occupancy mask or null
    int32_t occ_log2, nbx, nby, nbz;
};

struct Filter2DCall {
    Tex2DArgs tex;
    const float *q;
    int64_t n;
    int32_t filter, mode, spp, variant, shade;
    uint32_t seed;
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
    float *T;
    int32_t *taps;
};

// Launchers return hipSuccess or the launch error; arguments are validated.
hipError_t launch_filter2d(const Filter2DCall &c, hipStream_t s);
hipError_t launch_filter3d(const Filter3DCall &c, hipStream_t s);
hipError_t launch_raymarch(const RaymarchCall &c, hipStream_t s);
hipError_t launch_build_occupancy(const VolArgs &v, int32_t log2b, uint32_t *occ, int64_t words, hipStream_t s);
hipError_t launch_error_stats(const float *est, const double *ref, int64_t count, int32_t ch, double *out,
                              double *partials, int32_t nblocks, hipStream_t s);

}  // namespace sfk
