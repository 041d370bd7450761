// C ABI of libsf: argument validation on the host, derivation of per-call
// constants, and dispatch to the kernel launchers.  Nothing is enqueued
// unless every argument is valid.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "sf_internal.hpp"

namespace {

thread_local char g_err[512] = "";

sf_status fail(sf_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}

sf_status ok()
{
    g_err[0] = '\0';
    return SF_OK;
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// allow_split: the entry point implements SF_SPLIT (the 2-D filters).
sf_status check_sampling(const sf_sampling *smp, bool allow_split = false)
{
    if (!smp)
        return fail(SF_E_NULL, "sampling descriptor is NULL");
    if (smp->filter < SF_NEAREST || smp->filter > SF_MITCHELL)
        return fail(SF_E_RANGE, "filter %d out of range", smp->filter);
    if (smp->mode < SF_BEFORE || smp->mode > SF_SPLIT)
        return fail(SF_E_RANGE, "mode %d out of range", smp->mode);
    if (smp->mode == SF_SPLIT && !allow_split)
        return fail(SF_E_UNSUPPORTED, "split filtering is a mode of the 2-D filters");
    if (smp->spp < 1 || smp->spp > SF_MAX_SPP)
        return fail(SF_E_RANGE, "spp %d outside 1..%d", smp->spp, SF_MAX_SPP);
    if (smp->rng_variant != 0 && smp->rng_variant != 1)
        return fail(SF_E_RANGE, "rng_variant %d must be 0 or 1", smp->rng_variant);
    return SF_OK;
}

sf_status check_n(int64_t n)
{
    if (n < 0)
        return fail(SF_E_RANGE, "n = %lld is negative", (long long)n);
    if (n > 0x7fffffffLL)
        return fail(SF_E_RANGE, "n = %lld exceeds 2^31-1 (the hash key holds a 32-bit query index)", (long long)n);
    return SF_OK;
}

sf_status check_volume(const sf_volume *v, sfk::VolArgs &a)
{
    if (!v)
        return fail(SF_E_NULL, "volume descriptor is NULL");
    if (!v->base)
        return fail(SF_E_NULL, "volume base pointer is NULL");
    if (v->format != SF_R16F && v->format != SF_R32F)
        return fail(SF_E_UNSUPPORTED, "volume format %d unsupported (R16F or R32F)", v->format);
    if (v->nx < 1 || v->ny < 1 || v->nz < 1 || v->nx > 4096 || v->ny > 4096 || v->nz > 4096)
        return fail(SF_E_RANGE, "grid %d x %d x %d outside 1..4096 per axis", v->nx, v->ny, v->nz);
    const size_t esz = v->format == SF_R16F ? 2 : 4;
    const uint64_t bytes = (uint64_t)v->nx * v->ny * v->nz * esz;
    // one raw buffer resource addresses the grid with 32-bit byte offsets
    if (bytes > 0xffffffffULL || (uint64_t)v->ny * v->nz > (1ULL << 24))
        return fail(SF_E_UNSUPPORTED, "grid of %llu bytes exceeds the 4 GiB addressing of one buffer",
                    (unsigned long long)bytes);
    if (!aligned(v->base, esz))
        return fail(SF_E_RANGE, "volume base pointer misaligned");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(v->wmin[k]) || !std::isfinite(v->scale[k]) || v->scale[k] == 0.0f)
            return fail(SF_E_RANGE, "volume wmin/scale must be finite, scale non-zero");
    if (v->reserved != 0)
        return fail(SF_E_RANGE, "volume reserved field must be 0");
    a.occ = nullptr;
    a.occ_log2 = a.nbx = a.nby = a.nbz = a.occ_sx = a.occ_sy = 0;
    a.occ_bytes = 0;
    if (v->occupancy) {
        if (v->brick_log2 < 1 || v->brick_log2 > 6)
            return fail(SF_E_RANGE, "brick_log2 %d outside 1..6", v->brick_log2);
        if (!aligned(v->occupancy, 4))
            return fail(SF_E_RANGE, "occupancy pointer misaligned");
        const sfk::OccLayout o = sfk::occ_layout(v->nx, v->ny, v->nz, v->brick_log2);
        // the kernels form bit indices with signed 24-bit multiplies
        if (o.bits > sfk::kMaxOccBits || (int64_t)o.sy * (o.nbz + 1) >= (1LL << 23))
            return fail(SF_E_UNSUPPORTED, "occupancy mask of %lld bits exceeds 2^30 (use larger bricks)",
                        (long long)o.bits);
        a.occ = v->occupancy;
        a.occ_log2 = v->brick_log2;
        a.nbx = o.nbx;
        a.nby = o.nby;
        a.nbz = o.nbz;
        a.occ_sx = o.sx;
        a.occ_sy = o.sy;
        a.occ_bytes = (uint32_t)(o.words * 4);
    }
    a.lx = a.ly = -1;
    if ((v->nx & (v->nx - 1)) == 0 && (v->ny & (v->ny - 1)) == 0) {
        a.lx = __builtin_ctz((unsigned)v->nx);
        a.ly = __builtin_ctz((unsigned)v->ny);
    }
    a.base = v->base;
    a.nx = v->nx;
    a.ny = v->ny;
    a.nz = v->nz;
    a.fmt = v->format;
    a.bytes = (uint32_t)bytes;
    for (int k = 0; k < 3; ++k) {
        a.wmin[k] = v->wmin[k];
        a.scale[k] = v->scale[k];
    }
    return SF_OK;
}

sf_status ggx_constants(const sf_ggx *g, sfk::GgxConst &c)
{
    double n[3], wo[3], wi[3];
    for (int k = 0; k < 3; ++k) {
        n[k] = g->n[k];
        wo[k] = g->wo[k];
        wi[k] = g->wi[k];
    }
    double h[3] = {wo[0] + wi[0], wo[1] + wi[1], wo[2] + wi[2]};
    double hl = std::sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
    double no = n[0] * wo[0] + n[1] * wo[1] + n[2] * wo[2];
    double ni = n[0] * wi[0] + n[1] * wi[1] + n[2] * wi[2];
    if (!(no > 0.0) || !(ni > 0.0) || !(hl > 0.0))
        return fail(SF_E_RANGE, "GGX directions need n.wo > 0 and n.wi > 0");
    for (int k = 0; k < 3; ++k)
        h[k] /= hl;
    double nh = n[0] * h[0] + n[1] * h[1] + n[2] * h[2];
    double ih = wi[0] * h[0] + wi[1] * h[1] + wi[2] * h[2];
    double F = g->f0 + (1.0 - g->f0) * std::pow(1.0 - ih, 5.0);
    const double pi = 3.14159265358979323846;
    c.nh2 = (float)(nh * nh);
    c.no = (float)no;
    c.no2 = (float)(no * no);
    c.ni = (float)ni;
    c.ni2 = (float)(ni * ni);
    c.spec_c = (float)(F / pi);
    for (int k = 0; k < 3; ++k) {
        c.kd[k] = (float)(g->radiance[k] * ni / pi);
        c.ks[k] = (float)(g->radiance[k] * ni);
    }
    c.r_bias = g->r_bias;
    c.r_scale = g->r_scale;
    // tangent frame of n (Duff et al., JCGT 6(1), 2017) for normal-mapped shading
    const double sg = n[2] >= 0.0 ? 1.0 : -1.0;
    const double fa = -1.0 / (sg + n[2]), fb = n[0] * n[1] * fa;
    const double e1[3] = {1.0 + sg * n[0] * n[0] * fa, sg * fb, -sg * n[0]};
    const double e2[3] = {fb, sg + n[1] * n[1] * fa, -n[1]};
    const double *vs[2] = {wo, wi};
    float *ts[2] = {c.to, c.ti};
    for (int v = 0; v < 2; ++v) {
        const double *x = vs[v];
        ts[v][0] = (float)(e1[0] * x[0] + e1[1] * x[1] + e1[2] * x[2]);
        ts[v][1] = (float)(e2[0] * x[0] + e2[1] * x[1] + e2[2] * x[2]);
        ts[v][2] = (float)(n[0] * x[0] + n[1] * x[1] + n[2] * x[2]);
    }
    const double th[3] = {e1[0] * h[0] + e1[1] * h[1] + e1[2] * h[2], e2[0] * h[0] + e2[1] * h[1] + e2[2] * h[2],
                          n[0] * h[0] + n[1] * h[1] + n[2] * h[2]};
    for (int k = 0; k < 3; ++k) {
        c.th[k] = (float)th[k];
        c.thl[k] = (float)(th[k] - (double)c.th[k]);
    }
    c.th_defect = (float)(1.0 - (th[0] * th[0] + th[1] * th[1] + th[2] * th[2]));
    c.F = (float)F;
    for (int k = 0; k < 3; ++k) {
        c.rad[k] = g->radiance[k];
        c.kdn[k] = (float)(g->radiance[k] * 0.5 / pi);
    }
    return SF_OK;
}

sf_status device_status(hipError_t e)
{
    if (e != hipSuccess)
        return fail(SF_E_DEVICE, "HIP error %d: %s", (int)e, hipGetErrorString(e));
    return ok();
}

}  // namespace

extern "C" {

const char *sf_last_error(void) { return g_err; }
int32_t sf_abi_version(void) { return SF_ABI_VERSION; }
int32_t sf_rng_version(void) { return SF_RNG_VERSION; }

static sf_status check_tex2d(const sf_tex2d *tex)
{
    if (!tex->base)
        return fail(SF_E_NULL, "texture base pointer is NULL");
    if (tex->format != SF_RGBA32F && tex->format != SF_RGBA8_UNORM && tex->format != SF_DCT8)
        return fail(SF_E_UNSUPPORTED, "2-D texture format %d unsupported (RGBA32F, RGBA8_UNORM or DCT8)",
                    tex->format);
    if (tex->format == SF_DCT8 && (!tex->dct_range || !aligned(tex->dct_range, 16)))
        return fail(tex->dct_range ? SF_E_RANGE : SF_E_NULL, "a DCT8 texture needs 16-byte aligned dct_range");
    if (tex->width < 1 || tex->height < 1 || tex->width > 65536 || tex->height > 65536)
        return fail(SF_E_RANGE, "texture size %d x %d outside 1..65536", tex->width, tex->height);
    int maxlv = 1;
    while (((tex->width > tex->height ? tex->width : tex->height) >> maxlv) >= 1)
        ++maxlv;
    if (tex->levels < 1 || tex->levels > SF_MAX_LEVELS || tex->levels > maxlv)
        return fail(SF_E_RANGE, "levels %d outside 1..%d", tex->levels, maxlv < SF_MAX_LEVELS ? maxlv : SF_MAX_LEVELS);
    if (tex->wrap != SF_WRAP_REPEAT && tex->wrap != SF_WRAP_CLAMP)
        return fail(SF_E_RANGE, "wrap %d out of range", tex->wrap);
    if (tex->mip < SF_MIP_NONE || tex->mip > SF_MIP_LINEAR)
        return fail(SF_E_RANGE, "mip %d out of range", tex->mip);
    const size_t esz = tex->format == SF_RGBA8_UNORM ? 4 : 16;
    for (int l = 0; l < tex->levels; ++l)
        if (tex->level_offset[l] < 0 || !aligned((const uint8_t *)tex->base + tex->level_offset[l], esz))
            return fail(SF_E_RANGE, "level %d offset negative or misaligned", l);
    return SF_OK;
}

static void tex_args(const sf_tex2d *tex, sfk::Tex2DArgs &a)
{
    a.base = (const uint8_t *)tex->base;
    a.w = tex->width;
    a.h = tex->height;
    a.levels = tex->levels;
    a.fmt = tex->format;
    a.wrap = tex->wrap;
    a.mip = tex->mip;
    for (int l = 0; l < SF_MAX_LEVELS; ++l)
        a.off[l] = l < tex->levels ? tex->level_offset[l] : 0;
    a.dct_range = tex->format == SF_DCT8 ? tex->dct_range : nullptr;
}

static int level_dim(int n, int l) { return (n >> l) > 0 ? (n >> l) : 1; }

// Bytes from the texture's base pointer to the end of its last-placed level
// when the stochastic 2-D kernel can hold all of it in LDS (plain formats,
// at most kMaxLdsTexture bytes, 16-byte aligned base), else 0.
// SF_NO_LDS_TEXTURE=1 in the environment keeps every texture in global
// memory (so tests can compare both reads).
static int32_t lds_texture_bytes(const sf_tex2d *tex)
{
    if (tex->format == SF_DCT8 || !aligned(tex->base, 16))
        return 0;
    const char *e = getenv("SF_NO_LDS_TEXTURE");
    if (e && e[0] == '1')
        return 0;
    const int64_t esz = tex->format == SF_RGBA8_UNORM ? 4 : 16;
    int64_t end = 0;
    for (int l = 0; l < tex->levels; ++l)
        end = std::max<int64_t>(end, tex->level_offset[l] +
                                         esz * level_dim(tex->width, l) * level_dim(tex->height, l));
    return end <= sfk::kMaxLdsTexture ? (int32_t)end : 0;
}

sf_status sf_filter2d(const sf_tex2d *tex, const float *queries, int64_t n, const sf_sampling *smp, int32_t shade,
                      const sf_ggx *ggx, float *out, int32_t *dbg_taps, void *stream)
{
    sf_status st;
    if ((st = check_n(n)) != SF_OK)
        return st;
    if (n == 0)
        return ok();
    if (!tex || !queries || !out)
        return fail(SF_E_NULL, "tex, queries and out must be non-NULL");
    if ((st = check_sampling(smp, true)) != SF_OK)
        return st;
    if (smp->filter == SF_EWA)
        return fail(SF_E_UNSUPPORTED, "EWA needs the screen derivatives: use sf_filter2d_aniso");
    if (smp->mode == SF_SPLIT && ((smp->filter > SF_KEYS3 && smp->filter != SF_MITCHELL) || smp->rng_variant != 0))
        return fail(SF_E_UNSUPPORTED,
                    "split filtering takes NEAREST, LINEAR, BSPLINE3, KEYS3 or MITCHELL with rng_variant 0");
    if (smp->filter >= SF_KEYS3 && smp->rng_variant != 0)
        return fail(SF_E_UNSUPPORTED,
                    "the Keys, Mitchell, Gaussian and FIS filters draw independent uniforms (rng_variant 0)");
    if ((smp->filter == SF_GAUSS_FRS || smp->filter == SF_GAUSS_FIS) &&
        !(smp->sigma >= SF_SIGMA_MIN && smp->sigma <= SF_SIGMA_MAX))
        return fail(SF_E_RANGE, "sigma %g outside %g..%g", (double)smp->sigma, (double)SF_SIGMA_MIN,
                    (double)SF_SIGMA_MAX);
    if ((st = check_tex2d(tex)) != SF_OK)
        return st;
    if (shade != SF_SHADE_NONE && shade != SF_SHADE_GGX && shade != SF_SHADE_GGX_NORMAL)
        return fail(SF_E_RANGE, "shade %d out of range", shade);
    if (!aligned(queries, 4) || !aligned(out, shade == SF_SHADE_NONE ? 16 : 4))
        return fail(SF_E_RANGE, "queries or out misaligned");
    sfk::Filter2DCall c{};
    if (shade != SF_SHADE_NONE) {
        if (!ggx)
            return fail(SF_E_NULL, "GGX shading needs ggx parameters");
        if ((st = ggx_constants(ggx, c.g)) != SF_OK)
            return st;
    }
    tex_args(tex, c.tex);
    c.q = queries;
    c.n = n;
    c.filter = smp->filter;
    c.mode = smp->mode;
    c.spp = smp->spp;
    c.variant = smp->rng_variant;
    c.seed = smp->seed;
    c.sigma = smp->sigma;
    c.shade = shade;
    c.out = out;
    c.taps = smp->mode == SF_STOCHASTIC || smp->mode == SF_SPLIT ? dbg_taps : nullptr;
    c.lds_bytes = smp->mode == SF_STOCHASTIC ? lds_texture_bytes(tex) : 0;
    return device_status(sfk::launch_filter2d(c, (hipStream_t)stream));
}

sf_status sf_filter2d_aniso(const sf_tex2d *tex, const float *queries, int64_t n, const sf_sampling *smp,
                            int32_t aniso_max, int32_t shade, const sf_ggx *ggx, float *out, int32_t *dbg_taps,
                            void *stream)
{
    sf_status st;
    if ((st = check_n(n)) != SF_OK)
        return st;
    if (n == 0)
        return ok();
    if (!tex || !queries || !out)
        return fail(SF_E_NULL, "tex, queries and out must be non-NULL");
    if ((st = check_sampling(smp, true)) != SF_OK)
        return st;
    const int f = smp->filter;
    if (smp->mode == SF_SPLIT) {
        if (f > SF_KEYS3 && f != SF_MITCHELL)
            return fail(SF_E_UNSUPPORTED, "split filtering takes NEAREST, LINEAR, BSPLINE3, KEYS3 or MITCHELL");
    } else if (f != SF_NEAREST && f != SF_LINEAR && f != SF_BSPLINE3 && f != SF_GAUSS_FIS && f != SF_EWA) {
        return fail(SF_E_UNSUPPORTED, "anisotropic filtering takes NEAREST, LINEAR, BSPLINE3, GAUSS_FIS or EWA");
    }
    if (f == SF_GAUSS_FIS && smp->mode != SF_STOCHASTIC)
        return fail(SF_E_UNSUPPORTED, "the FIS Gaussian has no probe comparator here");
    if (smp->rng_variant != 0)
        return fail(SF_E_UNSUPPORTED, "anisotropic filtering draws independent uniforms (rng_variant 0)");
    if (f == SF_GAUSS_FIS && !(smp->sigma >= SF_SIGMA_MIN && smp->sigma <= SF_SIGMA_MAX))
        return fail(SF_E_RANGE, "sigma %g outside %g..%g", (double)smp->sigma, (double)SF_SIGMA_MIN,
                    (double)SF_SIGMA_MAX);
    if (aniso_max < 1 || aniso_max > SF_MAX_ANISO)
        return fail(SF_E_RANGE, "aniso_max %d outside 1..%d", aniso_max, SF_MAX_ANISO);
    if ((st = check_tex2d(tex)) != SF_OK)
        return st;
    if (f == SF_EWA) {
        if (aniso_max > SF_EWA_MAX_ANISO)
            return fail(SF_E_RANGE, "EWA: aniso_max %d above %d", aniso_max, SF_EWA_MAX_ANISO);
        const int32_t big = tex->width > tex->height ? tex->width : tex->height;
        const int32_t small = tex->width > tex->height ? tex->height : tex->width;
        int full = 1;
        while ((1 << (full - 1)) * 2 <= big)
            ++full;
        if (tex->levels != full)
            return fail(SF_E_UNSUPPORTED, "EWA needs the complete pyramid: %d levels for %dx%d, got %d", full,
                        tex->width, tex->height, tex->levels);
        if ((int64_t)big > (int64_t)SF_EWA_MAX_ASPECT * small)
            return fail(SF_E_UNSUPPORTED, "EWA: aspect %dx%d beyond %d:1", tex->width, tex->height,
                        SF_EWA_MAX_ASPECT);
    }
    if (shade != SF_SHADE_NONE && shade != SF_SHADE_GGX && shade != SF_SHADE_GGX_NORMAL)
        return fail(SF_E_RANGE, "shade %d out of range", shade);
    if (!aligned(queries, 4) || !aligned(out, shade == SF_SHADE_NONE ? 16 : 4))
        return fail(SF_E_RANGE, "queries or out misaligned");
    sfk::AnisoCall c{};
    if (shade != SF_SHADE_NONE) {
        if (!ggx)
            return fail(SF_E_NULL, "GGX shading needs ggx parameters");
        if ((st = ggx_constants(ggx, c.g)) != SF_OK)
            return st;
    }
    tex_args(tex, c.tex);
    c.q = queries;
    c.n = n;
    c.filter = f;
    c.mode = smp->mode;
    c.spp = smp->spp;
    c.seed = smp->seed;
    c.sigma = smp->sigma;
    c.amax = aniso_max;
    c.shade = shade;
    c.out = out;
    c.taps = smp->mode == SF_STOCHASTIC || smp->mode == SF_SPLIT ? dbg_taps : nullptr;
    return device_status(sfk::launch_aniso(c, (hipStream_t)stream));
}

int64_t sf_dct_layout(int32_t width, int32_t height, int32_t levels, int64_t *level_offset)
{
    if (width < 1 || height < 1 || width > 65536 || height > 65536 || levels < 1 || levels > SF_MAX_LEVELS)
        return -1;
    int64_t pos = 0;
    for (int l = 0; l < levels; ++l) {
        pos = (pos + 255) & ~(int64_t)255;
        if (level_offset)
            level_offset[l] = pos;
        const int64_t bw = (level_dim(width, l) + 7) / 8, bh = (level_dim(height, l) + 7) / 8;
        pos += 16 * bw * bh;
    }
    return pos;
}

sf_status sf_dct_encode(const sf_tex2d *src, void *dst_base, const int64_t *dst_level_offset, float *dst_range,
                        void *stream)
{
    sf_status st;
    if (!src || !dst_base || !dst_level_offset || !dst_range)
        return fail(SF_E_NULL, "src, dst_base, dst_level_offset and dst_range must be non-NULL");
    if ((st = check_tex2d(src)) != SF_OK)
        return st;
    if (src->format != SF_RGBA8_UNORM)
        return fail(SF_E_RANGE, "the DCT compressor takes an RGBA8_UNORM pyramid");
    if (!aligned(dst_range, 16))
        return fail(SF_E_RANGE, "dst_range must be 16-byte aligned");
    sfk::DctEncodeCall c{};
    c.src = (const uint8_t *)src->base;
    c.dst = (uint8_t *)dst_base;
    c.range = dst_range;
    c.w = src->width;
    c.h = src->height;
    c.levels = src->levels;
    c.first_block[0] = 0;
    for (int l = 0; l < src->levels; ++l) {
        if (dst_level_offset[l] < 0 || !aligned((const uint8_t *)dst_base + dst_level_offset[l], 16))
            return fail(SF_E_RANGE, "dst level %d offset negative or misaligned", l);
        c.src_off[l] = src->level_offset[l];
        c.dst_off[l] = dst_level_offset[l];
        const int64_t bw = (level_dim(c.w, l) + 7) / 8, bh = (level_dim(c.h, l) + 7) / 8;
        c.first_block[l + 1] = c.first_block[l] + bw * bh;
    }
    return device_status(sfk::launch_dct_encode(c, (hipStream_t)stream));
}

sf_status sf_triplanar(const sf_tex2d *tex, const float *queries, int64_t n, const sf_sampling *smp, float tex_scale,
                       int32_t plane_mode, int32_t shade, const sf_ggx *ggx, float *out, int32_t *dbg_taps,
                       void *stream)
{
    sf_status st;
    if ((st = check_n(n)) != SF_OK)
        return st;
    if (n == 0)
        return ok();
    if (!tex || !queries || !out)
        return fail(SF_E_NULL, "tex, queries and out must be non-NULL");
    if ((st = check_sampling(smp)) != SF_OK)
        return st;
    if (smp->filter > SF_BSPLINE3 || smp->rng_variant != 0)
        return fail(SF_E_UNSUPPORTED, "triplanar mapping takes NEAREST, LINEAR or BSPLINE3 with rng_variant 0");
    if (plane_mode != 0 && plane_mode != 1)
        return fail(SF_E_RANGE, "plane_mode %d must be 0 (blend) or 1 (pick one plane)", plane_mode);
    if (!(tex_scale > 0.0f) || !(tex_scale < 1e30f))
        return fail(SF_E_RANGE, "tex_scale must be positive and finite");
    if ((st = check_tex2d(tex)) != SF_OK)
        return st;
    if (shade != SF_SHADE_NONE && shade != SF_SHADE_GGX)
        return fail(SF_E_RANGE, "shade %d out of range", shade);
    if (!aligned(queries, 16) || !aligned(out, shade == SF_SHADE_NONE ? 16 : 4))
        return fail(SF_E_RANGE, "queries (16 B) or out misaligned");
    sfk::TriplanarCall c{};
    if (shade == SF_SHADE_GGX) {
        if (!ggx)
            return fail(SF_E_NULL, "GGX shading needs ggx parameters");
        if ((st = ggx_constants(ggx, c.g)) != SF_OK)
            return st;
    }
    tex_args(tex, c.tex);
    c.q = queries;
    c.n = n;
    c.filter = smp->filter;
    c.mode = smp->mode;
    c.spp = smp->spp;
    c.seed = smp->seed;
    c.scale = tex_scale;
    c.plane_mode = plane_mode;
    c.shade = shade;
    c.out = out;
    c.taps = plane_mode == 1 ? dbg_taps : nullptr;
    return device_status(sfk::launch_triplanar(c, (hipStream_t)stream));
}

sf_status sf_filter3d(const sf_volume *vol, const float *pos, int64_t n, const sf_sampling *smp, int32_t shade,
                      float ds, float *out, int32_t *dbg_taps, void *stream)
{
    sf_status st;
    if ((st = check_n(n)) != SF_OK)
        return st;
    if (n == 0)
        return ok();
    if (!pos || !out)
        return fail(SF_E_NULL, "pos and out must be non-NULL");
    if ((st = check_sampling(smp)) != SF_OK)
        return st;
    if (smp->filter > SF_BSPLINE3)
        return fail(SF_E_UNSUPPORTED, "the Keys, Gaussian and FIS filters are 2-D texture filters here");
    sfk::Filter3DCall c{};
    if ((st = check_volume(vol, c.vol)) != SF_OK)
        return st;
    if (shade != SF_SHADE_DENSITY && shade != SF_SHADE_TRANSMITTANCE && shade != SF_SHADE_PLANCK)
        return fail(SF_E_RANGE, "shade %d out of range", shade);
    if (!std::isfinite(ds))
        return fail(SF_E_RANGE, "ds must be finite");
    if (!aligned(pos, 4) || !aligned(out, 4))
        return fail(SF_E_RANGE, "pos or out misaligned");
    c.pos = pos;
    c.n = n;
    c.filter = smp->filter;
    c.mode = smp->mode;
    c.spp = smp->spp;
    c.variant = smp->rng_variant;
    c.seed = smp->seed;
    c.shade = shade;
    c.ds = ds;
    c.out = out;
    c.taps = smp->mode == SF_STOCHASTIC ? dbg_taps : nullptr;
    return device_status(sfk::launch_filter3d(c, (hipStream_t)stream));
}

sf_status sf_raymarch(const sf_volume *vol, const float *rays, int64_t n, int32_t steps, const sf_sampling *smp,
                      float *T, int32_t *dbg_taps, void *stream)
{
    sf_status st;
    if ((st = check_n(n)) != SF_OK)
        return st;
    if (steps < 1 || steps > SF_MAX_STEPS)
        return fail(SF_E_RANGE, "steps %d outside 1..%d", steps, SF_MAX_STEPS);
    if (n == 0)
        return ok();
    if (!rays || !T)
        return fail(SF_E_NULL, "rays and T must be non-NULL");
    if ((st = check_sampling(smp)) != SF_OK)
        return st;
    if (smp->filter > SF_BSPLINE3)
        return fail(SF_E_UNSUPPORTED, "the Keys, Gaussian and FIS filters are 2-D texture filters here");
    sfk::RaymarchCall c{};
    if ((st = check_volume(vol, c.vol)) != SF_OK)
        return st;
    if (!aligned(rays, 16) || !aligned(T, 4))
        return fail(SF_E_RANGE, "rays must be 16-byte aligned, T 4-byte aligned");
    c.rays = rays;
    c.n = n;
    c.steps = steps;
    c.filter = smp->filter;
    c.mode = smp->mode;
    c.spp = smp->spp;
    c.variant = smp->rng_variant;
    c.seed = smp->seed;
    c.T = T;
    c.taps = smp->mode == SF_STOCHASTIC ? dbg_taps : nullptr;
    return device_status(sfk::launch_raymarch(c, (hipStream_t)stream));
}

sf_status sf_raymarch_emission(const sf_volume *vol, const float *rays, int64_t n, int32_t steps,
                               const sf_sampling *smp, float footprint, float *L, int32_t *dbg_taps, void *stream)
{
    sf_status st;
    if ((st = check_n(n)) != SF_OK)
        return st;
    if (steps < 1 || steps > SF_MAX_STEPS)
        return fail(SF_E_RANGE, "steps %d outside 1..%d", steps, SF_MAX_STEPS);
    if (n == 0)
        return ok();
    if (!rays || !L)
        return fail(SF_E_NULL, "rays and L must be non-NULL");
    if ((st = check_sampling(smp)) != SF_OK)
        return st;
    if (smp->filter > SF_BSPLINE3)
        return fail(SF_E_UNSUPPORTED, "the Keys, Gaussian and FIS filters are 2-D texture filters here");
    sfk::RaymarchCall c{};
    if ((st = check_volume(vol, c.vol)) != SF_OK)
        return st;
    if (!aligned(rays, 16) || !aligned(L, 4))
        return fail(SF_E_RANGE, "rays must be 16-byte aligned, L 4-byte aligned");
    if (!(footprint >= 0.0f) || !(footprint < __builtin_inff()))
        return fail(SF_E_RANGE, "footprint %g must be finite and non-negative", (double)footprint);
    if (footprint > 0.0f && smp->mode != SF_STOCHASTIC)
        return fail(SF_E_UNSUPPORTED, "a footprint is sampled by the stochastic mode only");
    {
        const float smax = std::max(vol->scale[0], std::max(vol->scale[1], vol->scale[2]));
        if ((double)footprint * (double)smax > 1048576.0)
            return fail(SF_E_RANGE, "footprint %g spans more than 2^20 voxels", (double)footprint);
    }
    c.footprint = footprint;
    c.rays = rays;
    c.n = n;
    c.steps = steps;
    c.filter = smp->filter;
    c.mode = smp->mode;
    c.spp = smp->spp;
    c.variant = smp->rng_variant;
    c.seed = smp->seed;
    c.T = L;
    c.taps = smp->mode == SF_STOCHASTIC ? dbg_taps : nullptr;
    return device_status(sfk::launch_emission(c, (hipStream_t)stream));
}

int64_t sf_occupancy_words(int32_t nx, int32_t ny, int32_t nz, int32_t brick_log2)
{
    if (nx < 1 || ny < 1 || nz < 1 || brick_log2 < 1 || brick_log2 > 6)
        return 0;
    const sfk::OccLayout o = sfk::occ_layout(nx, ny, nz, brick_log2);
    return o.bits > sfk::kMaxOccBits || (int64_t)o.sy * (o.nbz + 1) >= (1LL << 23) ? 0 : o.words;
}

sf_status sf_build_occupancy(const sf_volume *vol, uint32_t *occupancy, int64_t words, void *stream)
{
    if (!vol || !occupancy)
        return fail(SF_E_NULL, "volume and occupancy must be non-NULL");
    sf_volume v = *vol;
    v.occupancy = occupancy;    // only to size the bricks below
    sfk::VolArgs a;
    sf_status st;
    if ((st = check_volume(&v, a)) != SF_OK)
        return st;
    const int64_t need = (int64_t)a.occ_bytes / 4;
    if (words < need)
        return fail(SF_E_RANGE, "occupancy needs %lld words, %lld given", (long long)need, (long long)words);
    return device_status(sfk::launch_build_occupancy(a, occupancy, (hipStream_t)stream));
}

// ---------------------------------------------------------------- neural
int64_t sf_mlp_nparams(int32_t in_dim, int32_t hidden, int32_t out_dim)
{
    if (in_dim < 1 || hidden < 1 || out_dim < 1)
        return 0;
    return (int64_t)in_dim * hidden + hidden + (int64_t)hidden * hidden + hidden + (int64_t)hidden * out_dim + out_dim;
}

static sf_status check_grid(const sf_latent_grid *g, bool need_data, sfk::LatentArgs &a)
{
    if (!g)
        return fail(SF_E_NULL, "latent grid descriptor is NULL");
    if (g->dims != 2 && g->dims != 3)
        return fail(SF_E_RANGE, "latent grid dims %d must be 2 or 3", g->dims);
    const int32_t r2 = g->dims == 2 ? 1 : g->res[2];
    if (g->res[0] < 1 || g->res[1] < 1 || r2 < 1 || g->res[0] > 65536 || g->res[1] > 65536 || r2 > 4096)
        return fail(SF_E_RANGE, "latent grid resolution out of range");
    if ((int64_t)g->res[0] * g->res[1] * r2 > (1LL << 31))
        return fail(SF_E_UNSUPPORTED, "more than 2^31 lattice points");
    if (g->channels != (g->dims == 2 ? 8 : 16))
        return fail(SF_E_UNSUPPORTED, "%d-D latent grids have %d channels here", g->dims, g->dims == 2 ? 8 : 16);
    if (g->format != SF_LATENT_BF16 && g->format != SF_LATENT_FP8E4M3)
        return fail(SF_E_UNSUPPORTED, "latent format %d: BF16 or E4M3", g->format);
    if (g->format == SF_LATENT_FP8E4M3 && (g->block_log2 < 1 || g->block_log2 > 6))
        return fail(SF_E_RANGE, "block_log2 %d outside 1..6", g->block_log2);
    if (need_data) {
        if (!g->latents || (g->format == SF_LATENT_FP8E4M3 && !g->block_scale))
            return fail(SF_E_NULL, "latents (and E4M3 block scales) must be non-NULL");
        if (!aligned(g->latents, 16) || (g->block_scale && !aligned(g->block_scale, 4)))
            return fail(SF_E_RANGE, "latents must be 16-byte aligned");
    }
    if (g->dims == 3)
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(g->wmin[k]) || !std::isfinite(g->scale[k]) || g->scale[k] == 0.0f)
                return fail(SF_E_RANGE, "latent grid wmin/scale must be finite, scale non-zero");
    a.latents = g->latents;
    a.scales = g->block_scale;
    a.dims = g->dims;
    a.res[0] = g->res[0];
    a.res[1] = g->res[1];
    a.res[2] = r2;
    a.C = g->channels;
    a.fmt = g->format;
    a.block_log2 = g->format == SF_LATENT_FP8E4M3 ? g->block_log2 : 0;
    for (int k = 0; k < 3; ++k) {
        a.wmin[k] = g->wmin[k];
        a.scale[k] = g->scale[k];
    }
    return SF_OK;
}

static sf_status check_mlp(const sf_mlp *m, const sfk::LatentArgs &g, sfk::MlpArgs &a)
{
    if (!m || !m->params)
        return fail(SF_E_NULL, "MLP descriptor or parameters NULL");
    const int32_t out = g.dims == 2 ? 4 : 1;
    if (m->in_dim != g.C || m->hidden != 64 || m->out_dim != out || m->reserved != 0)
        return fail(SF_E_UNSUPPORTED, "MLP %d-%d-%d: this grid needs %d-64-%d", m->in_dim, m->hidden, m->out_dim,
                    g.C, out);
    if (!aligned(m->params, 2))
        return fail(SF_E_RANGE, "MLP parameters misaligned");
    a.params = m->params;
    a.in_dim = m->in_dim;
    a.out_dim = m->out_dim;
    return SF_OK;
}

sf_status sf_neural_decode(const sf_latent_grid *grid, const sf_mlp *mlp, const float *queries, int64_t n,
                           const sf_sampling *smp, int32_t shade, const sf_ggx *ggx, float *out, int32_t *dbg_taps,
                           void *stream)
{
    sf_status st;
    if ((st = check_n(n)) != SF_OK)
        return st;
    if (n == 0)
        return ok();
    if (!queries || !out)
        return fail(SF_E_NULL, "queries and out must be non-NULL");
    if ((st = check_sampling(smp)) != SF_OK)
        return st;
    if (smp->rng_variant != 0 || smp->filter > SF_BSPLINE3)
        return fail(SF_E_UNSUPPORTED, "neural decoding: NEAREST, LINEAR or BSPLINE3 with independent uniforms");
    sfk::NeuralCall c{};
    if ((st = check_grid(grid, true, c.lat)) != SF_OK)
        return st;
    if (c.lat.dims != 2)
        return fail(SF_E_UNSUPPORTED, "sf_neural_decode takes a 2-D grid");
    if ((st = check_mlp(mlp, c.lat, c.mlp)) != SF_OK)
        return st;
    if (shade != SF_SHADE_NONE && shade != SF_SHADE_GGX)
        return fail(SF_E_RANGE, "shade %d out of range", shade);
    if (shade == SF_SHADE_GGX) {
        if (!ggx)
            return fail(SF_E_NULL, "GGX shading needs ggx parameters");
        if ((st = ggx_constants(ggx, c.g)) != SF_OK)
            return st;
    }
    if (!aligned(queries, 4) || !aligned(out, shade == SF_SHADE_NONE ? 16 : 4))
        return fail(SF_E_RANGE, "queries or out misaligned");
    c.q = queries;
    c.n = n;
    c.filter = smp->filter;
    c.mode = smp->mode;
    c.spp = smp->spp;
    c.seed = smp->seed;
    c.shade = shade;
    c.out = out;
    c.taps = smp->mode == SF_STOCHASTIC ? dbg_taps : nullptr;
    return device_status(sfk::launch_neural2d(c, (hipStream_t)stream));
}

sf_status sf_neural_raymarch(const sf_latent_grid *grid, const sf_mlp *mlp, const float *rays, int64_t n,
                             int32_t steps, const sf_sampling *smp, float *T, int32_t *dbg_taps, void *stream)
{
    sf_status st;
    if ((st = check_n(n)) != SF_OK)
        return st;
    if (steps < 1 || steps > SF_MAX_STEPS)
        return fail(SF_E_RANGE, "steps %d outside 1..%d", steps, SF_MAX_STEPS);
    if (n == 0)
        return ok();
    if (!rays || !T)
        return fail(SF_E_NULL, "rays and T must be non-NULL");
    if ((st = check_sampling(smp)) != SF_OK)
        return st;
    if (smp->mode != SF_STOCHASTIC || smp->rng_variant != 0 || smp->filter > SF_BSPLINE3)
        return fail(SF_E_UNSUPPORTED, "the neural ray march is stochastic (NEAREST, LINEAR or BSPLINE3) with "
                                      "independent uniforms");
    sfk::NeuralCall c{};
    if ((st = check_grid(grid, true, c.lat)) != SF_OK)
        return st;
    if (c.lat.dims != 3)
        return fail(SF_E_UNSUPPORTED, "sf_neural_raymarch takes a 3-D grid");
    if ((st = check_mlp(mlp, c.lat, c.mlp)) != SF_OK)
        return st;
    if (!aligned(rays, 16) || !aligned(T, 4))
        return fail(SF_E_RANGE, "rays must be 16-byte aligned, T 4-byte aligned");
    c.rays = rays;
    c.n = n;
    c.steps = steps;
    c.filter = smp->filter;
    c.mode = smp->mode;
    c.spp = smp->spp;
    c.seed = smp->seed;
    c.T = T;
    c.taps = dbg_taps;
    return device_status(sfk::launch_neural_ray(c, (hipStream_t)stream));
}

sf_status sf_neural_decode_lattice(const sf_latent_grid *grid, const sf_mlp *mlp, const int64_t *lattice_idx,
                                   int64_t n, float *out, void *stream)
{
    sf_status st;
    if ((st = check_n(n)) != SF_OK)
        return st;
    if (n == 0)
        return ok();
    if (!lattice_idx || !out)
        return fail(SF_E_NULL, "lattice_idx and out must be non-NULL");
    sfk::NeuralCall c{};
    if ((st = check_grid(grid, true, c.lat)) != SF_OK)
        return st;
    if ((st = check_mlp(mlp, c.lat, c.mlp)) != SF_OK)
        return st;
    if (!aligned(lattice_idx, 8) || !aligned(out, 4))
        return fail(SF_E_RANGE, "misaligned pointer");
    c.n = n;
    c.out = out;
    return device_status(sfk::launch_decode_lattice(c, lattice_idx, (hipStream_t)stream));
}

sf_status sf_to_bf16(const float *in, int64_t n, uint16_t *out, void *stream)
{
    if (n < 0)
        return fail(SF_E_RANGE, "n is negative");
    if (n == 0)
        return ok();
    if (!in || !out)
        return fail(SF_E_NULL, "in and out must be non-NULL");
    if (!aligned(in, 4) || !aligned(out, 2))
        return fail(SF_E_RANGE, "misaligned pointer");
    return device_status(sfk::launch_to_bf16(in, n, out, (hipStream_t)stream));
}

sf_status sf_neural_quantize(const float *latents, const sf_latent_grid *grid, void *out_latents, float *out_scales,
                             void *stream)
{
    sfk::LatentArgs a{};
    sf_status st;
    if ((st = check_grid(grid, false, a)) != SF_OK)
        return st;
    if (!latents || !out_latents || (a.fmt == SF_LATENT_FP8E4M3 && !out_scales))
        return fail(SF_E_NULL, "latents, out_latents (and E4M3 out_scales) must be non-NULL");
    if (!aligned(latents, 4) || !aligned(out_latents, 2) || (out_scales && !aligned(out_scales, 4)))
        return fail(SF_E_RANGE, "misaligned pointer");
    const int64_t count = (int64_t)a.res[0] * a.res[1] * a.res[2] * a.C;
    if (a.fmt == SF_LATENT_BF16)
        return device_status(sfk::launch_to_bf16(latents, count, (uint16_t *)out_latents, (hipStream_t)stream));
    return device_status(sfk::launch_quant_fp8(latents, a, (uint8_t *)out_latents, out_scales, (hipStream_t)stream));
}

static int train_parts(int64_t batch)
{
    int64_t p = (batch + 15) / 16;
    return (int)(p < 1 ? 1 : (p > 2048 ? 2048 : p));
}

// One wavefront per 16-sample tile up to 1024 wavefronts (one per SIMD of
// a 256-CU device: each holds the registers of one), then longer chunks.
// Never more than train_parts(batch), so one workspace size serves both modes.
static int train_parts_mfma(int64_t batch)
{
    int64_t p = (batch + 15) / 16;
    return (int)(p < 1 ? 1 : (p > 1024 ? 1024 : p));
}

size_t sf_neural_train_workspace(int32_t channels, int32_t out_dim, int64_t batch)
{
    if (!((channels == 8 && out_dim == 4) || (channels == 16 && out_dim == 1)) || batch < 1)
        return 0;
    const int parts = train_parts(batch);
    return (size_t)(parts + sfk::train_reduce_chunks(parts)) * (size_t)(sfk::train_nparams(channels, out_dim) + 1) *
           sizeof(float);
}

sf_status sf_neural_train_step(const sf_train_state *stt, const int32_t *batch_idx, const float *targets,
                               int64_t batch, int32_t step, float lr_latent, float lr_mlp, float *loss_out,
                               float *grad_params, float *grad_latents, void *workspace, size_t workspace_bytes,
                               void *stream)
{
    if (!stt)
        return fail(SF_E_NULL, "training state is NULL");
    if (!((stt->channels == 8 && stt->out_dim == 4) || (stt->channels == 16 && stt->out_dim == 1)) ||
        stt->hidden != 64)
        return fail(SF_E_UNSUPPORTED, "training shapes: 8-64-4 or 16-64-1");
    if (stt->compute != SF_TRAIN_BF16 && stt->compute != SF_TRAIN_FP32)
        return fail(SF_E_RANGE, "compute %d must be SF_TRAIN_BF16 or SF_TRAIN_FP32", stt->compute);
    if (batch < 1 || batch > stt->n_lattice || stt->n_lattice < 1 || stt->n_lattice > (1LL << 31) || step < 1)
        return fail(SF_E_RANGE, "batch must be in 1..n_lattice and step >= 1");
    if (!std::isfinite(lr_latent) || !std::isfinite(lr_mlp))
        return fail(SF_E_RANGE, "learning rates must be finite");
    if (!stt->latents || !stt->params || !stt->m_latents || !stt->v_latents || !stt->m_params || !stt->v_params ||
        !batch_idx || !targets || !loss_out)
        return fail(SF_E_NULL, "training arrays, batch_idx, targets and loss_out must be non-NULL");
    const size_t need = sf_neural_train_workspace(stt->channels, stt->out_dim, batch);
    if (!workspace || workspace_bytes < need)
        return fail(SF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? workspace_bytes : 0);
    sfk::TrainCall t{};
    t.latents = stt->latents;
    t.params = stt->params;
    t.m_lat = stt->m_latents;
    t.v_lat = stt->v_latents;
    t.m_par = stt->m_params;
    t.v_par = stt->v_params;
    t.idx = batch_idx;
    t.targets = targets;
    t.batch = batch;
    t.n_lattice = stt->n_lattice;
    t.C = stt->channels;
    t.O = stt->out_dim;
    t.lr_latent = lr_latent;
    t.lr_mlp = lr_mlp;
    t.bc1 = (float)(1.0 - std::pow(0.9, step));
    t.bc2 = (float)(1.0 - std::pow(0.999, step));
    t.inv_bc1 = (float)(1.0 / (1.0 - std::pow(0.9, step)));
    t.inv_bc2 = (float)(1.0 / (1.0 - std::pow(0.999, step)));
    t.loss_out = loss_out;
    t.grad_params = grad_params;
    t.grad_latents = grad_latents;
    if (stt->compute == SF_TRAIN_BF16) {
        // fewer, longer chunks than the FP32 path (at most as many partials):
        // a wavefront loads its weight fragments once for 8 tiles of 16
        const int parts = train_parts_mfma(batch);
        const int64_t chunk = ((batch + parts - 1) / parts + 15) / 16 * 16;
        hipError_t e = sfk::launch_train_mfma(t, (float *)workspace, parts, chunk, (hipStream_t)stream);
        if (e == hipSuccess)
            e = sfk::launch_train_reduce(t, (float *)workspace, parts, (hipStream_t)stream);
        return device_status(e);
    }
    const int parts = train_parts(batch);
    const int64_t chunk = (batch + parts - 1) / parts;
    return device_status(sfk::launch_train(t, (float *)workspace, parts, chunk, (hipStream_t)stream));
}

static int32_t err_blocks(int64_t count)
{
    int64_t b = (count + 1023) / 1024;
    return (int32_t)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

size_t sf_error_stats_workspace(int64_t count)
{
    if (count < 0)
        count = 0;
    return (size_t)err_blocks(count) * 8 * sizeof(double);
}

sf_status sf_error_stats(const float *est, const double *ref, int64_t n, int32_t ch, double *out, void *workspace,
                         size_t workspace_bytes, void *stream)
{
    if (n < 0 || ch < 1)
        return fail(SF_E_RANGE, "n must be >= 0 and ch >= 1");
    if (!out)
        return fail(SF_E_NULL, "out must be non-NULL");
    const int64_t count = n * (int64_t)ch;
    if (count > 0 && (!est || !ref))
        return fail(SF_E_NULL, "est and ref must be non-NULL");
    const size_t need = sf_error_stats_workspace(count);
    if (!workspace || workspace_bytes < need)
        return fail(SF_E_WORKSPACE, "workspace of %zu bytes needed, %zu given", need, workspace ? workspace_bytes : 0);
    if (!aligned(out, 8) || !aligned(workspace, 8) || (ref && !aligned(ref, 8)) || (est && !aligned(est, 4)))
        return fail(SF_E_RANGE, "misaligned pointer");
    return device_status(
        sfk::launch_error_stats(est, ref, count, ch, out, (double *)workspace, err_blocks(count), (hipStream_t)stream));
}

}  // extern "C"

// Scratch of sf_error_stats_noalloc: the per-block partial rows of the
// reduction, one copy per device, held until the process ends.  Every row
// that the final pass reads is written by the first pass of the same call,
// so nothing needs clearing between calls.
namespace {

constexpr int kNoallocRows = 1024;   // err_blocks() never asks for more
static __device__ __align__(256) double scratch[kNoallocRows * 8];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_ptr[kMaxDevices] = {};

// The device address of this device's copy of `scratch`, looked up once per
// device with that device current (the host-side name of the array is not a
// device address).
sf_status scratch_for_current_device(double **ptr)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0)
        return fail(SF_E_DEVICE, "hipGetDevice failed");
    if (dev >= kMaxDevices)
        return fail(SF_E_UNSUPPORTED, "device %d beyond the %d devices the static scratch supports", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SF_E_DEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *ptr = g_scratch_ptr[dev];
    return SF_OK;
}

}  // namespace

extern "C" {

size_t sf_error_stats_noalloc_max_bytes(void) { return sizeof(scratch); }

sf_status sf_error_stats_noalloc(const float *est, const double *ref, int64_t n, int32_t ch, double *out,
                                 void *stream)
{
    if (n < 0 || ch < 1)
        return fail(SF_E_RANGE, "n must be >= 0 and ch >= 1");
    if (!out)
        return fail(SF_E_NULL, "out must be non-NULL");
    if (n > 0 && ch > INT64_MAX / n)
        return fail(SF_E_RANGE, "n * ch overflows");
    const int64_t count = n * (int64_t)ch;
    if (count > 0 && (!est || !ref))
        return fail(SF_E_NULL, "est and ref must be non-NULL");
    const size_t need = sf_error_stats_workspace(count);
    if (need > sizeof(scratch))
        return fail(SF_E_RANGE, "this call needs %zu bytes of scratch, beyond the %zu bytes of the static scratch",
                    need, sizeof(scratch));
    if (!aligned(out, 8) || (ref && !aligned(ref, 8)) || (est && !aligned(est, 4)))
        return fail(SF_E_RANGE, "misaligned pointer");
    double *ws = nullptr;
    const sf_status st = scratch_for_current_device(&ws);
    if (st != SF_OK)
        return st;
    return device_status(
        sfk::launch_error_stats(est, ref, count, ch, out, ws, err_blocks(count), (hipStream_t)stream));
}

}  // extern "C"
