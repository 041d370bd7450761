/*
 * sf.h — C ABI of libsf, stochastic texture filtering with filtering after
 * shading on AMD Instinct MI355X (gfx950).
 *
 * Method: Pharr, Wronski, Salvi, Fajardo, "Filtering After Shading With
 * Stochastic Texture Filtering" (2024).  For each query the library builds
 * the separable filter weights, picks ONE texel per sample by inverse CDF on
 * those weights (Sec. 2.2 "Sampling arrays", eq. stochastic-sum; Sec. 4.1
 * FRS), shades that texel and averages: an unbiased estimate of filtering
 * after shading (Sec. 3, eq. filtering-after-shading).  The deterministic
 * filter-before-shading (eq. filter-before-shading) and exact
 * filter-after-shading sums run beside it.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is a DEVICE pointer (HBM of the current HIP
 *    device); descriptor structs are HOST structs whose pointer members are
 *    device pointers.  The caller owns all memory; the library allocates
 *    nothing and keeps no state besides the thread-local error string.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued asynchronously; results are valid after the stream
 *    is synchronised.  No call synchronises on its own.
 *  - Arguments are validated on the host BEFORE anything is enqueued.  On an
 *    error nothing is enqueued and the status names the class; sf_last_error()
 *    gives the message.  n == 0 is a no-op returning SF_OK.
 *  - Coordinates are raster coordinates with texel centres at integers: a
 *    texture coordinate u in [0,1) maps to p = u*N - 0.5 (one fused
 *    multiply-add in binary32); the lookup point sits at fraction
 *    t = p - floor(p) past texel i0 = floor(p).
 *  - Random numbers: SF_RNG_VERSION 1 = the 4-D PCG hash of Jarzynski and
 *    Olano (JCGT 2020) on the key (query index, sample index, step index,
 *    seed); each 32-bit output word w gives the uniform (w >> 8) * 2^-24.
 *    Words 0,1,2 drive the x,y,z tap picks, word 3 the MIP level pick.
 *  - Picks: per axis, the tap index j = #{k : u >= C_k} over the running sums
 *    C_k of the axis weights, evaluated in binary32 in a fixed operation
 *    order (the "decision contract"), so that the integer decisions match an
 *    IEEE-binary32 reference bit for bit.
 *  - Queries with a non-finite coordinate give NaN and the sentinel tap
 *    SF_TAP_NONE.
 */
#ifndef SF_H
#define SF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SF_ABI_VERSION 3
#define SF_RNG_VERSION 1
#define SF_TAP_NONE INT32_MIN
#define SF_MAX_LEVELS 16
#define SF_MAX_STEPS 65536
#define SF_MAX_SPP 65536
#define SF_MAX_ANISO 64
#define SF_EWA_MAX_ANISO 16  /* EWA: anisotropy limit (bounds the ellipse's box)    */
#define SF_EWA_MAX_ASPECT 8  /* EWA: max(width, height) <= 8 min(width, height)     */

typedef int32_t sf_status;
enum {
    SF_OK = 0,
    SF_E_NULL = 1,        /* a required pointer is NULL                       */
    SF_E_RANGE = 2,       /* a size / count / enum value is out of range      */
    SF_E_UNSUPPORTED = 3, /* a valid but unsupported combination              */
    SF_E_DEVICE = 4,      /* the HIP runtime reported an error while enqueuing */
    SF_E_WORKSPACE = 5    /* workspace missing or too small                   */
};

/* Separable reconstruction filter per axis (Suppl. S.2): box K0 (nearest),
 * tent K1 (bi/trilinear), cubic B-spline K_bs (bi/tricubic, eq. cubic-bspline),
 * and the interpolating cubic K3 with a = -1/2 (Keys), whose negative lobes
 * the stochastic mode handles by positivisation (Sec. 2.2 "Positivization"):
 * one tap drawn from the positive and one from the negative product
 * weights, estimate W+ f(t+) - W- f(t-).  SF_KEYS3 is a 2-D texture filter. */
enum { SF_NEAREST = 0, SF_LINEAR = 1, SF_BSPLINE3 = 2, SF_KEYS3 = 3, SF_GAUSS_FRS = 4, SF_GAUSS_FIS = 5,
       SF_BSPLINE3_FIS = 6, SF_EWA = 7, SF_MITCHELL = 8 };
/* SF_MITCHELL: the Mitchell-Netravali cubic, B = C = 1/3 (Mitchell and
 * Netravali 1988; the other reading of the paper's "Mitchell" filter of
 * Sec. 5 and the bicubic listing of Suppl. S.4), on taps i0-1..i0+2, a 2-D
 * texture filter.  Its outer lobe changes sign at |x| = 8/7, so the
 * stochastic mode positivises by per-tap sign (as the listing's two
 * reservoirs do): binary32 weights, s = 1-t,
 *   w0 = ((s s) fma(-7, t, 1)) fl(1/18),  w1 = fma(t t, fma(fl(7/6), t, -2), fl(8/9)),
 *   w2 likewise in s,                     w3 = ((t t) fma(7, t, -6)) fl(1/18);
 * per axis the positive set holds the taps with w > 0 and the negative set
 * those with w < 0, P+ / P- their |w| summed in tap order; inside a set the
 * tap is the first whose running sum c satisfies u P < c (else its last);
 * blocks, keys and the estimate (A + B) f(t+) - (Cn + Dn) f(t-) as SF_KEYS3;
 * dbg_taps n x spp x {level, x+, y+, x-, y-}. */
/* SF_EWA: the elliptically weighted average over the pixel footprint, and
 * its stochastic form (one texel per sample drawn from the EWA weights);
 * sf_filter2d_aniso only (it needs the screen derivatives). */
/* Gaussian filters and filter importance sampling (2-D textures only):
 *   SF_GAUSS_FRS    discrete Gaussian of standard deviation sigma (texels) on
 *                   the nearest 4x4 texels, sampled per axis by its running
 *                   sum (FRS, Sec. 4.1; Suppl. S.4.2, discrete sampling);
 *   SF_GAUSS_FIS    Gaussian filter importance sampling: a Box-Muller offset
 *                   of standard deviation sigma, then the nearest texel
 *                   (Sec. 4.2; Suppl. S.4.2); the filter it realises is the
 *                   Gaussian convolved with the unit box (cell masses);
 *   SF_BSPLINE3_FIS the cubic B-spline by FIS: offset xi1 + xi2 + xi3 - 3/2
 *                   (quadratic B-spline density), then the nearest texel
 *                   (Sec. 4.2, Cox-de Boor); deterministic modes = SF_BSPLINE3.
 * Their binary32 decision contract (raster p = i0 + t as for every filter):
 *   ln, exp, cos/sin(2 pi v) are evaluated by the written-out sequences
 *   documented in the oracle (frexp reduction + atanh series; Cody-Waite
 *   reduction + Taylor to r^7; quadrant fold + Taylor to x^9 / x^10);
 *   GAUSS_FRS: h = 0.5/(sigma sigma); a_k = (d d) h, d = (k-1) - t;
 *     g_k = exp(min a - a_k); C0 = g0/W, C1 = (g0+g1)/W, C2 = (g0+g1+g2)/W,
 *     W = ((g0+g1)+g2)+g3; offset -1 + #{C_j <= u};
 *   GAUSS_FIS: r = sigma sqrt(-2 ln(1 - u0)); (c, s) = cos/sin(2 pi u1);
 *     offsets floor((t + 1/2) + r c), floor((t + 1/2) + r s);
 *   BSPLINE3_FIS: S = (w0>>8)+(w1>>8)+(w2>>8) = 2^24 q + r (words 0..2 of
 *     the key with step 0 for x, step 1 for y); offset q - 1 + [r 2^-24 >= 1 - t]. */
/* SF_BEFORE: shade(sum_i w_i t_i)            (eq. filter-before-shading)
 * SF_AFTER_EXACT: sum_i w_i shade(t_i)        (eq. filtering-after-shading)
 * SF_STOCHASTIC: mean over spp of shade(t_j), P(j) = w_j (eq. stochastic-sum)
 * SF_SPLIT (2-D filters only): the split-filtering estimator (Sec. 3 eq.
 *   split-filtering-shading, Sec. 4): per sample the low-pass filter is
 *   sampled — the MIP level (sf_filter2d: key word 3, as SF_STOCHASTIC), and
 *   for sf_filter2d_aniso also the jitter over the pixel (key words 0, 1, 2,
 *   as SF_STOCHASTIC) — and the reconstruction filter is evaluated on that
 *   level before shading: mean over spp of shade(sum_i w_i t_i).  Filters
 *   NEAREST, LINEAR, BSPLINE3, KEYS3 (binary32 weights), rng_variant 0;
 *   dbg_taps hold {level, SF_TAP_NONE, SF_TAP_NONE} per sample. */
enum { SF_BEFORE = 0, SF_AFTER_EXACT = 1, SF_STOCHASTIC = 2, SF_SPLIT = 3 };
enum { SF_RGBA32F = 0, SF_RGBA8_UNORM = 1, SF_R16F = 2, SF_R32F = 3, SF_DCT8 = 4 };
enum { SF_WRAP_REPEAT = 0, SF_WRAP_CLAMP = 1 };
/* MIP level use (Sec. 2.1 pyramids; single stochastic level, Sec. 4.2.1):
 * NONE = level 0 only; NEAREST = level round(lambda); LINEAR = levels
 * floor(lambda) and floor(lambda)+1 with weights (1-f, f), f = frac(lambda)
 * (a stochastic mode picks ONE of them with those probabilities). */
enum { SF_MIP_NONE = 0, SF_MIP_NEAREST = 1, SF_MIP_LINEAR = 2 };
enum { SF_SHADE_NONE = 0, SF_SHADE_GGX = 1, SF_SHADE_GGX_NORMAL = 2 }; /* 2-D */
/* SF_SHADE_GGX_NORMAL (sf_filter2d, sf_filter2d_aniso): a normal-mapped grey
 * material (Sec. 3 "Normal maps": filtering the normals before shading
 * changes a minified surface's appearance).  The texel's RGB encodes the
 * tangent-space normal m = 2 rgb - 1, renormalised (z for m = 0), A the
 * roughness parameter as for SF_SHADE_GGX; the tangent frame (e1, e2, n) of
 * the sf_ggx normal n is sg = sign(n_z), a = -1/(sg + n_z), b = n_x n_y a,
 * e1 = (1 + sg n_x^2 a, sg b, -sg n_x), e2 = (b, sg + n_y^2 a, -n_y) (Duff et
 * al., JCGT 6(1), 2017); the GGX + Lambert model of SF_SHADE_GGX with albedo
 * 1/2 is evaluated at the shading normal with its cosines clamped at 0 and
 * the masking factors divided by their cosines analytically (G1(c)/c =
 * 2/(c + sqrt(a^2 + (1 - a^2) c^2))), a continuous function that is 0 where
 * the normal faces away from wi.  Filtering before shading shades the
 * filtered (shortened, then renormalised) normal.  Output: RGB. */
enum { SF_SHADE_DENSITY = 0, SF_SHADE_TRANSMITTANCE = 1, SF_SHADE_PLANCK = 2 }; /* 3-D points */
/* SF_SHADE_PLANCK: the grid holds temperatures in kelvin, shaded by black-body
 * emission (Sec. 5 "Filtering nonlinear physical properties"): the spectral
 * radiance in W sr^-1 m^-2 nm^-1 at the three wavelengths 700, 546.1 and
 * 435.8 nm (the CIE 1931 RGB primaries),
 *   B(lambda, T) = 2 h c^2 / (lambda^5 (exp(h c / (lambda k T)) - 1)) * 1e-9,
 * lambda in metres, exact SI h, c, k; T <= 0 emits nothing, NaN gives NaN.
 * Values (not decisions) in binary32 on the transcendental unit: relative
 * error about (x + 3) * 2^-24, x = h c / (lambda k T). */

typedef struct sf_sampling {
    int32_t filter;      /* SF_NEAREST .. SF_MITCHELL (see above)                    */
    int32_t mode;        /* SF_BEFORE | SF_AFTER_EXACT | SF_STOCHASTIC | SF_SPLIT     */
    int32_t spp;         /* samples per query, 1..SF_MAX_SPP (deterministic: ignored) */
    uint32_t seed;       /* fourth word of the hash key                              */
    int32_t rng_variant; /* 0: one uniform per axis; 1: one uniform for all spatial
                            axes, re-derived after each pick by uniform sample reuse
                            (Sec. 2.2 eq. uniform-sample-reuse): u' = (u-lo)/(hi-lo)
                            over the picked bin [lo, hi), clamped to 1 - 2^-24      */
    float sigma;         /* Gaussian filters: standard deviation in texels of the
                            level read, SF_SIGMA_MIN..SF_SIGMA_MAX; else ignored     */
} sf_sampling;
#define SF_SIGMA_MIN 0.0625f
#define SF_SIGMA_MAX 4.0f

/* A 2-D texture with an optional MIP pyramid.  Level l has
 * max(1, width >> l) x max(1, height >> l) texels, row-major, 4 channels,
 * at base + level_offset[l] (bytes).  RGBA8_UNORM channels decode as c/255.
 * Channels are (albedo R, G, B, roughness parameter A) when shaded. */
typedef struct sf_tex2d {
    const void *base;
    int32_t width, height, levels; /* levels in 1..SF_MAX_LEVELS                 */
    int32_t format;                /* SF_RGBA32F | SF_RGBA8_UNORM | SF_DCT8       */
    int32_t wrap;                  /* SF_WRAP_REPEAT | SF_WRAP_CLAMP              */
    int32_t mip;                   /* SF_MIP_NONE | SF_MIP_NEAREST | SF_MIP_LINEAR */
    int64_t level_offset[SF_MAX_LEVELS];
    const float *dct_range;        /* SF_DCT8: AC range of channel c on level l at
                                      [4 l + c] (device); NULL otherwise          */
} sf_tex2d;

/* SF_DCT8 — DCT-compressed texture (Sec. 5 "Texture compression").  Level l
 * holds ceil(w_l/8) x ceil(h_l/8) blocks of 8x8 texels, row-major, 16 bytes
 * each: one 32-bit word per channel (R, G, B, A) with the six
 * lowest-frequency coefficients of the orthonormal 2-D DCT-II of the texel
 * values v = byte/255, in zigzag order (u horizontal, v vertical frequency)
 * (0,0), (1,0), (0,1), (0,2), (1,1), (2,0):
 *   bits 0..6   DC code d, coefficient d * 8/127;
 *   bits 7..31  five 5-bit AC codes a (0..30), coefficient (a - 15) R/15,
 *               R = dct_range[4 l + c].
 * A texel decodes to clamp(sum_k coef_k c_uk(x) c_vk(y), 0, 1) with
 * c_0 = sqrt(1/8), c_k(x) = cos((2x+1) k pi/16)/2: one block read and 24
 * multiply-adds, independent of the filter — the decode that stochastic
 * filtering performs once per sample instead of once per tap. */

/* GGX microfacet specular + Lambert diffuse times the cosine (the paper's
 * BSDF-times-cosine f-hat, Sec. 3) for one directional light of `radiance`.
 * Unit vectors n, wo, wi with n.wo > 0 and n.wi > 0.  The texel's A channel
 * gives roughness r = r_bias + r_scale*A, alpha = r^2; D is the GGX normal
 * distribution, G the separable Smith term, F Schlick's with f0. */
typedef struct sf_ggx {
    float n[3], wo[3], wi[3], radiance[3];
    float f0, r_bias, r_scale;
} sf_ggx;

/* A dense 3-D grid of scalar density (x fastest, then y, then z) occupying
 * the world box from wmin; scale = voxels per world unit per axis.  World
 * point x maps to raster p = (x - wmin)*scale - 0.5 (subtract, then one fused
 * multiply-add).  Taps outside the grid read zero (empty space).  A grid
 * holds at most 4 GiB (it is addressed with 32-bit byte offsets) and
 * ny*nz <= 2^24.
 * occupancy: NULL, or the brick mask sf_build_occupancy wrote for this grid
 * and brick_log2 (the mask must be rebuilt whenever the grid changes).  The
 * ray march then skips every step whose lookup point lies in a brick whose
 * 2-voxel dilation holds only zeros: such a step can only read zeros, so the
 * stochastic result is bit-identical with and without the mask (Sec. 5: the
 * sparse NanoVDB grid of the paper's offline renderer plays this role). */
typedef struct sf_volume {
    const void *base;
    int32_t nx, ny, nz;
    int32_t format; /* SF_R16F | SF_R32F */
    float wmin[3], scale[3];
    const uint32_t *occupancy; /* device, sf_occupancy_words(...) words, or NULL */
    int32_t brick_log2;        /* brick side 2^brick_log2 voxels, 1..6 (with occupancy) */
    int32_t reserved;          /* must be 0 */
} sf_volume;

/*
 * sf_filter2d — filtered (and optionally shaded) lookups in a 2-D texture.
 *   queries : n x {u, v, lambda} float32; lambda = level of detail (ignored
 *             with SF_MIP_NONE), clamped to [0, levels-1].
 *   shade   : SF_SHADE_NONE -> out is n x 4 float32 (filtered RGBA);
 *             SF_SHADE_GGX  -> out is n x 3 float32 (RGB radiance); ggx required.
 *   dbg_taps: NULL, or n x spp x {level, x, y} int32 (stochastic mode only):
 *             the texel each sample read, after wrapping; with SF_KEYS3
 *             n x spp x {level, x+, y+, x-, y-} (SF_TAP_NONE when the negative
 *             weights vanish).  Keys decisions (binary32): per axis
 *             m0 = (t/2)(s s), m3 = (s/2)(t t), p1 = fma(t t, fma(3/2, t, -5/2), 1),
 *             p2 likewise in s = 1-t, P+ = p1 + p2, P- = m0 + m3; a positive pair
 *             takes its first tap iff u P+ < p1, a negative pair iff u P- < m0;
 *             the positive sample is in block (+,+) iff u (A+B) < A, A = P+x P+y,
 *             B = P-x P-y; the negative one in (+,-) iff u (C+D) < C, C = P+x P-y,
 *             D = P-x P+y; uniforms: words 0,1,2 of the sample's key for the
 *             positive draw (x, y, block) and of its key with step 1 for the
 *             negative draw.
 * Stochastic NEAREST / LINEAR / BSPLINE3 lookups in a plain-format texture
 * of at most 64 KiB (from base to the end of its last level, 16-byte aligned
 * base) read a copy of it in LDS when the launch has at most one 256-lane
 * tile per resident workgroup; SF_NO_LDS_TEXTURE=1 in the environment keeps
 * the reads in global memory (results are equal).
 * Defines: Sec. 2.2 eqs. filtered-texture and stochastic-sum; Sec. 3 eqs.
 * filter-before-shading and filtering-after-shading; Sec. 4.1 eq.
 * bicubic-bspline-texfilt; Suppl. S.1 stochastic bilerp; MIP level pick of
 * Sec. 4.2.1.
 * Errors: SF_E_NULL (tex, base, queries, out, smp, or ggx when shading);
 *         SF_E_RANGE (n < 0 or n > 2^31-1, bad enum, spp outside 1..SF_MAX_SPP,
 *         size <= 0, levels outside 1..SF_MAX_LEVELS or beyond the pyramid,
 *         sigma outside SF_SIGMA_MIN..SF_SIGMA_MAX for a Gaussian filter);
 *         SF_E_UNSUPPORTED (rng_variant 1 with SF_KEYS3 or a Gaussian / FIS filter);
 *         SF_E_DEVICE (launch failure).
 */
sf_status sf_filter2d(const sf_tex2d *tex, const float *queries, int64_t n, const sf_sampling *smp,
                      int32_t shade, const sf_ggx *ggx, float *out, int32_t *dbg_taps, void *stream);

/*
 * sf_filter2d_aniso — minification with anisotropic footprints by
 * screen-space jitter (Sec. 4.2.1 "Screen-Space Anisotropic Minification";
 * the level of detail of Suppl. S.4.3; Sec. 5 "Anisotropic filtering and
 * minification").
 *   queries : n x {u, v, du/dx, dv/dx, du/dy, dv/dy} float32 (24 B): the
 *             pixel centre's texture coordinate and its screen derivatives.
 *   smp     : filter NEAREST | LINEAR | BSPLINE3 (FRS) | GAUSS_FIS (stochastic
 *             only, with smp->sigma) | EWA (below); rng_variant 0.
 *   aniso_max: 1..SF_MAX_ANISO (the paper's limit is 64).
 *   tex->mip is ignored: the level comes from the footprint.  Footprint
 *   axes in level-0 texels a = (W du/dx, H dv/dx), b = (W du/dy, H dv/dy);
 *   minor = the shorter, lengthened to major/aniso_max if the ratio exceeds
 *   aniso_max (as major/(minor aniso_max) * minor); lambda = log2(minor)
 *   (binary32 contract: frexp reduction + atanh series, as the Gaussian
 *   filters' ln).
 *   SF_STOCHASTIC, per sample: key (query, sample, 0, seed) words 0, 1 give
 *     the jitter j = u - 1/2 and word 2 the level uniform; key (.., 1, ..)
 *     words 0, 1 the filter's uniforms.  uv' = fma(jy, d/dy, fma(jx, d/dx, uv)),
 *     level = floor(clamp(lambda + (u_l - 1/2), 0, levels-1) + 1/2), then
 *     one texel of that level at uv'.  dbg_taps: n x spp x {level, x, y}.
 *   SF_BEFORE / SF_AFTER_EXACT: the probe comparator (hardware-style
 *     anisotropic filtering): N = clamp(ceil(major/minor), 1, aniso_max)
 *     probes at offsets (k + 1/2)/N - 1/2 of the major-axis derivative, each
 *     filtered on levels floor(lambda), floor(lambda)+1 (weights 1-f, f),
 *     averaged; before shades the average, after averages shaded texels.
 * SF_EWA (Sec. 4.1, stochastic EWA: a level chosen from the ellipse's
 *   extent, then one texel drawn from all the EWA weights; the EWA kernel of
 *   Greene and Heckbert).  Needs a complete pyramid
 *   (levels = floor(log2(max(W, H))) + 1, the last level 1 x 1), aspect
 *   max(W, H) <= SF_EWA_MAX_ASPECT min(W, H) and aniso_max <=
 *   SF_EWA_MAX_ANISO, which bound the ellipse's box at a level a sample
 *   reads to (4 r_x aniso_max + 3) x (4 r_y aniso_max + 3) cells,
 *   r_x = max(W, H)/W, r_y = max(W, H)/H.  Binary32 contract, in this order
 *   (no contraction):
 *   J in level-0 texels: jsx = W du/dx, jtx = H dv/dx, jsy = W du/dy,
 *   jty = H dv/dy; m = max |j..|, m >= 2^40 gives lod = +inf; else
 *   S = J J^T: Sss = jsx jsx + jsy jsy, Stt = jtx jtx + jty jty,
 *   Sst = jsx jtx + jsy jty; dJ = jsx jty - jtx jsy, det = dJ dJ;
 *   lp = (Sss + Stt)/2 + sqrt(((Sss - Stt)/2)^2 + Sst^2), s1 = sqrt(lp),
 *   minor = lp > 0 ? |dJ| / s1 : 0; if minor aniso_max < s1:
 *   lm = det / lp, minor = s1 / aniso_max,
 *   k = lp > lm ? (minor^2 - lm)/(lp - lm) : 1, Sss += k (lp - Sss),
 *   Stt += k (lp - Stt), Sst -= k Sst, det = lp minor^2;
 *   lod = minor > 0 ? max(0, log2(minor)) : 0 (contract log2).
 *   lod > levels-1: every mode returns the (shaded) texel of the 1 x 1
 *   level.  Else at level l (W_l x H_l): fs = W_l/W, ft = H_l/H,
 *   a = Sss fs^2 + 1, c = Stt ft^2 + 1, D = ((det fs^2 ft^2 + Sss fs^2)
 *   + Stt ft^2) + 1; V^-1 = (c/D, a/D, -(2 Sst fs ft)/D) for (ss, tt, 2 st);
 *   s = u W_l - 1/2, t = v H_l - 1/2 (u, v wrapped); s0 = ceil(s - sqrt(a)),
 *   s1 = floor(s + sqrt(a)), t0, t1 likewise with sqrt(c); rows it = t0..t1,
 *   columns is = s0..s1: r^2 = (qss ds^2 + qtt dt^2) + q2st ds dt,
 *   ds = is - s, dt = it - t; weight e^(-2 r^2) - e^(-2) (contract exp) for
 *   r^2 < 1, else 0; cells of weight <= 0 skipped.
 *   SF_STOCHASTIC, per sample: key (query, sample, 0, seed); word 3 picks
 *     level floor(lod) + [u_3 >= 1 - frac(lod)] (at most levels-1); word 0
 *     is the uniform u: W = sum of the weights in scan order, then the first
 *     cell whose running sum exceeds u W (the last positive cell if none).
 *     dbg_taps: n x spp x {level, x, y} of the picked (wrapped) texel.
 *   SF_BEFORE / SF_AFTER_EXACT: the EWA sums on levels floor(lod) and
 *     floor(lod)+1 (weights 1-f, f), each divided by its weight total;
 *     before shades the blend of texels, after blends shaded texels.
 * Queries with a non-finite value, or whose extreme jittered coordinate
 * |u| + |du/dx| + |du/dy| (or the same for v) overflows binary32, give NaN.
 * Errors: as sf_filter2d; SF_E_UNSUPPORTED for other filters or variants;
 *         SF_E_RANGE for aniso_max or sigma out of range (EWA: aniso_max above
 *         SF_EWA_MAX_ANISO); SF_E_UNSUPPORTED for EWA on an incomplete
 *         pyramid or beyond the aspect limit.
 */
sf_status sf_filter2d_aniso(const sf_tex2d *tex, const float *queries, int64_t n, const sf_sampling *smp,
                            int32_t aniso_max, int32_t shade, const sf_ggx *ggx, float *out, int32_t *dbg_taps,
                            void *stream);

/*
 * sf_dct_layout — byte offsets (256-byte aligned, written to level_offset)
 * of the SF_DCT8 levels of a width x height pyramid with `levels` levels;
 * returns the total bytes, or -1 for sizes out of range.
 */
int64_t sf_dct_layout(int32_t width, int32_t height, int32_t levels, int64_t *level_offset);

/*
 * sf_dct_encode — compress an SF_RGBA8_UNORM pyramid into SF_DCT8 (the
 * compressor of Sec. 5 "Texture compression").  dst_base (device,
 * sf_dct_layout bytes) receives the blocks at dst_level_offset[l];
 * dst_range (device, 4 x levels floats) the AC ranges R = max |AC| over the
 * level's blocks per channel.  Codes are decided in binary32: rows
 * R_u(y) = fma-chain over x = 0..7 of c_u(x) v(x, y) with v = byte/255.0f,
 * then C = fma-chain over y of c_v(y) R_u(y); c_k(x) the binary32 roundings
 * of the basis; blocks past the level's edge replicate its edge texels;
 * d = clamp(floor(C0 * 15.875 + 1/2), 0, 127);
 * a = R > 0 ? clamp(floor(Ck * (15/R) + 1/2), -15, 15) + 15 : 15.
 * Errors: SF_E_NULL, SF_E_RANGE (src not RGBA8, levels, misaligned offsets).
 */
sf_status sf_dct_encode(const sf_tex2d *src, void *dst_base, const int64_t *dst_level_offset, float *dst_range,
                        void *stream);

/*
 * sf_triplanar — triplanar mapping (Sec. 5 "Triplanar mapping").
 *   queries : n x {p.x, p.y, p.z, n.x, n.y, n.z, lambda, unused} float32
 *             (32 B): surface point, unit normal, level of detail.
 *   The three planar projections read the texture at (p.y, p.z), (p.x, p.z)
 *   and (p.x, p.y) times tex_scale; their blend weights are
 *   b_i = n_i^4 / sum_j n_j^4.  plane_mode 0 blends all three planes;
 *   plane_mode 1 picks one plane per sample with probability b_i (a
 *   stochastic estimate of the blend, eq. stochastic-sum): binary32
 *   a_i = n_i n_i, w_i = a_i a_i, W = (w0 + w1) + w2,
 *   plane = [u >= w0/W] + [u >= (w0 + w1)/W], u from word 2 of the sample's
 *   key.  smp: NEAREST | LINEAR | BSPLINE3, any mode (the filter on a plane
 *   is as sf_filter2d's, words 0, 1, 3 of the same key); plane_mode 1 with a
 *   deterministic filter averages spp samples of the picked plane's
 *   deterministic value.  SF_BEFORE shades the blended filtered texel.
 *   dbg_taps (plane_mode 1 only): n x spp x {plane, level, x, y} (level, x, y
 *   SF_TAP_NONE for a deterministic filter).
 *   Queries with a non-finite value or a projected coordinate p_k tex_scale
 *   that overflows binary32 give NaN.
 * Errors: as sf_filter2d; SF_E_UNSUPPORTED for other filters or variants.
 */
sf_status sf_triplanar(const sf_tex2d *tex, const float *queries, int64_t n, const sf_sampling *smp,
                       float tex_scale, int32_t plane_mode, int32_t shade, const sf_ggx *ggx, float *out,
                       int32_t *dbg_taps, void *stream);

/*
 * sf_filter3d — filtered point lookups in a density grid.
 *   pos     : n x {x, y, z} float32 world positions.
 *   shade   : SF_SHADE_DENSITY -> out[i] = filtered sigma;
 *             SF_SHADE_TRANSMITTANCE -> out[i] = filtered exp(-sigma*ds);
 *             SF_SHADE_PLANCK -> out[3i..3i+2] = B at the three wavelengths
 *             of the filtered temperature (before) / filtered B (after) /
 *             mean B of the picked voxels (stochastic).
 *   out     : n float32 (n x 3 for SF_SHADE_PLANCK).
 *   dbg_taps: NULL, or n x spp x {x, y, z} int32 raw tap indices (before the
 *             zero-outside rule), stochastic mode only.
 * Points whose raster coordinate exceeds 2^22 in magnitude give NaN.
 * Defines: Sec. 4.1 (n-dimensional FRS, 4^n lookups -> 1); Sec. 5 offline
 * rendering (density lookups).
 * Errors: as sf_filter2d.
 */
sf_status sf_filter3d(const sf_volume *vol, const float *pos, int64_t n, const sf_sampling *smp,
                      int32_t shade, float ds, float *out, int32_t *dbg_taps, void *stream);

/*
 * sf_raymarch — transmittance along rays through a density grid by fixed-step
 * ray marching, filtering the density at every step.
 *   rays : n x {ox, oy, oz, dx, dy, dz, t0, t1} float32, d of unit length,
 *          [t0, t1] the segment to march (already clipped to the grid box by
 *          the caller; t1 <= t0 means an empty segment, T = 1).
 *   steps: S in 1..SF_MAX_STEPS.  dt = (t1 - t0)/S; the raster position of
 *          step k is p_k = (k + 1/2)*G + E per axis with E = t0*B + A and
 *          G = dt*B (fused multiply-adds), A = (o - wmin)*scale - 0.5 and
 *          B = d*scale.
 *   T    : n float32.  SF_STOCHASTIC: mean over spp of exp(-dt * sum_k sigma_k)
 *          with ONE picked voxel per step (the sum over steps and the mean
 *          over spp are compensated binary32 sums);
 *          SF_BEFORE: exp(-dt * sum_k sum_i w_i sigma_i);
 *          SF_AFTER_EXACT: prod_k sum_i w_i exp(-dt*sigma_i).
 *   dbg_taps: NULL, or n x spp x S x {x, y, z} int32 (stochastic only).
 * Rays with a non-finite component, or whose raster positions exceed 2^22 in
 * magnitude, give NaN.
 * Defines: Sec. 5 "Offline rendering" (density lookups of a volumetric path
 * tracer with trilinear / tricubic and stochastic variants); Sec. 4.1 FRS;
 * the transmittance is the shading nonlinearity exp(-sigma*dt) filtered after
 * shading (Sec. 3).
 * Errors: as sf_filter2d, plus SF_E_RANGE for steps outside 1..SF_MAX_STEPS.
 */
sf_status sf_raymarch(const sf_volume *vol, const float *rays, int64_t n, int32_t steps,
                      const sf_sampling *smp, float *T, int32_t *dbg_taps, void *stream);

/*
 * sf_raymarch_emission — radiance gathered along rays through an emitting,
 * non-absorbing grid of temperatures (kelvin), shaded by black-body emission
 * (Sec. 5 "Filtering nonlinear physical properties": filtering the
 * temperatures before Planck's law differs from filtering the emission
 * after it, and the stochastic filter gives the latter with one voxel per
 * step).
 *   rays, steps: as sf_raymarch (same raster positions, keys and picks).
 *   L    : n x 3 float32, the radiance at 700, 546.1, 435.8 nm (see
 *          SF_SHADE_PLANCK) integrated over the segment: dt * sum_k E_k with
 *          SF_STOCHASTIC: E_k = B(T_j) of the one picked voxel (mean over spp);
 *          SF_BEFORE: E_k = B(sum_i w_i T_i); SF_AFTER_EXACT: sum_i w_i B(T_i).
 *          Sums over steps are compensated binary32 sums.  An empty segment
 *          gives 0.
 *   footprint: standard deviation (world units) of a Gaussian pixel
 *          footprint in the plane perpendicular to the ray, sampled per step
 *          (stochastic only; 0 = none; footprint * max scale <= 2^20): the
 *          plane's basis from d by Duff et al. (JCGT 6(1), 2017),
 *          sg = copysign(1, d_z), a = -1/(sg + d_z), b = (d_x d_y) a,
 *          e1 = (1 + ((sg d_x) d_x) a, sg b, -sg d_x), e2 = (b, sg + (d_y d_y) a, -d_y),
 *          A_i = (footprint e1_i) scale_i, B_i likewise; per step the key
 *          (ray, sample | 2^31, step, seed) words 0, 1 give u0, u1,
 *          r = sqrt(-2 ln(1 - u0)), g = r (cos, sin)(2 pi u1) with the
 *          contract ln / cos / sin, and p_k becomes
 *          fma(g2, B, fma(g1, A, p_k)) before the pick (Sec. 5: filtering
 *          after shading under minification with a Gaussian perpendicular
 *          to the ray; a prefiltered coarse grid passed with footprint 0 is
 *          the filter-before comparator).
 *   dbg_taps: NULL, or n x spp x S x {x, y, z} int32 (stochastic only).
 *   An occupancy mask (vol->occupancy, built by sf_build_occupancy from the
 *   temperatures) skips bricks at 0 K exactly (tested at the jittered
 *   position).
 * Rays with a non-finite component, or whose raster positions exceed 2^22 in
 * magnitude, give NaN.
 * Errors: as sf_raymarch; SF_E_RANGE for a negative, non-finite or too wide
 *         footprint, SF_E_UNSUPPORTED for a footprint with a deterministic mode.
 */
sf_status sf_raymarch_emission(const sf_volume *vol, const float *rays, int64_t n, int32_t steps,
                               const sf_sampling *smp, float footprint, float *L, int32_t *dbg_taps,
                               void *stream);

/*
 * sf_build_occupancy — brick occupancy mask of a density grid for empty-space
 * skipping in sf_raymarch.
 *   vol->brick_log2 sets the brick side B = 2^brick_log2 (vol->occupancy is
 *   ignored).  With nbx = ceil(nx/B) bricks along x (likewise y, z), the mask
 *   holds one bit per brick in nbz planes of sy = nby + 1 rows of
 *   sx = nbx + 1 bits: brick (bx, by, bz) is bit b = (bz*sy + by)*sx + bx,
 *   bit (b & 31) of word b >> 5, which is 1 iff every voxel within 2 voxels
 *   of the brick (the support of a cubic B-spline tap around any point of the
 *   brick) is zero, else 0; the last bit of every row, the last row of every
 *   plane and the bits past the last plane are 0.  The padding lets the
 *   march test a lookup point's brick without clamping its coordinates (a
 *   point just outside the grid meets a 0 and is marched).
 *   occupancy: device buffer of `words` uint32, at least
 *   sf_occupancy_words() = ceil(sx*sy*nbz/32); the mask holds at most 2^30
 *   bits (sf_occupancy_words returns 0 beyond that: use larger bricks).
 * Errors: SF_E_NULL, SF_E_RANGE (brick_log2 outside 1..6, words too small),
 *         SF_E_UNSUPPORTED (grid as in sf_raymarch, mask over 2^30 bits),
 *         SF_E_DEVICE.
 */
sf_status sf_build_occupancy(const sf_volume *vol, uint32_t *occupancy, int64_t words, void *stream);
int64_t sf_occupancy_words(int32_t nx, int32_t ny, int32_t nz, int32_t brick_log2);

/* --------------------------------------------------------------------------
 * Neural latent textures and volumes.  A lattice of latent vectors z_c is
 * decoded by a 3-layer MLP, D_c = W3^T relu(W2^T relu(W1^T z_c + b1) + b2) + b3
 * (hidden width 64).  Filtering picks lattice points exactly as the plain
 * filters pick texels, so the stochastic estimator decodes ONE latent per
 * sample instead of all 16 (bicubic) or 64 (tricubic) taps (Sec. 4.1 FRS; the
 * paper motivates stochastic filtering by the cost of evaluating an expensive
 * decoder per tap, Sec. 1 and the compressed-texture results of Sec. 5).
 * Supported shapes: 2-D with 8 channels and 4 outputs (RGBA), 3-D with 16
 * channels and 1 output (density).  Decoding runs on the matrix cores with
 * BF16 operands and FP32 accumulation.
 * ------------------------------------------------------------------------ */
enum { SF_LATENT_F32 = 0, SF_LATENT_BF16 = 1, SF_LATENT_FP8E4M3 = 2 };

/* Lattice point (x, y, z) stores channels at latents + ((z*res[1] + y)*res[0]
 * + x)*channels.  SF_LATENT_FP8E4M3 (OCP E4M3, saturating): the MLP reads
 * bf16(code * block_scale[b]), the binary32 product rounded to BF16 (nearest
 * even), b the block of side 2^block_log2 lattice points holding the point,
 * blocks numbered x fastest.  2-D grids use res[2] = 1 and map a
 * texture coordinate u to raster p = u*res - 0.5 with repeat wrap; 3-D grids
 * map world x to p = (x - wmin)*scale - 0.5 and read zero outside. */
typedef struct sf_latent_grid {
    const void *latents;
    const float *block_scale; /* E4M3 only */
    int32_t dims;             /* 2 or 3 */
    int32_t res[3];
    int32_t channels;         /* 8 (2-D) or 16 (3-D) */
    int32_t format;           /* SF_LATENT_BF16 | SF_LATENT_FP8E4M3 for decoding */
    int32_t block_log2;       /* E4M3 block side 2^block_log2, 1..6 */
    float wmin[3], scale[3];  /* 3-D only */
} sf_latent_grid;

/* Packed MLP parameters W1 [in x 64], b1 [64], W2 [64 x 64], b2 [64],
 * W3 [64 x out], b3 [out], row-major; BF16 bits for decoding. */
typedef struct sf_mlp {
    const void *params;
    int32_t in_dim, hidden, out_dim;
    int32_t reserved; /* must be 0 */
} sf_mlp;

/* Number of packed MLP parameters (in*h + h + h*h + h + h*out + out). */
int64_t sf_mlp_nparams(int32_t in_dim, int32_t hidden, int32_t out_dim);

/*
 * sf_neural_decode — filtered lookups in a 2-D neural texture.
 *   As sf_filter2d on level 0 with repeat wrap, the decoded texel of lattice
 *   point c being clamp(D_c, 0, 1) = (albedo RGB, roughness parameter A).
 *   SF_STOCHASTIC: one decode per sample; SF_AFTER_EXACT: sum_c w_c
 *   shade(D_c); SF_BEFORE: shade(sum_c w_c D_c).  dbg_taps: n x spp x {x, y}.
 * Errors: as sf_filter2d; SF_E_UNSUPPORTED for other shapes or formats.
 */
sf_status sf_neural_decode(const sf_latent_grid *grid, const sf_mlp *mlp, const float *queries, int64_t n,
                           const sf_sampling *smp, int32_t shade, const sf_ggx *ggx, float *out, int32_t *dbg_taps,
                           void *stream);

/*
 * sf_neural_raymarch — sf_raymarch through a 3-D neural density volume,
 * sigma_c = max(D_c, 0).  SF_STOCHASTIC only (the deterministic forms would
 * decode 8 or 64 lattice points per step; the CPU reference computes them).
 *   Latents of at most 2^31 bytes are read through 32-bit buffer offsets,
 *   larger lattices with 64-bit addresses (the environment variable
 *   SF_NEURAL_ADDR64=1 forces the latter, for testing; results are equal).
 * Errors: as sf_raymarch; SF_E_UNSUPPORTED for other modes, shapes, formats.
 */
sf_status sf_neural_raymarch(const sf_latent_grid *grid, const sf_mlp *mlp, const float *rays, int64_t n,
                             int32_t steps, const sf_sampling *smp, float *T, int32_t *dbg_taps, void *stream);

/*
 * sf_neural_decode_lattice — raw MLP outputs (no clamp) at n lattice points.
 *   lattice_idx: n int64 linear lattice indices; out: n x out_dim float32.
 */
sf_status sf_neural_decode_lattice(const sf_latent_grid *grid, const sf_mlp *mlp, const int64_t *lattice_idx,
                                   int64_t n, float *out, void *stream);

/*
 * sf_to_bf16 — binary32 -> bfloat16 bits, round to nearest even (n values).
 */
sf_status sf_to_bf16(const float *in, int64_t n, uint16_t *out, void *stream);

/*
 * sf_neural_quantize — FP32 latents -> the format grid->format names:
 *   BF16: round to nearest even; E4M3: per block s = amax/448 (binary32,
 *   1 for an all-zero block), code = E4M3(z/s) round to nearest even,
 *   saturating.  Writes out_latents (and out_scales, one per block, E4M3).
 */
sf_status sf_neural_quantize(const float *latents, const sf_latent_grid *grid, void *out_latents, float *out_scales,
                             void *stream);

/* Training state, all FP32 device arrays updated in place by a step:
 * latents [n_lattice x channels], params (packed, sf_mlp layout), and the
 * Adam moments of both (FP32 master copies in either compute mode). */
typedef struct sf_train_state {
    float *latents, *params, *m_latents, *v_latents, *m_params, *v_params;
    int64_t n_lattice;
    int32_t channels, hidden, out_dim;
    int32_t compute; /* SF_TRAIN_BF16 (0) or SF_TRAIN_FP32 (1) */
} sf_train_state;

/* How a training step computes its products:
 *   SF_TRAIN_BF16  matrix cores: BF16 operands (latents, weights, hidden
 *                  activations and the pre-activation gradients rounded to
 *                  nearest even), FP32 accumulation; forward, backward and
 *                  the weight gradients (K = the batch's samples) on
 *                  v_mfma_f32_16x16x{16,32}_bf16.
 *   SF_TRAIN_FP32  the vector ALU in FP32 throughout (reference mode). */
enum { SF_TRAIN_BF16 = 0, SF_TRAIN_FP32 = 1 };

/*
 * sf_neural_train_step — one Adam step (beta 0.9/0.999, eps 1e-8, bias
 * correction with `step` >= 1) on the loss (1/B) sum_s ||D(z_{i_s}) -
 * t_{i_s}||^2 over the batch lattice points i_s = batch_idx[s] (distinct:
 * each batch entry updates its own latent; duplicates race).  All gradients
 * are taken at the current values, then latents and parameters move.
 *   targets: n_lattice x out_dim; loss_out: 1 float (device), the batch loss;
 *   grad_params (nullable): the summed parameter gradient; grad_latents
 *   (nullable): batch x channels latent gradients.
 *   workspace: sf_neural_train_workspace() bytes of device scratch.
 *   st->compute selects the matrix-core BF16 step or the FP32 one; both
 *   keep the state in FP32 and reduce the parameter gradients in a fixed
 *   order (bit-reproducible for a given batch).
 * Defines: the training of the learned stand-in (the paper trains no
 * network; the objective is this library's reading, a lattice-point
 * autodecoder fitted to texels the plain method generates).
 * Errors: SF_E_NULL, SF_E_RANGE (also compute outside 0..1),
 * SF_E_UNSUPPORTED (shape), SF_E_WORKSPACE.
 */
sf_status sf_neural_train_step(const sf_train_state *st, const int32_t *batch_idx, const float *targets,
                               int64_t batch, int32_t step, float lr_latent, float lr_mlp, float *loss_out,
                               float *grad_params, float *grad_latents, void *workspace, size_t workspace_bytes,
                               void *stream);
size_t sf_neural_train_workspace(int32_t channels, int32_t out_dim, int64_t batch);

/*
 * sf_error_stats — error statistics of an estimate against a reference,
 * reduced in float64 on the GPU in a fixed order (bit-reproducible).
 *   est: n*ch float32; ref: n*ch float64; out: 8 float64 (device):
 *   {sum err^2, sum err, max |err|, max |err|/|ref| (ref != 0), count,
 *    sum ref^2, count of non-finite est, unused}, err = est - ref, taken over
 *   the finite entries.
 *   workspace: device scratch of sf_error_stats_workspace(n*ch) bytes.
 * Defines: the MSE measure of Sec. 5 (offline rendering).
 * Errors: SF_E_NULL, SF_E_RANGE (n < 0, ch < 1), SF_E_WORKSPACE.
 */
sf_status sf_error_stats(const float *est, const double *ref, int64_t n, int32_t ch, double *out,
                         void *workspace, size_t workspace_bytes, void *stream);
size_t sf_error_stats_workspace(int64_t count);

/*
 * sf_error_stats_noalloc — sf_error_stats for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels and the same result, bit for bit,
 * with the reduction's partial rows kept in a static device array of the
 * library instead of a caller workspace.  It calls no hipMalloc / hipFree and
 * no allocating library routine.
 *   est, ref, n, ch, out, stream: as sf_error_stats (device pointers, owned by
 *   the caller).
 *   Scratch: sf_error_stats_noalloc_max_bytes() bytes (64 KiB) per device,
 *   taken on the first call on a device and held until the process ends.
 *   Every call on one device shares that device's array: calls that overlap
 *   on one device (two streams, two threads) race and give undefined results.
 * Errors: SF_E_NULL, SF_E_RANGE (n < 0, ch < 1, n * ch overflowing, a call
 * whose partial rows exceed the static scratch, misaligned pointers),
 * SF_E_DEVICE (the scratch's device address cannot be found),
 * SF_E_UNSUPPORTED (a device index of 64 or more).
 */
sf_status sf_error_stats_noalloc(const float *est, const double *ref, int64_t n, int32_t ch, double *out,
                                 void *stream);
size_t sf_error_stats_noalloc_max_bytes(void);

/* Message of the last error on the calling thread ("" if none). */
const char *sf_last_error(void);
int32_t sf_abi_version(void);
int32_t sf_rng_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SF_H */
