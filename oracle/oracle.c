/*
 * CPU ORACLE for stochastic texture filtering with filtering after shading
 * (Pharr, Wronski, Salvi, Fajardo, "Filtering After Shading With Stochastic
 * Texture Filtering", 2024).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or constant generator with the HIP library; it is the plain,
 * slow, obviously-correct statement of what the GPU path must compute.
 *
 * Numbers: every texel value, weight used in a deterministic sum, shading
 * result and accumulation is IEEE binary64.  The few *decisions* (which texel
 * a sample picks, which MIP level, the raster position of a ray step) are made
 * in IEEE binary32 with every operation written out (compile with
 * -ffp-contract=off; fmaf is called explicitly where the decision contract
 * specifies a fused multiply-add), so that a GPU following the same contract
 * reaches the same integer decisions bit for bit.
 *
 * Paper passages followed (section / equation / listing):
 *   texture as a lattice of samples ............ Sec. 2.1, eq. texture-definition
 *   filtered texture as a weighted sum ......... Sec. 2.2, eq. filtered-texture
 *   one-texel stochastic estimator ............. Sec. 2.2, eq. stochastic-sum
 *   sampling an array by its running sum ....... Sec. 2.2 "Sampling arrays"
 *   uniform sample reuse ....................... Sec. 2.2, eq. uniform-sample-reuse
 *   separable sampling ......................... Sec. 2.2 "Separable functions"
 *   filter before / after shading .............. Sec. 3, eqs. filter-before-shading,
 *                                                filtering-after-shading
 *   FRS on the separable B-spline .............. Sec. 4.1, eq. bicubic-bspline-texfilt
 *   tent and cubic B-spline kernels ............ Suppl. S.2, eq. cubic-bspline
 *   stochastic lerp / bilerp ................... Suppl. S.1
 *   stochastic MIP level selection ............. Sec. 4.2.1
 *   positivisation of negative lobes ........... Sec. 2.2 "Positivization"
 *   screen-space anisotropic minification ...... Sec. 4.2.1; Suppl. S.4.3; Sec. 5 "Anisotropic
 *                                                filtering and minification"
 *   DCT-compressed textures, triplanar mapping . Sec. 5 "Texture compression", "Triplanar mapping"
 *   stochastic EWA by reservoir sampling ....... Sec. 4.1 (EWA paragraph); Suppl. S.4 (EWA listing)
 *   filter importance sampling (FIS) ........... Sec. 4.2; Sec. 5 "Magnification, Filter
 *                                                Importance Sampling"; Suppl. S.4.2
 *   transmittance in a density grid ............ Sec. 5 (offline rendering)
 *   black-body emission of a temperature grid .. Sec. 5 "Filtering nonlinear physical properties"
 *
 * Readings where the paper is silent (the GPU side follows the same ones):
 *   - raster coordinates put texel centres at integers: p = u*N - 0.5;
 *   - uniforms are 24-bit: u = (w >> 8) * 2^-24, so u lies in [0, 1);
 *   - the running-sum thresholds of the cubic B-spline are evaluated in the
 *     factored forms below (algebraically equal to the kernel of S.2);
 *   - ties advance: the pick is the number of thresholds C_k with u >= C_k;
 *   - the random stream is the 4-D PCG hash "pcg4d" of Jarzynski and Olano,
 *     "Hash Functions for GPU Rendering" (JCGT 9(3), 2020), keyed on
 *     (query, sample, step, seed);
 *   - 2-D textures repeat or clamp; 3-D grids read zero outside.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_EXPORT __attribute__((visibility("default")))

enum { F_NEAREST = 0, F_LINEAR = 1, F_BSPLINE3 = 2, F_KEYS3 = 3, F_GAUSS_FRS = 4, F_GAUSS_FIS = 5,
       F_BSPLINE3_FIS = 6, F_EWA = 7, F_MITCHELL = 8 };
enum { M_BEFORE = 0, M_AFTER = 1, M_STOCH = 2, M_SPLIT = 3 };
enum { FMT_RGBA32F = 0, FMT_RGBA8 = 1, FMT_R16F = 2, FMT_R32F = 3, FMT_DCT8 = 4 };
enum { WRAP_REPEAT = 0, WRAP_CLAMP = 1 };
enum { MIP_NONE = 0, MIP_NEAREST = 1, MIP_LINEAR = 2 };

static const double PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* Random stream: pcg4d, from its published definition (JCGT 2020).         */
/* An LCG step on every word, a cross-multiplying mix, a 16-bit xorshift and */
/* a second cross-multiplying mix.  All arithmetic is modulo 2^32.           */
/* ------------------------------------------------------------------------ */
ORC_EXPORT void orc_pcg4d(const uint32_t in[4], uint32_t out[4])
{
    uint32_t x = in[0] * 1664525u + 1013904223u;
    uint32_t y = in[1] * 1664525u + 1013904223u;
    uint32_t z = in[2] * 1664525u + 1013904223u;
    uint32_t w = in[3] * 1664525u + 1013904223u;
    x += y * w;
    y += z * x;
    z += x * y;
    w += y * z;
    x ^= x >> 16;
    y ^= y >> 16;
    z ^= z >> 16;
    w ^= w >> 16;
    x += y * w;
    y += z * x;
    z += x * y;
    w += y * z;
    out[0] = x;
    out[1] = y;
    out[2] = z;
    out[3] = w;
}

ORC_EXPORT void orc_pcg4d_batch(const uint32_t *in, uint32_t *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        orc_pcg4d(in + 4 * i, out + 4 * i);
}

/* 24-bit uniform in [0,1): exactly representable in binary32. */
static float uniform24(uint32_t w)
{
    return (float)(w >> 8) * 0x1p-24f;
}

/* ------------------------------------------------------------------------ */
/* Filter kernels (Suppl. S.2), binary64 closed forms.                      */
/* ------------------------------------------------------------------------ */
ORC_EXPORT double orc_kbs(double x)
{
    double a = fabs(x);
    if (a <= 1.0)
        return (4.0 - 3.0 * a * a * (2.0 - a)) / 6.0;
    if (a <= 2.0)
        return (2.0 - a) * (2.0 - a) * (2.0 - a) / 6.0;
    return 0.0;
}

/* Interpolating cubic K3 of S.2 with a = -1/2 (Keys): negative lobes on
 * 1 < |x| < 2. */
ORC_EXPORT double orc_k3(double x)
{
    const double a = -0.5;
    double t = fabs(x);
    if (t < 1.0)
        return (a + 2.0) * t * t * t - (a + 3.0) * t * t + 1.0;
    if (t < 2.0)
        return a * t * t * t - 5.0 * a * t * t + 8.0 * a * t - 4.0 * a;
    return 0.0;
}

/* The Mitchell-Netravali cubic with B = C = 1/3 (Mitchell and Netravali,
 * "Reconstruction Filters in Computer Graphics", 1988), the other reading of
 * the paper's "Mitchell" filter: (7|x|^3 - 12|x|^2 + 16/3)/6 on |x| < 1 and
 * (-7/3 |x|^3 + 12|x|^2 - 20|x| + 32/3)/6 on 1 <= |x| < 2, whose outer lobe
 * changes sign at |x| = 8/7. */
ORC_EXPORT double orc_kmn(double x)
{
    double t = fabs(x);
    if (t < 1.0)
        return (7.0 * t * t * t - 12.0 * t * t + 16.0 / 3.0) / 6.0;
    if (t < 2.0)
        return (-7.0 / 3.0 * t * t * t + 12.0 * t * t - 20.0 * t + 32.0 / 3.0) / 6.0;
    return 0.0;
}

ORC_EXPORT double orc_ktent(double x)
{
    double a = fabs(x);
    return a < 1.0 ? 1.0 - a : 0.0;
}

/* Taps and binary64 weights of one axis.  The lookup point sits at fraction
 * t past texel i0; the cubic B-spline touches i0-1..i0+2 (Sec. 4.1), the tent
 * i0..i0+1 and the box the nearest texel. Returns the tap count. */
static int axis_weights(int filter, double t, int *first_off, double w[4])
{
    if (filter == F_BSPLINE3) {
        *first_off = -1;
        for (int k = 0; k < 4; ++k)
            w[k] = orc_kbs(t - (double)(k - 1));
        return 4;
    }
    if (filter == F_LINEAR) {
        *first_off = 0;
        w[0] = orc_ktent(t);
        w[1] = orc_ktent(t - 1.0);
        return 2;
    }
    if (filter == F_KEYS3) {
        *first_off = -1;
        for (int k = 0; k < 4; ++k)
            w[k] = orc_k3(t - (double)(k - 1));
        return 4;
    }
    if (filter == F_MITCHELL) {
        *first_off = -1;
        for (int k = 0; k < 4; ++k)
            w[k] = orc_kmn(t - (double)(k - 1));
        return 4;
    }
    /* nearest (box, S.2 K0): the texel whose cell contains the point */
    *first_off = (t >= 0.5) ? 1 : 0;
    w[0] = 1.0;
    return 1;
}

ORC_EXPORT void orc_axis_weights64(int filter, double t, double w[4])
{
    int off;
    w[0] = w[1] = w[2] = w[3] = 0.0;
    axis_weights(filter, t, &off, w);
}

/* Running-sum thresholds of the axis weights in binary32: the pick is the
 * first tap j with u < C_j (Sec. 2.2 "Sampling arrays"; the weights already
 * sum to one).  Returns the number of thresholds (taps - 1).
 * Cubic B-spline, s = 1 - t:
 *   C0 = w0          = ((s*s)*s) * (1/6)
 *   C1 = w0 + w1,  w1 = 2/3 - t^2 (1 - t/2)   (one fused op per product below)
 *   C2 = 1 - w3,   w3 = ((t*t)*t) * (1/6)
 * Tent: C0 = 1 - t. */
ORC_EXPORT int orc_thresholds(int filter, float t, float C[3])
{
    if (filter == F_BSPLINE3) {
        const float k6 = 1.0f / 6.0f, k23 = 2.0f / 3.0f;
        float s = 1.0f - t;
        float w0 = ((s * s) * s) * k6;
        float t2 = t * t;
        float half = fmaf(-0.5f, t, 1.0f);
        float w1 = fmaf(-t2, half, k23);
        float w3 = (t2 * t) * k6;
        C[0] = w0;
        C[1] = w0 + w1;
        C[2] = 1.0f - w3;
        return 3;
    }
    if (filter == F_LINEAR) {
        C[0] = 1.0f - t;
        return 1;
    }
    return 0;
}

/* Sampling an array of unnormalised weights (Sec. 2.2 "Sampling arrays"):
 * the first j whose normalised running sum exceeds xi.  binary64. */
ORC_EXPORT int orc_sample_array(const double *w, int n, double xi)
{
    double total = 0.0, run = 0.0;
    for (int i = 0; i < n; ++i)
        total += w[i];
    for (int j = 0; j < n; ++j) {
        run += w[j];
        if (xi < run / total)
            return j;
    }
    return n - 1;
}

/* Positivisation of the separable Keys cubic (Sec. 2.2 "Positivization").
 * Per axis, taps i0-1..i0+2 carry weights (-m0, p1, p2, -m3) with
 * m0 = t s^2/2, m3 = s t^2/2, p1 = 1 - 5t^2/2 + 3t^3/2, p2 the same in s = 1-t
 * (S.2's K3 at a = -1/2, factored); their sums are P+ = p1 + p2 and
 * P- = m0 + m3.  A 2-D product weight is positive on (+,+) and (-,-) and
 * negative on (+,-) and (-,+).  One tap is drawn from each set in proportion
 * to |w|: first the block (by the block sums), then one tap per axis inside
 * the axis' positive or negative pair.  binary32 decision contract:
 * s = 1-t; m0 = (0.5 t)(s s); m3 = (0.5 s)(t t); Pm = m0 + m3;
 * p1 = fma(t t, fma(1.5, t, -2.5), 1); p2 likewise in s; Pp = p1 + p2;
 * inside the positive pair the first tap is taken iff u*Pp < p1, inside the
 * negative pair iff u*Pm < m0; block (+,+) iff u*(A+B) < A with A = Ppx*Ppy,
 * B = Pmx*Pmy; block (+,-) iff u*(Cn+Dn) < Cn with Cn = Ppx*Pmy, Dn = Pmx*Ppy. */
typedef struct {
    float m0, m3, Pm, p1, p2, Pp;
} keys_axis;

static keys_axis keys_axis_of(float t)
{
    keys_axis k;
    float s = 1.0f - t;
    k.m0 = (0.5f * t) * (s * s);
    k.m3 = (0.5f * s) * (t * t);
    k.Pm = k.m0 + k.m3;
    k.p1 = fmaf(t * t, fmaf(1.5f, t, -2.5f), 1.0f);
    k.p2 = fmaf(s * s, fmaf(1.5f, s, -2.5f), 1.0f);
    k.Pp = k.p1 + k.p2;
    return k;
}

/* Tap offsets (relative to i0) of the positive and negative samples; *has_neg
 * is 0 when the negative set is empty (t = 0 on both axes' lobes). */
ORC_EXPORT void orc_keys_pick(float tx, float ty, const float u[6], int off[4], int *has_neg)
{
    keys_axis kx = keys_axis_of(tx), ky = keys_axis_of(ty);
    float A = kx.Pp * ky.Pp, B = kx.Pm * ky.Pm;
    int pp = u[2] * (A + B) < A;               /* positive block: (+,+) or (-,-) */
    if (pp) {
        off[0] = (u[0] * kx.Pp < kx.p1) ? 0 : 1;
        off[1] = (u[1] * ky.Pp < ky.p1) ? 0 : 1;
    } else {
        off[0] = (u[0] * kx.Pm < kx.m0) ? -1 : 2;
        off[1] = (u[1] * ky.Pm < ky.m0) ? -1 : 2;
    }
    float Cn = kx.Pp * ky.Pm, Dn = kx.Pm * ky.Pp;
    *has_neg = (Cn + Dn) > 0.0f;
    int xpos = u[5] * (Cn + Dn) < Cn;          /* negative block: (+,-) or (-,+) */
    if (xpos) {
        off[2] = (u[3] * kx.Pp < kx.p1) ? 0 : 1;
        off[3] = (u[4] * ky.Pm < ky.m0) ? -1 : 2;
    } else {
        off[2] = (u[3] * kx.Pm < kx.m0) ? -1 : 2;
        off[3] = (u[4] * ky.Pp < ky.p1) ? 0 : 1;
    }
}

/* binary64 block sums of the positive and negative product weights. */
static void keys_block_sums(double tx, double ty, double *Wp, double *Wm)
{
    double wx[4], wy[4];
    for (int k = 0; k < 4; ++k) {
        wx[k] = orc_k3(tx - (double)(k - 1));
        wy[k] = orc_k3(ty - (double)(k - 1));
    }
    double Ppx = wx[1] + wx[2], Pmx = -(wx[0] + wx[3]);
    double Ppy = wy[1] + wy[2], Pmy = -(wy[0] + wy[3]);
    *Wp = Ppx * Ppy + Pmx * Pmy;
    *Wm = Ppx * Pmy + Pmx * Ppy;
}

/* Positivisation of the separable Mitchell-Netravali cubic (Sec. 2.2
 * "Positivization"; the paper's listing sorts each weight into a positive
 * or a negative reservoir by its sign).  Per axis the weights of taps
 * i0-1..i0+2 in factored binary32 form, s = 1-t:
 *   w0 = ((s s) fma(-7, t, 1)) K18, w1 = fma(t t, fma(K76, t, -2), K89),
 *   w2 = fma(s s, fma(K76, s, -2), K89), w3 = ((t t) fma(7, t, -6)) K18,
 * K18 = fl(1/18), K76 = fl(7/6), K89 = fl(8/9) (the inner taps are always
 * positive; w0 is positive for t < 1/7 and w3 for t > 6/7).  The positive
 * set of an axis is its taps with w > 0, the negative set those with w < 0;
 * P+ and P- are their |w| summed in tap order.  Inside a set the tap is the
 * first (in tap order) whose running sum c of |w| satisfies u P < c (the
 * set's last tap otherwise).  Blocks and their decisions as for the Keys
 * cubic: (+,+) iff u (A + B) < A with A = P+x P+y, B = P-x P-y; (+,-) iff
 * u (Cn + Dn) < Cn with Cn = P+x P-y, Dn = P-x P+y; the estimate is
 * (A + B) f(t+) - (Cn + Dn) f(t-). */
typedef struct {
    float w[4], Pp, Pm;
} pn_axis;

static pn_axis mitchell_axis_of(float t)
{
    const float K18 = 1.0f / 18.0f, K76 = 7.0f / 6.0f, K89 = 8.0f / 9.0f;
    pn_axis a;
    float s = 1.0f - t;
    a.w[0] = ((s * s) * fmaf(-7.0f, t, 1.0f)) * K18;
    a.w[1] = fmaf(t * t, fmaf(K76, t, -2.0f), K89);
    a.w[2] = fmaf(s * s, fmaf(K76, s, -2.0f), K89);
    a.w[3] = ((t * t) * fmaf(7.0f, t, -6.0f)) * K18;
    a.Pp = 0.0f;
    a.Pm = 0.0f;
    for (int k = 0; k < 4; ++k) {
        if (a.w[k] > 0.0f)
            a.Pp = a.Pp + a.w[k];
        else if (a.w[k] < 0.0f)
            a.Pm = a.Pm + (-a.w[k]);
    }
    return a;
}

/* tap (0..3) of the positive (sign > 0) or negative set of one axis */
static int pn_pick(const pn_axis *a, int sign, float u)
{
    const float P = sign > 0 ? a->Pp : a->Pm;
    const float uP = u * P;
    float c = 0.0f;
    int last = -1;
    for (int k = 0; k < 4; ++k) {
        float m = sign > 0 ? a->w[k] : -a->w[k];
        if (!(m > 0.0f))
            continue;
        c = c + m;
        last = k;
        if (uP < c)
            return k;
    }
    return last;
}

ORC_EXPORT void orc_mitchell_axis(float t, float w[4], float *Pp, float *Pm)
{
    pn_axis a = mitchell_axis_of(t);
    for (int k = 0; k < 4; ++k)
        w[k] = a.w[k];
    *Pp = a.Pp;
    *Pm = a.Pm;
}

/* Tap offsets (relative to i0) of the positive and negative samples. */
ORC_EXPORT void orc_mitchell_pick(float tx, float ty, const float u[6], int off[4], int *has_neg)
{
    pn_axis ax = mitchell_axis_of(tx), ay = mitchell_axis_of(ty);
    float A = ax.Pp * ay.Pp, B = ax.Pm * ay.Pm;
    int pp = u[2] * (A + B) < A;
    off[0] = pn_pick(&ax, pp ? 1 : -1, u[0]) - 1;
    off[1] = pn_pick(&ay, pp ? 1 : -1, u[1]) - 1;
    float Cn = ax.Pp * ay.Pm, Dn = ax.Pm * ay.Pp;
    *has_neg = (Cn + Dn) > 0.0f;
    int xpos = u[5] * (Cn + Dn) < Cn;
    off[2] = pn_pick(&ax, xpos ? 1 : -1, u[3]) - 1;
    off[3] = pn_pick(&ay, xpos ? -1 : 1, u[4]) - 1;
}

/* binary64 block sums of the positive and negative product weights of the
 * Mitchell-Netravali cubic */
static void mitchell_block_sums(double tx, double ty, double *Wp, double *Wm)
{
    double px = 0, mx = 0, py = 0, my = 0;
    for (int k = 0; k < 4; ++k) {
        double a = orc_kmn(tx - (double)(k - 1)), b = orc_kmn(ty - (double)(k - 1));
        if (a > 0)
            px += a;
        else
            mx -= a;
        if (b > 0)
            py += b;
        else
            my -= b;
    }
    *Wp = px * py + mx * my;
    *Wm = px * my + mx * py;
}

/* Index of the picked tap among the filter's taps (0..3), ties advance. */
ORC_EXPORT int orc_pick(int filter, float t, float u)
{
    float C[3];
    int nc = orc_thresholds(filter, t, C);
    if (nc == 0)
        return t >= 0.5f ? 1 : 0; /* nearest: offset from i0 */
    int j = 0;
    for (int k = 0; k < nc; ++k)
        if (u >= C[k])
            ++j;
    return j;
}

/* Uniform sample reuse (Sec. 2.2 eq. uniform-sample-reuse) generalised to
 * the bin [lo, hi) that the pick fell into: u' = (u - lo) / (hi - lo). */
ORC_EXPORT float orc_reuse(int filter, float t, float u, int j)
{
    float C[3];
    int nc = orc_thresholds(filter, t, C);
    if (nc == 0)
        return u;
    float lo = (j == 0) ? 0.0f : C[j - 1];
    float hi = (j == nc) ? 1.0f : C[j];
    float r = (u - lo) / (hi - lo);
    const float top = 0x1.fffffep-1f;
    return r > top ? top : r;
}

/* Exact probability that a 24-bit uniform selects tap j: the uniforms are
 * k*2^-24, k = 0..2^24-1, and u >= C  <=>  k >= ceil(C*2^24). */
ORC_EXPORT void orc_pick_pmf(int filter, float t, double P[4])
{
    float C[3];
    int nc = orc_thresholds(filter, t, C);
    P[0] = P[1] = P[2] = P[3] = 0.0;
    if (nc == 0) {
        P[0] = 1.0;
        return;
    }
    double prev = 0.0;
    for (int j = 0; j <= nc; ++j) {
        double c = (j == nc) ? 16777216.0 : ceil((double)C[j] * 16777216.0);
        if (c < 0.0)
            c = 0.0;
        if (c > 16777216.0)
            c = 16777216.0;
        P[j] = (c - prev) / 16777216.0;
        if (c > prev)
            prev = c;
    }
}

/* ------------------------------------------------------------------------ */
/* Binary32 elementary functions of the decision contract.  The Gaussian     */
/* samplers decide texels through exp, log, sin and cos; for the GPU to       */
/* reach the same decisions bit for bit, both sides evaluate these with one  */
/* written-out sequence of correctly rounded binary32 operations (+ - * /,   */
/* sqrt, fma, floor, frexp, ldexp).  Accuracy is pinned against libm.        */
/* ------------------------------------------------------------------------ */
static const float LN2_HI = 0x1.62e4p-1f;      /* ln 2 to 17 bits: n * LN2_HI is exact for |n| < 128 */
static const float LN2_LO = 1.42860677e-6f;    /* ln 2 - LN2_HI */

/* ln x for x in (0, 1]: x = m 2^e with m in [sqrt(1/2), sqrt(2)); ln m =
 * 2 atanh(s), s = (m - 1)/(m + 1), by the series 2 s (1 + s^2/3 + s^4/5 +
 * s^6/7 + s^8/9) (|s| <= 0.1716); ln x = e ln 2 + ln m with ln 2 in two
 * parts (the reduction of Cody and Waite). */
ORC_EXPORT float orc_lnc(float x)
{
    int e;
    float m = frexpf(x, &e);
    if (m < 0.70710678f) {
        m = m * 2.0f;
        e = e - 1;
    }
    float s = (m - 1.0f) / (m + 1.0f);
    float z = s * s;
    float p = fmaf(z, fmaf(z, fmaf(z, fmaf(z, 1.0f / 9.0f, 1.0f / 7.0f), 1.0f / 5.0f), 1.0f / 3.0f), 1.0f);
    float r = (2.0f * s) * p;
    float fe = (float)e;
    return fmaf(fe, LN2_HI, fmaf(fe, LN2_LO, r));
}

/* e^x for x in [-80, 0] (0 below): n = floor(x log2 e + 1/2), r = x - n ln 2
 * (two parts), e^r by its Taylor polynomial to r^7 (|r| <= 0.35), times 2^n. */
ORC_EXPORT float orc_expc(float x)
{
    if (!(x >= -80.0f))
        return 0.0f;
    float n = floorf(fmaf(x, 1.44269504f, 0.5f));
    float r = fmaf(-n, LN2_HI, x);
    r = fmaf(-n, LN2_LO, r);
    float p = fmaf(r, 1.0f / 5040.0f, 1.0f / 720.0f);
    p = fmaf(r, p, 1.0f / 120.0f);
    p = fmaf(r, p, 1.0f / 24.0f);
    p = fmaf(r, p, 1.0f / 6.0f);
    p = fmaf(r, p, 0.5f);
    p = fmaf(r, p, 1.0f);
    p = fmaf(r, p, 1.0f);
    return ldexpf(p, (int)n);
}

/* cos and sin of 2 pi v, v in [0, 1): the quadrant from 4v (exact), the rest
 * folded into an angle x in [0, pi/4], Taylor series to x^9 (sin) and x^10
 * (cos), then rotated into the quadrant. */
ORC_EXPORT void orc_sincos2pi(float v, float *c, float *s)
{
    float a = 4.0f * v;
    float qf = floorf(a);
    float f = a - qf;
    int q = (int)qf & 3;
    int fold = f > 0.5f;
    float h = fold ? 1.0f - f : f;
    float x = h * 1.57079637f;
    float z = x * x;
    float sp = fmaf(z, 1.0f / 362880.0f, -1.0f / 5040.0f);
    sp = fmaf(z, sp, 1.0f / 120.0f);
    sp = fmaf(z, sp, -1.0f / 6.0f);
    sp = fmaf(z, sp, 1.0f);
    float sn = x * sp;
    float cp = fmaf(z, -1.0f / 3628800.0f, 1.0f / 40320.0f);
    cp = fmaf(z, cp, -1.0f / 720.0f);
    cp = fmaf(z, cp, 1.0f / 24.0f);
    cp = fmaf(z, cp, -0.5f);
    float cs = fmaf(z, cp, 1.0f);
    float c0 = fold ? sn : cs, s0 = fold ? cs : sn;
    switch (q) {
    case 0: *c = c0; *s = s0; break;
    case 1: *c = -s0; *s = c0; break;
    case 2: *c = -c0; *s = -s0; break;
    default: *c = s0; *s = -c0; break;
    }
}

ORC_EXPORT void orc_elementary_batch(int which, const float *x, float *y, float *y2, int64_t n)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        if (which == 0)
            y[i] = orc_lnc(x[i]);
        else if (which == 1)
            y[i] = orc_expc(x[i]);
        else
            orc_sincos2pi(x[i], &y[i], &y2[i]);
    }
}

/* Gaussian filter importance sampling (Sec. 4.2, FIS): an offset drawn from
 * the isotropic normal of standard deviation sigma (texels) by the
 * Box-Muller transform (Box and Muller 1958) of two uniforms, radius
 * sigma sqrt(-2 ln(1 - u1)) (1 - u1 lies in (0, 1]), angle 2 pi u2.  The
 * nearest texel of the offset point is then read: with raster position
 * p = i0 + t the tap offset is floor((t + 1/2) + d).  Its probability is the
 * Gaussian's mass over the texel's cell, so FIS with nearest lookup realises
 * the Gaussian convolved with the unit box. */
ORC_EXPORT void orc_fis_gauss_offset(float u1, float u2, float sigma, float *dx, float *dy)
{
    float r = sigma * sqrtf(-2.0f * orc_lnc(1.0f - u1));
    float c, s;
    orc_sincos2pi(u2, &c, &s);
    *dx = r * c;
    *dy = r * s;
}

ORC_EXPORT int orc_fis_nearest(float t, float d) { return (int)floorf((t + 0.5f) + d); }

/* Cubic B-spline by FIS (Sec. 4.2): the cubic B-spline is the quadratic one
 * convolved with the unit box (Cox-de Boor), and the sum of three uniforms
 * has the quadratic B-spline density on [0, 3]; so the nearest texel of
 * p + (xi1 + xi2 + xi3 - 3/2) is distributed by the cubic B-spline weights.
 * Decision: S = a + b + c of the three 24-bit words (exact integer),
 * S = 2^24 q + r; tap offset q - 1 + [r 2^-24 >= 1 - t], which is
 * floor(t + S 2^-24 - 1) whenever 1 - t is a multiple of 2^-24. */
ORC_EXPORT int orc_fis_bspline_pick(float t, uint32_t a, uint32_t b, uint32_t c)
{
    uint32_t S = (a >> 8) + (b >> 8) + (c >> 8);
    int q = (int)(S >> 24);
    float r = (float)(S & 0xffffffu) * 0x1p-24f;
    return q - 1 + (r >= 1.0f - t ? 1 : 0);
}

/* Exact probabilities of the four offsets of orc_fis_bspline_pick over all
 * 2^72 word triples: the number of triples of 24-bit integers with sum
 * below X is sum_j (-1)^j C(3,j) C(X - j 2^24 + 2, 3) (stars and bars with
 * inclusion-exclusion). */
static unsigned __int128 below3(int64_t X)
{
    const int64_t M = 1 << 24;
    __int128 acc = 0;
    const int sgn[4] = {1, -3, 3, -1};
    for (int j = 0; j < 4; ++j) {
        __int128 n = (__int128)X - (__int128)j * M + 2;
        if (n >= 3)
            acc += (__int128)sgn[j] * (n * (n - 1) * (n - 2) / 6);
    }
    return (unsigned __int128)acc;
}

ORC_EXPORT void orc_fis_bspline_pmf(float t, double P[4])
{
    const int64_t M = 1 << 24;
    /* smallest r with r 2^-24 >= 1 - t */
    int64_t R = (int64_t)ceil((double)(1.0f - t) * 16777216.0);
    if (R < 0)
        R = 0;
    if (R > M)
        R = M;
    const long double total = (long double)M * (long double)M * (long double)M;
    for (int k = 0; k < 4; ++k)
        P[k] = 0.0;
    for (int q = 0; q < 3; ++q) {
        int64_t a = q * M, b = q * M + R, c = (q + 1) * M;
        P[q] += (double)((long double)(below3(b) - below3(a)) / total);      /* offset q - 1 */
        P[q + 1] += (double)((long double)(below3(c) - below3(b)) / total);  /* offset q */
    }
}

/* Discrete Gaussian on the nearest 4x4 texels (FRS, Sec. 4.1; the comparison
 * of Sec. 5 "Magnification, Filter Importance Sampling"; Suppl. S.4.2),
 * sampled per axis by its running sum: with
 * h = 1/(2 sigma^2), a_k = (d_k d_k) h for d_k = (k - 1) - t, k = 0..3, the
 * weights g_k = e^(a_min - a_k) (the common factor e^(-a_min) cancels in
 * the normalisation and keeps the largest weight at 1), W = g0+g1+g2+g3,
 * C0 = g0/W, C1 = (g0+g1)/W, C2 = (g0+g1+g2)/W.  The 2-D weight is the
 * product of the axis weights, so the separable pick has the 2-D weights'
 * distribution over the 16 texels. */
ORC_EXPORT void orc_gauss_thresholds(float t, float h, float C[3])
{
    float a[4], g[4];
    for (int k = 0; k < 4; ++k) {
        float d = (float)(k - 1) - t;
        a[k] = (d * d) * h;
    }
    float amin = fminf(fminf(a[0], a[1]), fminf(a[2], a[3]));
    for (int k = 0; k < 4; ++k)
        g[k] = orc_expc(amin - a[k]);
    float s1 = g[0] + g[1];
    float s2 = s1 + g[2];
    float W = s2 + g[3];
    C[0] = g[0] / W;
    C[1] = s1 / W;
    C[2] = s2 / W;
}

ORC_EXPORT float orc_gauss_h(float sigma) { return 0.5f / (sigma * sigma); }

/* Exact pick probabilities for the discrete Gaussian over the 24-bit lattice. */
ORC_EXPORT void orc_gauss_pick_pmf(float t, float h, double P[4])
{
    float C[3];
    orc_gauss_thresholds(t, h, C);
    double prev = 0.0;
    for (int j = 0; j < 4; ++j) {
        double c = (j == 3) ? 16777216.0 : ceil((double)C[j] * 16777216.0);
        if (c > 16777216.0)
            c = 16777216.0;
        if (c < prev)
            c = prev;
        P[j] = (c - prev) / 16777216.0;
        prev = c;
    }
}

/* Binary64 weights of the Gaussian filters.  Discrete: e^(-d_k^2 h) over the
 * 4 taps, normalised.  FIS with nearest lookup: the mass of N(0, sigma^2)
 * over each texel's cell, Phi((k + 1/2 - t)/sigma) - Phi((k - 1/2 - t)/sigma),
 * for offsets k in [-R, R+1], R = ceil(7 sigma) + 1 (the mass left outside
 * is below 2 Phi(-7) = 2.6e-12 per axis). */
static int gauss_fis_radius(double sigma) { return (int)ceil(7.0 * sigma) + 1; }

static double gauss_cell(double sigma, double t, int k)
{
    double r2 = sqrt(2.0) * sigma;
    return 0.5 * (erfc(((double)k - 0.5 - t) / r2) - erfc(((double)k + 0.5 - t) / r2));
}

/* ------------------------------------------------------------------------ */
/* Scalar formats                                                            */
/* ------------------------------------------------------------------------ */

/* IEEE 754 binary16 -> binary64, from the format definition. */
ORC_EXPORT double orc_half_to_double(uint16_t h)
{
    int sign = (h >> 15) & 1;
    int e = (h >> 10) & 0x1f;
    int m = h & 0x3ff;
    double v;
    if (e == 0)
        v = ldexp((double)m, -24);
    else if (e == 31)
        v = m ? NAN : INFINITY;
    else
        v = ldexp((double)(m | 0x400), e - 25);
    return sign ? -v : v;
}

/* ------------------------------------------------------------------------ */
/* Shading: GGX microfacet specular + Lambert diffuse, times the cosine      */
/* (the paper's f-hat is BSDF x cosine, Sec. 3), under one directional light. */
/* p[16]: n[3], wo[3], wi[3], radiance[3], f0, r_bias, r_scale, unused.       */
/* The texel supplies albedo (RGB) and a roughness parameter A; the          */
/* perceptual roughness r = r_bias + r_scale*A, alpha = r^2.                 */
/* ------------------------------------------------------------------------ */
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

ORC_EXPORT void orc_shade_ggx(const double *p, const double rgba[4], double out[3])
{
    const double *n = p, *wo = p + 3, *wi = p + 6, *rad = p + 9;
    double f0 = p[12], rb = p[13], rs = p[14];
    double h[3] = {wo[0] + wi[0], wo[1] + wi[1], wo[2] + wi[2]};
    double hl = sqrt(dot3(h, h));
    h[0] /= hl;
    h[1] /= hl;
    h[2] /= hl;
    double nh = dot3(n, h), no = dot3(n, wo), ni = dot3(n, wi), ih = dot3(wi, h);
    double r = rb + rs * rgba[3];
    double a = r * r, a2 = a * a;
    double dd = nh * nh * (a2 - 1.0) + 1.0;
    double D = a2 / (PI * dd * dd);
    double G1o = 2.0 * no / (no + sqrt(a2 + (1.0 - a2) * no * no));
    double G1i = 2.0 * ni / (ni + sqrt(a2 + (1.0 - a2) * ni * ni));
    double F = f0 + (1.0 - f0) * pow(1.0 - ih, 5.0);
    double spec = D * G1o * G1i * F / (4.0 * no * ni);
    for (int c = 0; c < 3; ++c)
        out[c] = rad[c] * (rgba[c] / PI + spec) * ni;
}

/* ------------------------------------------------------------------------ */
/* 2-D textures                                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    const uint8_t *base;
    int w, h, levels, fmt, wrap, mip;
    const int64_t *off;
    const float *dct_range; /* FMT_DCT8: AC range of channel c on level l at [4 l + c] */
} tex2d;

static int lvl_dim(int n, int l)
{
    int d = n >> l;
    return d < 1 ? 1 : d;
}

/* ------------------------------------------------------------------------ */
/* DCT texture compression (Sec. 5 "Texture compression"): 8x8 texel blocks, */
/* per channel the six lowest-frequency coefficients of the orthonormal 2-D  */
/* DCT-II in zigzag order, DC in 7 bits and the five AC in 5 bits each: one  */
/* 32-bit word per channel, 16 bytes per RGBA block (16x smaller than RGBA8).*/
/* Readings: coefficients of the texel values v = byte/255; blocks past the  */
/* level's edge replicate the edge texels; DC = 8 x block mean in [0, 8] is  */
/* quantised uniformly to 0..127; AC uniformly to -15..15 over [-R, R] with  */
/* R the largest |AC| of that channel on that level (stored beside the       */
/* blocks); decoded values are clamped to [0, 1].                            */
/* ------------------------------------------------------------------------ */
/* zigzag order (u = horizontal, v = vertical frequency) */
static const int DCT_U[6] = {0, 1, 0, 0, 1, 2};
static const int DCT_V[6] = {0, 0, 1, 2, 1, 0};

/* binary64 basis alpha(k) cos((2x+1) k pi / 16), alpha(0) = sqrt(1/8), else 1/2 */
static double dct_basis64(int k, int x)
{
    double a = k == 0 ? sqrt(0.125) : 0.5;
    return a * cos((2.0 * x + 1.0) * k * PI / 16.0);
}

/* the same rounded to binary32: the encoder's constants */
ORC_EXPORT float orc_dct_basis32(int k, int x) { return (float)dct_basis64(k, x); }

/* Six coefficients of one channel of one block in binary32: rows first,
 * R_u(y) = sum_x c_u(x) v(x, y), then C(u, v) = sum_y c_v(y) R_u(y), each
 * sum a chain of fused multiply-adds in increasing index from 0. */
static void dct_block_coeffs(const uint8_t *lv, int wl, int hl, int bx, int by, int c, float C[6])
{
    float R[3][8];
    for (int y = 0; y < 8; ++y) {
        int yy = by * 8 + y < hl ? by * 8 + y : hl - 1;
        float v[8];
        for (int x = 0; x < 8; ++x) {
            int xx = bx * 8 + x < wl ? bx * 8 + x : wl - 1;
            v[x] = (float)lv[4 * ((int64_t)yy * wl + xx) + c] / 255.0f;
        }
        for (int u = 0; u < 3; ++u) {
            float acc = 0.0f;
            for (int x = 0; x < 8; ++x)
                acc = fmaf(orc_dct_basis32(u, x), v[x], acc);
            R[u][y] = acc;
        }
    }
    for (int k = 0; k < 6; ++k) {
        float acc = 0.0f;
        for (int y = 0; y < 8; ++y)
            acc = fmaf(orc_dct_basis32(DCT_V[k], y), R[DCT_U[k]][y], acc);
        C[k] = acc;
    }
}

/* Encode one RGBA8 level (wl x hl) into ceil(wl/8) x ceil(hl/8) blocks of
 * four words and its four AC ranges.  Codes (binary32 decisions):
 *   DC: clamp(floor(C0 * 15.875 + 1/2), 0, 127);
 *   AC: R > 0 ? clamp(floor(Ck * (15/R) + 1/2), -15, 15) + 15 : 15;
 *   word = DC | AC1 << 7 | AC2 << 12 | AC3 << 17 | AC4 << 22 | AC5 << 27. */
ORC_EXPORT void orc_dct_encode_level(const uint8_t *lv, int wl, int hl, uint32_t *blocks, float range[4])
{
    int bw = (wl + 7) / 8, bh = (hl + 7) / 8;
    for (int c = 0; c < 4; ++c) {
        float r = 0.0f;
        for (int by = 0; by < bh; ++by)
            for (int bx = 0; bx < bw; ++bx) {
                float C[6];
                dct_block_coeffs(lv, wl, hl, bx, by, c, C);
                for (int k = 1; k < 6; ++k)
                    r = fmaxf(r, fabsf(C[k]));
            }
        range[c] = r;
        float sc = r > 0.0f ? 15.0f / r : 0.0f;
        for (int by = 0; by < bh; ++by)
            for (int bx = 0; bx < bw; ++bx) {
                float C[6];
                dct_block_coeffs(lv, wl, hl, bx, by, c, C);
                int dc = (int)floorf(C[0] * 15.875f + 0.5f);
                dc = dc < 0 ? 0 : (dc > 127 ? 127 : dc);
                uint32_t word = (uint32_t)dc;
                for (int k = 1; k < 6; ++k) {
                    int a = 15;
                    if (r > 0.0f) {
                        a = (int)floorf(C[k] * sc + 0.5f);
                        a = (a < -15 ? -15 : (a > 15 ? 15 : a)) + 15;
                    }
                    word |= (uint32_t)a << (7 + 5 * (k - 1));
                }
                blocks[4 * ((int64_t)by * bw + bx) + c] = word;
            }
    }
}

/* Decoded texel (binary64 arithmetic, basis in binary64), clamped to [0, 1]. */
static void dct_decode(const uint32_t *blk, const float *range, int x, int y, double out[4])
{
    for (int c = 0; c < 4; ++c) {
        uint32_t wd = blk[c];
        double v = (double)(wd & 127u) * (8.0 / 127.0) * dct_basis64(0, x) * dct_basis64(0, y);
        for (int k = 1; k < 6; ++k) {
            int a = (int)((wd >> (7 + 5 * (k - 1))) & 31u) - 15;
            double coef = (double)a * (double)range[c] / 15.0;
            v += coef * dct_basis64(DCT_U[k], x) * dct_basis64(DCT_V[k], y);
        }
        out[c] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
    }
}

static void fetch2d(const tex2d *t, int l, int x, int y, double out[4])
{
    int wl = lvl_dim(t->w, l);
    int64_t idx = (int64_t)y * wl + x;
    const uint8_t *lv = t->base + t->off[l];
    if (t->fmt == FMT_DCT8) {
        int bw = (wl + 7) / 8;
        const uint32_t *blk = (const uint32_t *)lv + 4 * ((int64_t)(y / 8) * bw + x / 8);
        dct_decode(blk, t->dct_range + 4 * l, x % 8, y % 8, out);
        return;
    }
    if (t->fmt == FMT_RGBA32F) {
        const float *f = (const float *)lv + 4 * idx;
        for (int c = 0; c < 4; ++c)
            out[c] = (double)f[c];
    } else {
        const uint8_t *b = lv + 4 * idx;
        for (int c = 0; c < 4; ++c)
            out[c] = (double)b[c] / 255.0;
    }
}

static float wrap_coord(int wrap, float u)
{
    if (wrap == WRAP_REPEAT)
        return u - floorf(u);
    return fminf(fmaxf(u, 0.0f), 1.0f);
}

static int wrap_tap(int wrap, int i, int n)
{
    if (wrap == WRAP_REPEAT) {
        int r = i % n;
        return r < 0 ? r + n : r;
    }
    return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

/* Raster position of coordinate u on an axis of n texels (centres at
 * integers): p = u*n - 0.5 as one fused operation; i0 = floor(p), t = p - i0. */
static void raster(float u, int n, int *i0, float *t)
{
    float p = fmaf(u, (float)n, -0.5f);
    float f = floorf(p);
    *i0 = (int)f;
    *t = p - f;
}

/* MIP level(s) and their weights from the level of detail lambda
 * (Sec. 2.1 pyramids; the stochastic single-level choice of Sec. 4.2.1). */
static void levels_of(const tex2d *t, float lam, int *l0, int *l1, float *f)
{
    if (t->mip == MIP_NONE) {
        *l0 = *l1 = 0;
        *f = 0.0f;
        return;
    }
    float lc = fminf(fmaxf(lam, 0.0f), (float)(t->levels - 1));
    float fl = floorf(lc);
    float fr = lc - fl;
    int a = (int)fl;
    if (t->mip == MIP_NEAREST) {
        a += (fr >= 0.5f) ? 1 : 0;
        if (a > t->levels - 1)
            a = t->levels - 1;
        *l0 = *l1 = a;
        *f = 0.0f;
        return;
    }
    *l0 = a;
    *l1 = a + 1 <= t->levels - 1 ? a + 1 : t->levels - 1;
    *f = fr;
}

/* Normal-mapped GGX (Sec. 3 "Normal maps": filtering normals before shading
 * changes appearance).  The texel's RGB encodes a tangent-space normal
 * m = 2 rgb - 1, A the roughness parameter as for GGX; the shading normal
 * is m/|m| (z if m = 0) in the frame (e1, e2, n) of the geometric normal n
 * (branchless basis of Duff et al., JCGT 6(1), 2017); a grey material,
 * albedo 1/2, is shaded with the GGX + Lambert model above with the
 * cosines clamped at 0 and the masking factors divided by their cosines
 * analytically, G1(c)/c = 2/(c + sqrt(a^2 + (1 - a^2) c^2)): the result is
 * continuous, 0 where the shading normal faces away from the light, and
 * grazing (c = 0) where it faces away from the viewer. */
ORC_EXPORT void orc_shade_ggx_normal(const double *p, const double rgba[4], double out[3])
{
    const double *n = p, *wo = p + 3, *wi = p + 6, *rad = p + 9;
    double f0 = p[12], rb = p[13], rs = p[14];
    double sg = n[2] >= 0.0 ? 1.0 : -1.0;
    double a_ = -1.0 / (sg + n[2]), b_ = n[0] * n[1] * a_;
    double e1[3] = {1.0 + sg * n[0] * n[0] * a_, sg * b_, -sg * n[0]};
    double e2[3] = {b_, sg + n[1] * n[1] * a_, -n[1]};
    double m[3] = {2.0 * rgba[0] - 1.0, 2.0 * rgba[1] - 1.0, 2.0 * rgba[2] - 1.0};
    double ml = sqrt(dot3(m, m));
    double ns[3];
    if (ml > 0.0) {
        for (int c = 0; c < 3; ++c)
            ns[c] = (m[0] * e1[c] + m[1] * e2[c] + m[2] * n[c]) / ml;
    } else {
        ns[0] = n[0], ns[1] = n[1], ns[2] = n[2];
    }
    double h[3] = {wo[0] + wi[0], wo[1] + wi[1], wo[2] + wi[2]};
    double hl = sqrt(dot3(h, h));
    h[0] /= hl;
    h[1] /= hl;
    h[2] /= hl;
    double nh = dot3(ns, h), no = fmax(dot3(ns, wo), 0.0), ni = fmax(dot3(ns, wi), 0.0), ih = dot3(wi, h);
    double r = rb + rs * rgba[3];
    double a = r * r, a2 = a * a;
    double dd = nh * nh * (a2 - 1.0) + 1.0;
    double D = a2 / (PI * dd * dd);
    double go = 2.0 / (no + sqrt(a2 + (1.0 - a2) * no * no)); /* G1(no)/no */
    double gi = 2.0 / (ni + sqrt(a2 + (1.0 - a2) * ni * ni));
    double F = f0 + (1.0 - f0) * pow(1.0 - ih, 5.0);
    double spec = D * go * gi * F / 4.0;
    for (int c = 0; c < 3; ++c)
        out[c] = rad[c] * (0.5 / PI + spec) * ni;
}

static void shade2d(int shade, const double *ggx, const double rgba[4], double *out)
{
    if (shade == 1)
        orc_shade_ggx(ggx, rgba, out);
    else if (shade == 2)
        orc_shade_ggx_normal(ggx, rgba, out);
    else
        for (int c = 0; c < 4; ++c)
            out[c] = rgba[c];
}

static int query_finite(const tex2d *t, const float *q)
{
    if (!isfinite(q[0]) || !isfinite(q[1]))
        return 0;
    if (t->mip != MIP_NONE && !isfinite(q[2]))
        return 0;
    return 1;
}

/* Widest axis window: the FIS Gaussian at sigma = 4 texels (2 R + 2 = 60 taps). */
#define AXIS_TAPS_MAX 64
static int axis_weights_s(int filter, float sigma, double t, int *first_off, double *w);

/* The reconstruction filter alone at level l: sum_i w_i t_i (binary64
 * weights and sums) at the wrapped coordinate (uu, vv). */
static void recon_level(const tex2d *t, float uu, float vv, int l, int filter, float sigma, double rgba[4])
{
    int wl = lvl_dim(t->w, l), hl = lvl_dim(t->h, l);
    int ix, iy;
    float tx, ty;
    raster(uu, wl, &ix, &tx);
    raster(vv, hl, &iy, &ty);
    double wx[AXIS_TAPS_MAX], wy[AXIS_TAPS_MAX];
    int ox, oy;
    int nx = axis_weights_s(filter, sigma, (double)tx, &ox, wx);
    int ny = axis_weights_s(filter, sigma, (double)ty, &oy, wy);
    for (int c = 0; c < 4; ++c)
        rgba[c] = 0.0;
    for (int b = 0; b < ny; ++b)
        for (int a = 0; a < nx; ++a) {
            double texel[4];
            fetch2d(t, l, wrap_tap(t->wrap, ix + ox + a, wl), wrap_tap(t->wrap, iy + oy + b, hl), texel);
            for (int c = 0; c < 4; ++c)
                rgba[c] += wx[a] * wy[b] * texel[c];
        }
}

/* One query of the 2-D filter.  out has 4 (shade none) or 3 (GGX) channels.
 * M_SPLIT (the split-filtering estimator of Sec. 3 eq. split-filtering-shading
 * and Sec. 4: the low-pass filter sampled, the reconstruction filter
 * evaluated before shading): per sample the stochastic level of the key's
 * word 3, then shade(sum_i w_i t_i) on that level; mean over samples. */
static void filter2d_one(const tex2d *t, const float *q, int64_t qi, int filter, int mode, int spp,
                         uint32_t seed, int variant, float sigma, int shade, const double *ggx, double *out,
                         int32_t *taps)
{
    int ch = shade != 0 ? 3 : 4;
    if (!query_finite(t, q)) {
        for (int c = 0; c < ch; ++c)
            out[c] = NAN;
        if (taps && (mode == M_STOCH || mode == M_SPLIT))
            for (int s = 0; s < ((filter == F_KEYS3 || filter == F_MITCHELL) && mode == M_STOCH ? 5 : 3) * spp; ++s)
                taps[s] = INT32_MIN;
        return;
    }
    float uu = wrap_coord(t->wrap, q[0]);
    float vv = wrap_coord(t->wrap, q[1]);
    int l0, l1;
    float f;
    levels_of(t, q[2], &l0, &l1, &f);

    if (mode == M_SPLIT) {
        double acc[4] = {0, 0, 0, 0};
        for (int s = 0; s < spp; ++s) {
            uint32_t key[4] = {(uint32_t)qi, (uint32_t)s, 0u, seed}, w[4];
            orc_pcg4d(key, w);
            int l = (uniform24(w[3]) >= 1.0f - f) ? l1 : l0;
            if (taps) {
                taps[3 * s] = l;
                taps[3 * s + 1] = taps[3 * s + 2] = INT32_MIN;
            }
            double rgba[4], v[4];
            recon_level(t, uu, vv, l, filter, sigma, rgba);
            shade2d(shade, ggx, rgba, v);
            for (int c = 0; c < ch; ++c)
                acc[c] += v[c];
        }
        for (int c = 0; c < ch; ++c)
            out[c] = acc[c] / (double)spp;
        return;
    }

    if (mode == M_STOCH) {
        double acc[4] = {0, 0, 0, 0};
        for (int s = 0; s < spp; ++s) {
            uint32_t key[4] = {(uint32_t)qi, (uint32_t)s, 0u, seed}, w[4];
            orc_pcg4d(key, w);
            float ux = uniform24(w[0]), uy = uniform24(w[1]), ul = uniform24(w[3]);
            /* level: stochastic choice between l0 and l1 with P(l1) = f */
            int l = (ul >= 1.0f - f) ? l1 : l0;
            int wl = lvl_dim(t->w, l), hl = lvl_dim(t->h, l);
            int ix, iy;
            float tx, ty;
            raster(uu, wl, &ix, &tx);
            raster(vv, hl, &iy, &ty);
            if (filter == F_KEYS3 || filter == F_MITCHELL) {
                /* positivised estimator: W+ shade(t+) - W- shade(t-) */
                uint32_t key2[4] = {(uint32_t)qi, (uint32_t)s, 1u, seed}, w2[4];
                orc_pcg4d(key2, w2);
                float u6[6] = {ux, uy, uniform24(w[2]), uniform24(w2[0]), uniform24(w2[1]), uniform24(w2[2])};
                int off[4], has_neg;
                double Wp, Wm;
                if (filter == F_KEYS3) {
                    orc_keys_pick(tx, ty, u6, off, &has_neg);
                    keys_block_sums((double)tx, (double)ty, &Wp, &Wm);
                } else {
                    orc_mitchell_pick(tx, ty, u6, off, &has_neg);
                    mitchell_block_sums((double)tx, (double)ty, &Wp, &Wm);
                }
                int xp = wrap_tap(t->wrap, ix + off[0], wl), yp = wrap_tap(t->wrap, iy + off[1], hl);
                int xn = wrap_tap(t->wrap, ix + off[2], wl), yn = wrap_tap(t->wrap, iy + off[3], hl);
                if (taps) {
                    int32_t *q5 = taps + 5 * s;
                    q5[0] = l;
                    q5[1] = xp;
                    q5[2] = yp;
                    q5[3] = has_neg ? xn : INT32_MIN;
                    q5[4] = has_neg ? yn : INT32_MIN;
                }
                double texel[4], v[4], vn[4];
                fetch2d(t, l, xp, yp, texel);
                shade2d(shade, ggx, texel, v);
                for (int c = 0; c < ch; ++c)
                    acc[c] += Wp * v[c];
                if (has_neg) {
                    fetch2d(t, l, xn, yn, texel);
                    shade2d(shade, ggx, texel, vn);
                    for (int c = 0; c < ch; ++c)
                        acc[c] -= Wm * vn[c];
                }
                continue;
            }
            int ox, oy;
            if (filter == F_GAUSS_FRS) {
                /* discrete Gaussian: running-sum pick per axis on the 4 taps */
                float h = orc_gauss_h(sigma), Cx[3], Cy[3];
                orc_gauss_thresholds(tx, h, Cx);
                orc_gauss_thresholds(ty, h, Cy);
                ox = -1 + (ux >= Cx[0]) + (ux >= Cx[1]) + (ux >= Cx[2]);
                oy = -1 + (uy >= Cy[0]) + (uy >= Cy[1]) + (uy >= Cy[2]);
            } else if (filter == F_GAUSS_FIS) {
                /* Box-Muller offset, then the nearest texel */
                float dx, dy;
                orc_fis_gauss_offset(ux, uy, sigma, &dx, &dy);
                ox = orc_fis_nearest(tx, dx);
                oy = orc_fis_nearest(ty, dy);
            } else if (filter == F_BSPLINE3_FIS) {
                /* three uniforms per axis: words 0, 1, 2 of the key with
                 * step 0 for x, of the key with step 1 for y */
                uint32_t key2[4] = {(uint32_t)qi, (uint32_t)s, 1u, seed}, w2[4];
                orc_pcg4d(key2, w2);
                ox = orc_fis_bspline_pick(tx, w[0], w[1], w[2]);
                oy = orc_fis_bspline_pick(ty, w2[0], w2[1], w2[2]);
            } else {
                int first = filter == F_BSPLINE3 ? -1 : 0;
                int jx = orc_pick(filter, tx, ux);
                if (variant == 1)
                    uy = orc_reuse(filter, tx, ux, jx);
                int jy = orc_pick(filter, ty, uy);
                ox = first + jx;
                oy = first + jy;
            }
            int x = wrap_tap(t->wrap, ix + ox, wl);
            int y = wrap_tap(t->wrap, iy + oy, hl);
            if (taps) {
                taps[3 * s] = l;
                taps[3 * s + 1] = x;
                taps[3 * s + 2] = y;
            }
            double texel[4], v[4];
            fetch2d(t, l, x, y, texel);
            shade2d(shade, ggx, texel, v);
            for (int c = 0; c < ch; ++c)
                acc[c] += v[c];
        }
        for (int c = 0; c < ch; ++c)
            out[c] = acc[c] / (double)spp;
        return;
    }

    /* deterministic: before = shade(sum w*texel), after = sum w*shade(texel) */
    double sum[4] = {0, 0, 0, 0};
    int lv[2] = {l0, l1};
    double pl[2] = {1.0 - (double)f, (double)f};
    for (int li = 0; li < 2; ++li) {
        if (pl[li] == 0.0)
            continue;
        int l = lv[li];
        int wl = lvl_dim(t->w, l), hl = lvl_dim(t->h, l);
        int ix, iy;
        float tx, ty;
        raster(uu, wl, &ix, &tx);
        raster(vv, hl, &iy, &ty);
        double wx[AXIS_TAPS_MAX], wy[AXIS_TAPS_MAX];
        int ox, oy;
        int nx = axis_weights_s(filter, sigma, (double)tx, &ox, wx);
        int ny = axis_weights_s(filter, sigma, (double)ty, &oy, wy);
        for (int b = 0; b < ny; ++b)
            for (int a = 0; a < nx; ++a) {
                double wgt = pl[li] * wx[a] * wy[b];
                double texel[4], v[4];
                fetch2d(t, l, wrap_tap(t->wrap, ix + ox + a, wl), wrap_tap(t->wrap, iy + oy + b, hl), texel);
                if (mode == M_BEFORE) {
                    for (int c = 0; c < 4; ++c)
                        sum[c] += wgt * texel[c];
                } else {
                    shade2d(shade, ggx, texel, v);
                    for (int c = 0; c < ch; ++c)
                        sum[c] += wgt * v[c];
                }
            }
    }
    if (mode == M_BEFORE)
        shade2d(shade, ggx, sum, out);
    else
        for (int c = 0; c < ch; ++c)
            out[c] = sum[c];
}

/* Axis weights of every 2-D filter, including the Gaussians (binary64):
 * the discrete Gaussian's normalised e^(-d^2 h) on taps -1..2, the FIS
 * Gaussian's cell masses on -R..R+1, and the B-spline FIS = the cubic
 * B-spline (the filter it realises). */
static int axis_weights_s(int filter, float sigma, double t, int *first_off, double *w)
{
    if (filter == F_GAUSS_FRS) {
        double h = 0.5 / ((double)sigma * (double)sigma), W = 0.0;
        *first_off = -1;
        for (int k = 0; k < 4; ++k) {
            double d = (double)(k - 1) - t;
            w[k] = exp(-d * d * h);
            W += w[k];
        }
        for (int k = 0; k < 4; ++k)
            w[k] /= W;
        return 4;
    }
    if (filter == F_GAUSS_FIS) {
        int R = gauss_fis_radius(sigma);
        *first_off = -R;
        for (int k = -R; k <= R + 1; ++k)
            w[k + R] = gauss_cell(sigma, t, k);
        return 2 * R + 2;
    }
    return axis_weights(filter == F_BSPLINE3_FIS ? F_BSPLINE3 : filter, t, first_off, w);
}


/* queries: n x {u, v, lambda}.  If subset is non-null only the nsub listed
 * queries are computed (out and taps indexed by position in the subset, the
 * random key by the query's own index). */
ORC_EXPORT int orc_filter2d(const void *base, int w, int h, int levels, int fmt, int wrap, int mip,
                            const int64_t *level_off, const float *dct_range, const float *q, int64_t n,
                            int filter, int mode,
                            int spp, uint32_t seed, int variant, float sigma, int shade, const double *ggx,
                            double *out, int32_t *taps, const int64_t *subset, int64_t nsub)
{
    tex2d t = {(const uint8_t *)base, w, h, levels, fmt, wrap, mip, level_off, dct_range};
    int ch = shade != 0 ? 3 : 4;
    int64_t m = subset ? nsub : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
        int64_t qi = subset ? subset[i] : i;
        int tw = (filter == F_KEYS3 || filter == F_MITCHELL) && mode == M_STOCH ? 5 : 3;
        filter2d_one(&t, q + 3 * qi, qi, filter, mode, spp, seed, variant, sigma, shade, ggx, out + ch * i,
                     taps ? taps + (int64_t)tw * spp * i : NULL);
    }
    return 0;
}

/* Exact expectation of the stochastic estimator with independent 24-bit
 * uniforms per axis and level: sum over every (level, tap x, tap y) of the
 * exact pick probabilities times the shaded texel.  Filters: nearest,
 * linear, cubic B-spline, discrete Gaussian and B-spline FIS (returns -1
 * for the others). */
ORC_EXPORT int orc_filter2d_expect(const void *base, int w, int h, int levels, int fmt, int wrap, int mip,
                                   const int64_t *level_off, const float *dct_range, const float *q, int64_t n,
                                   int filter,
                                   float sigma, int shade, const double *ggx, double *out)
{
    if (filter == F_KEYS3 || filter == F_MITCHELL || filter == F_GAUSS_FIS)
        return -1;
    tex2d t = {(const uint8_t *)base, w, h, levels, fmt, wrap, mip, level_off, dct_range};
    int ch = shade != 0 ? 3 : 4;
    for (int64_t i = 0; i < n; ++i) {
        const float *qq = q + 3 * i;
        double *o = out + ch * i;
        float uu = wrap_coord(t.wrap, qq[0]), vv = wrap_coord(t.wrap, qq[1]);
        int l0, l1;
        float f;
        levels_of(&t, qq[2], &l0, &l1, &f);
        /* level probability: P(u >= 1-f) over the 24-bit lattice */
        double c = ceil((double)(1.0f - f) * 16777216.0);
        double p1 = (16777216.0 - c) / 16777216.0;
        double pl[2] = {1.0 - p1, p1};
        int lv[2] = {l0, l1};
        for (int c2 = 0; c2 < ch; ++c2)
            o[c2] = 0.0;
        for (int li = 0; li < 2; ++li) {
            if (pl[li] == 0.0)
                continue;
            int l = lv[li];
            int wl = lvl_dim(t.w, l), hl = lvl_dim(t.h, l);
            int ix, iy;
            float tx, ty;
            raster(uu, wl, &ix, &tx);
            raster(vv, hl, &iy, &ty);
            double Px[4], Py[4];
            if (filter == F_GAUSS_FRS) {
                orc_gauss_pick_pmf(tx, orc_gauss_h(sigma), Px);
                orc_gauss_pick_pmf(ty, orc_gauss_h(sigma), Py);
            } else if (filter == F_BSPLINE3_FIS) {
                orc_fis_bspline_pmf(tx, Px);
                orc_fis_bspline_pmf(ty, Py);
            } else {
                orc_pick_pmf(filter, tx, Px);
                orc_pick_pmf(filter, ty, Py);
            }
            int cubic = filter == F_BSPLINE3 || filter == F_GAUSS_FRS || filter == F_BSPLINE3_FIS;
            int off = cubic ? -1 : 0;
            int ntap = cubic ? 4 : (filter == F_LINEAR ? 2 : 1);
            int nearx = filter == F_NEAREST ? (tx >= 0.5f) : 0;
            int neary = filter == F_NEAREST ? (ty >= 0.5f) : 0;
            for (int b = 0; b < ntap; ++b)
                for (int a = 0; a < ntap; ++a) {
                    double pr = pl[li] * Px[a] * Py[b];
                    if (pr == 0.0)
                        continue;
                    double texel[4], v[4];
                    fetch2d(&t, l, wrap_tap(t.wrap, ix + off + a + nearx, wl),
                            wrap_tap(t.wrap, iy + off + b + neary, hl), texel);
                    shade2d(shade, ggx, texel, v);
                    for (int c2 = 0; c2 < ch; ++c2)
                        o[c2] += pr * v[c2];
                }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Anisotropic minification by screen-space jitter (Sec. 4.2.1; the level of  */
/* detail of Suppl. S.4.3; Sec. 5 "Anisotropic filtering and minification").  */
/* A query is a pixel: uv and its screen derivatives (du/dx, dv/dx, du/dy,    */
/* dv/dy).  A sample jitters uv uniformly over the pixel's parallelogram      */
/* (first-order image of the pixel square), reads ONE level chosen from the   */
/* minor axis of the footprint with a uniform jitter of the level, and ONE    */
/* texel of it with the reconstruction filter.                                */
/* ------------------------------------------------------------------------ */

/* log2 x for positive normal x (binary32 contract): the same frexp
 * reduction and atanh series as orc_lnc, then e + ln(m) log2(e); -inf for
 * x < 2^-126 or NaN, +inf for +inf. */
ORC_EXPORT float orc_log2c(float x)
{
    if (!(x >= 0x1p-126f))
        return -INFINITY;
    if (x == INFINITY)
        return INFINITY;
    int e;
    float m = frexpf(x, &e);
    if (m < 0.70710678f) {
        m = m * 2.0f;
        e = e - 1;
    }
    float s = (m - 1.0f) / (m + 1.0f);
    float z = s * s;
    float p = fmaf(z, fmaf(z, fmaf(z, fmaf(z, 1.0f / 9.0f, 1.0f / 7.0f), 1.0f / 5.0f), 1.0f / 3.0f), 1.0f);
    float r = (2.0f * s) * p;
    return fmaf(r, 1.44269504f, (float)e);
}

/* Footprint axes of a pixel in level-0 texels: x-axis (W du/dx, H dv/dx),
 * y-axis (W du/dy, H dv/dy).  The shorter is the minor axis; if the
 * anisotropy exceeds amax the minor axis is lengthened to major/amax (the
 * listing's rescaling, in its operation order).  Returns lambda = log2 of
 * the minor length; *major_y tells which derivative is the major axis;
 * *nprobe = the probe count of the deterministic comparator,
 * clamp(ceil(major/minor), 1, amax) (amax when the minor axis vanishes
 * and the major does not). */
ORC_EXPORT float orc_aniso_lod(int W, int H, const float d[4], int amax, int *major_y, int *nprobe)
{
    float ax = (float)W * d[0], ay = (float)H * d[1];
    float bx = (float)W * d[2], by = (float)H * d[3];
    float la2 = ax * ax + ay * ay, lb2 = bx * bx + by * by;
    int swap = la2 > lb2;
    float lmin = sqrtf(swap ? lb2 : la2), lmax = sqrtf(swap ? la2 : lb2);
    *major_y = !swap;
    float A = (float)amax;
    if (lmin > 0.0f && lmin * A < lmax) {
        float scale = lmax / (lmin * A);
        lmin = lmin * scale;
    }
    int np;
    if (lmin > 0.0f) {
        float r = ceilf(lmax / lmin);
        np = r < 1.0f ? 1 : (!(r <= A) ? amax : (int)r);
    } else {
        np = lmax > 0.0f ? amax : 1;
    }
    *nprobe = np;
    return orc_log2c(lmin);
}

/* A query is usable when its six values are finite and so are the extreme
 * jittered coordinates |u| + |du/dx| + |du/dy| (and for v) in binary32. */
static int aniso_query_finite(const float *q)
{
    for (int k = 0; k < 6; ++k)
        if (!isfinite(q[k]))
            return 0;
    float eu = (fabsf(q[0]) + fabsf(q[2])) + fabsf(q[4]);
    float ev = (fabsf(q[1]) + fabsf(q[3])) + fabsf(q[5]);
    return isfinite(eu) && isfinite(ev);
}

/* Deterministic filter of one point at the level pair of lambda
 * (weights 1-f, f), as filter2d's deterministic sums; adds weight * value
 * (texel for before, shaded texel for after) into sum. */
static void det_point(const tex2d *t, float u, float v, float lam, int filter, float sigma, int mode, int shade,
                      const double *ggx, double weight, double *sum)
{
    int ch = shade != 0 ? 3 : 4;
    float uu = wrap_coord(t->wrap, u), vv = wrap_coord(t->wrap, v);
    int l0, l1;
    float f;
    levels_of(t, lam, &l0, &l1, &f);
    int lv[2] = {l0, l1};
    double pl[2] = {1.0 - (double)f, (double)f};
    for (int li = 0; li < 2; ++li) {
        if (pl[li] == 0.0)
            continue;
        int l = lv[li];
        int wl = lvl_dim(t->w, l), hl = lvl_dim(t->h, l);
        int ix, iy;
        float tx, ty;
        raster(uu, wl, &ix, &tx);
        raster(vv, hl, &iy, &ty);
        double wx[AXIS_TAPS_MAX], wy[AXIS_TAPS_MAX];
        int ox, oy;
        int nx = axis_weights_s(filter, sigma, (double)tx, &ox, wx);
        int ny = axis_weights_s(filter, sigma, (double)ty, &oy, wy);
        for (int b = 0; b < ny; ++b)
            for (int a = 0; a < nx; ++a) {
                double wgt = weight * pl[li] * wx[a] * wy[b];
                double texel[4], val[4];
                fetch2d(t, l, wrap_tap(t->wrap, ix + ox + a, wl), wrap_tap(t->wrap, iy + oy + b, hl), texel);
                if (mode == M_BEFORE) {
                    for (int c = 0; c < 4; ++c)
                        sum[c] += wgt * texel[c];
                } else {
                    shade2d(shade, ggx, texel, val);
                    for (int c = 0; c < ch; ++c)
                        sum[c] += wgt * val[c];
                }
            }
    }
}

/* One pixel.  Stochastic: per sample, key (q, s, 0, seed) gives the jitter
 * (words 0, 1: j = u - 1/2 along du/dx and du/dy) and the level uniform
 * (word 2); key (q, s, 1, seed) gives the filter's uniforms (words 0, 1).
 *   uv' = uv + jx d/dx + jy d/dy  (two fused operations per coordinate),
 *   level = floor(clamp(lambda + (u_l - 1/2), 0, L-1) + 1/2),
 *   then one texel of that level by the filter's pick at uv'.
 * Deterministic (the comparators): N probes at offsets (k + 1/2)/N - 1/2
 * of the major-axis derivative, each filtered on the levels floor(lambda),
 * floor(lambda)+1 with weights (1-f, f); mean over probes; before shades
 * the filtered texel, after sums shaded texels. */
static void aniso_one(const tex2d *t, const float *q, int64_t qi, int filter, int mode, int spp, uint32_t seed,
                      float sigma, int amax, int shade, const double *ggx, double *out, int32_t *taps)
{
    int ch = shade != 0 ? 3 : 4;
    if (!aniso_query_finite(q)) {
        for (int c = 0; c < ch; ++c)
            out[c] = NAN;
        if (taps && (mode == M_STOCH || mode == M_SPLIT))
            for (int s = 0; s < 3 * spp; ++s)
                taps[s] = INT32_MIN;
        return;
    }
    int major_y, np;
    float lam = orc_aniso_lod(t->w, t->h, q + 2, amax, &major_y, &np);
    const float lmax = (float)(t->levels - 1);
    if (mode == M_SPLIT) {
        /* split filtering: the low-pass filter (jitter over the pixel and the
         * jittered level, key words 0, 1, 2 as the stochastic mode) sampled,
         * the reconstruction filter evaluated before shading */
        double acc[4] = {0, 0, 0, 0};
        for (int s = 0; s < spp; ++s) {
            uint32_t k0[4] = {(uint32_t)qi, (uint32_t)s, 0u, seed}, w0[4];
            orc_pcg4d(k0, w0);
            float jx = uniform24(w0[0]) - 0.5f, jy = uniform24(w0[1]) - 0.5f;
            float u = fmaf(jy, q[4], fmaf(jx, q[2], q[0]));
            float v = fmaf(jy, q[5], fmaf(jx, q[3], q[1]));
            float lj = lam + (uniform24(w0[2]) - 0.5f);
            lj = fminf(fmaxf(lj, 0.0f), lmax);
            int l = (int)floorf(lj + 0.5f);
            if (taps) {
                taps[3 * s] = l;
                taps[3 * s + 1] = taps[3 * s + 2] = INT32_MIN;
            }
            double rgba[4], val[4];
            recon_level(t, wrap_coord(t->wrap, u), wrap_coord(t->wrap, v), l, filter, sigma, rgba);
            shade2d(shade, ggx, rgba, val);
            for (int c = 0; c < ch; ++c)
                acc[c] += val[c];
        }
        for (int c = 0; c < ch; ++c)
            out[c] = acc[c] / (double)spp;
        return;
    }
    if (mode == M_STOCH) {
        double acc[4] = {0, 0, 0, 0};
        for (int s = 0; s < spp; ++s) {
            uint32_t k0[4] = {(uint32_t)qi, (uint32_t)s, 0u, seed}, w0[4];
            uint32_t k1[4] = {(uint32_t)qi, (uint32_t)s, 1u, seed}, w1[4];
            orc_pcg4d(k0, w0);
            orc_pcg4d(k1, w1);
            float jx = uniform24(w0[0]) - 0.5f, jy = uniform24(w0[1]) - 0.5f;
            float u = fmaf(jy, q[4], fmaf(jx, q[2], q[0]));
            float v = fmaf(jy, q[5], fmaf(jx, q[3], q[1]));
            float lj = lam + (uniform24(w0[2]) - 0.5f);
            lj = fminf(fmaxf(lj, 0.0f), lmax);
            int l = (int)floorf(lj + 0.5f);
            int wl = lvl_dim(t->w, l), hl = lvl_dim(t->h, l);
            int ix, iy;
            float tx, ty;
            raster(wrap_coord(t->wrap, u), wl, &ix, &tx);
            raster(wrap_coord(t->wrap, v), hl, &iy, &ty);
            float ux = uniform24(w1[0]), uy = uniform24(w1[1]);
            int ox, oy;
            if (filter == F_GAUSS_FIS) {
                float dx, dy;
                orc_fis_gauss_offset(ux, uy, sigma, &dx, &dy);
                ox = orc_fis_nearest(tx, dx);
                oy = orc_fis_nearest(ty, dy);
            } else {
                int first = filter == F_BSPLINE3 ? -1 : 0;
                ox = first + orc_pick(filter, tx, ux);
                oy = first + orc_pick(filter, ty, uy);
            }
            int x = wrap_tap(t->wrap, ix + ox, wl), y = wrap_tap(t->wrap, iy + oy, hl);
            if (taps) {
                taps[3 * s] = l;
                taps[3 * s + 1] = x;
                taps[3 * s + 2] = y;
            }
            double texel[4], val[4];
            fetch2d(t, l, x, y, texel);
            shade2d(shade, ggx, texel, val);
            for (int c = 0; c < ch; ++c)
                acc[c] += val[c];
        }
        for (int c = 0; c < ch; ++c)
            out[c] = acc[c] / (double)spp;
        return;
    }
    double sum[4] = {0, 0, 0, 0};
    float mu = major_y ? q[4] : q[2], mv = major_y ? q[5] : q[3];
    for (int k = 0; k < np; ++k) {
        float o = ((float)k + 0.5f) / (float)np - 0.5f;
        float u = fmaf(o, mu, q[0]), v = fmaf(o, mv, q[1]);
        det_point(t, u, v, lam, filter, sigma, mode, shade, ggx, 1.0 / (double)np, sum);
    }
    if (mode == M_BEFORE)
        shade2d(shade, ggx, sum, out);
    else
        for (int c = 0; c < ch; ++c)
            out[c] = sum[c];
}

/* ------------------------------------------------------------------------ */
/* Elliptically weighted average (EWA) and its stochastic form (Sec. 4.1: a  */
/* MIP level chosen from the ellipse's extent, then all EWA weights are      */
/* computed and one texel is drawn from their distribution).                 */
/*                                                                          */
/* The ellipse (Greene and Heckbert's EWA): the footprint Jacobian J maps    */
/* the pixel's unit circle to texture space, so the footprint is the         */
/* ellipse of covariance S = J J^T; adding the unit covariance of one texel  */
/* (reconstruction) gives V = S + I, and a texel at offset d from the lookup */
/* point has radius r^2 = d^T V^-1 d and weight e^(-2 r^2) - e^(-2) inside   */
/* r^2 < 1 (a Gaussian truncated to the ellipse).                            */
/* Level of detail: from the singular values s1 >= s2 of J in level-0        */
/* texels (the ellipse's semi-axes): the minor axis is lengthened to         */
/* s1/amax when s2 amax < s1, by adding (s1^2/amax^2 - s2^2) times the       */
/* projector on the minor eigenvector, (s1^2 I - S)/(s1^2 - s2^2), to S;     */
/* lod = max(0, log2(minor)) (a zero footprint has lod 0).  A footprint     */
/* wider than the texture (lod > L-1) reads the last (1 x 1) level.          */
/* Sampling (Sec. 2.2, "Sampling arrays"): the weights of the cells of the   */
/* ellipse's bounding box are summed in scan order (rows t, then columns s), */
/* and the sample takes the first cell whose running sum exceeds u W; the    */
/* box's half-extents are sqrt(V_ss) and sqrt(V_tt), the ellipse's support   */
/* along s and t.  Comparators: the EWA sums on levels floor(lod),           */
/* floor(lod)+1 (weights 1-f, f), each normalised by its weight total.       */
/* Binary32 decisions in the order written here, without contraction (the    */
/* GPU follows the same sequence); the Gaussian uses the contract exp.       */
/* ------------------------------------------------------------------------ */
typedef struct {
    float lod;
    float vss, vtt, vst, det; /* S after the anisotropy limit (level-0 texels^2), det S */
} ewa_frame;

static ewa_frame ewa_setup(const float *q, int w, int h, int amax)
{
    ewa_frame e;
    /* J: columns d(s,t)/dx and d(s,t)/dy in level-0 texels */
    const float jsx = (float)w * q[2], jtx = (float)h * q[3];
    const float jsy = (float)w * q[4], jty = (float)h * q[5];
    const float m = fmaxf(fmaxf(fabsf(jsx), fabsf(jtx)), fmaxf(fabsf(jsy), fabsf(jty)));
    if (!(m < 0x1p40f)) {
        /* s1 >= m, so the minor axis is at least 2^40/amax texels: beyond the
         * last level of any pyramid (at most 2^15 texels wide) */
        e.lod = INFINITY;
        e.vss = e.vtt = e.vst = e.det = 0.0f;
        return e;
    }
    float vss = jsx * jsx + jsy * jsy;
    float vtt = jtx * jtx + jty * jty;
    float vst = jsx * jtx + jsy * jty;
    const float dj = jsx * jty - jtx * jsy;
    float det = dj * dj;
    const float half = (vss - vtt) * 0.5f, mean = (vss + vtt) * 0.5f;
    const float lp = mean + sqrtf(half * half + vst * vst); /* larger eigenvalue of S */
    const float s1 = sqrtf(lp);
    float minor = lp > 0.0f ? fabsf(dj) / s1 : 0.0f;
    if (minor * (float)amax < s1) {
        const float lm = det / lp; /* smaller eigenvalue */
        minor = s1 / (float)amax;
        const float k = lp > lm ? (minor * minor - lm) / (lp - lm) : 1.0f;
        vss = vss + k * (lp - vss);
        vtt = vtt + k * (lp - vtt);
        vst = vst - k * vst;
        det = lp * (minor * minor);
    }
    e.vss = vss, e.vtt = vtt, e.vst = vst, e.det = det;
    e.lod = minor > 0.0f ? fmaxf(0.0f, orc_log2c(minor)) : 0.0f;
    return e;
}

ORC_EXPORT float orc_ewa_lod(const float *q, int w, int h, int amax)
{
    return ewa_setup(q, w, h, amax).lod;
}

typedef struct {
    float s, t;            /* lookup point in the level's raster coordinates */
    float qss, qtt, q2st;  /* V^-1 (its off-diagonal doubled) */
    int s0, s1, t0, t1;    /* bounding box of the ellipse */
} ewa_level;

static ewa_level ewa_at(const tex2d *tx, const float *q, const ewa_frame *e, int l)
{
    ewa_level v;
    const int wl = lvl_dim(tx->w, l), hl = lvl_dim(tx->h, l);
    const float fs = (float)wl / (float)tx->w, ft = (float)hl / (float)tx->h;
    const float lss = e->vss * (fs * fs), ltt = e->vtt * (ft * ft), lst = e->vst * (fs * ft);
    const float ldet = e->det * ((fs * fs) * (ft * ft));
    const float a = lss + 1.0f, c = ltt + 1.0f;          /* V = S_l + I */
    const float D = ((ldet + lss) + ltt) + 1.0f;          /* det V, a sum of non-negative terms */
    v.qss = c / D;
    v.qtt = a / D;
    v.q2st = -(2.0f * lst) / D;
    const float ex = sqrtf(a), ey = sqrtf(c);
    v.s = wrap_coord(tx->wrap, q[0]) * (float)wl - 0.5f;
    v.t = wrap_coord(tx->wrap, q[1]) * (float)hl - 0.5f;
    v.s0 = (int)ceilf(v.s - ex);
    v.s1 = (int)floorf(v.s + ex);
    v.t0 = (int)ceilf(v.t - ey);
    v.t1 = (int)floorf(v.t + ey);
    return v;
}

/* The truncated Gaussian of the ellipse radius; 0 outside (r^2 >= 1). */
static float ewa_gauss(float r2)
{
    if (!(r2 < 1.0f))
        return 0.0f;
    return orc_expc(-2.0f * r2) - orc_expc(-2.0f);
}

ORC_EXPORT float orc_ewa_gauss(float r2)
{
    return ewa_gauss(r2);
}

static float ewa_weight(const ewa_level *v, int is, int it)
{
    const float ds = (float)is - v->s, dt = (float)it - v->t;
    const float r2 = (v->qss * (ds * ds) + v->qtt * (dt * dt)) + v->q2st * (ds * dt);
    return ewa_gauss(r2);
}

/* One texel by inverse CDF over the positive weights in scan order; returns
 * 0 when no weight is positive (the sample then reads nothing). */
static int ewa_pick(const ewa_level *v, float u, int *px, int *py)
{
    float W = 0.0f;
    for (int it = v->t0; it <= v->t1; ++it)
        for (int is = v->s0; is <= v->s1; ++is) {
            const float w = ewa_weight(v, is, it);
            if (w > 0.0f)
                W = W + w;
        }
    if (!(W > 0.0f))
        return 0;
    const float thr = u * W;
    float S = 0.0f;
    for (int it = v->t0; it <= v->t1; ++it)
        for (int is = v->s0; is <= v->s1; ++is) {
            const float w = ewa_weight(v, is, it);
            if (!(w > 0.0f))
                continue;
            S = S + w;
            *px = is, *py = it; /* the last positive cell if u W rounds up to W */
            if (S > thr)
                return 1;
        }
    return 1;
}

static void ewa_one(const tex2d *tx, const float *q, int64_t qi, int mode, int spp, uint32_t seed, int amax,
                    int shade, const double *ggx, double *out, int32_t *taps)
{
    int ch = shade != 0 ? 3 : 4;
    ewa_frame e = ewa_setup(q, tx->w, tx->h, amax);
    const float lmax = (float)(tx->levels - 1);
    if (e.lod > lmax) {
        /* a footprint wider than the whole texture reads the one texel of the
         * coarsest level */
        double texel[4], val[4];
        fetch2d(tx, tx->levels - 1, 0, 0, texel);
        shade2d(shade, ggx, texel, val);
        for (int c = 0; c < ch; ++c)
            out[c] = val[c];
        if (taps && mode == M_STOCH)
            for (int s = 0; s < spp; ++s) {
                taps[3 * s] = tx->levels - 1;
                taps[3 * s + 1] = taps[3 * s + 2] = 0;
            }
        return;
    }
    const float fl = floorf(e.lod);
    if (mode == M_STOCH) {
        double acc[4] = {0, 0, 0, 0};
        for (int s = 0; s < spp; ++s) {
            uint32_t key[4] = {(uint32_t)qi, (uint32_t)s, 0u, seed}, w[4];
            orc_pcg4d(key, w);
            int l = (int)fl + (uniform24(w[3]) >= 1.0f - (e.lod - fl) ? 1 : 0);
            if (l > tx->levels - 1)
                l = tx->levels - 1;
            ewa_level v = ewa_at(tx, q, &e, l);
            int x = 0, y = 0;
            int found = ewa_pick(&v, uniform24(w[0]), &x, &y);
            int wl = lvl_dim(tx->w, l), hl = lvl_dim(tx->h, l);
            if (taps) {
                taps[3 * s] = found ? l : INT32_MIN;
                taps[3 * s + 1] = found ? wrap_tap(tx->wrap, x, wl) : INT32_MIN;
                taps[3 * s + 2] = found ? wrap_tap(tx->wrap, y, hl) : INT32_MIN;
            }
            if (!found)
                continue;
            double texel[4], val[4];
            fetch2d(tx, l, wrap_tap(tx->wrap, x, wl), wrap_tap(tx->wrap, y, hl), texel);
            shade2d(shade, ggx, texel, val);
            for (int c = 0; c < ch; ++c)
                acc[c] += val[c];
        }
        for (int c = 0; c < ch; ++c)
            out[c] = acc[c] / (double)spp;
        return;
    }
    double sum[4] = {0, 0, 0, 0};
    int lv[2] = {(int)fl, (int)fl + 1 > tx->levels - 1 ? tx->levels - 1 : (int)fl + 1};
    double pl[2] = {1.0 - (double)(e.lod - fl), (double)(e.lod - fl)};
    for (int li = 0; li < 2; ++li) {
        if (pl[li] == 0.0)
            continue;
        ewa_level v = ewa_at(tx, q, &e, lv[li]);
        int wl = lvl_dim(tx->w, lv[li]), hl = lvl_dim(tx->h, lv[li]);
        double part[4] = {0, 0, 0, 0}, W = 0.0;
        for (int it = v.t0; it <= v.t1; ++it)
            for (int is = v.s0; is <= v.s1; ++is) {
                const float w = ewa_weight(&v, is, it);
                if (!(w > 0.0f))
                    continue;
                double texel[4], val[4];
                fetch2d(tx, lv[li], wrap_tap(tx->wrap, is, wl), wrap_tap(tx->wrap, it, hl), texel);
                W += (double)w;
                if (mode == M_BEFORE) {
                    for (int c = 0; c < 4; ++c)
                        part[c] += (double)w * texel[c];
                } else {
                    shade2d(shade, ggx, texel, val);
                    for (int c = 0; c < ch; ++c)
                        part[c] += (double)w * val[c];
                }
            }
        for (int c = 0; c < 4; ++c)
            sum[c] += W > 0.0 ? pl[li] * part[c] / W : 0.0;
    }
    if (mode == M_BEFORE)
        shade2d(shade, ggx, sum, out);
    else
        for (int c = 0; c < ch; ++c)
            out[c] = sum[c];
}

/* Exact pick probabilities at one level, by running the pick on all 2^24
 * uniforms; P[(it - t0) * nx + (is - s0)]. */
ORC_EXPORT int orc_ewa_pick_pmf(int w, int h, int levels, int wrap, const float *q, int amax, int level, double *P,
                                int maxcells, int32_t *box)
{
    const int64_t off0 = 0;
    tex2d tx = {NULL, w, h, levels, FMT_RGBA32F, wrap, MIP_LINEAR, &off0, NULL};
    ewa_frame e = ewa_setup(q, w, h, amax);
    ewa_level v = ewa_at(&tx, q, &e, level);
    int nx = v.s1 - v.s0 + 1, ny = v.t1 - v.t0 + 1;
    box[0] = v.s0, box[1] = v.s1, box[2] = v.t0, box[3] = v.t1;
    if (nx * ny > maxcells || nx <= 0 || ny <= 0)
        return -1;
    int64_t *cnt = (int64_t *)calloc((size_t)nx * ny, sizeof(int64_t));
#pragma omp parallel
    {
        int64_t *loc = (int64_t *)calloc((size_t)nx * ny, sizeof(int64_t));
#pragma omp for schedule(static)
        for (int64_t k = 0; k < (1 << 24); ++k) {
            int x, y;
            if (ewa_pick(&v, (float)k * 0x1p-24f, &x, &y))
                loc[(y - v.t0) * nx + (x - v.s0)]++;
        }
#pragma omp critical
        for (int i = 0; i < nx * ny; ++i)
            cnt[i] += loc[i];
        free(loc);
    }
    for (int i = 0; i < nx * ny; ++i)
        P[i] = (double)cnt[i] / 16777216.0;
    free(cnt);
    return nx * ny;
}

/* The ellipse's bounding box (s0, s1, t0, t1) at one level. */
ORC_EXPORT void orc_ewa_box(int w, int h, int levels, const float *q, int amax, int level, int32_t *box)
{
    const int64_t off0 = 0;
    tex2d tx = {NULL, w, h, levels, FMT_RGBA32F, WRAP_REPEAT, MIP_LINEAR, &off0, NULL};
    ewa_frame e = ewa_setup(q, w, h, amax);
    ewa_level v = ewa_at(&tx, q, &e, level);
    box[0] = v.s0, box[1] = v.s1, box[2] = v.t0, box[3] = v.t1;
}

/* The normalised EWA weights at one level on the same box (binary64 of the
 * binary32 weights). */
ORC_EXPORT int orc_ewa_weights(int w, int h, int levels, int wrap, const float *q, int amax, int level, double *P,
                               int maxcells)
{
    const int64_t off0 = 0;
    tex2d tx = {NULL, w, h, levels, FMT_RGBA32F, wrap, MIP_LINEAR, &off0, NULL};
    ewa_frame e = ewa_setup(q, w, h, amax);
    ewa_level v = ewa_at(&tx, q, &e, level);
    int nx = v.s1 - v.s0 + 1, ny = v.t1 - v.t0 + 1;
    if (nx * ny > maxcells || nx <= 0 || ny <= 0)
        return -1;
    double W = 0.0;
    for (int it = v.t0; it <= v.t1; ++it)
        for (int is = v.s0; is <= v.s1; ++is) {
            const float wt = ewa_weight(&v, is, it);
            const double x = wt > 0.0f ? (double)wt : 0.0;
            P[(it - v.t0) * nx + (is - v.s0)] = x;
            W += x;
        }
    for (int i = 0; i < nx * ny; ++i)
        P[i] /= W;
    return nx * ny;
}

/* The level-0 footprint frame after the anisotropy limit:
 * {lod, S_ss, S_tt, S_st, det S}. */
ORC_EXPORT void orc_ewa_frame(const float *q, int w, int h, int amax, float *out5)
{
    ewa_frame e = ewa_setup(q, w, h, amax);
    out5[0] = e.lod, out5[1] = e.vss, out5[2] = e.vtt, out5[3] = e.vst, out5[4] = e.det;
}

/* queries: n x {u, v, du/dx, dv/dx, du/dy, dv/dy}; the texture's mip field
 * is ignored (the level comes from the footprint). */
ORC_EXPORT int orc_filter2d_aniso(const void *base, int w, int h, int levels, int fmt, int wrap,
                                  const int64_t *level_off, const float *dct_range, const float *q, int64_t n,
                                  int filter, int mode, int spp,
                                  uint32_t seed, float sigma, int amax, int shade, const double *ggx, double *out,
                                  int32_t *taps, const int64_t *subset, int64_t nsub)
{
    tex2d t = {(const uint8_t *)base, w, h, levels, fmt, wrap, MIP_LINEAR, level_off, dct_range};
    int ch = shade != 0 ? 3 : 4;
    int64_t m = subset ? nsub : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
        int64_t qi = subset ? subset[i] : i;
        const float *qq = q + 6 * qi;
        int32_t *tp = taps ? taps + (int64_t)3 * spp * i : NULL;
        if (filter == F_EWA && aniso_query_finite(qq))
            ewa_one(&t, qq, qi, mode, spp, seed, amax, shade, ggx, out + ch * i, tp);
        else
            aniso_one(&t, qq, qi, filter, mode, spp, seed, sigma, amax, shade, ggx, out + ch * i, tp);
    }
    return 0;
}

/* Pixel-integral reference: the mean over K x K stratum centres of the pixel
 * (offsets (i + 1/2)/K - 1/2 along d/dx and d/dy) of the exact
 * filter-after value on level 0 alone (no prefiltered level), i.e. filtering
 * after shading over the whole pixel footprint. */
ORC_EXPORT int orc_aniso_reference(const void *base, int w, int h, int fmt, int wrap, const float *dct_range,
                                   const float *q, int64_t n,
                                   int K, int filter, float sigma, int shade, const double *ggx, double *out,
                                   const int64_t *subset, int64_t nsub)
{
    const int64_t off0 = 0;
    tex2d t = {(const uint8_t *)base, w, h, 1, fmt, wrap, MIP_NONE, &off0, dct_range};
    int ch = shade != 0 ? 3 : 4;
    int64_t m = subset ? nsub : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        const float *qq = q + 6 * (subset ? subset[i] : i);
        double *o = out + ch * i;
        if (!aniso_query_finite(qq)) {
            for (int c = 0; c < ch; ++c)
                o[c] = NAN;
            continue;
        }
        double sum[4] = {0, 0, 0, 0};
        for (int a = 0; a < K; ++a)
            for (int b = 0; b < K; ++b) {
                double jx = ((double)a + 0.5) / K - 0.5, jy = ((double)b + 0.5) / K - 0.5;
                float u = (float)((double)qq[0] + jx * qq[2] + jy * qq[4]);
                float v = (float)((double)qq[1] + jx * qq[3] + jy * qq[5]);
                det_point(&t, u, v, 0.0f, filter, sigma, M_AFTER, shade, ggx, 1.0 / ((double)K * K), sum);
            }
        for (int c = 0; c < ch; ++c)
            o[c] = sum[c];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Triplanar mapping (Sec. 5 "Triplanar mapping").  A surface point p with   */
/* unit normal n is textured from three planar projections, uv = (p.y, p.z), */
/* (p.x, p.z), (p.x, p.y) times the texture scale, blended with weights      */
/* b_i = n_i^4 / sum_j n_j^4 (reading: the usual sharpness 4; the paper does */
/* not fix the blend).  The blend is a weighted mean of three filtered       */
/* values, so one plane picked with probability b_i estimates it             */
/* (eq. stochastic-sum).  Binary32 decision contract: a_i = n_i n_i,         */
/* w_i = a_i a_i, W = (w0 + w1) + w2, plane = [u >= w0/W] + [u >= (w0+w1)/W] */
/* with u = word 2 of the sample's key; words 0, 1 and 3 drive the filter's  */
/* x and y picks and the MIP level pick as in filter2d.                      */
/* ------------------------------------------------------------------------ */
static void tri_weights32(const float *nrm, float w[3], float *W)
{
    for (int i = 0; i < 3; ++i) {
        float a = nrm[i] * nrm[i];
        w[i] = a * a;
    }
    *W = (w[0] + w[1]) + w[2];
}

ORC_EXPORT int orc_tri_pick(const float nrm[3], float u)
{
    float w[3], W;
    tri_weights32(nrm, w, &W);
    return (u >= w[0] / W) + (u >= (w[0] + w[1]) / W);
}

static void tri_uv(const float *p, int plane, float scale, float *u, float *v)
{
    const float a = plane == 0 ? p[1] : p[0];
    const float b = plane == 2 ? p[1] : p[2];
    *u = a * scale;
    *v = b * scale;
}

/* One stochastic single-texel lookup at (u, v, lambda) with uniforms
 * (ux, uy, ul): level pick, raster, per-axis pick, fetch, shade. */
static void stoch_point(const tex2d *t, float u, float v, float lam, int filter, float ux, float uy, float ul,
                        int shade, const double *ggx, double *val, int32_t *tap3)
{
    float uu = wrap_coord(t->wrap, u), vv = wrap_coord(t->wrap, v);
    int l0, l1;
    float f;
    levels_of(t, lam, &l0, &l1, &f);
    int l = (ul >= 1.0f - f) ? l1 : l0;
    int wl = lvl_dim(t->w, l), hl = lvl_dim(t->h, l);
    int ix, iy;
    float tx, ty;
    raster(uu, wl, &ix, &tx);
    raster(vv, hl, &iy, &ty);
    int first = filter == F_BSPLINE3 ? -1 : 0;
    int x = wrap_tap(t->wrap, ix + first + orc_pick(filter, tx, ux), wl);
    int y = wrap_tap(t->wrap, iy + first + orc_pick(filter, ty, uy), hl);
    if (tap3) {
        tap3[0] = l;
        tap3[1] = x;
        tap3[2] = y;
    }
    double texel[4];
    fetch2d(t, l, x, y, texel);
    shade2d(shade, ggx, texel, val);
}

/* queries: n x {p.x, p.y, p.z, n.x, n.y, n.z, lambda, unused}.
 * plane_mode 0 blends the three planes (weights b in binary64), 1 picks one
 * plane per sample.  Filter modes: stochastic (per sample, one texel per
 * plane used), before (shade the blend of the filtered texels), after
 * (blend of filtered shaded texels).  With plane_mode 1 and a deterministic
 * filter the result is the mean over spp samples of the picked plane's
 * deterministic value.  taps (plane_mode 1 only): n x spp x {plane, level,
 * x, y}, the last three TAP_NONE for a deterministic filter. */
ORC_EXPORT int orc_triplanar(const void *base, int w, int h, int levels, int fmt, int wrap, int mip,
                             const int64_t *level_off, const float *dct_range, const float *q, int64_t n,
                             float scale, int plane_mode, int filter, int mode, int spp, uint32_t seed, int shade,
                             const double *ggx, double *out, int32_t *taps, const int64_t *subset, int64_t nsub)
{
    tex2d t = {(const uint8_t *)base, w, h, levels, fmt, wrap, mip, level_off, dct_range};
    int ch = shade != 0 ? 3 : 4;
    int64_t m = subset ? nsub : n;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < m; ++i) {
        int64_t qi = subset ? subset[i] : i;
        const float *qq = q + 8 * qi;
        double *o = out + ch * i;
        int32_t *tp = taps ? taps + (int64_t)4 * spp * i : NULL;
        int finite = 1;
        for (int k = 0; k < 7; ++k)
            finite &= isfinite(qq[k]) != 0;
        for (int k = 0; k < 3; ++k)
            finite &= isfinite(qq[k] * scale) != 0;     /* projected coordinates */
        if (!finite) {
            for (int c = 0; c < ch; ++c)
                o[c] = NAN;
            if (tp)
                for (int k = 0; k < 4 * spp; ++k)
                    tp[k] = INT32_MIN;
            continue;
        }
        double b[3], B = 0.0;
        for (int k = 0; k < 3; ++k) {
            double a = (double)qq[3 + k] * (double)qq[3 + k];
            b[k] = a * a;
            B += b[k];
        }
        for (int k = 0; k < 3; ++k)
            b[k] /= B;
        double acc[4] = {0, 0, 0, 0};
        if (plane_mode == 0 && mode != M_STOCH) {
            for (int j = 0; j < 3; ++j) {
                float u, v;
                tri_uv(qq, j, scale, &u, &v);
                det_point(&t, u, v, qq[6], filter, 0.5f, mode, shade, ggx, b[j], acc);
            }
            if (mode == M_BEFORE)
                shade2d(shade, ggx, acc, o);
            else
                for (int c = 0; c < ch; ++c)
                    o[c] = acc[c];
            continue;
        }
        for (int s = 0; s < spp; ++s) {
            uint32_t key[4] = {(uint32_t)qi, (uint32_t)s, 0u, seed}, wd[4];
            orc_pcg4d(key, wd);
            float ux = uniform24(wd[0]), uy = uniform24(wd[1]), up = uniform24(wd[2]), ul = uniform24(wd[3]);
            if (plane_mode == 0) {
                for (int j = 0; j < 3; ++j) {
                    float u, v;
                    double val[4];
                    tri_uv(qq, j, scale, &u, &v);
                    stoch_point(&t, u, v, qq[6], filter, ux, uy, ul, shade, ggx, val, NULL);
                    for (int c = 0; c < ch; ++c)
                        acc[c] += b[j] * val[c];
                }
                continue;
            }
            int j = orc_tri_pick(qq + 3, up);
            float u, v;
            tri_uv(qq, j, scale, &u, &v);
            if (tp)
                tp[4 * s] = j;
            if (mode == M_STOCH) {
                double val[4];
                stoch_point(&t, u, v, qq[6], filter, ux, uy, ul, shade, ggx, val, tp ? tp + 4 * s + 1 : NULL);
                for (int c = 0; c < ch; ++c)
                    acc[c] += val[c];
            } else {
                double sum[4] = {0, 0, 0, 0}, val[4];
                det_point(&t, u, v, qq[6], filter, 0.5f, mode, shade, ggx, 1.0, sum);
                if (mode == M_BEFORE)
                    shade2d(shade, ggx, sum, val);
                for (int c = 0; c < ch; ++c)
                    acc[c] += mode == M_BEFORE ? val[c] : sum[c];
                if (tp)
                    tp[4 * s + 1] = tp[4 * s + 2] = tp[4 * s + 3] = INT32_MIN;
            }
        }
        for (int c = 0; c < ch; ++c)
            o[c] = acc[c] / (double)spp;
    }
    return 0;
}

/* Fraction of the 2^24 uniforms u with u*P < p in binary32 (brute force). */
static double frac_lt(float P, float p)
{
    int64_t c = 0;
    for (uint32_t k = 0; k < (1u << 24); ++k)
        c += ((float)k * 0x1p-24f) * P < p;
    return (double)c / 16777216.0;
}

/* Exact expectation of the positivised Keys estimator (level 0, shade as in
 * filter2d) over the 24-bit uniforms: every decision's probability counted
 * by brute force, the block sums in binary64. */
ORC_EXPORT int orc_keys_expect2d(const void *base, int w, int h, int fmt, int wrap, const float *q, int64_t n,
                                 int shade, const double *ggx, double *out)
{
    const int64_t off0 = 0;
    tex2d t = {(const uint8_t *)base, w, h, 1, fmt, wrap, MIP_NONE, &off0};
    int ch = shade != 0 ? 3 : 4;
    for (int64_t i = 0; i < n; ++i) {
        float uu = wrap_coord(wrap, q[3 * i]), vv = wrap_coord(wrap, q[3 * i + 1]);
        int ix, iy;
        float tx, ty;
        raster(uu, w, &ix, &tx);
        raster(vv, h, &iy, &ty);
        keys_axis kx = keys_axis_of(tx), ky = keys_axis_of(ty);
        double Wp, Wm;
        keys_block_sums((double)tx, (double)ty, &Wp, &Wm);
        /* per-axis pair probabilities: P(first tap | positive pair), P(first | negative pair) */
        double pxp = frac_lt(kx.Pp, kx.p1), pxm = frac_lt(kx.Pm, kx.m0);
        double pyp = frac_lt(ky.Pp, ky.p1), pym = frac_lt(ky.Pm, ky.m0);
        float A = kx.Pp * ky.Pp, B = kx.Pm * ky.Pm, Cn = kx.Pp * ky.Pm, Dn = kx.Pm * ky.Pp;
        double pblk = frac_lt(A + B, A), nblk = (Cn + Dn) > 0.0f ? frac_lt(Cn + Dn, Cn) : 0.0;
        double PX[2][4] = {{0, pxp, 1 - pxp, 0}, {pxm, 0, 0, 1 - pxm}}; /* [pos/neg pair][tap] */
        double PY[2][4] = {{0, pyp, 1 - pyp, 0}, {pym, 0, 0, 1 - pym}};
        double acc[4] = {0, 0, 0, 0};
        for (int b = 0; b < 4; ++b)
            for (int a = 0; a < 4; ++a) {
                double texel[4], v[4];
                fetch2d(&t, 0, wrap_tap(wrap, ix - 1 + a, w), wrap_tap(wrap, iy - 1 + b, h), texel);
                shade2d(shade, ggx, texel, v);
                double ppos = pblk * PX[0][a] * PY[0][b] + (1 - pblk) * PX[1][a] * PY[1][b];
                double pneg = nblk * PX[0][a] * PY[1][b] + (1 - nblk) * PX[1][a] * PY[0][b];
                for (int c = 0; c < ch; ++c)
                    acc[c] += Wp * ppos * v[c] - ((Cn + Dn) > 0.0f ? Wm * pneg * v[c] : 0.0);
            }
        for (int c = 0; c < ch; ++c)
            out[ch * i + c] = acc[c];
    }
    return 0;
}

/* Per-tap probabilities of pn_pick on the positive (row 0) and negative
 * (row 1) set of one axis over the 24-bit lattice. */
static void pn_probs(const pn_axis *a, double P[2][4])
{
    for (int r = 0; r < 2; ++r) {
        const float Ps = r == 0 ? a->Pp : a->Pm;
        float c = 0.0f;
        double prev = 0.0;
        int last = -1;
        for (int k = 0; k < 4; ++k) {
            P[r][k] = 0.0;
            float m = r == 0 ? a->w[k] : -a->w[k];
            if (!(m > 0.0f))
                continue;
            c = c + m;
            double cur = frac_lt(Ps, c);
            P[r][k] = cur - prev;
            prev = cur;
            last = k;
        }
        if (last >= 0)
            P[r][last] += 1.0 - prev;   /* the set's last tap takes the rest */
    }
}

/* Exact expectation of the positivised Mitchell-Netravali estimator (level
 * 0), as orc_keys_expect2d. */
ORC_EXPORT int orc_mitchell_expect2d(const void *base, int w, int h, int fmt, int wrap, const float *q, int64_t n,
                                     int shade, const double *ggx, double *out)
{
    const int64_t off0 = 0;
    tex2d t = {(const uint8_t *)base, w, h, 1, fmt, wrap, MIP_NONE, &off0};
    int ch = shade != 0 ? 3 : 4;
    for (int64_t i = 0; i < n; ++i) {
        float uu = wrap_coord(wrap, q[3 * i]), vv = wrap_coord(wrap, q[3 * i + 1]);
        int ix, iy;
        float tx, ty;
        raster(uu, w, &ix, &tx);
        raster(vv, h, &iy, &ty);
        pn_axis ax = mitchell_axis_of(tx), ay = mitchell_axis_of(ty);
        double Wp, Wm;
        mitchell_block_sums((double)tx, (double)ty, &Wp, &Wm);
        double PX[2][4], PY[2][4];
        pn_probs(&ax, PX);
        pn_probs(&ay, PY);
        float A = ax.Pp * ay.Pp, B = ax.Pm * ay.Pm, Cn = ax.Pp * ay.Pm, Dn = ax.Pm * ay.Pp;
        double pblk = frac_lt(A + B, A), nblk = (Cn + Dn) > 0.0f ? frac_lt(Cn + Dn, Cn) : 0.0;
        double acc[4] = {0, 0, 0, 0};
        for (int b = 0; b < 4; ++b)
            for (int a = 0; a < 4; ++a) {
                double texel[4], v[4];
                fetch2d(&t, 0, wrap_tap(wrap, ix - 1 + a, w), wrap_tap(wrap, iy - 1 + b, h), texel);
                shade2d(shade, ggx, texel, v);
                double ppos = pblk * PX[0][a] * PY[0][b] + (1 - pblk) * PX[1][a] * PY[1][b];
                double pneg = nblk * PX[0][a] * PY[1][b] + (1 - nblk) * PX[1][a] * PY[0][b];
                for (int c = 0; c < ch; ++c)
                    acc[c] += Wp * ppos * v[c] - ((Cn + Dn) > 0.0f ? Wm * pneg * v[c] : 0.0);
            }
        for (int c = 0; c < ch; ++c)
            out[ch * i + c] = acc[c];
    }
    return 0;
}

/* Distribution of (jx, jy) under the reuse variant, by running every one of
 * the 2^24 uniforms through the pick-and-remap chain.  counts[16]. */
ORC_EXPORT void orc_reuse_histogram2(int filter, float tx, float ty, int64_t counts[16])
{
    memset(counts, 0, 16 * sizeof(int64_t));
    for (uint32_t k = 0; k < (1u << 24); ++k) {
        float u = (float)k * 0x1p-24f;
        int jx = orc_pick(filter, tx, u);
        float u2 = orc_reuse(filter, tx, u, jx);
        int jy = orc_pick(filter, ty, u2);
        counts[jy * 4 + jx]++;
    }
}

/* ------------------------------------------------------------------------ */
/* 3-D grids                                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    const uint8_t *base;
    int nx, ny, nz, fmt;
    float wmin[3], scale[3];
} grid3d;

static double fetch3d(const grid3d *g, int x, int y, int z)
{
    if (x < 0 || y < 0 || z < 0 || x >= g->nx || y >= g->ny || z >= g->nz)
        return 0.0; /* empty space outside the grid */
    int64_t idx = ((int64_t)z * g->ny + y) * g->nx + x;
    if (g->fmt == FMT_R16F)
        return orc_half_to_double(((const uint16_t *)g->base)[idx]);
    return (double)((const float *)g->base)[idx];
}

static double shade3d(int shade, double sigma, double ds)
{
    return shade == 1 ? exp(-sigma * ds) : sigma;
}

/* Black-body emission (Sec. 5, "Filtering nonlinear physical properties": a
 * grid of temperatures shaded by Planck's law, filtered before or after the
 * shading).  Spectral radiance per nanometre of wavelength, in
 * W sr^-1 m^-2 nm^-1, of a black body at temperature T (kelvin):
 *   B(lambda, T) = 2 h c^2 / (lambda^5 (exp(h c / (lambda k T)) - 1)) * 1e-9,
 * lambda in metres, with the exact SI values of h, c and k.  T <= 0 (empty
 * space) emits nothing; NaN stays NaN.  The three wavelengths of an emission
 * result are the CIE 1931 RGB primaries, 700, 546.1 and 435.8 nm. */
static const double PLANCK_NM[3] = {700.0, 546.1, 435.8};

ORC_EXPORT double orc_planck(double lambda_nm, double T)
{
    if (isnan(T))
        return NAN;
    if (!(T > 0.0))
        return 0.0;
    const double h = 6.62607015e-34, c = 299792458.0, k = 1.380649e-23;
    const double l = lambda_nm * 1e-9;
    return 2.0 * h * c * c / (pow(l, 5.0) * expm1(h * c / (l * k * T))) * 1e-9;
}

static void planck3(double T, double *out)
{
    for (int c = 0; c < 3; ++c)
        out[c] = orc_planck(PLANCK_NM[c], T);
}

/* Three axis picks from the sample's uniforms; variant 1 reuses one. */
static void pick3(int filter, const float t[3], const uint32_t w[4], int variant, int j[3])
{
    float u = uniform24(w[0]);
    for (int a = 0; a < 3; ++a) {
        if (variant == 0)
            u = uniform24(w[a]);
        j[a] = orc_pick(filter, t[a], u);
        if (variant == 1)
            u = orc_reuse(filter, t[a], u, j[a]);
    }
}

static int pos_finite(const float *x)
{
    return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
}

/* Point lookups.  shade: 0 the filtered value, 1 the transmittance
 * exp(-value ds) of a segment of length ds, 2 black-body emission of the
 * value as a temperature (three wavelengths: out is n x 3). */
ORC_EXPORT int orc_filter3d(const void *base, int nx, int ny, int nz, int fmt, const float *wmin,
                            const float *scale, const float *pos, int64_t n, int filter, int mode,
                            int spp, uint32_t seed, int variant, int shade, float ds, double *out,
                            int32_t *taps, const int64_t *subset, int64_t nsub)
{
    grid3d g = {(const uint8_t *)base, nx, ny, nz, fmt, {wmin[0], wmin[1], wmin[2]}, {scale[0], scale[1], scale[2]}};
    int64_t m = subset ? nsub : n;
    const int ch = shade == 2 ? 3 : 1;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t ii = 0; ii < m; ++ii) {
        int64_t i = subset ? subset[ii] : ii;
        const float *x = pos + 3 * i;
        double *o_ = out + ch * ii;
        int32_t *tp = taps ? taps + (int64_t)3 * spp * ii : NULL;
        int ok = pos_finite(x);
        float p[3], t[3];
        int i0[3];
        for (int a = 0; a < 3 && ok; ++a) {
            p[a] = fmaf(x[a] - g.wmin[a], g.scale[a], -0.5f);
            if (!(fabsf(p[a]) <= 4194304.0f))
                ok = 0;
        }
        if (!ok) {
            for (int c = 0; c < ch; ++c)
                o_[c] = NAN;
            if (tp && mode == M_STOCH)
                for (int k = 0; k < 3 * spp; ++k)
                    tp[k] = INT32_MIN;
            continue;
        }
        for (int a = 0; a < 3; ++a) {
            float fl = floorf(p[a]);
            i0[a] = (int)fl;
            t[a] = p[a] - fl;
        }
        int off = filter == F_BSPLINE3 ? -1 : 0;
        double e[3];
        if (mode == M_STOCH) {
            double acc[3] = {0.0, 0.0, 0.0};
            for (int s = 0; s < spp; ++s) {
                uint32_t key[4] = {(uint32_t)i, (uint32_t)s, 0u, seed}, w[4];
                orc_pcg4d(key, w);
                int j[3];
                pick3(filter, t, w, variant, j);
                int tx = i0[0] + off + j[0], ty = i0[1] + off + j[1], tz = i0[2] + off + j[2];
                if (tp) {
                    tp[3 * s] = tx;
                    tp[3 * s + 1] = ty;
                    tp[3 * s + 2] = tz;
                }
                double v = fetch3d(&g, tx, ty, tz);
                if (shade == 2) {
                    planck3(v, e);
                    for (int c = 0; c < 3; ++c)
                        acc[c] += e[c];
                } else {
                    acc[0] += shade3d(shade, v, (double)ds);
                }
            }
            for (int c = 0; c < ch; ++c)
                o_[c] = acc[c] / (double)spp;
        } else {
            double w[3][4];
            int o[3], nt[3];
            for (int a = 0; a < 3; ++a)
                nt[a] = axis_weights(filter, (double)t[a], &o[a], w[a]);
            double sum[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < nt[2]; ++c)
                for (int b = 0; b < nt[1]; ++b)
                    for (int a = 0; a < nt[0]; ++a) {
                        double wgt = w[0][a] * w[1][b] * w[2][c];
                        double sg = fetch3d(&g, i0[0] + o[0] + a, i0[1] + o[1] + b, i0[2] + o[2] + c);
                        if (mode == M_BEFORE) {
                            sum[0] += wgt * sg;
                        } else if (shade == 2) {
                            planck3(sg, e);
                            for (int q = 0; q < 3; ++q)
                                sum[q] += wgt * e[q];
                        } else {
                            sum[0] += wgt * shade3d(shade, sg, (double)ds);
                        }
                    }
            if (mode == M_BEFORE && shade == 2)
                planck3(sum[0], o_);
            else if (mode == M_BEFORE)
                o_[0] = shade3d(shade, sum[0], (double)ds);
            else
                for (int c = 0; c < ch; ++c)
                    o_[c] = sum[c];
        }
    }
    return 0;
}

/* Ray-step raster positions (binary32 contract).  For a ray (o, d, t0, t1)
 * and S steps: dt = (t1 - t0)/S, the raster origin A = (o - wmin)*scale - 0.5
 * (fused), direction B = d*scale, entry E = t0*B + A (fused), step G = dt*B,
 * and the midpoint of step k is p_k = (k + 1/2)*G + E (fused). */
typedef struct {
    float E[3], G[3], dt;
    int ok, empty;
} ray_setup;

static ray_setup setup_ray(const grid3d *g, const float *r, int steps)
{
    ray_setup rs;
    memset(&rs, 0, sizeof rs);
    rs.ok = 1;
    for (int k = 0; k < 8; ++k)
        if (!isfinite(r[k]))
            rs.ok = 0;
    if (!rs.ok)
        return rs;
    if (!(r[7] > r[6])) {
        rs.empty = 1;
        return rs;
    }
    rs.dt = (r[7] - r[6]) / (float)steps;
    for (int a = 0; a < 3; ++a) {
        float A = fmaf(r[a] - g->wmin[a], g->scale[a], -0.5f);
        float B = r[3 + a] * g->scale[a];
        rs.E[a] = fmaf(r[6], B, A);
        rs.G[a] = rs.dt * B;
        float pa = fmaf(0.5f, rs.G[a], rs.E[a]);
        float pb = fmaf((float)(steps - 1) + 0.5f, rs.G[a], rs.E[a]);
        if (!(fabsf(pa) <= 4194304.0f) || !(fabsf(pb) <= 4194304.0f))
            rs.ok = 0;
    }
    return rs;
}

static void step_pos(const ray_setup *rs, int k, int i0[3], float t[3])
{
    float kh = (float)k + 0.5f;
    for (int a = 0; a < 3; ++a) {
        float p = fmaf(kh, rs->G[a], rs->E[a]);
        float fl = floorf(p);
        i0[a] = (int)fl;
        t[a] = p - fl;
    }
}

static double raymarch_one(const grid3d *g, const float *r, int64_t ri, int steps, int filter, int mode,
                           int spp, uint32_t seed, int variant, int32_t *tp)
{
    ray_setup rs = setup_ray(g, r, steps);
    if (!rs.ok || rs.empty) {
        if (tp && mode == M_STOCH)
            for (int64_t k = 0; k < (int64_t)3 * spp * steps; ++k)
                tp[k] = INT32_MIN;
        return rs.ok ? 1.0 : NAN;
    }
    double dt = (double)rs.dt;
    int off = filter == F_BSPLINE3 ? -1 : 0;
    if (mode == M_STOCH) {
        /* one texel per step and sample; per-sample transmittance
         * exp(-dt * sum of the picked densities), averaged over samples */
        double Tsum = 0.0;
        for (int s = 0; s < spp; ++s) {
            double tau = 0.0;
            for (int k = 0; k < steps; ++k) {
                int i0[3], j[3];
                float t[3];
                step_pos(&rs, k, i0, t);
                uint32_t key[4] = {(uint32_t)ri, (uint32_t)s, (uint32_t)k, seed}, w[4];
                orc_pcg4d(key, w);
                pick3(filter, t, w, variant, j);
                int x = i0[0] + off + j[0], y = i0[1] + off + j[1], z = i0[2] + off + j[2];
                if (tp) {
                    int32_t *q = tp + ((int64_t)s * steps + k) * 3;
                    q[0] = x;
                    q[1] = y;
                    q[2] = z;
                }
                tau += fetch3d(g, x, y, z);
            }
            Tsum += exp(-dt * tau);
        }
        return Tsum / (double)spp;
    }
    /* deterministic: before = exp(-dt * sum_k sum_i w_i sigma_i);
     * after = prod_k sum_i w_i exp(-dt sigma_i) */
    double tau = 0.0, T = 1.0;
    for (int k = 0; k < steps; ++k) {
        int i0[3], o[3], nt[3];
        float t[3];
        double w[3][4];
        step_pos(&rs, k, i0, t);
        for (int a = 0; a < 3; ++a)
            nt[a] = axis_weights(filter, (double)t[a], &o[a], w[a]);
        double sum = 0.0;
        for (int c = 0; c < nt[2]; ++c)
            for (int b = 0; b < nt[1]; ++b)
                for (int a = 0; a < nt[0]; ++a) {
                    double wgt = w[0][a] * w[1][b] * w[2][c];
                    double sg = fetch3d(g, i0[0] + o[0] + a, i0[1] + o[1] + b, i0[2] + o[2] + c);
                    sum += wgt * (mode == M_BEFORE ? sg : exp(-dt * sg));
                }
        if (mode == M_BEFORE)
            tau += sum;
        else
            T *= sum;
    }
    return mode == M_BEFORE ? exp(-dt * tau) : T;
}

/* rays: n x {ox,oy,oz,dx,dy,dz,t0,t1}.  If subset is non-null only the nsub
 * listed rays are computed (T and taps are then indexed by position in the
 * subset, the RNG key still by the ray's own index). */
ORC_EXPORT int orc_raymarch(const void *base, int nx, int ny, int nz, int fmt, const float *wmin,
                            const float *scale, const float *rays, int64_t n, int steps, int filter,
                            int mode, int spp, uint32_t seed, int variant, double *T, int32_t *taps,
                            const int64_t *subset, int64_t nsub)
{
    grid3d g = {(const uint8_t *)base, nx, ny, nz, fmt, {wmin[0], wmin[1], wmin[2]}, {scale[0], scale[1], scale[2]}};
    int64_t m = subset ? nsub : n;
    int64_t per = (int64_t)3 * spp * steps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        int64_t ri = subset ? subset[i] : i;
        T[i] = raymarch_one(&g, rays + 8 * ri, ri, steps, filter, mode, spp, seed, variant,
                            taps ? taps + per * i : NULL);
    }
    return 0;
}

/* Exact expectation of the stochastic transmittance with independent
 * uniforms: picks at different steps are independent, so
 * E[T] = prod_k sum_{taps} P(tap) exp(-dt sigma_tap), with the exact 24-bit
 * pick probabilities. */
ORC_EXPORT int orc_raymarch_expect(const void *base, int nx, int ny, int nz, int fmt, const float *wmin,
                                   const float *scale, const float *rays, int64_t n, int steps,
                                   int filter, double *T)
{
    grid3d g = {(const uint8_t *)base, nx, ny, nz, fmt, {wmin[0], wmin[1], wmin[2]}, {scale[0], scale[1], scale[2]}};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        ray_setup rs = setup_ray(&g, rays + 8 * i, steps);
        if (!rs.ok || rs.empty) {
            T[i] = rs.ok ? 1.0 : NAN;
            continue;
        }
        double dt = (double)rs.dt, prod = 1.0;
        int off = filter == F_BSPLINE3 ? -1 : 0;
        int ntap = filter == F_BSPLINE3 ? 4 : (filter == F_LINEAR ? 2 : 1);
        for (int k = 0; k < steps; ++k) {
            int i0[3];
            float t[3];
            double P[3][4];
            step_pos(&rs, k, i0, t);
            int near[3] = {0, 0, 0};
            for (int a = 0; a < 3; ++a) {
                orc_pick_pmf(filter, t[a], P[a]);
                if (filter == F_NEAREST)
                    near[a] = t[a] >= 0.5f;
            }
            double e = 0.0;
            for (int c = 0; c < ntap; ++c)
                for (int b = 0; b < ntap; ++b)
                    for (int a = 0; a < ntap; ++a) {
                        double pr = P[0][a] * P[1][b] * P[2][c];
                        if (pr == 0.0)
                            continue;
                        double sg = fetch3d(&g, i0[0] + off + a + near[0], i0[1] + off + b + near[1],
                                            i0[2] + off + c + near[2]);
                        e += pr * exp(-dt * sg);
                    }
            prod *= e;
        }
        T[i] = prod;
    }
    return 0;
}

/* Emission ray march through a temperature grid (Sec. 5, "Filtering
 * nonlinear physical properties"): an emitting, non-absorbing medium, so the
 * radiance a ray gathers is dt * sum over its steps of the step's emission
 * at three wavelengths.  The step's emission is B(sum_i w_i T_i) before
 * shading, sum_i w_i B(T_i) after, and B(T_j) of the one picked voxel in the
 * stochastic mode (mean over samples).  Picks, keys and raster positions as
 * in the transmittance ray march; with a footprint sigma > 0 (stochastic
 * only) each step's position is first jittered by the perpendicular
 * Gaussian below.  L: n x 3; a ray that misses reads 0, a ray with a
 * non-finite value or an overflowing raster position NaN. */
/* Gaussian footprint perpendicular to a ray (Sec. 5: filtering after
 * shading under minification with a Gaussian in the plane perpendicular to
 * the ray).  Basis of that plane from the unit direction d by the branchless
 * construction of Duff et al., "Building an Orthonormal Basis, Revisited"
 * (JCGT 6(1), 2017), binary32:
 *   sg = copysign(1, d_z), a = -1/(sg + d_z), b = (d_x d_y) a,
 *   e1 = (1 + ((sg d_x) d_x) a, sg b, -sg d_x), e2 = (b, sg + (d_y d_y) a, -d_y);
 * raster-space axes A_i = (sigma e1_i) scale_i, B_i = (sigma e2_i) scale_i.
 * Per step, the key (ray, sample | 2^31, step, seed) gives u0, u1 (words 0,
 * 1); Box-Muller with the contract ln and cos/sin: r = sqrt(-2 ln(1 - u0)),
 * g1 = r cos(2 pi u1), g2 = r sin(2 pi u1); the step's raster position p
 * becomes fma(g2, B, fma(g1, A, p)) before the tap pick. */
typedef struct {
    float A[3], B[3];
} perp_frame;

static perp_frame perp_setup(const grid3d *g, const float *r, float sigma)
{
    const float dx = r[3], dy = r[4], dz = r[5];
    const float sg = copysignf(1.0f, dz);
    const float a = -1.0f / (sg + dz);
    const float b = (dx * dy) * a;
    const float e1[3] = {1.0f + ((sg * dx) * dx) * a, sg * b, -sg * dx};
    const float e2[3] = {b, sg + (dy * dy) * a, -dy};
    perp_frame f;
    for (int i = 0; i < 3; ++i) {
        f.A[i] = (sigma * e1[i]) * g->scale[i];
        f.B[i] = (sigma * e2[i]) * g->scale[i];
    }
    return f;
}

static void perp_jitter(const perp_frame *f, int64_t ri, int s, int k, uint32_t seed, float p[3])
{
    uint32_t key[4] = {(uint32_t)ri, (uint32_t)s | 0x80000000u, (uint32_t)k, seed}, w[4];
    orc_pcg4d(key, w);
    const float u0 = uniform24(w[0]), u1 = uniform24(w[1]);
    const float rr = sqrtf(-2.0f * orc_lnc(1.0f - u0));
    float c, sn;
    orc_sincos2pi(u1, &c, &sn);
    const float g1 = rr * c, g2 = rr * sn;
    for (int i = 0; i < 3; ++i)
        p[i] = fmaf(g2, f->B[i], fmaf(g1, f->A[i], p[i]));
}

/* the raster positions of one step, jittered */
ORC_EXPORT void orc_perp_jitter(const float *wmin, const float *scale, const float *ray, int steps, float sigma,
                                int64_t ri, int s, int k, uint32_t seed, float *p_out)
{
    grid3d g = {NULL, 1, 1, 1, FMT_R32F, {wmin[0], wmin[1], wmin[2]}, {scale[0], scale[1], scale[2]}};
    ray_setup rs = setup_ray(&g, ray, steps);
    perp_frame f = perp_setup(&g, ray, sigma);
    float kh = (float)k + 0.5f;
    for (int a = 0; a < 3; ++a)
        p_out[a] = fmaf(kh, rs.G[a], rs.E[a]);
    perp_jitter(&f, ri, s, k, seed, p_out);
}

static void emission_one(const grid3d *g, const float *r, int64_t ri, int steps, int filter, int mode, int spp,
                         uint32_t seed, int variant, float footprint, double *L, int32_t *tp)
{
    ray_setup rs = setup_ray(g, r, steps);
    if (!rs.ok || rs.empty) {
        if (tp && mode == M_STOCH)
            for (int64_t k = 0; k < (int64_t)3 * spp * steps; ++k)
                tp[k] = INT32_MIN;
        for (int c = 0; c < 3; ++c)
            L[c] = rs.ok ? 0.0 : NAN;
        return;
    }
    const double dt = (double)rs.dt;
    const int off = filter == F_BSPLINE3 ? -1 : 0;
    double e[3], acc[3] = {0.0, 0.0, 0.0};
    if (mode == M_STOCH) {
        const perp_frame pf = perp_setup(g, r, footprint);
        for (int s = 0; s < spp; ++s)
            for (int k = 0; k < steps; ++k) {
                int i0[3], j[3];
                float t[3];
                if (footprint > 0.0f) {
                    float p[3], kh = (float)k + 0.5f;
                    for (int a = 0; a < 3; ++a)
                        p[a] = fmaf(kh, rs.G[a], rs.E[a]);
                    perp_jitter(&pf, ri, s, k, seed, p);
                    for (int a = 0; a < 3; ++a) {
                        float fl = floorf(p[a]);
                        i0[a] = (int)fl;
                        t[a] = p[a] - fl;
                    }
                } else {
                    step_pos(&rs, k, i0, t);
                }
                uint32_t key[4] = {(uint32_t)ri, (uint32_t)s, (uint32_t)k, seed}, w[4];
                orc_pcg4d(key, w);
                pick3(filter, t, w, variant, j);
                int x = i0[0] + off + j[0], y = i0[1] + off + j[1], z = i0[2] + off + j[2];
                if (tp) {
                    int32_t *q = tp + ((int64_t)s * steps + k) * 3;
                    q[0] = x;
                    q[1] = y;
                    q[2] = z;
                }
                planck3(fetch3d(g, x, y, z), e);
                for (int c = 0; c < 3; ++c)
                    acc[c] += e[c];
            }
        for (int c = 0; c < 3; ++c)
            L[c] = dt * acc[c] / (double)spp;
        return;
    }
    for (int k = 0; k < steps; ++k) {
        int i0[3], o[3], nt[3];
        float t[3];
        double w[3][4], sum[3] = {0.0, 0.0, 0.0};
        step_pos(&rs, k, i0, t);
        for (int a = 0; a < 3; ++a)
            nt[a] = axis_weights(filter, (double)t[a], &o[a], w[a]);
        for (int c = 0; c < nt[2]; ++c)
            for (int b = 0; b < nt[1]; ++b)
                for (int a = 0; a < nt[0]; ++a) {
                    double wgt = w[0][a] * w[1][b] * w[2][c];
                    double T = fetch3d(g, i0[0] + o[0] + a, i0[1] + o[1] + b, i0[2] + o[2] + c);
                    if (mode == M_BEFORE) {
                        sum[0] += wgt * T;
                    } else {
                        planck3(T, e);
                        for (int q = 0; q < 3; ++q)
                            sum[q] += wgt * e[q];
                    }
                }
        if (mode == M_BEFORE)
            planck3(sum[0], sum);
        for (int c = 0; c < 3; ++c)
            acc[c] += sum[c];
    }
    for (int c = 0; c < 3; ++c)
        L[c] = dt * acc[c];
}

ORC_EXPORT int orc_raymarch_emission(const void *base, int nx, int ny, int nz, int fmt, const float *wmin,
                                     const float *scale, const float *rays, int64_t n, int steps, int filter,
                                     int mode, int spp, uint32_t seed, int variant, float footprint, double *L,
                                     int32_t *taps, const int64_t *subset, int64_t nsub)
{
    grid3d g = {(const uint8_t *)base, nx, ny, nz, fmt, {wmin[0], wmin[1], wmin[2]}, {scale[0], scale[1], scale[2]}};
    int64_t m = subset ? nsub : n;
    int64_t per = (int64_t)3 * spp * steps;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        int64_t ri = subset ? subset[i] : i;
        emission_one(&g, rays + 8 * ri, ri, steps, filter, mode, spp, seed, variant, footprint, L + 3 * i,
                     taps ? taps + per * i : NULL);
    }
    return 0;
}

/* Exact expectation of the stochastic emission with independent uniforms:
 * dt * sum_k sum_taps P(tap) B(T_tap), with the exact 24-bit pick
 * probabilities. */
ORC_EXPORT int orc_raymarch_emission_expect(const void *base, int nx, int ny, int nz, int fmt, const float *wmin,
                                            const float *scale, const float *rays, int64_t n, int steps,
                                            int filter, double *L)
{
    grid3d g = {(const uint8_t *)base, nx, ny, nz, fmt, {wmin[0], wmin[1], wmin[2]}, {scale[0], scale[1], scale[2]}};
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        ray_setup rs = setup_ray(&g, rays + 8 * i, steps);
        if (!rs.ok || rs.empty) {
            for (int c = 0; c < 3; ++c)
                L[3 * i + c] = rs.ok ? 0.0 : NAN;
            continue;
        }
        int off = filter == F_BSPLINE3 ? -1 : 0;
        int ntap = filter == F_BSPLINE3 ? 4 : (filter == F_LINEAR ? 2 : 1);
        double acc[3] = {0.0, 0.0, 0.0}, e[3];
        for (int k = 0; k < steps; ++k) {
            int i0[3];
            float t[3];
            double P[3][4];
            step_pos(&rs, k, i0, t);
            int near[3] = {0, 0, 0};
            for (int a = 0; a < 3; ++a) {
                orc_pick_pmf(filter, t[a], P[a]);
                if (filter == F_NEAREST)
                    near[a] = t[a] >= 0.5f;
            }
            for (int c = 0; c < ntap; ++c)
                for (int b = 0; b < ntap; ++b)
                    for (int a = 0; a < ntap; ++a) {
                        double pr = P[0][a] * P[1][b] * P[2][c];
                        if (pr == 0.0)
                            continue;
                        planck3(fetch3d(&g, i0[0] + off + a + near[0], i0[1] + off + b + near[1],
                                        i0[2] + off + c + near[2]), e);
                        for (int q = 0; q < 3; ++q)
                            acc[q] += pr * e[q];
                    }
        }
        for (int c = 0; c < 3; ++c)
            L[3 * i + c] = (double)rs.dt * acc[c];
    }
    return 0;
}

/* Brick occupancy: bit b of the mask is set iff some voxel within 2 voxels
 * of brick b (side 2^lg, x fastest) is non-zero or not a number. */
ORC_EXPORT void orc_build_occupancy(const void *base, int nx, int ny, int nz, int fmt, int lg, uint32_t *words)
{
    grid3d g = {(const uint8_t *)base, nx, ny, nz, fmt, {0, 0, 0}, {1, 1, 1}};
    int B = 1 << lg;
    int nbx = (nx + B - 1) / B, nby = (ny + B - 1) / B, nbz = (nz + B - 1) / B;
    int64_t nb = (int64_t)nbx * nby * nbz;
    memset(words, 0, (size_t)((nb + 31) / 32) * sizeof(uint32_t));
    for (int bz = 0; bz < nbz; ++bz)
        for (int by = 0; by < nby; ++by)
            for (int bx = 0; bx < nbx; ++bx) {
                int any = 0;
                for (int z = bz * B - 2; z < bz * B + B + 2 && !any; ++z)
                    for (int y = by * B - 2; y < by * B + B + 2 && !any; ++y)
                        for (int x = bx * B - 2; x < bx * B + B + 2 && !any; ++x) {
                            double v = fetch3d(&g, x, y, z);
                            if (!(v == 0.0))
                                any = 1;
                        }
                int64_t b = ((int64_t)bz * nby + by) * nbx + bx;
                if (any)
                    words[b >> 5] |= 1u << (b & 31);
            }
}

ORC_EXPORT int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
