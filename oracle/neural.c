/*
 * CPU ORACLE, neural part: a latent grid decoded by a small MLP, trained on
 * texels the plain filter generates, and filtered stochastically with ONE
 * decode per sample (the paper motivates this by avoiding repeated
 * evaluation of an expensive decompression per pixel: Sec. 1, Sec. 5 "DCT"
 * results; neural texture compression is its cited example).
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.c).  Shares no code with the HIP
 * library.  binary64 throughout, except where the GPU's storage formats are
 * emulated on purpose (bfloat16 and OCP float8 E4M3 values, and the bfloat16
 * rounding of the hidden activations that feed the matrix cores), each
 * written from the format definitions.
 *
 * MLP: y = W3^T relu(W2^T relu(W1^T z + b1) + b2) + b3, parameters packed
 * as W1 [C x H], b1 [H], W2 [H x H], b2 [H], W3 [H x O], b3 [O], row-major.
 * Loss of a batch: (1/B) sum_s sum_o (y_so - t_so)^2.  relu'(0) = 0.
 * Adam (Kingma & Ba 2015) with bias correction; latents are updated only
 * where the batch touched them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EXPORT __attribute__((visibility("default")))

/* from oracle.c */
void orc_pcg4d(const uint32_t in[4], uint32_t out[4]);
int orc_pick(int filter, float t, float u);
void orc_shade_ggx(const double *p, const double rgba[4], double out[3]);
double orc_kbs(double x);
void orc_axis_weights64(int filter, double t, double w[4]);

enum { F_NEAREST = 0, F_LINEAR = 1, F_BSPLINE3 = 2 };
enum { M_BEFORE = 0, M_AFTER = 1, M_STOCH = 2 };
enum { LAT_F32 = 0, LAT_BF16 = 1, LAT_FP8 = 2 };

/* ------------------------------------------------------------- formats  */
/* binary32 -> bfloat16, round to nearest, ties to even (NaN kept quiet). */
ORC_EXPORT uint16_t orc_f32_to_bf16(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u)
        return (uint16_t)((u >> 16) | 0x40);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

ORC_EXPORT double orc_bf16_to_double(uint16_t h)
{
    uint32_t u = (uint32_t)h << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* OCP float8 E4M3 ("FN"): 1 sign, 4 exponent (bias 7), 3 mantissa bits; no
 * infinities; 0x7f / 0xff are NaN; largest finite 448; subnormals m*2^-9. */
ORC_EXPORT double orc_fp8_to_double(uint8_t b)
{
    int s = b >> 7, e = (b >> 3) & 15, m = b & 7;
    double v;
    if (e == 15 && m == 7)
        return NAN;
    if (e == 0)
        v = ldexp((double)m, -9);
    else
        v = ldexp(1.0 + m / 8.0, e - 7);
    return s ? -v : v;
}

/* binary32 -> E4M3, round to nearest even, saturating at +-448.  Chosen by
 * scanning the 127 non-negative finite codes for the nearest (ties to the
 * even code), which follows the format definition directly. */
ORC_EXPORT uint8_t orc_f32_to_fp8(float f)
{
    if (isnan(f))
        return 0x7f;
    double a = fabs((double)f);
    uint8_t sign = signbit(f) ? 0x80 : 0;
    if (a >= 448.0)
        return sign | 0x7e;
    int best = 0;
    double bd = INFINITY;
    for (int c = 0; c < 0x7f; ++c) {
        double d = fabs(orc_fp8_to_double((uint8_t)c) - a);
        if (d < bd || (d == bd && (c & 1) == 0 && (best & 1) == 1)) {
            bd = d;
            best = c;
        }
    }
    return sign | (uint8_t)best;
}

/* Per-block scales and E4M3 codes of a latent grid: block of side 2^lg
 * lattice points per axis (all C channels); s = amax/448 in binary32
 * (1 for an all-zero block); code = E4M3(z / s) with both operations in
 * binary32. */
ORC_EXPORT void orc_quantize_fp8(const float *lat, int dims, const int *res, int C, int lg, uint8_t *codes,
                                 float *scales)
{
    int B = 1 << lg;
    int nb[3] = {1, 1, 1}, r[3] = {res[0], dims > 1 ? res[1] : 1, dims > 2 ? res[2] : 1};
    for (int a = 0; a < dims; ++a)
        nb[a] = (r[a] + B - 1) / B;
    for (int bz = 0; bz < nb[2]; ++bz)
        for (int by = 0; by < nb[1]; ++by)
            for (int bx = 0; bx < nb[0]; ++bx) {
                float amax = 0.0f;
                for (int z = bz * B; z < (bz + 1) * B && z < r[2]; ++z)
                    for (int y = by * B; y < (by + 1) * B && y < r[1]; ++y)
                        for (int x = bx * B; x < (bx + 1) * B && x < r[0]; ++x)
                            for (int c = 0; c < C; ++c) {
                                float v = fabsf(lat[(((int64_t)z * r[1] + y) * r[0] + x) * C + c]);
                                if (v > amax)
                                    amax = v;
                            }
                float s = amax > 0.0f ? amax / 448.0f : 1.0f;
                scales[((int64_t)bz * nb[1] + by) * nb[0] + bx] = s;
                for (int z = bz * B; z < (bz + 1) * B && z < r[2]; ++z)
                    for (int y = by * B; y < (by + 1) * B && y < r[1]; ++y)
                        for (int x = bx * B; x < (bx + 1) * B && x < r[0]; ++x)
                            for (int c = 0; c < C; ++c) {
                                int64_t i = (((int64_t)z * r[1] + y) * r[0] + x) * C + c;
                                codes[i] = orc_f32_to_fp8(lat[i] / s);
                            }
            }
}

/* The value an E4M3 latent feeds to the MLP, whose operands are BF16: the
 * code's value times its block scale, that product rounded to binary32, and
 * the binary32 product rounded to BF16 (nearest, ties to even).  codes: n x C;
 * scale: one per lattice point (its block's); out: n x C binary64. */
ORC_EXPORT void orc_dequant_fp8(const uint8_t *codes, const float *scale, int64_t n, int C, double *out)
{
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < C; ++c) {
            float p = (float)orc_fp8_to_double(codes[i * C + c]) * scale[i];
            out[i * C + c] = orc_bf16_to_double(orc_f32_to_bf16(p));
        }
}

/* ----------------------------------------------------------------- MLP  */
typedef struct {
    int C, H, O;
} dims_t;

static int64_t nparams(dims_t d) { return (int64_t)d.C * d.H + d.H + (int64_t)d.H * d.H + d.H + (int64_t)d.H * d.O + d.O; }

/* Forward pass.  If act_bf16, the two hidden activations are rounded to
 * bfloat16 before the next layer (the matrix-core decoder's storage). */
static void mlp_forward(dims_t d, const double *P, const double *z, int act_bf16, double *a1, double *h1,
                        double *a2, double *h2, double *y)
{
    const double *W1 = P, *b1 = W1 + d.C * d.H, *W2 = b1 + d.H, *b2 = W2 + d.H * d.H, *W3 = b2 + d.H,
                 *b3 = W3 + d.H * d.O;
    for (int h = 0; h < d.H; ++h) {
        double s = b1[h];
        for (int c = 0; c < d.C; ++c)
            s += z[c] * W1[c * d.H + h];
        a1[h] = s;
        h1[h] = s > 0.0 ? s : 0.0;
        if (act_bf16)
            h1[h] = orc_bf16_to_double(orc_f32_to_bf16((float)h1[h]));
    }
    for (int h = 0; h < d.H; ++h) {
        double s = b2[h];
        for (int k = 0; k < d.H; ++k)
            s += h1[k] * W2[k * d.H + h];
        a2[h] = s;
        h2[h] = s > 0.0 ? s : 0.0;
        if (act_bf16)
            h2[h] = orc_bf16_to_double(orc_f32_to_bf16((float)h2[h]));
    }
    for (int o = 0; o < d.O; ++o) {
        double s = b3[o];
        for (int k = 0; k < d.H; ++k)
            s += h2[k] * W3[k * d.O + o];
        y[o] = s;
    }
}

/* Decoded outputs of a batch of latent vectors. */
ORC_EXPORT void orc_mlp_forward(int C, int H, int O, const double *P, const double *Z, int64_t n, int act_bf16,
                                double *Y)
{
    dims_t d = {C, H, O};
    double a1[256], h1[256], a2[256], h2[256];
#pragma omp parallel for private(a1, h1, a2, h2) schedule(static)
    for (int64_t i = 0; i < n; ++i)
        mlp_forward(d, P, Z + i * C, act_bf16, a1, h1, a2, h2, Y + i * O);
}

/* Gradients of the batch loss (1/B) sum_s ||y_s - t_s||^2 with respect to
 * the packed parameters (gP, summed over the batch) and to each sample's
 * latent (gZ, B x C).  Returns the loss.  act_bf16: the hidden activations
 * are stored in BF16 as a matrix-core implementation reads them (the same
 * reading as the decoder's); everything else is FP64. */
ORC_EXPORT double orc_mlp_grad(int C, int H, int O, const double *P, const double *Z, const double *T, int64_t B,
                               int act_bf16, double *gP, double *gZ)
{
    dims_t d = {C, H, O};
    const double *W1 = P, *W2 = W1 + C * H + H, *W3 = W2 + H * H + H;
    int64_t np = nparams(d);
    memset(gP, 0, np * sizeof(double));
    double *gW1 = gP, *gb1 = gW1 + C * H, *gW2 = gb1 + H, *gb2 = gW2 + H * H, *gW3 = gb2 + H, *gb3 = gW3 + H * O;
    double loss = 0.0;
    double a1[256], h1[256], a2[256], h2[256], y[16], dy[16], da2[256], da1[256];
    for (int64_t s = 0; s < B; ++s) {
        const double *z = Z + s * C;
        mlp_forward(d, P, z, act_bf16, a1, h1, a2, h2, y);
        for (int o = 0; o < O; ++o) {
            double e = y[o] - T[s * O + o];
            loss += e * e;
            dy[o] = 2.0 * e / (double)B;
        }
        for (int o = 0; o < O; ++o) {
            gb3[o] += dy[o];
            for (int k = 0; k < H; ++k)
                gW3[k * O + o] += h2[k] * dy[o];
        }
        for (int k = 0; k < H; ++k) {
            double g = 0.0;
            for (int o = 0; o < O; ++o)
                g += W3[k * O + o] * dy[o];
            da2[k] = a2[k] > 0.0 ? g : 0.0;
        }
        for (int h = 0; h < H; ++h) {
            gb2[h] += da2[h];
            for (int k = 0; k < H; ++k)
                gW2[k * H + h] += h1[k] * da2[h];
        }
        for (int k = 0; k < H; ++k) {
            double g = 0.0;
            for (int h = 0; h < H; ++h)
                g += W2[k * H + h] * da2[h];
            da1[k] = a1[k] > 0.0 ? g : 0.0;
        }
        for (int h = 0; h < H; ++h) {
            gb1[h] += da1[h];
            for (int c = 0; c < C; ++c)
                gW1[c * H + h] += z[c] * da1[h];
        }
        for (int c = 0; c < C; ++c) {
            double g = 0.0;
            for (int h = 0; h < H; ++h)
                g += W1[c * H + h] * da1[h];
            gZ[s * C + c] = g;
        }
    }
    return loss / (double)B;
}

/* One Adam step on n values (theta, m, v updated in place). */
ORC_EXPORT void orc_adam(double *theta, double *m, double *v, const double *g, int64_t n, int step, double lr)
{
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        theta[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* ------------------------------------------------ neural filtering paths */
/* A latent grid: res[0] x res[1] (x res[2]) lattice points, C channels,
 * latents already decoded to binary64 (from BF16 or E4M3 x block scale).
 * The decoded texel of lattice point c is clamp(MLP(z_c), 0, 1) (2-D, RGBA)
 * or max(MLP(z_c), 0) (3-D, density); act_bf16 as in mlp_forward. */
typedef struct {
    int dims, res[3], C, H, O, act_bf16;
    const double *Z, *P;
} net_t;

static void decode(const net_t *n, int64_t idx, double *out)
{
    double a1[256], h1[256], a2[256], h2[256];
    dims_t d = {n->C, n->H, n->O};
    mlp_forward(d, n->P, n->Z + idx * n->C, n->act_bf16, a1, h1, a2, h2, out);
    for (int o = 0; o < n->O; ++o) {
        double v = out[o] > 0.0 ? out[o] : 0.0;
        if (n->dims == 2 && v > 1.0)
            v = 1.0;
        out[o] = v;
    }
}

static int wrapi(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

/* 2-D neural texture, repeat wrap, lattice raster p = u*R - 0.5 (fused),
 * taps picked exactly as the plain 2-D filter picks texels of level 0.
 * shade: 0 none (RGBA), 1 GGX (needs O = 4). */
ORC_EXPORT void orc_neural_filter2d(int R0, int R1, int C, int H, int O, const double *Z, const double *P,
                                    int act_bf16, const float *q, int64_t n, int filter, int mode, int spp,
                                    uint32_t seed, int shade, const double *ggx, double *out, int32_t *taps,
                                    const int64_t *subset, int64_t nsub)
{
    net_t net = {2, {R0, R1, 1}, C, H, O, act_bf16, Z, P};
    int ch = shade == 1 ? 3 : O;
    int64_t m = subset ? nsub : n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t ii = 0; ii < m; ++ii) {
        int64_t qi = subset ? subset[ii] : ii;
        double *o = out + ii * ch;
        const float *qq = q + 3 * qi;
        if (!isfinite(qq[0]) || !isfinite(qq[1])) {
            for (int c = 0; c < ch; ++c)
                o[c] = NAN;
            if (taps && mode == M_STOCH)
                for (int s = 0; s < 2 * spp; ++s)
                    taps[ii * 2 * spp + s] = INT32_MIN;
            continue;
        }
        float u = qq[0] - floorf(qq[0]), v = qq[1] - floorf(qq[1]);
        float px = fmaf(u, (float)R0, -0.5f), py = fmaf(v, (float)R1, -0.5f);
        float fx = floorf(px), fy = floorf(py);
        int ix = (int)fx, iy = (int)fy;
        float tx = px - fx, ty = py - fy;
        int off = filter == F_BSPLINE3 ? -1 : 0;
        double D[16], sh[4], acc[4] = {0, 0, 0, 0};
        if (mode == M_STOCH) {
            for (int s = 0; s < spp; ++s) {
                uint32_t key[4] = {(uint32_t)qi, (uint32_t)s, 0u, seed}, w[4];
                orc_pcg4d(key, w);
                float ux = (float)(w[0] >> 8) * 0x1p-24f, uy = (float)(w[1] >> 8) * 0x1p-24f;
                int x = wrapi(ix + off + orc_pick(filter, tx, ux), R0);
                int y = wrapi(iy + off + orc_pick(filter, ty, uy), R1);
                if (taps) {
                    taps[(ii * spp + s) * 2] = x;
                    taps[(ii * spp + s) * 2 + 1] = y;
                }
                decode(&net, (int64_t)y * R0 + x, D);
                if (shade == 1)
                    orc_shade_ggx(ggx, D, sh);
                for (int c = 0; c < ch; ++c)
                    acc[c] += shade == 1 ? sh[c] : D[c];
            }
            for (int c = 0; c < ch; ++c)
                o[c] = acc[c] / spp;
            continue;
        }
        double wx[4], wy[4];
        orc_axis_weights64(filter, (double)tx, wx);
        orc_axis_weights64(filter, (double)ty, wy);
        int nt = filter == F_BSPLINE3 ? 4 : (filter == F_LINEAR ? 2 : 1);
        int ox = filter == F_NEAREST ? (tx >= 0.5f) : off, oy = filter == F_NEAREST ? (ty >= 0.5f) : off;
        double sum[4] = {0, 0, 0, 0};
        for (int b = 0; b < nt; ++b)
            for (int a = 0; a < nt; ++a) {
                double wgt = wx[a] * wy[b];
                decode(&net, (int64_t)wrapi(iy + oy + b, R1) * R0 + wrapi(ix + ox + a, R0), D);
                if (mode == M_BEFORE) {
                    for (int c = 0; c < O; ++c)
                        sum[c] += wgt * D[c];
                } else {
                    if (shade == 1)
                        orc_shade_ggx(ggx, D, sh);
                    for (int c = 0; c < ch; ++c)
                        sum[c] += wgt * (shade == 1 ? sh[c] : D[c]);
                }
            }
        if (mode == M_BEFORE && shade == 1)
            orc_shade_ggx(ggx, sum, o);
        else
            for (int c = 0; c < ch; ++c)
                o[c] = sum[c];
    }
}

/* 3-D neural volume ray march: the same ray-step contract as the plain
 * march (see oracle.c), densities decoded from the latent lattice; taps
 * outside the lattice read zero without a decode. */
ORC_EXPORT void orc_neural_raymarch(int R0, int R1, int R2, int C, int H, const double *Z, const double *P,
                                    int act_bf16, const float *wmin, const float *scale, const float *rays,
                                    int64_t n, int steps, int filter, int mode, int spp, uint32_t seed, double *T,
                                    int32_t *taps, const int64_t *subset, int64_t nsub)
{
    net_t net = {3, {R0, R1, R2}, C, H, 1, act_bf16, Z, P};
    int res[3] = {R0, R1, R2};
    int64_t m = subset ? nsub : n;
    int64_t per = (int64_t)3 * spp * steps;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t ii = 0; ii < m; ++ii) {
        int64_t ri = subset ? subset[ii] : ii;
        const float *r = rays + 8 * ri;
        int ok = 1;
        for (int k = 0; k < 8; ++k)
            ok &= isfinite(r[k]) != 0;
        int32_t *tp = taps ? taps + per * ii : NULL;
        if (!ok || !(r[7] > r[6])) {
            T[ii] = ok ? 1.0 : NAN;
            if (tp && mode == M_STOCH)
                for (int64_t k = 0; k < per; ++k)
                    tp[k] = INT32_MIN;
            continue;
        }
        float dtf = (r[7] - r[6]) / (float)steps;
        float E[3], G[3];
        for (int a = 0; a < 3; ++a) {
            float A = fmaf(r[a] - wmin[a], scale[a], -0.5f);
            float Bd = r[3 + a] * scale[a];
            E[a] = fmaf(r[6], Bd, A);
            G[a] = dtf * Bd;
            float pa = fmaf(0.5f, G[a], E[a]), pb = fmaf((float)(steps - 1) + 0.5f, G[a], E[a]);
            if (!(fabsf(pa) <= 4194304.0f) || !(fabsf(pb) <= 4194304.0f))
                ok = 0;
        }
        if (!ok) {
            T[ii] = NAN;
            if (tp && mode == M_STOCH)
                for (int64_t k = 0; k < per; ++k)
                    tp[k] = INT32_MIN;
            continue;
        }
        double dt = (double)dtf;
        int off = filter == F_BSPLINE3 ? -1 : 0;
        double D[1];
        if (mode == M_STOCH) {
            double Tsum = 0.0;
            for (int s = 0; s < spp; ++s) {
                double tau = 0.0;
                for (int k = 0; k < steps; ++k) {
                    int i0[3], j[3];
                    float t[3];
                    for (int a = 0; a < 3; ++a) {
                        float p = fmaf((float)k + 0.5f, G[a], E[a]);
                        float fl = floorf(p);
                        i0[a] = (int)fl;
                        t[a] = p - fl;
                    }
                    uint32_t key[4] = {(uint32_t)ri, (uint32_t)s, (uint32_t)k, seed}, w[4];
                    orc_pcg4d(key, w);
                    for (int a = 0; a < 3; ++a)
                        j[a] = i0[a] + off + orc_pick(filter, t[a], (float)(w[a] >> 8) * 0x1p-24f);
                    if (tp) {
                        int32_t *q = tp + ((int64_t)s * steps + k) * 3;
                        q[0] = j[0];
                        q[1] = j[1];
                        q[2] = j[2];
                    }
                    if (j[0] < 0 || j[1] < 0 || j[2] < 0 || j[0] >= R0 || j[1] >= R1 || j[2] >= R2)
                        continue;
                    decode(&net, ((int64_t)j[2] * R1 + j[1]) * R0 + j[0], D);
                    tau += D[0];
                }
                Tsum += exp(-dt * tau);
            }
            T[ii] = Tsum / spp;
            continue;
        }
        double tau = 0.0, Tp = 1.0;
        int nt = filter == F_BSPLINE3 ? 4 : (filter == F_LINEAR ? 2 : 1);
        for (int k = 0; k < steps; ++k) {
            int i0[3], o3[3];
            float t[3];
            double w[3][4];
            for (int a = 0; a < 3; ++a) {
                float p = fmaf((float)k + 0.5f, G[a], E[a]);
                float fl = floorf(p);
                i0[a] = (int)fl;
                t[a] = p - fl;
                orc_axis_weights64(filter, (double)t[a], w[a]);
                o3[a] = filter == F_NEAREST ? (t[a] >= 0.5f) : off;
            }
            double sum = 0.0;
            for (int c = 0; c < nt; ++c)
                for (int b = 0; b < nt; ++b)
                    for (int a = 0; a < nt; ++a) {
                        int x = i0[0] + o3[0] + a, y = i0[1] + o3[1] + b, z = i0[2] + o3[2] + c;
                        double sg = 0.0;
                        if (x >= 0 && y >= 0 && z >= 0 && x < res[0] && y < res[1] && z < res[2]) {
                            decode(&net, ((int64_t)z * R1 + y) * R0 + x, D);
                            sg = D[0];
                        }
                        double wgt = w[0][a] * w[1][b] * w[2][c];
                        sum += wgt * (mode == M_BEFORE ? sg : exp(-dt * sg));
                    }
            if (mode == M_BEFORE)
                tau += sum;
            else
                Tp *= sum;
        }
        T[ii] = mode == M_BEFORE ? exp(-dt * tau) : Tp;
    }
}
