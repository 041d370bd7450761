// Neural latent textures / volumes of libsf.
//
// A lattice of latent vectors z_c is decoded by a small MLP
// D_c = W3^T relu(W2^T relu(W1^T z_c + b1) + b2) + b3.  Stochastic filtering
// picks ONE lattice point per sample with the same inverse-CDF contract as
// the plain texture (Sec. 4.1 FRS) and therefore runs ONE decode per sample
// instead of 16 (bicubic) or 64 (tricubic).
//
//  - Training in FP32 on the vector ALU (the SF_TRAIN_FP32 step; the default
//    matrix-core step is in train.hip): one wavefront streams a chunk of the
//    batch; lane h owns hidden unit h, so both matrix-vector products of a
//    sample are 64-lane broadcasts from LDS.  Per-wavefront parameter
//    gradients of either step are summed in a fixed order by two kernels here,
//    the second of which applies Adam; latent gradients are applied at once
//    (each batch entry owns its latent).
//  - Decoding (BF16 matrix cores, FP32 accumulation): 16 samples form the
//    columns of one v_mfma_f32_16x16x32_bf16 tile with hidden units as rows,
//    so one layer's accumulators are, lane for lane, the next layer's B
//    operand (the weights' K order is permuted to match, see kperm()).
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "sf_device.hpp"
#include "sf_internal.hpp"
#include "volume_dev.hpp"

#pragma clang fp contract(off)

namespace sfk {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int HID = 64;

// ------------------------------------------------------------------ formats
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7fffffffu) > 0x7f800000u)
        return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_bits_to_f32(uint16_t h) { return __builtin_bit_cast(float, (uint32_t)h << 16); }

// binary32 -> E4M3, round to nearest even, saturating at +-448.
__device__ __forceinline__ uint8_t f32_to_fp8_rne(float f)
{
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    const uint32_t sign = (u >> 24) & 0x80u;
    if ((u & 0x7fffffffu) > 0x7f800000u)
        return 0x7f;
    const float a = __builtin_fabsf(f);
    if (a >= 448.0f)
        return (uint8_t)(sign | 0x7eu);
    if (a < 0x1p-6f) {   // subnormal range: multiples of 2^-9
        float m = __builtin_rintf(a * 512.0f);   // exact scaling, RNE
        return (uint8_t)(sign | (uint32_t)m);    // m == 8 is the smallest normal, code 0x08
    }
    const uint32_t au = __builtin_bit_cast(uint32_t, a);
    uint32_t e = (au >> 23) - 120u;          // E4M3 exponent field, 1..15
    uint32_t m3 = (au >> 20) & 7u;
    const uint32_t rem = au & 0xfffffu, halfway = 0x80000u;
    if (rem > halfway || (rem == halfway && (m3 & 1u)))
        ++m3;
    uint32_t code = (e << 3) + m3;          // a mantissa carry rolls into the exponent
    return (uint8_t)(sign | (code > 0x7eu ? 0x7eu : code));
}

// ------------------------------------------------------------ quantization
__global__ __launch_bounds__(256) void k_to_bf16(const float *in, int64_t n, uint16_t *out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        out[i] = f32_to_bf16_rne(in[i]);
}

// One workgroup per block of lattice points: amax over the block (all
// channels), s = amax/448 (1 for an all-zero block), code = E4M3(z/s).
__global__ __launch_bounds__(256) void k_quant_fp8(const float *lat, LatentArgs g, uint8_t *codes, float *scales)
{
    __shared__ float red[256];
    const int B = 1 << g.block_log2;
    const int nbx = (g.res[0] + B - 1) / B, nby = (g.res[1] + B - 1) / B;
    const int64_t b = blockIdx.x;
    const int bx = (int)(b % nbx), by = (int)((b / nbx) % nby), bz = (int)(b / ((int64_t)nbx * nby));
    const int ex = min(B, g.res[0] - bx * B), ey = min(B, g.res[1] - by * B), ez = min(B, g.res[2] - bz * B);
    const int64_t count = (int64_t)ex * ey * ez * g.C;
    float amax = 0.0f;
    for (int64_t k = threadIdx.x; k < count; k += 256) {
        const int c = (int)(k % g.C);
        const int64_t p = k / g.C;
        const int x = bx * B + (int)(p % ex), y = by * B + (int)((p / ex) % ey), z = bz * B + (int)(p / ((int64_t)ex * ey));
        const int64_t idx = (((int64_t)z * g.res[1] + y) * g.res[0] + x) * g.C + c;
        amax = __builtin_fmaxf(amax, __builtin_fabsf(lat[idx]));
    }
    red[threadIdx.x] = amax;
    __syncthreads();
    for (int m = 128; m >= 1; m >>= 1) {
        if ((int)threadIdx.x < m)
            red[threadIdx.x] = __builtin_fmaxf(red[threadIdx.x], red[threadIdx.x + m]);
        __syncthreads();
    }
    const float s = red[0] > 0.0f ? red[0] / 448.0f : 1.0f;
    if (threadIdx.x == 0)
        scales[b] = s;
    for (int64_t k = threadIdx.x; k < count; k += 256) {
        const int c = (int)(k % g.C);
        const int64_t p = k / g.C;
        const int x = bx * B + (int)(p % ex), y = by * B + (int)((p / ex) % ey), z = bz * B + (int)(p / ((int64_t)ex * ey));
        const int64_t idx = (((int64_t)z * g.res[1] + y) * g.res[0] + x) * g.C + c;
        codes[idx] = f32_to_fp8_rne(lat[idx] / s);
    }
}

// ----------------------------------------------------------------- training
// Packed parameter offsets: W1 [C x H], b1 [H], W2 [H x H], b2 [H], W3 [H x O], b3 [O].
struct POff {
    int w1, b1, w2, b2, w3, b3, n;
    __host__ __device__ POff(int C, int O)
    {
        w1 = 0;
        b1 = C * HID;
        w2 = b1 + HID;
        b2 = w2 + HID * HID;
        w3 = b2 + HID;
        b3 = w3 + HID * O;
        n = b3 + O;
    }
};

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        v += __shfl_xor(v, m);
    return v;
}

// One wavefront (= one workgroup) per chunk of the batch.  Lane h holds
// hidden unit h: its column of W1, its row of W3 and the matching gradient
// accumulators; W2 and W1 sit in LDS with rows padded to HID + 1 words, so
// that lane h reads column h (W2[k][h], layer 2 forward) and row h (W2[h][k],
// W1[h][k], the backward sums) without bank conflicts, and the wavefront
// keeps few enough registers to share a SIMD.  S consecutive samples are
// processed together: their loads and their multiply-add chains are
// independent, so they overlap, while every per-sample sum and every
// accumulator update keeps the sample order (the results equal those of one
// sample at a time).
template <int C, int O, int S>
__global__ __launch_bounds__(64) void k_train(TrainCall t, int64_t chunk, float *partials)
{
    constexpr int LD = HID + 1;
    __shared__ float sw2[HID * LD], sw1[C * LD];
    __shared__ float sh_h1[HID][S], sh_da[HID][S];
    const POff P(C, O);
    const int h = threadIdx.x;
    const float *W = t.params;
    float w1c[C], w3r[O];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        w1c[c] = W[P.w1 + c * HID + h];
        sw1[c * LD + h] = w1c[c];
    }
    for (int k = 0; k < HID; ++k)
        sw2[k * LD + h] = W[P.w2 + k * HID + h];
#pragma unroll
    for (int o = 0; o < O; ++o)
        w3r[o] = W[P.w3 + h * O + o];
    __syncthreads();
    const float b1 = W[P.b1 + h], b2 = W[P.b2 + h];
    float b3[O];
#pragma unroll
    for (int o = 0; o < O; ++o)
        b3[o] = W[P.b3 + o];

    float g1[C], g2[HID], g3[O], gb1 = 0.0f, gb2 = 0.0f, gb3[O], loss = 0.0f;
#pragma unroll
    for (int c = 0; c < C; ++c)
        g1[c] = 0.0f;
#pragma unroll
    for (int k = 0; k < HID; ++k)
        g2[k] = 0.0f;
#pragma unroll
    for (int o = 0; o < O; ++o)
        g3[o] = gb3[o] = 0.0f;

    const float inv_b = 2.0f / (float)t.batch;
    const int64_t s0 = (int64_t)blockIdx.x * chunk;
    const int64_t s1 = min(s0 + chunk, t.batch);
    // Software pipeline over the groups of S samples, unrolled twice over two
    // register sets so that no value still in flight is ever copied: while a
    // group is computed, the next group's latents and targets and the batch
    // indices of the group after it are being read, and the group's own Adam
    // moments and latent values are read at its start.  The batch indices are
    // distinct, so no value read ahead is one that an earlier group updates.
    // An index outside the lattice (or past the chunk) contributes nothing.
    // Every read ahead is unconditional, from element 0 where a sample is
    // unused (past the chunk, or an index outside the lattice), and no value
    // read ahead is selected on before its use: a select would make the wave
    // wait for the load at once.  An unused sample's values only feed its
    // own sums, which every update, store and gradient gates on use[j].
    struct Group {
        int32_t raw[S];   // batch indices as read
        bool in[S];       // inside the chunk
        float z[S][C], tg[S][O];
    };
    Group A, B;
    const auto read_idx = [&](int64_t sb, Group &G) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            G.in[j] = sb + j < s1;
            G.raw[j] = t.idx[min(sb + j, s1 - 1)];
        }
    };
    const auto usable = [&](const Group &G, int j) {
        return G.in[j] && (uint64_t)(int64_t)G.raw[j] < (uint64_t)t.n_lattice;
    };
    const auto read_group = [&](Group &G) {
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const int64_t p = usable(G, j) ? (int64_t)G.raw[j] : 0;
#pragma unroll
            for (int c = 0; c < C; ++c)
                G.z[j][c] = t.latents[p * C + c];
#pragma unroll
            for (int o = 0; o < O; ++o)
                G.tg[j][o] = t.targets[p * O + o];
        }
    };
    const auto step = [&](int64_t sb, Group &cur, Group &nxt) {
        int64_t li[S];
        bool use[S];
        float mq[S], vq[S], zq[S];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            use[j] = usable(cur, j);
            li[j] = cur.raw[j];
            const int64_t q = use[j] && h < C ? li[j] * C + h : 0;   // lane c < C owns channel c
            mq[j] = t.m_lat[q];
            vq[j] = t.v_lat[q];
            zq[j] = t.latents[q];
        }
        read_group(nxt);              // nxt's indices were read one group earlier
        read_idx(sb + 2 * S, cur);    // the group after nxt
        float a1[S], a2[S];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            a1[j] = b1;
#pragma unroll
            for (int c = 0; c < C; ++c)
                a1[j] = __builtin_fmaf(cur.z[j][c], w1c[c], a1[j]);
            sh_h1[h][j] = a1[j] > 0.0f ? a1[j] : 0.0f;
            a2[j] = b2;
        }
        __syncthreads();
#pragma unroll 16
        for (int k = 0; k < HID; ++k) {
            const float w = sw2[k * LD + h];   // W2[k][h]
#pragma unroll
            for (int j = 0; j < S; ++j)
                a2[j] = __builtin_fmaf(sh_h1[k][j], w, a2[j]);
        }
        float da2[S];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            const float h2 = a2[j] > 0.0f ? a2[j] : 0.0f;
            float dh2 = 0.0f;
#pragma unroll
            for (int o = 0; o < O; ++o) {
                const float y = wave_sum(h2 * w3r[o]) + b3[o];
                const float e = y - cur.tg[j][o];
                const float dy = e * inv_b;
                if (use[j]) {
                    loss = __builtin_fmaf(e, e, loss);
                    g3[o] = __builtin_fmaf(h2, dy, g3[o]);
                    gb3[o] += dy;
                }
                dh2 = __builtin_fmaf(w3r[o], dy, dh2);
            }
            da2[j] = use[j] && a2[j] > 0.0f ? dh2 : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < S; ++j) {
            if (!use[j])
                continue;
            gb2 += da2[j];
#pragma unroll
            for (int k = 0; k < HID; ++k)
                g2[k] = __builtin_fmaf(sh_h1[k][j], da2[j], g2[k]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < S; ++j)
            sh_da[h][j] = da2[j];
        __syncthreads();
        float dh1[S];
#pragma unroll
        for (int j = 0; j < S; ++j)
            dh1[j] = 0.0f;
#pragma unroll 16
        for (int k = 0; k < HID; ++k) {
            const float w = sw2[h * LD + k];   // W2[h][k]
#pragma unroll
            for (int j = 0; j < S; ++j)
                dh1[j] = __builtin_fmaf(w, sh_da[k][j], dh1[j]);
        }
        float da1[S];
#pragma unroll
        for (int j = 0; j < S; ++j) {
            da1[j] = a1[j] > 0.0f ? dh1[j] : 0.0f;
            if (!use[j])
                continue;
            gb1 += da1[j];
#pragma unroll
            for (int c = 0; c < C; ++c)
                g1[c] = __builtin_fmaf(cur.z[j][c], da1[j], g1[c]);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < S; ++j)
            sh_da[h][j] = da1[j];
        __syncthreads();
        // latent gradients and their Adam steps
        if (h < C) {
            float gz[S];
#pragma unroll
            for (int j = 0; j < S; ++j)
                gz[j] = 0.0f;
#pragma unroll 16
            for (int k = 0; k < HID; ++k) {
                const float w = sw1[h * LD + k];   // W1[h][k]
#pragma unroll
                for (int j = 0; j < S; ++j)
                    gz[j] = __builtin_fmaf(w, sh_da[k][j], gz[j]);
            }
#pragma unroll
            for (int j = 0; j < S; ++j) {
                if (!use[j])
                    continue;
                if (t.grad_latents)
                    t.grad_latents[(sb + j) * C + h] = gz[j];
                const int64_t q = li[j] * C + h;
                const float m = 0.9f * mq[j] + 0.1f * gz[j];
                const float v = 0.999f * vq[j] + 0.001f * gz[j] * gz[j];
                t.m_lat[q] = m;
                t.v_lat[q] = v;
                t.latents[q] = zq[j] - t.lr_latent * (m / t.bc1) / (__builtin_sqrtf(v / t.bc2) + 1e-8f);
            }
        }
        __syncthreads();
    };
    read_idx(s0, A);
    read_idx(s0 + S, B);
    read_group(A);
    for (int64_t sb = s0; sb < s1; sb += 2 * S) {
        step(sb, A, B);
        if (sb + S < s1)
            step(sb + S, B, A);
    }
    // per-wavefront partial gradients in the packed layout, then the loss
    float *out = partials + (int64_t)blockIdx.x * (P.n + 1);
#pragma unroll
    for (int c = 0; c < C; ++c)
        out[P.w1 + c * HID + h] = g1[c];
    out[P.b1 + h] = gb1;
#pragma unroll
    for (int k = 0; k < HID; ++k)
        out[P.w2 + k * HID + h] = g2[k];
    out[P.b2 + h] = gb2;
#pragma unroll
    for (int o = 0; o < O; ++o)
        out[P.w3 + h * O + o] = g3[o];
    if (h == 0) {
#pragma unroll
        for (int o = 0; o < O; ++o)
            out[P.b3 + o] = gb3[o];
        out[P.n] = loss;
    }
}

constexpr int TRAIN_GROUP = 2;   // samples per iteration of k_train

// First stage of the gradient sum: chunk c (blockIdx.y) of REDUCE_CHUNK
// consecutive per-wavefront partials, summed in order.
constexpr int REDUCE_CHUNK = 64;

// All REDUCE_CHUNK loads are issued before the first addition (a partial
// past the last reads the last one's address and adds +0).
__global__ __launch_bounds__(256) void k_train_chunks(int nparts, const float *partials, int npar, float *chunks)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p > npar)
        return;
    const int w0 = blockIdx.y * REDUCE_CHUNK, w1 = min(w0 + REDUCE_CHUNK, nparts);
    float v[REDUCE_CHUNK];
#pragma unroll
    for (int j = 0; j < REDUCE_CHUNK; ++j) {
        const float x = partials[(int64_t)min(w0 + j, w1 - 1) * (npar + 1) + p];
        v[j] = w0 + j < w1 ? x : 0.0f;
    }
    float g = 0.0f;
#pragma unroll
    for (int j = 0; j < REDUCE_CHUNK; ++j)
        g += v[j];
    chunks[(int64_t)blockIdx.y * (npar + 1) + p] = g;
}

// Sum the chunk sums in order (a fixed order overall: the result does not
// depend on scheduling) and take one Adam step per parameter; the loss lands
// in loss_out.
__global__ __launch_bounds__(256) void k_train_reduce(TrainCall t, int nchunks, const float *chunks, int npar)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p > npar)
        return;
    // the chunk sums in order, loaded MAX_CHUNKS at a time before they are added
    constexpr int MAX_CHUNKS = 32;
    float g = 0.0f;
    for (int w0 = 0; w0 < nchunks; w0 += MAX_CHUNKS) {
        float v[MAX_CHUNKS];
#pragma unroll
        for (int j = 0; j < MAX_CHUNKS; ++j) {
            const float x = chunks[(int64_t)min(w0 + j, nchunks - 1) * (npar + 1) + p];
            v[j] = w0 + j < nchunks ? x : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < MAX_CHUNKS; ++j)
            g += v[j];
    }
    if (p == npar) {
        t.loss_out[0] = g / (float)t.batch;
        return;
    }
    if (t.grad_params)
        t.grad_params[p] = g;
    const float m = 0.9f * t.m_par[p] + 0.1f * g;
    const float v = 0.999f * t.v_par[p] + 0.001f * g * g;
    t.m_par[p] = m;
    t.v_par[p] = v;
    t.params[p] -= t.lr_mlp * (m / t.bc1) / (__builtin_sqrtf(v / t.bc2) + 1e-8f);
}

// ------------------------------------------------------- matrix-core decoder
// Lane l of a 16x16x32 tile: column n = l % 16, K block g = l / 16 (8 K values
// for A and B), accumulator rows 4g..4g+3.  Hidden unit at K position
// 8g + j of K step ks: two accumulator tiles (2ks, 2ks+1) interleaved.
// Layer 1 (C = 8 or 16 inputs) uses the 16x16x16 tile: K block g holds the
// 4 input channels 4g..4g+3, the accumulator layout is the same.
__device__ __forceinline__ int kperm(int ks, int g, int j) { return 16 * (2 * ks + (j >> 2)) + 4 * g + (j & 3); }

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

template <int C, int O>
struct MlpFrags {
    bf16x4 a1[4];
    bf16x8 a2[4][2], a3[2];
    f32x4 b1[4], b2[4], b3;
};

__device__ __forceinline__ float pbf(const uint16_t *P, int i) { return bf16_bits_to_f32(P[i]); }

template <int C, int O>
__device__ __forceinline__ void load_frags(const uint16_t *P, MlpFrags<C, O> &F)
{
    const POff off(C, O);
    const int l = threadIdx.x & 63, n = l & 15, g = l >> 4;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = 4 * g + j;
            F.a1[m][j] = (__bf16)(c < C ? pbf(P, off.w1 + c * HID + 16 * m + n) : 0.0f);
        }
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int j = 0; j < 8; ++j)
                F.a2[m][ks][j] = (__bf16)pbf(P, off.w2 + kperm(ks, g, j) * HID + 16 * m + n);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            F.b1[m][j] = pbf(P, off.b1 + 16 * m + 4 * g + j);
            F.b2[m][j] = pbf(P, off.b2 + 16 * m + 4 * g + j);
        }
    }
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int j = 0; j < 8; ++j)
            F.a3[ks][j] = (__bf16)(n < O ? pbf(P, off.w3 + kperm(ks, g, j) * O + n) : 0.0f);
#pragma unroll
    for (int j = 0; j < 4; ++j)
        F.b3[j] = (4 * g + j < O) ? pbf(P, off.b3 + 4 * g + j) : 0.0f;
}

typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two floats -> one word of two bfloat16 (round to nearest even, one packed
// conversion).
__device__ __forceinline__ uint32_t pack_bf16(float a, float b)
{
    const f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

// A packed word of two bfloat16 with its negative halves (-0 included)
// zeroed: a negative bfloat16 is a negative int16.
__device__ __forceinline__ uint32_t relu_bf16x2(uint32_t w)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, w), (s16x2)0));
}

// bfloat16(max(x, 0)) for eight accumulators: rounding first and rectifying
// the rounded values gives the same numbers.
__device__ __forceinline__ bf16x8 relu_pack(f32x4 lo, f32x4 hi)
{
    const uint4 w = make_uint4(relu_bf16x2(pack_bf16(lo[0], lo[1])), relu_bf16x2(pack_bf16(lo[2], lo[3])),
                               relu_bf16x2(pack_bf16(hi[0], hi[1])), relu_bf16x2(pack_bf16(hi[2], hi[3])));
    return __builtin_bit_cast(bf16x8, w);
}

// Four OCP E4M3 codes (one word) times their block scale s, as the MLP's
// BF16 operands: each code's value (exact in binary32) times s, rounded to
// binary32, then to bfloat16 (nearest even).
__device__ __forceinline__ bf16x4 fp8x4_dequant(uint32_t w, float s)
{
    const f32x2 a0 = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, false), a1 = __builtin_amdgcn_cvt_pk_f32_fp8((int)w, true);
    return __builtin_bit_cast(bf16x4, make_uint2(pack_bf16(a0.x * s, a0.y * s), pack_bf16(a1.x * s, a1.y * s)));
}

// The MLP on the 16 samples whose latents (K block of this lane, BF16, E4M3
// latents already scaled) are in zb; each layer's bias enters its matrix
// product as the accumulator.  Returns the layer-3 accumulators: lanes
// 0..15 hold outputs 0..3 of sample (lane).
template <int C, int O>
__device__ __forceinline__ f32x4 mlp16(const MlpFrags<C, O> &F, bf16x4 zb)
{
    f32x4 d1[4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
        d1[m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(F.a1[m], zb, F.b1[m], 0, 0, 0);
    const bf16x8 h1a = relu_pack(d1[0], d1[1]), h1b = relu_pack(d1[2], d1[3]);
    f32x4 d2[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        d2[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a2[m][0], h1a, F.b2[m], 0, 0, 0);
        d2[m] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a2[m][1], h1b, d2[m], 0, 0, 0);
    }
    const bf16x8 h2a = relu_pack(d2[0], d2[1]), h2b = relu_pack(d2[2], d2[3]);
    f32x4 d3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a3[0], h2a, F.b3, 0, 0, 0);
    d3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(F.a3[1], h2b, d3, 0, 0, 0);
    return d3;
}

// This lane's K block of the latent of lattice point idx as BF16 operands
// (zeros past C, or for idx < 0); blk is the point's scale block (E4M3
// latents).
template <int C, int FMT>
__device__ __forceinline__ bf16x4 latent_frag(const LatentArgs &g, int64_t idx, int blk)
{
    const int kb = (threadIdx.x & 63) >> 4;
    bf16x4 r;
    if (4 * kb >= C || idx < 0) {
#pragma unroll
        for (int j = 0; j < 4; ++j)
            r[j] = (__bf16)0.0f;
        return r;
    }
    if constexpr (FMT == SF_LATENT_BF16) {
        const uint2 v = *reinterpret_cast<const uint2 *>(static_cast<const uint16_t *>(g.latents) + idx * C + 4 * kb);
        r = __builtin_bit_cast(bf16x4, v);
    } else {
        const uint32_t v = *reinterpret_cast<const uint32_t *>(static_cast<const uint8_t *>(g.latents) + idx * C + 4 * kb);
        r = fp8x4_dequant(v, g.scales[blk]);
    }
    return r;
}

// Decode one lattice point per lane for the whole wavefront (every lane must
// take part; idx < 0 marks a lane with nothing to decode).  blk is the
// point's scale block (E4M3 latents only).  Returns this lane's O raw outputs.
template <int C, int O, int FMT>
__device__ __forceinline__ void decode_wave(const LatentArgs &g, const MlpFrags<C, O> &F, int64_t idx, int blk,
                                            float y[O])
{
    const int lane = threadIdx.x & 63;
    // the four groups' latents are gathered first, so their loads overlap
    bf16x4 zb[4];
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const int src = 16 * G + (lane & 15);
        const int64_t sidx = ((int64_t)__shfl((int)(idx >> 32), src) << 32) | (uint32_t)__shfl((int)idx, src);
        const int sblk = FMT == SF_LATENT_BF16 ? 0 : __shfl(blk, src);
        zb[G] = latent_frag<C, FMT>(g, sidx, sblk);
    }
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const f32x4 d3 = mlp16<C, O>(F, zb[G]);
#pragma unroll
        for (int o = 0; o < O; ++o) {
            const float v = __shfl(d3[o], lane & 15);
            if ((lane >> 4) == G)
                y[o] = v;
        }
    }
}

__device__ __forceinline__ int wrapi(int i, int n)
{
    int r = i % n;
    return r < 0 ? r + n : r;
}

// 2-D neural texture lookups (repeat wrap).  Decoded texel = clamp(MLP, 0, 1).
// One query per lane: filter the decoded latent texture at query q (every
// lane of the wave takes part in the decodes; q >= n marks a lane with
// nothing to do).
template <int F_, int SHADE, int MODE, int FMT>
__device__ __forceinline__ void neural2d_query(const NeuralCall &c, const MlpFrags<8, 4> &Fr, int64_t q)
{
    constexpr int C = 8, O = 4;
    const bool active = q < c.n;
    float qx = 0.f, qy = 0.f;
    if (active) {
        qx = c.q[3 * q];
        qy = c.q[3 * q + 1];
    }
    const bool ok = active && __builtin_isfinite(qx) && __builtin_isfinite(qy);
    const int R0 = c.lat.res[0], R1 = c.lat.res[1];
    int ix = 0, iy = 0;
    float tx = 0.f, ty = 0.f;
    if (ok) {
        const float u = qx - __builtin_floorf(qx), v = qy - __builtin_floorf(qy);
        const float px = __builtin_fmaf(u, (float)R0, -0.5f), py = __builtin_fmaf(v, (float)R1, -0.5f);
        const float fx = __builtin_floorf(px), fy = __builtin_floorf(py);
        ix = (int)fx;
        iy = (int)fy;
        tx = px - fx;
        ty = py - fy;
    }
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    float y[O];
    if constexpr (MODE == STOCH) {
        for (int s = 0; s < c.spp; ++s) {
            int64_t idx = -1;
            int blk = 0;
            if (ok) {
                const uint4 w = pcg4d(make_uint4((uint32_t)q, (uint32_t)s, 0u, c.seed));
                const int x = wrapi(ix + pick_off_2p24<F_>(tx, u24i(w.x)), R0);
                const int yy = wrapi(iy + pick_off_2p24<F_>(ty, u24i(w.y)), R1);
                idx = (int64_t)yy * R0 + x;
                blk = c.lat.block_at(x, yy, 0);
                if (c.taps) {
                    c.taps[(q * c.spp + s) * 2] = x;
                    c.taps[(q * c.spp + s) * 2 + 1] = yy;
                }
            } else if (active && c.taps) {
                c.taps[(q * c.spp + s) * 2] = c.taps[(q * c.spp + s) * 2 + 1] = SF_TAP_NONE;
            }
            decode_wave<C, O, FMT>(c.lat, Fr, idx, blk, y);
            float4 d = make_float4(__builtin_fminf(__builtin_fmaxf(y[0], 0.f), 1.f),
                                   __builtin_fminf(__builtin_fmaxf(y[1], 0.f), 1.f),
                                   __builtin_fminf(__builtin_fmaxf(y[2], 0.f), 1.f),
                                   __builtin_fminf(__builtin_fmaxf(y[3], 0.f), 1.f));
            if constexpr (SHADE == SF_SHADE_GGX) {
                const float3 r = shade_ggx_dev(c.g, d);
                acc[0] += r.x;
                acc[1] += r.y;
                acc[2] += r.z;
            } else {
                acc[0] += d.x;
                acc[1] += d.y;
                acc[2] += d.z;
                acc[3] += d.w;
            }
        }
        const float inv = 1.0f / (float)c.spp;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            acc[k] *= inv;
    } else {
        constexpr int NT = Taps<F_>::n;
        constexpr int F0 = Taps<F_>::first;
        float wx[4], wy[4];
        axis_weights<F_>(tx, wx);
        axis_weights<F_>(ty, wy);
        if constexpr (F_ == NEAREST) {
            ix += tx >= 0.5f;
            iy += ty >= 0.5f;
        }
        for (int b = 0; b < NT; ++b)
            for (int a = 0; a < NT; ++a) {
                const int xx = wrapi(ix + F0 + a, R0), yy = wrapi(iy + F0 + b, R1);
                const int64_t idx = ok ? (int64_t)yy * R0 + xx : -1;
                decode_wave<C, O, FMT>(c.lat, Fr, idx, c.lat.block_at(xx, yy, 0), y);
                const float w = wx[a] * wy[b];
                float4 d = make_float4(__builtin_fminf(__builtin_fmaxf(y[0], 0.f), 1.f),
                                       __builtin_fminf(__builtin_fmaxf(y[1], 0.f), 1.f),
                                       __builtin_fminf(__builtin_fmaxf(y[2], 0.f), 1.f),
                                       __builtin_fminf(__builtin_fmaxf(y[3], 0.f), 1.f));
                if (MODE == AFTER && SHADE == SF_SHADE_GGX) {
                    const float3 r = shade_ggx_dev(c.g, d);
                    acc[0] = __builtin_fmaf(w, r.x, acc[0]);
                    acc[1] = __builtin_fmaf(w, r.y, acc[1]);
                    acc[2] = __builtin_fmaf(w, r.z, acc[2]);
                } else {
                    acc[0] = __builtin_fmaf(w, d.x, acc[0]);
                    acc[1] = __builtin_fmaf(w, d.y, acc[1]);
                    acc[2] = __builtin_fmaf(w, d.z, acc[2]);
                    acc[3] = __builtin_fmaf(w, d.w, acc[3]);
                }
            }
        if (MODE == BEFORE && SHADE == SF_SHADE_GGX) {
            const float3 r = shade_ggx_dev(c.g, make_float4(acc[0], acc[1], acc[2], acc[3]));
            acc[0] = r.x;
            acc[1] = r.y;
            acc[2] = r.z;
        }
    }
    if (!active)
        return;
    if (!ok) {
        acc[0] = acc[1] = acc[2] = acc[3] = __builtin_nanf("");
    }
    if constexpr (SHADE == SF_SHADE_GGX) {
        c.out[3 * q] = acc[0];
        c.out[3 * q + 1] = acc[1];
        c.out[3 * q + 2] = acc[2];
    } else {
        reinterpret_cast<float4 *>(c.out)[q] = make_float4(acc[0], acc[1], acc[2], acc[3]);
    }
}

// The MLP's fragments are loaded into registers once per workgroup, which
// then walks the query stream in tiles of 256 (a grid of as many
// workgroups as the device holds at once), so their load is spread over
// several tiles.  The tile base is uniform over the workgroup.

template <int F_, int SHADE, int MODE, int FMT>
__global__ __launch_bounds__(256) void k_neural2d(NeuralCall c)
{
    MlpFrags<8, 4> Fr;
    load_frags<8, 4>(static_cast<const uint16_t *>(c.mlp.params), Fr);
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t base = (int64_t)blockIdx.x * 256; base < c.n; base += stride)
        neural2d_query<F_, SHADE, MODE, FMT>(c, Fr, base + threadIdx.x);
}

// Decoded outputs at given lattice points (no filtering, no clamping).
template <int C, int O, int FMT>
__global__ __launch_bounds__(256) void k_decode_lattice(NeuralCall c, const int64_t *idx_in)
{
    MlpFrags<C, O> Fr;
    load_frags<C, O>(static_cast<const uint16_t *>(c.mlp.params), Fr);
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t npts = (int64_t)c.lat.res[0] * c.lat.res[1] * c.lat.res[2];
    int64_t idx = i < c.n ? idx_in[i] : -1;
    const bool valid = (uint64_t)idx < (uint64_t)npts;
    if (!valid)
        idx = -1;   // outside the lattice: no load, NaN result
    int blk = 0;
    if (FMT != SF_LATENT_BF16 && idx >= 0) {
        const int64_t plane = (int64_t)c.lat.res[0] * c.lat.res[1];
        const int z = (int)(idx / plane), y = (int)((idx % plane) / c.lat.res[0]), x = (int)(idx % c.lat.res[0]);
        blk = c.lat.block_at(x, y, z);
    }
    float y[O];
    decode_wave<C, O, FMT>(c.lat, Fr, idx, blk, y);
    if (i < c.n)
#pragma unroll
        for (int o = 0; o < O; ++o)
            c.out[i * O + o] = valid ? y[o] : __builtin_nanf("");
}

// The march's lattice point of one ray step, per lane: `at` is the byte
// offset of the point's latent (OFF32: the latents span at most 2^31 bytes
// and are read through a buffer resource) or its linear index, and
// kNoLatent (negative as int32) when the tap is outside the lattice or the
// lane has no ray; cs is the point's block scale (E4M3 latents).  The loads
// of one step for the wave's four 16-sample groups are issued before the
// MLPs of the previous step, so one step of gathers stays in flight behind
// the matrix-core work.
constexpr uint32_t kNoLatent = 0x80000000u;

template <int FMT>
struct StepLatents {
    using Raw = typename std::conditional<FMT == SF_LATENT_BF16, uint2, uint32_t>::type;
    Raw raw[4];     // this lane's K block of group G's sample latents, as loaded
    uint32_t at;    // this lane's own point (validity of its sample)
    float cs;       // this lane's own block scale, shuffled to the groups at decode time
};

template <int FMT, bool OFF32>
__device__ __forceinline__ void issue_latents(const LatentArgs &g, __amdgpu_buffer_rsrc_t rs, uint32_t at, float cs,
                                              StepLatents<FMT> &L)
{
    constexpr uint32_t kBytes = FMT == SF_LATENT_BF16 ? 8u : 4u;   // one K block: 4 channels
    const int lane = threadIdx.x & 63, kb = lane >> 4;
    L.at = at;
    L.cs = cs;
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        const uint32_t sat = __shfl(at, 16 * G + (lane & 15));
        if constexpr (OFF32) {
            // a point outside the lattice reads past the buffer's end: zeros
            const uint32_t off = sat + kb * kBytes;
            if constexpr (FMT == SF_LATENT_BF16) {
                typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
                const u32x2 v = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
                L.raw[G] = make_uint2(v.x, v.y);
            } else {
                L.raw[G] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
            }
        } else {
            const uint8_t *p = static_cast<const uint8_t *>(g.latents) + (uint64_t)sat * (4 * kBytes) + kb * kBytes;
            if constexpr (FMT == SF_LATENT_BF16)
                L.raw[G] = (int32_t)sat >= 0 ? *reinterpret_cast<const uint2 *>(p) : make_uint2(0u, 0u);
            else
                L.raw[G] = (int32_t)sat >= 0 ? *reinterpret_cast<const uint32_t *>(p) : 0u;
        }
    }
}

// The wave's MLPs on one step's loaded latents; returns this lane's raw
// output (density before the clamp at zero).
template <int C, int FMT>
__device__ __forceinline__ float decode_loaded(const MlpFrags<C, 1> &F, const StepLatents<FMT> &L)
{
    const int lane = threadIdx.x & 63;
    float y = 0.0f;
#pragma unroll
    for (int G = 0; G < 4; ++G) {
        bf16x4 zb;
        if constexpr (FMT == SF_LATENT_BF16)
            zb = __builtin_bit_cast(bf16x4, L.raw[G]);
        else
            zb = fp8x4_dequant(L.raw[G], __shfl(L.cs, 16 * G + (lane & 15)));
        const f32x4 d3 = mlp16<C, 1>(F, zb);
        const float v = __shfl(d3[0], lane & 15);
        if ((lane >> 4) == G)
            y = v;
    }
    return y;
}

// Ray march through a neural density volume: per step the lookup point's
// picked lattice point is decoded (sigma = max(MLP, 0)); taps outside the
// lattice read zero and are not decoded.  Every lane walks the same number
// of steps so the wavefront can batch its decodes on the matrix cores; the
// step loop is unrolled twice so the two steps' latent registers alternate.
// Three wavefronts per SIMD overlap one wavefront's vector work with
// another's matrix work.
template <int F_, int FMT, bool DBG, bool OFF32>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_neural_ray(NeuralCall c, uint32_t nb_pad)
{
    constexpr int C = 16;
    constexpr uint32_t kPointBytes = FMT == SF_LATENT_BF16 ? 32u : 16u;
    MlpFrags<C, 1> Fr;
    load_frags<C, 1>(static_cast<const uint16_t *>(c.mlp.params), Fr);
    const int64_t i = (int64_t)xcd_block(blockIdx.x, nb_pad) * 256 + threadIdx.x;
    const bool active = i < c.n;
    RayGeom g = {};
    int st = 1;
    if (active)
        st = ray_setup_dev(c.lat.wmin, c.lat.scale, c.rays + 8 * i, c.steps, g);
    const bool march = active && st == 0;
    const uint32_t npts = (uint32_t)c.lat.res[0] * (uint32_t)c.lat.res[1] * (uint32_t)c.lat.res[2];
    __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(c.lat.latents), 0,
                                                                  OFF32 ? (int)(npts * kPointBytes) : 0, kBufferFlags);
    // compensated binary32 sums, as in the plain march
    CompSum Tsum;
    Tsum.init();
    // the block scales through a buffer resource too: an index outside the
    // block array reads zero
    const uint32_t nblk = (uint32_t)c.lat.nblocks();
    __amdgpu_buffer_rsrc_t srs = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(c.lat.scales), 0,
                                                                   FMT != SF_LATENT_BF16 ? (int)(nblk * 4u) : 0,
                                                                   kBufferFlags);
    if (!march)
        g = RayGeom{};   // lanes without a ray walk a dummy ray whose points are all discarded
    // lattice point (and block scale) of step k of this lane's ray.  Computed
    // by every lane without branches, so the compiler can schedule it among
    // the matrix products of the step before; kNoLatent for lanes without a
    // ray, steps past the last and taps outside the lattice.
    auto step_point = [&](const StepHash &h, int k, int s, uint32_t &at, float &cs) {
        int i0[3], o[3];
        float t[3];
        const float kh = (float)k + 0.5f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float p = __builtin_fmaf(kh, g.G[a], g.E[a]);
            const float fl = __builtin_floorf(p);
            i0[a] = (int)fl;
            t[a] = p - fl;
        }
        const uint3 w = h.at((uint32_t)k);
        o[0] = pick_off_2p24<F_>(t[0], u24i(w.x));
        o[1] = pick_off_2p24<F_>(t[1], u24i(w.y));
        o[2] = pick_off_2p24<F_>(t[2], u24i(w.z));
        const int x = i0[0] + o[0], y = i0[1] + o[1], z = i0[2] + o[2];
        if constexpr (DBG) {
            if (march && k < c.steps) {
                int32_t *tp = c.taps + (((int64_t)i * c.spp + s) * c.steps + k) * 3;
                tp[0] = x;
                tp[1] = y;
                tp[2] = z;
            }
        }
        const bool in = march & (k < c.steps) & ((uint32_t)x < (uint32_t)c.lat.res[0]) &
                        ((uint32_t)y < (uint32_t)c.lat.res[1]) & ((uint32_t)z < (uint32_t)c.lat.res[2]);
        const uint32_t pt = ((uint32_t)z * (uint32_t)c.lat.res[1] + (uint32_t)y) * (uint32_t)c.lat.res[0] + (uint32_t)x;
        // (a select written as an OR, which keeps the compiler from branching here)
        at = (OFF32 ? pt * kPointBytes : pt) | ((uint32_t)!in << 31);
        cs = 0.0f;
        if constexpr (FMT != SF_LATENT_BF16)
            cs = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(srs, (uint32_t)c.lat.block_at(x, y, z) * 4u,
                                                                                0, 0));
    };
    for (int s = 0; s < c.spp; ++s) {
        StepHash h;
        h.init((uint32_t)i, (uint32_t)s, c.seed);
        CompSum tau;
        tau.init();
        StepLatents<FMT> A, B;
        uint32_t at;
        float cs;
        step_point(h, 0, s, at, cs);
        issue_latents<FMT, OFF32>(c.lat, rs, at, cs, A);
        for (int k = 0; k < c.steps; k += 2) {
            step_point(h, k + 1, s, at, cs);
            issue_latents<FMT, OFF32>(c.lat, rs, at, cs, B);   // step k+1 in flight
            // adding +0 for a point not decoded leaves the compensated sum as it is
            float y = decode_loaded<C, FMT>(Fr, A);             // step k
            tau.add((int32_t)A.at >= 0 ? __builtin_fmaxf(y, 0.0f) : 0.0f);
            if (k + 1 >= c.steps)
                break;
            step_point(h, k + 2, s, at, cs);
            issue_latents<FMT, OFF32>(c.lat, rs, at, cs, A);   // step k+2 in flight
            y = decode_loaded<C, FMT>(Fr, B);                   // step k+1
            tau.add((int32_t)B.at >= 0 ? __builtin_fmaxf(y, 0.0f) : 0.0f);
        }
        Tsum.add(expf(-(g.dt * tau.value())));
    }
    if (!active)
        return;
    if (st != 0) {
        c.T[i] = st == 1 ? 1.0f : __builtin_nanf("");
        if constexpr (DBG) {
            const int64_t per = (int64_t)3 * c.spp * c.steps;
            for (int64_t k = 0; k < per; ++k)
                c.taps[per * i + k] = SF_TAP_NONE;
        }
        return;
    }
    c.T[i] = Tsum.value() / (float)c.spp;
}

// ---------------------------------------------------------------- launchers
hipError_t launch_to_bf16(const float *in, int64_t n, uint16_t *out, hipStream_t s)
{
    k_to_bf16<<<dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s>>>(in, n, out);
    return hipGetLastError();
}

hipError_t launch_quant_fp8(const float *lat, const LatentArgs &g, uint8_t *codes, float *scales, hipStream_t s)
{
    k_quant_fp8<<<dim3((uint32_t)g.nblocks()), dim3(256), 0, s>>>(lat, g, codes, scales);
    return hipGetLastError();
}

hipError_t launch_train(const TrainCall &t, float *workspace, int nparts, int64_t chunk, hipStream_t s)
{
    if (t.C == 8 && t.O == 4)
        k_train<8, 4, TRAIN_GROUP><<<dim3(nparts), dim3(64), 0, s>>>(t, chunk, workspace);
    else
        k_train<16, 1, TRAIN_GROUP><<<dim3(nparts), dim3(64), 0, s>>>(t, chunk, workspace);
    return launch_train_reduce(t, workspace, nparts, s);
}

hipError_t launch_train_reduce(const TrainCall &t, float *workspace, int nparts, hipStream_t s)
{
    const int npar = POff(t.C, t.O).n;
    const int nchunks = (nparts + REDUCE_CHUNK - 1) / REDUCE_CHUNK;
    float *chunks = workspace + (int64_t)nparts * (npar + 1);
    k_train_chunks<<<dim3((npar + 1 + 255) / 256, nchunks), dim3(256), 0, s>>>(nparts, workspace, npar, chunks);
    k_train_reduce<<<dim3((npar + 1 + 255) / 256), dim3(256), 0, s>>>(t, nchunks, chunks, npar);
    return hipGetLastError();
}

int train_reduce_chunks(int nparts) { return (nparts + REDUCE_CHUNK - 1) / REDUCE_CHUNK; }

int train_nparams(int C, int O) { return POff(C, O).n; }

// Workgroups of 256 lanes of kernel K resident on the current device at
// once (occupancy x compute units), at least 1.
template <typename K>
static int64_t resident_blocks(K kernel)
{
    int dev = 0, ncu = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, 256, 0) != hipSuccess)
        return 1024;
    return std::max<int64_t>(1, (int64_t)std::max(per_cu, 1) * std::max(ncu, 1));
}

template <int F_, int SHADE, int MODE, int FMT>
static void launch_n2_k(const NeuralCall &c, hipStream_t s)
{
    static const int64_t resident = resident_blocks(k_neural2d<F_, SHADE, MODE, FMT>);
    const int64_t tiles = (c.n + 255) / 256;
    k_neural2d<F_, SHADE, MODE, FMT><<<dim3((uint32_t)std::min(tiles, resident)), dim3(256), 0, s>>>(c);
}

template <int F_, int SHADE, int MODE>
static void launch_n2_m(const NeuralCall &c, hipStream_t s)
{
    if (c.lat.fmt == SF_LATENT_BF16)
        launch_n2_k<F_, SHADE, MODE, SF_LATENT_BF16>(c, s);
    else
        launch_n2_k<F_, SHADE, MODE, SF_LATENT_FP8E4M3>(c, s);
}

template <int F_, int SHADE>
static void launch_n2_s(const NeuralCall &c, hipStream_t s)
{
    if (c.mode == STOCH)
        launch_n2_m<F_, SHADE, STOCH>(c, s);
    else if (c.mode == BEFORE)
        launch_n2_m<F_, SHADE, BEFORE>(c, s);
    else
        launch_n2_m<F_, SHADE, AFTER>(c, s);
}

template <int F_>
static void launch_n2_f(const NeuralCall &c, hipStream_t s)
{
    if (c.shade == SF_SHADE_GGX)
        launch_n2_s<F_, SF_SHADE_GGX>(c, s);
    else
        launch_n2_s<F_, SF_SHADE_NONE>(c, s);
}

hipError_t launch_neural2d(const NeuralCall &c, hipStream_t s)
{
    switch (c.filter) {
    case NEAREST:
        launch_n2_f<NEAREST>(c, s);
        break;
    case LINEAR:
        launch_n2_f<LINEAR>(c, s);
        break;
    default:
        launch_n2_f<BSPLINE3>(c, s);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_decode_lattice(const NeuralCall &c, const int64_t *idx, hipStream_t s)
{
    dim3 grid((uint32_t)((c.n + 255) / 256)), block(256);
    if (c.mlp.in_dim == 8) {
        if (c.lat.fmt == SF_LATENT_BF16)
            k_decode_lattice<8, 4, SF_LATENT_BF16><<<grid, block, 0, s>>>(c, idx);
        else
            k_decode_lattice<8, 4, SF_LATENT_FP8E4M3><<<grid, block, 0, s>>>(c, idx);
    } else {
        if (c.lat.fmt == SF_LATENT_BF16)
            k_decode_lattice<16, 1, SF_LATENT_BF16><<<grid, block, 0, s>>>(c, idx);
        else
            k_decode_lattice<16, 1, SF_LATENT_FP8E4M3><<<grid, block, 0, s>>>(c, idx);
    }
    return hipGetLastError();
}

// SF_NEURAL_ADDR64=1 in the environment sends every neural march through
// the 64-bit addressing variant that lattices of more than 2^31 bytes of
// latents take (so tests can run it on small lattices).
static bool addr64_forced()
{
    const char *e = getenv("SF_NEURAL_ADDR64");
    return e && e[0] == '1';
}

template <int F_, int FMT>
static void launch_nr_m(const NeuralCall &c, hipStream_t s, dim3 grid, uint32_t nb_pad)
{
    dim3 block(256);
    const uint64_t bytes = (uint64_t)c.lat.res[0] * c.lat.res[1] * c.lat.res[2] * (FMT == SF_LATENT_BF16 ? 32u : 16u);
    const bool off32 = bytes <= (uint64_t)kNoLatent && !addr64_forced();
    if (c.taps) {
        if (off32)
            k_neural_ray<F_, FMT, true, true><<<grid, block, 0, s>>>(c, nb_pad);
        else
            k_neural_ray<F_, FMT, true, false><<<grid, block, 0, s>>>(c, nb_pad);
    } else {
        if (off32)
            k_neural_ray<F_, FMT, false, true><<<grid, block, 0, s>>>(c, nb_pad);
        else
            k_neural_ray<F_, FMT, false, false><<<grid, block, 0, s>>>(c, nb_pad);
    }
}

template <int F_>
static void launch_nr_f(const NeuralCall &c, hipStream_t s, dim3 grid, uint32_t nb_pad)
{
    if (c.lat.fmt == SF_LATENT_BF16)
        launch_nr_m<F_, SF_LATENT_BF16>(c, s, grid, nb_pad);
    else
        launch_nr_m<F_, SF_LATENT_FP8E4M3>(c, s, grid, nb_pad);
}

hipError_t launch_neural_ray(const NeuralCall &c, hipStream_t s)
{
    const uint32_t nb = (uint32_t)((c.n + 255) / 256);
    const uint32_t nb_pad = (nb + 7u) & ~7u;
    dim3 grid(nb_pad);
    switch (c.filter) {
    case NEAREST:
        launch_nr_f<NEAREST>(c, s, grid, nb_pad);
        break;
    case LINEAR:
        launch_nr_f<LINEAR>(c, s, grid, nb_pad);
        break;
    default:
        launch_nr_f<BSPLINE3>(c, s, grid, nb_pad);
        break;
    }
    return hipGetLastError();
}

}  // namespace sfk
