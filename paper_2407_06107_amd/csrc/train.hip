// Neural training step on the matrix cores (the learned stand-in's
// autodecoder: lattice latents z_c and the MLP D(z) = W3^T relu(W2^T
// relu(W1^T z + b1) + b2) + b3, loss (1/B) sum_s ||D(z_s) - t_s||^2).
//
// BF16 operands, FP32 accumulation, FP32 master copies of latents and
// parameters (and their Adam moments).  One wavefront walks a chunk of the
// batch in tiles of 16 samples:
//  - forward and backward products are 16-row tiles of hidden units times
//    the 16 samples as columns (v_mfma_f32_16x16x16_bf16 for the 8/16-input
//    and the <= 4-output layers, v_mfma_f32_16x16x32_bf16 for the 64 x 64
//    layers), so one product's accumulators are, lane for lane, the next
//    product's B operand (the weights' K order is permuted to match);
//  - weight gradients sum over samples, so the tile's activations and
//    pre-activation gradients go through LDS in [sample][feature] order and
//    come back as A / B operands whose K dimension is the 16 samples;
//    the wavefront's dW accumulators stay in registers over its whole chunk;
//  - bias gradients and the loss are per-lane sums reduced once at the end;
//  - each sample's latent gradient (16 x 16 tile: channels x samples) gets
//    its Adam step at once (batch entries own distinct latents).
// The per-wavefront parameter gradients are then summed in a fixed order and
// Adam moves the parameters (the same second stage as the FP32 path).
#include "sf_device.hpp"
#include "sf_internal.hpp"

#pragma clang fp contract(off)

namespace sfk {

namespace {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

constexpr int H = 64;

// Packed parameter offsets: W1 [C x H], b1 [H], W2 [H x H], b2 [H], W3 [H x O], b3 [O].
struct Off {
    int w1, b1, w2, b2, w3, b3, n;
    __device__ Off(int C, int O)
    {
        w1 = 0;
        b1 = C * H;
        w2 = b1 + H;
        b2 = w2 + H * H;
        w3 = b2 + H;
        b3 = w3 + H * O;
        n = b3 + O;
    }
};

// B-operand K position 8g + j of K step ks of a 16x16x32 product whose B
// operand is the previous product's accumulators (tiles 2ks, 2ks+1, rows
// 4g..4g+3): hidden unit 16 (2 ks + j/4) + 4 g + j%4.
__device__ __forceinline__ int kp(int ks, int g, int j) { return 16 * (2 * ks + (j >> 2)) + 4 * g + (j & 3); }

__device__ __forceinline__ uint32_t pk(float a, float b)
{
    const f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}

__device__ __forceinline__ uint32_t relu2(uint32_t w)
{
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(s16x2, w), (s16x2)0));
}

__device__ __forceinline__ bf16x4 to_bf16x4(f32x4 v)
{
    return __builtin_bit_cast(bf16x4, make_uint2(pk(v[0], v[1]), pk(v[2], v[3])));
}

// two accumulator tiles -> one 8-wide B operand; RELU rectifies the rounded
// values (the same numbers as rounding the rectified ones)
template <bool RELU>
__device__ __forceinline__ uint4 pack8(f32x4 lo, f32x4 hi)
{
    uint4 w = make_uint4(pk(lo[0], lo[1]), pk(lo[2], lo[3]), pk(hi[0], hi[1]), pk(hi[2], hi[3]));
    if constexpr (RELU) {
        w.x = relu2(w.x);
        w.y = relu2(w.y);
        w.z = relu2(w.z);
        w.w = relu2(w.w);
    }
    return w;
}

__device__ __forceinline__ bf16x8 as8(uint4 w) { return __builtin_bit_cast(bf16x8, w); }

__device__ __forceinline__ __bf16 bw(const float *P, int i) { return (__bf16)P[i]; }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// LDS rows of 16-bit values, [sample][feature]; RS keeps rows 8-byte
// aligned and spreads the column reads of a fragment over the banks.
constexpr int RS = H + 4, RS16 = 16 + 4;

// A / B fragment of a K = 16-sample product: feature column f, samples
// 4g..4g+3.
template <int STRIDE>
__device__ __forceinline__ bf16x4 col4(const uint16_t *s, int g, int f)
{
    const uint32_t a = s[(4 * g) * STRIDE + f], b = s[(4 * g + 1) * STRIDE + f];
    const uint32_t c = s[(4 * g + 2) * STRIDE + f], d = s[(4 * g + 3) * STRIDE + f];
    return __builtin_bit_cast(bf16x4, make_uint2(a | (b << 16), c | (d << 16)));
}

__device__ __forceinline__ float sum16(float v)
{
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    v += __shfl_xor(v, 4);
    v += __shfl_xor(v, 8);
    return v;
}

}  // namespace

template <int C, int O>
__global__ __launch_bounds__(64) void k_train_mfma(TrainCall t, int64_t chunk, float *partials)
{
    static_assert(C == 8 || C == 16, "8 or 16 latent channels");
    static_assert(O >= 1 && O <= 4, "at most 4 outputs");
    __shared__ __attribute__((aligned(16))) uint16_t sH1[16 * RS], sA2[16 * RS], sA1[16 * RS], sH2[16 * RS];
    __shared__ __attribute__((aligned(16))) uint16_t sZ[16 * RS16], sY[16 * RS16];
    const Off P(C, O);
    const float *W = t.params;
    const int l = threadIdx.x, n = l & 15, g = l >> 4;

    // weight fragments (BF16 of the FP32 master parameters)
    bf16x4 a1f[4], ab3[4];
    bf16x8 a2f[4][2], ab2[4][2], a3f[2], ab1[2];
    f32x4 b1i[4], b2i[4], b3i;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int c = 4 * g + j, o = 4 * g + j;
            a1f[m][j] = c < C ? bw(W, P.w1 + c * H + 16 * m + n) : (__bf16)0.0f;          // W1[c][16m+n]
            ab3[m][j] = o < O ? bw(W, P.w3 + (16 * m + n) * O + o) : (__bf16)0.0f;        // W3[16m+n][o]
            b1i[m][j] = W[P.b1 + 16 * m + 4 * g + j];
            b2i[m][j] = W[P.b2 + 16 * m + 4 * g + j];
        }
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                a2f[m][ks][j] = bw(W, P.w2 + kp(ks, g, j) * H + 16 * m + n);   // W2[k][16m+n]
                ab2[m][ks][j] = bw(W, P.w2 + (16 * m + n) * H + kp(ks, g, j));   // W2[16m+n][k]
            }
    }
#pragma unroll
    for (int ks = 0; ks < 2; ++ks)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            a3f[ks][j] = n < O ? bw(W, P.w3 + kp(ks, g, j) * O + n) : (__bf16)0.0f;   // W3[k][n]
            ab1[ks][j] = n < C ? bw(W, P.w1 + n * H + kp(ks, g, j)) : (__bf16)0.0f;   // W1[n][k]
        }
#pragma unroll
    for (int j = 0; j < 4; ++j)
        b3i[j] = 4 * g + j < O ? W[P.b3 + 4 * g + j] : 0.0f;

    const f32x4 zero = {0.0f, 0.0f, 0.0f, 0.0f};
    f32x4 gw2[4][4], gw1[4], gw3[4];
    float gb1[4][4], gb2[4][4], gb3[4], loss = 0.0f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gw1[a] = zero;
        gw3[a] = zero;
        gb3[a] = 0.0f;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            gw2[a][b] = zero;
            gb1[a][b] = gb2[a][b] = 0.0f;
        }
    }

    const float inv_b = 2.0f / (float)t.batch;
    const int64_t s0 = (int64_t)blockIdx.x * chunk;
    const int64_t s1 = min(s0 + chunk, t.batch);
    // The tiles are software-pipelined: the batch indices of tile k+2 and
    // the latents, targets and latent Adam moments of tile k+1 are loaded
    // while tile k computes (batch entries own distinct latents, so the
    // Adam step of tile k never writes what tile k+1 has read).
    // Batch index of this lane's column of the tile at sb (an address inside
    // the chunk also past its end).
    auto index_at = [&](int64_t sb) -> int32_t { return t.idx[min(sb + n, s1 - 1)]; };
    struct TileIn {
        bool use;       // the column holds a sample of the chunk inside the lattice
        int64_t si, p;  // its batch entry and lattice point (0 for unused columns)
        f32x4 z, mq, vq;
        float tg[4];
    };
    // unused columns read element 0 and contribute nothing
    auto load_tile = [&](int64_t sb, int32_t raw, TileIn &T) {
        T.si = sb + n;
        T.use = T.si < s1 && (uint64_t)(int64_t)raw < (uint64_t)t.n_lattice;
        T.p = T.use ? (int64_t)raw : 0;
        T.z = zero;
        T.mq = zero;
        T.vq = zero;
        if (4 * g < C) {
            const int64_t q = T.p * C + 4 * g;
            T.z = *reinterpret_cast<const f32x4 *>(t.latents + q);
            T.mq = *reinterpret_cast<const f32x4 *>(t.m_lat + q);
            T.vq = *reinterpret_cast<const f32x4 *>(t.v_lat + q);
        }
#pragma unroll
        for (int o = 0; o < 4; ++o)
            T.tg[o] = (g == 0 && o < O) ? t.targets[T.p * O + o] : 0.0f;
    };
    TileIn cur, nxt;
    int32_t raw_next = 0;
    if (s0 < s1) {
        load_tile(s0, index_at(s0), cur);
        raw_next = index_at(s0 + 16);
    }
    for (int64_t sb = s0; sb < s1; sb += 16) {
        if (sb + 16 < s1)
            load_tile(sb + 16, raw_next, nxt);   // tile k+1
        raw_next = index_at(sb + 32);             // tile k+2
        const bool use = cur.use;
        const int64_t si = cur.si, p = cur.p;
        // finite inputs for unused columns, so that their zero gradients stay zero
        const f32x4 z = use ? cur.z : zero;
        const float *tg = cur.tg;
        const bf16x4 zb = to_bf16x4(z);

        // forward: A1, H1, A2, H2, Y (columns = samples)
        f32x4 a1[4], a2[4];
#pragma unroll
        for (int m = 0; m < 4; ++m)
            a1[m] = mfma16(a1f[m], zb, b1i[m]);
        const uint4 h1w[2] = {pack8<true>(a1[0], a1[1]), pack8<true>(a1[2], a1[3])};
#pragma unroll
        for (int m = 0; m < 4; ++m)
            a2[m] = mfma32(a2f[m][1], as8(h1w[1]), mfma32(a2f[m][0], as8(h1w[0]), b2i[m]));
        const uint4 h2w[2] = {pack8<true>(a2[0], a2[1]), pack8<true>(a2[2], a2[3])};
        const f32x4 y = mfma32(a3f[1], as8(h2w[1]), mfma32(a3f[0], as8(h2w[0]), b3i));

        // dL/dY on rows 4g + j < O (lanes g = 0)
        f32x4 dy = zero;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const bool row = g == 0 && j < O && use;
            const float e = y[j] - tg[j];
            loss = row ? __builtin_fmaf(e, e, loss) : loss;
            dy[j] = row ? e * inv_b : 0.0f;
            gb3[j] += dy[j];
        }
        const bf16x4 dyb = to_bf16x4(dy);

        // backward: dA2 = W3 dY (rectified), dA1 = W2 dA2 (rectified), dZ = W1 dA1
        f32x4 da2[4], da1[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const f32x4 d = mfma16(ab3[m], dyb, zero);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                da2[m][j] = a2[m][j] > 0.0f ? d[j] : 0.0f;
                gb2[m][j] += da2[m][j];
            }
        }
        const uint4 d2w[2] = {pack8<false>(da2[0], da2[1]), pack8<false>(da2[2], da2[3])};
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const f32x4 d = mfma32(ab2[m][1], as8(d2w[1]), mfma32(ab2[m][0], as8(d2w[0]), zero));
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                da1[m][j] = a1[m][j] > 0.0f ? d[j] : 0.0f;
                gb1[m][j] += da1[m][j];
            }
        }
        const uint4 d1w[2] = {pack8<false>(da1[0], da1[1]), pack8<false>(da1[2], da1[3])};
        const f32x4 dz = mfma32(ab1[1], as8(d1w[1]), mfma32(ab1[0], as8(d1w[0]), zero));

        // the latent's gradient (channels 4g..4g+3 of sample n) and its Adam step
        if (use && 4 * g < C) {
            if (t.grad_latents)
                *reinterpret_cast<f32x4 *>(t.grad_latents + si * C + 4 * g) = dz;
            const int64_t q = p * C + 4 * g;
            const f32x4 mq = cur.mq, vq = cur.vq;
            f32x4 mo, vo, zo;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                mo[j] = 0.9f * mq[j] + 0.1f * dz[j];
                vo[j] = 0.999f * vq[j] + 0.001f * dz[j] * dz[j];
                // bias corrections by the reciprocals, the step by the hardware
                // square root and reciprocal (1 ulp each)
                const float den = __builtin_amdgcn_sqrtf(vo[j] * t.inv_bc2) + 1e-8f;
                zo[j] = z[j] - t.lr_latent * (mo[j] * t.inv_bc1) * __builtin_amdgcn_rcpf(den);
            }
            *reinterpret_cast<f32x4 *>(t.m_lat + q) = mo;
            *reinterpret_cast<f32x4 *>(t.v_lat + q) = vo;
            *reinterpret_cast<f32x4 *>(t.latents + q) = zo;
        }

        // stage the tile in LDS as [sample][feature]
        {
            uint2 *h1 = reinterpret_cast<uint2 *>(sH1 + n * RS + 4 * g);
            uint2 *h2 = reinterpret_cast<uint2 *>(sH2 + n * RS + 4 * g);
            uint2 *e2 = reinterpret_cast<uint2 *>(sA2 + n * RS + 4 * g);
            uint2 *e1 = reinterpret_cast<uint2 *>(sA1 + n * RS + 4 * g);
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                h1[(32 * ks) / 4] = make_uint2(h1w[ks].x, h1w[ks].y);        // tile 2ks
                h1[(32 * ks + 16) / 4] = make_uint2(h1w[ks].z, h1w[ks].w);   // tile 2ks+1
                h2[(32 * ks) / 4] = make_uint2(h2w[ks].x, h2w[ks].y);
                h2[(32 * ks + 16) / 4] = make_uint2(h2w[ks].z, h2w[ks].w);
                e2[(32 * ks) / 4] = make_uint2(d2w[ks].x, d2w[ks].y);
                e2[(32 * ks + 16) / 4] = make_uint2(d2w[ks].z, d2w[ks].w);
                e1[(32 * ks) / 4] = make_uint2(d1w[ks].x, d1w[ks].y);
                e1[(32 * ks + 16) / 4] = make_uint2(d1w[ks].z, d1w[ks].w);
            }
            *reinterpret_cast<uint2 *>(sZ + n * RS16 + 4 * g) = __builtin_bit_cast(uint2, zb);
            *reinterpret_cast<uint2 *>(sY + n * RS16 + 4 * g) = __builtin_bit_cast(uint2, dyb);
        }
        __syncthreads();
        // weight gradients, K = the tile's 16 samples
        bf16x4 ca[4], cb[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            ca[m] = col4<RS>(sH1, g, 16 * m + n);   // H1[16m+n][s]
            cb[m] = col4<RS>(sA2, g, 16 * m + n);   // dA2[16m+n][s]
        }
#pragma unroll
        for (int mi = 0; mi < 4; ++mi)
#pragma unroll
            for (int mo = 0; mo < 4; ++mo)
                gw2[mi][mo] = mfma16(ca[mi], cb[mo], gw2[mi][mo]);
        const bf16x4 zc = col4<RS16>(sZ, g, n);      // Z[n][s]
#pragma unroll
        for (int m = 0; m < 4; ++m)
            gw1[m] = mfma16(zc, col4<RS>(sA1, g, 16 * m + n), gw1[m]);
        const bf16x4 yc = col4<RS16>(sY, g, n);      // dY[n][s]
#pragma unroll
        for (int m = 0; m < 4; ++m)
            gw3[m] = mfma16(col4<RS>(sH2, g, 16 * m + n), yc, gw3[m]);
        __syncthreads();
        cur = nxt;
    }

    // this wavefront's partial gradients in the packed layout, then the loss
    float *out = partials + (int64_t)blockIdx.x * (P.n + 1);
#pragma unroll
    for (int mi = 0; mi < 4; ++mi)
#pragma unroll
        for (int mo = 0; mo < 4; ++mo)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                out[P.w2 + (16 * mi + 4 * g + j) * H + 16 * mo + n] = gw2[mi][mo][j];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (4 * g + j < C)
                out[P.w1 + (4 * g + j) * H + 16 * m + n] = gw1[m][j];
            if (n < O)
                out[P.w3 + (16 * m + 4 * g + j) * O + n] = gw3[m][j];
            // bias sums over the lanes of one row group (same g, all columns n)
            const float s1v = sum16(gb1[m][j]), s2v = sum16(gb2[m][j]);
            if (n == 0) {
                out[P.b1 + 16 * m + 4 * g + j] = s1v;
                out[P.b2 + 16 * m + 4 * g + j] = s2v;
            }
        }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float s3 = sum16(gb3[j]);
        if (l == 0 && j < O)
            out[P.b3 + j] = s3;
    }
    float lsum = loss;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        lsum += __shfl_xor(lsum, m);
    if (l == 0)
        out[P.n] = lsum;
}

hipError_t launch_train_mfma(const TrainCall &t, float *partials, int nparts, int64_t chunk, hipStream_t s)
{
    if (t.C == 8 && t.O == 4)
        k_train_mfma<8, 4><<<dim3(nparts), dim3(64), 0, s>>>(t, chunk, partials);
    else
        k_train_mfma<16, 1><<<dim3(nparts), dim3(64), 0, s>>>(t, chunk, partials);
    return hipGetLastError();
}

}  // namespace sfk
