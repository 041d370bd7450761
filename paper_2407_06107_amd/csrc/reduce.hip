// Float64 error statistics of an estimate against a reference (the MSE
// measure of Sec. 5), reduced on the GPU in a fixed order: each block folds a
// fixed strided slice in lane order, then a fixed tree in LDS, then one block
// folds the per-block partials in order.  The result is bit-reproducible for
// a given (count, block count).
#include "sf_internal.hpp"

namespace sfk {

constexpr int kStats = 8;  // sum e^2, sum e, max|e|, max|e|/|r|, count, sum r^2, non-finite, unused

struct Acc {
    double v[kStats];
};

__device__ __forceinline__ void acc_init(Acc &a)
{
#pragma unroll
    for (int k = 0; k < kStats; ++k)
        a.v[k] = 0.0;
}

__device__ __forceinline__ void acc_merge(Acc &a, const Acc &b)
{
    a.v[0] += b.v[0];
    a.v[1] += b.v[1];
    a.v[2] = fmax(a.v[2], b.v[2]);
    a.v[3] = fmax(a.v[3], b.v[3]);
    a.v[4] += b.v[4];
    a.v[5] += b.v[5];
    a.v[6] += b.v[6];
}

__device__ void block_reduce(Acc &a, double *lds /* 256 * kStats */)
{
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < kStats; ++k)
        lds[k * 256 + t] = a.v[k];
    __syncthreads();
    for (int m = 128; m >= 1; m >>= 1) {
        if (t < m) {
            Acc b;
#pragma unroll
            for (int k = 0; k < kStats; ++k) {
                a.v[k] = lds[k * 256 + t];
                b.v[k] = lds[k * 256 + t + m];
            }
            acc_merge(a, b);
#pragma unroll
            for (int k = 0; k < kStats; ++k)
                lds[k * 256 + t] = a.v[k];
        }
        __syncthreads();
    }
    if (t == 0)
#pragma unroll
        for (int k = 0; k < kStats; ++k)
            a.v[k] = lds[k * 256];
}

__global__ __launch_bounds__(256) void k_err_partial(const float *est, const double *ref, int64_t count,
                                                     double *partials)
{
    __shared__ double lds[256 * kStats];
    Acc a;
    acc_init(a);
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count; i += stride) {
        double e = (double)est[i];
        double r = ref[i];
        if (!__builtin_isfinite(e) || !__builtin_isfinite(r)) {
            a.v[6] += 1.0;
            continue;
        }
        double d = e - r;
        a.v[0] += d * d;
        a.v[1] += d;
        a.v[2] = fmax(a.v[2], fabs(d));
        if (r != 0.0)
            a.v[3] = fmax(a.v[3], fabs(d) / fabs(r));
        a.v[4] += 1.0;
        a.v[5] += r * r;
    }
    block_reduce(a, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < kStats; ++k)
            partials[(int64_t)blockIdx.x * kStats + k] = a.v[k];
}

__global__ __launch_bounds__(256) void k_err_final(const double *partials, int nblocks, double *out)
{
    __shared__ double lds[256 * kStats];
    Acc a;
    acc_init(a);
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        Acc p;
        for (int k = 0; k < kStats; ++k)
            p.v[k] = partials[(int64_t)b * kStats + k];
        acc_merge(a, p);
    }
    block_reduce(a, lds);
    if (threadIdx.x == 0)
        for (int k = 0; k < kStats; ++k)
            out[k] = a.v[k];
}

hipError_t launch_error_stats(const float *est, const double *ref, int64_t count, int32_t ch, double *out,
                              double *partials, int32_t nblocks, hipStream_t s)
{
    (void)ch;
    k_err_partial<<<dim3(nblocks), dim3(256), 0, s>>>(est, ref, count, partials);
    k_err_final<<<dim3(1), dim3(256), 0, s>>>(partials, nblocks, out);
    return hipGetLastError();
}

}  // namespace sfk
