// Benchmark-only library libsf_bench.so (not part of libsf: nothing in
// include/ declares it, and no product path loads it).
//
// Issue rates of single vector-ALU instructions: each lane runs kIter passes
// over kChains independent chains of one instruction (written in inline
// assembly so that the instruction and its operand kinds are exactly those
// named), with no memory access but one store of the chains' xor per lane.
// The wall time of a launch that keeps 32 wavefronts on every compute unit
// gives the compute-unit cycles one wave64 instruction of that kind takes:
// the ceiling of a kernel whose instructions are all of that kind.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sfb {

constexpr int kIter = 2000;
constexpr int kChains = 8;

// %0 the chain's value, %1 a wave-uniform value in a scalar register, %2 the
// next chain's value, %3 a loop-invariant vector register
#define SFB_RATE_KERNEL(NAME, INS, T, INIT, ...)                                                     \
    __global__ __launch_bounds__(256) void NAME(uint32_t *out, uint32_t s)                          \
    {                                                                                                \
        T a[kChains];                                                                                \
        for (int c = 0; c < kChains; ++c)                                                            \
            a[c] = INIT;                                                                             \
        T inv;                                                                                       \
        asm volatile("v_mov_b32 %0, %1" : "=v"(inv) : "s"(s));                                      \
        for (int i = 0; i < kIter; ++i) {                                                            \
            _Pragma("unroll") for (int c = 0; c < kChains; ++c)                                      \
                asm volatile(INS : "+v"(a[c]) : "s"(s), "v"(a[(c + 1) % kChains]), "v"(inv) __VA_ARGS__); \
        }                                                                                            \
        uint32_t r = 0;                                                                              \
        for (int c = 0; c < kChains; ++c)                                                            \
            r ^= __builtin_bit_cast(uint32_t, a[c]);                                                 \
        out[blockIdx.x * blockDim.x + threadIdx.x] = r;                                              \
    }

SFB_RATE_KERNEL(k_fma_vvv, "v_fma_f32 %0, %0, %2, %3", float, 1.0f + (float)threadIdx.x)
SFB_RATE_KERNEL(k_fma_vvs, "v_fma_f32 %0, %0, %2, %1", float, 1.0f + (float)threadIdx.x)
SFB_RATE_KERNEL(k_mul_f32_vv, "v_mul_f32 %0, %0, %2", float, 1.0f + (float)threadIdx.x)
SFB_RATE_KERNEL(k_add_u32_vv, "v_add_u32 %0, %3, %0", uint32_t, threadIdx.x + c)
SFB_RATE_KERNEL(k_add_u32_sv, "v_add_u32 %0, %1, %0", uint32_t, threadIdx.x + c)
SFB_RATE_KERNEL(k_max_f32_vv, "v_max_f32 %0, %0, %2", float, 1.0f + (float)threadIdx.x)
SFB_RATE_KERNEL(k_cvt_f32_u32, "v_cvt_f32_u32 %0, %0", uint32_t, threadIdx.x + c)
SFB_RATE_KERNEL(k_cmp_f32, "v_cmp_le_f32 vcc, %0, %2", float, 1.0f + (float)threadIdx.x, : "vcc")
SFB_RATE_KERNEL(k_bfe_u32, "v_bfe_u32 %0, %0, %2, 1", uint32_t, threadIdx.x + c)
SFB_RATE_KERNEL(k_mad_u64_u32, "v_mad_u64_u32 v[40:41], vcc, %0, %3, 0", uint32_t, threadIdx.x + c,
                : "vcc", "v40", "v41")
SFB_RATE_KERNEL(k_xor_sdwa,
                "v_xor_b32_sdwa %0, %0, %0 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:WORD_1 src1_sel:DWORD",
                uint32_t, threadIdx.x + c)
SFB_RATE_KERNEL(k_exp_f32, "v_exp_f32 %0, %0", float, 1.0f + (float)threadIdx.x)

// two instructions per chain step: a binary32 add and a slower-class
// instruction on another register
SFB_RATE_KERNEL(k_add_cvt, "v_add_f32 %0, %0, %2\n\tv_cvt_f32_u32 v40, %0", float, 1.0f + (float)threadIdx.x, : "v40")
SFB_RATE_KERNEL(k_add_cmp, "v_add_f32 %0, %0, %2\n\tv_cmp_le_f32 vcc, %0, %3", float, 1.0f + (float)threadIdx.x,
                : "vcc")

#undef SFB_RATE_KERNEL

typedef void (*RateKernel)(uint32_t *, uint32_t);
struct Case {
    const char *name;
    RateKernel k;
};
const Case kCases[] = {
    {"v_fma_f32 v,v,v", k_fma_vvv},
    {"v_fma_f32 v,v,s", k_fma_vvs},
    {"v_mul_f32 v,v", k_mul_f32_vv},
    {"v_add_u32 v,v", k_add_u32_vv},
    {"v_add_u32 s,v", k_add_u32_sv},
    {"v_max_f32 v,v", k_max_f32_vv},
    {"v_cvt_f32_u32 v", k_cvt_f32_u32},
    {"v_cmp_le_f32 vcc,v,v", k_cmp_f32},
    {"v_bfe_u32 v,v,1", k_bfe_u32},
    {"v_mad_u64_u32 v,v,0", k_mad_u64_u32},
    {"v_xor_b32 sdwa", k_xor_sdwa},
    {"v_exp_f32 v", k_exp_f32},
    {"v_add_f32 v,v + v_cvt_f32_u32 (pairs)", k_add_cvt},
    {"v_add_f32 v,v + v_cmp_le_f32 (pairs)", k_add_cmp},
};

}  // namespace sfb

// Number of cases, and the name of case `which` (NULL outside 0..n-1).
extern "C" int sfb_valu_rate_cases(void) { return (int)(sizeof(sfb::kCases) / sizeof(sfb::kCases[0])); }
extern "C" const char *sfb_valu_rate_name(int which)
{
    return which >= 0 && which < sfb_valu_rate_cases() ? sfb::kCases[which].name : nullptr;
}

// One launch of case `which`: blocks x 256 lanes, each writing one uint32 to
// out (blocks * 256 words, device memory).  Wave64 instructions per lane:
// kIter * kChains (the value sfb_valu_rate_insts returns), twice that for the
// cases named "(pairs)".  Returns 0, -1
// for arguments outside these limits, or the HIP error of the launch.
extern "C" int sfb_valu_rate_insts(void) { return sfb::kIter * sfb::kChains; }
extern "C" int sfb_valu_rate_launch(int which, uint32_t *out, int blocks, void *stream)
{
    if (which < 0 || which >= sfb_valu_rate_cases() || !out || blocks < 1)
        return -1;
    sfb::kCases[which].k<<<dim3(blocks), dim3(256), 0, (hipStream_t)stream>>>(out, 3u);
    return (int)hipGetLastError();
}
