// Microbenchmarks of the ceilings of include/fdk_peaks.h: HBM stream read,
// LDS reads (plain widths and the back-projector's own tap patterns) and the
// float32 FMA issue rate.  The values read or computed are folded into one
// word so that no load or FMA can be dropped; `sink` is written only when that
// word takes a value the inputs never produce.
#include <hip/hip_runtime.h>

#include "fdk_peaks.h"
#include "internal.h"

namespace fdk {
namespace {

constexpr int kPT = 256;                 // threads per block
constexpr int kLdsWords = 8192;          // 32 KiB of LDS per block
constexpr int kReads = 16;               // LDS read instructions per lane per iteration
constexpr unsigned kNever = 0x9e3779b9u; // checksum value that triggers the sink write

__global__ __launch_bounds__(kPT) void hbm_read_kernel(const uint4* __restrict__ p, int64_t n,
                                                       unsigned* sink)
{
    const int64_t stride = (int64_t)gridDim.x * kPT;
    int64_t i = (int64_t)blockIdx.x * kPT + threadIdx.x;
    unsigned a = 0u;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const uint4 x0 = p[i], x1 = p[i + stride], x2 = p[i + 2 * stride], x3 = p[i + 3 * stride];
        a ^= x0.x ^ x0.y ^ x0.z ^ x0.w ^ x1.x ^ x1.y ^ x1.z ^ x1.w;
        a ^= x2.x ^ x2.y ^ x2.z ^ x2.w ^ x3.x ^ x3.y ^ x3.z ^ x3.w;
    }
    for (; i < n; i += stride) {
        const uint4 x = p[i];
        a ^= x.x ^ x.y ^ x.z ^ x.w;
    }
    if (a == kNever) sink[0] = a;
}

// Word offsets of the 16 read steps of an iteration (kernel arguments, so the
// compiler can neither merge nor fold reads it cannot prove distinct).
struct LdsSteps {
    int off[kReads];
};

template <int MODE>
__global__ __launch_bounds__(kPT) void lds_read_kernel(int iters, const LdsSteps S, unsigned* sink)
{
    __shared__ unsigned buf[kLdsWords];
    // single-width reads through a volatile view: one instruction per read,
    // immediate offsets, no pairing into ds_read2
    typedef __attribute__((address_space(3))) volatile unsigned lds_vu32;
    typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
    typedef __attribute__((address_space(3))) volatile u32x2 lds_vu64;
    lds_vu32* vbuf = (lds_vu32*)(size_t)(__attribute__((address_space(3))) unsigned*)buf;
    const unsigned lds_base = (unsigned)(size_t)(__attribute__((address_space(3))) unsigned*)buf;
    for (int i = threadIdx.x; i < kLdsWords; i += kPT) buf[i] = (unsigned)i * 2654435761u + blockIdx.x;
    __syncthreads();
    const int tid = threadIdx.x, lane = tid & 63;
    // column of voxel (lx, ly) of a 16 x 16 tile at 1.6 pixels per voxel, 30 degrees
    const int lx = tid & 15, ly = tid >> 4;
    const int col = 2 + (int)(1.6f * (0.8660254f * (float)lx + 0.5f * (float)ly));
    unsigned a = 0u, b = 0u;
    for (int it = 0; it < iters; ++it) {
        asm volatile("" ::: "memory");   // the reads are repeated every iteration
#pragma unroll
        for (int q = 0; q < kReads; ++q) {
            if constexpr (MODE == FDK_LDS_B32) {
                a ^= vbuf[lane + 64 * q];
            } else if constexpr (MODE == FDK_LDS_READ2_B32) {
                const int w = lane + 8 * (q & 7) + 1024 * (q >> 3);
                a ^= buf[w];
                b ^= buf[w + 36];
            } else if constexpr (MODE == FDK_LDS_B64) {
                const u32x2 x = ((lds_vu64*)vbuf)[lane + 64 * q];
                a ^= x.x;
                b ^= x.y;
            } else if constexpr (MODE == FDK_LDS_B128) {
                const uint4 x = reinterpret_cast<const uint4*>(buf)[lane + 64 * q];
                a ^= x.x ^ x.y;
                b ^= x.z ^ x.w;
            } else if constexpr (MODE == FDK_LDS_B64_ASM || MODE == FDK_LDS_B64_ASM_DWORD) {
                // four reads in flight, waited for inside the same block; steps
                // q = 0, 4, 8, 12 issue them (the others do nothing)
                if ((q & 3) == 0) {
                    const unsigned addr = lds_base + 8u * (unsigned)lane + 2048u * (unsigned)(q >> 2) +
                                          (MODE == FDK_LDS_B64_ASM_DWORD ? 4u : 0u);
                    u32x2 r0, r1, r2, r3;
                    asm volatile(
                        "ds_read_b64 %0, %4\n"
                        "ds_read_b64 %1, %4 offset:512\n"
                        "ds_read_b64 %2, %4 offset:1024\n"
                        "ds_read_b64 %3, %4 offset:1536\n"
                        "s_waitcnt lgkmcnt(0)"
                        : "=&v"(r0), "=&v"(r1), "=&v"(r2), "=&v"(r3)
                        : "v"(addr)
                        : "memory");
                    a ^= r0.x ^ r1.x ^ r2.x ^ r3.x;
                    b ^= r0.y ^ r1.y ^ r2.y ^ r3.y;
                }
            } else if constexpr (MODE == FDK_LDS_TAPS_F16) {
                const int w = S.off[q] * 36 + col;
                a ^= buf[w];
                b ^= buf[w + 36];
            } else {
                const int w = S.off[q] * 72 + col;
                a ^= buf[w] ^ buf[w + 1];
                b ^= buf[w + 72] ^ buf[w + 73];
            }
        }
    }
    if ((a ^ b) == kNever) sink[0] = a ^ b;
}

__global__ __launch_bounds__(kPT) void valu_fma_kernel(int iters, float* sink)
{
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = (float)(threadIdx.x + j) * 1e-3f;
    const float m = 0.999999f, c = 1e-6f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
#pragma unroll
            for (int j = 0; j < 8; ++j) x[j] = fmaf(x[j], m, c);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += x[j];
    if (s == -1.0f) sink[0] = s;
}

// One instruction of fdk_valu_op on chain register x (c, d: loop-invariant
// operands).  Each form reads and writes x, so the 8 chains of a thread stay
// independent and no instruction can be dropped or hoisted.
template <int OP>
__device__ __forceinline__ void valu_step(float& x, float c, unsigned d)
{
    if constexpr (OP == FDK_OP_FMA_F32) asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(x) : "v"(c));
    else if constexpr (OP == FDK_OP_FMAC_F32) asm volatile("v_fmac_f32 %0, %1, %1" : "+v"(x) : "v"(c));
    else if constexpr (OP == FDK_OP_SUB_F32) asm volatile("v_sub_f32 %0, %0, %1" : "+v"(x) : "v"(c));
    else if constexpr (OP == FDK_OP_FRACT_F32) asm volatile("v_fract_f32 %0, %0" : "+v"(x));
    else if constexpr (OP == FDK_OP_CVT_I32_F32) asm volatile("v_cvt_i32_f32 %0, %0" : "+v"(x));
    else if constexpr (OP == FDK_OP_MAD_U32_U24) asm volatile("v_mad_u32_u24 %0, %0, %1, %1" : "+v"(x) : "v"(d));
    else if constexpr (OP == FDK_OP_FMA_MIX_F32)
        asm volatile("v_fma_mix_f32 %0, %1, %0, %0 op_sel_hi:[1,0,0]" : "+v"(x) : "v"(d));
    else if constexpr (OP == FDK_OP_CVT_F32_F16) asm volatile("v_cvt_f32_f16 %0, %0" : "+v"(x));
    else if constexpr (OP == FDK_OP_DOT2_F32_F16) asm volatile("v_dot2_f32_f16 %0, %1, %1, %0" : "+v"(x) : "v"(d));
    else if constexpr (OP == FDK_OP_PK_FMA_F16) asm volatile("v_pk_fma_f16 %0, %0, %1, %1" : "+v"(x) : "v"(d));
    else if constexpr (OP == FDK_OP_ADD_U32) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x) : "v"(d));
    else asm volatile("v_floor_f32 %0, %0" : "+v"(x));
}

template <int OP>
__global__ __launch_bounds__(kPT) void valu_op_kernel(int iters, float* sink)
{
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = (float)(threadIdx.x + j) * 1e-3f;
    const float c = 0.5f;
    const unsigned d = 0x3c003c00u + threadIdx.x;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
#pragma unroll
            for (int j = 0; j < 8; ++j) valu_step<OP>(x[j], c, d);
        }
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += x[j];
    if (s == -1.0f) sink[0] = s;
}

// bytes a lane reads per LDS read instruction, and instructions per read
// step (kReads steps per iteration)
int64_t lds_bytes_per_lane_step(int pattern)
{
    switch (pattern) {
        case FDK_LDS_B32: return 4;
        case FDK_LDS_READ2_B32: return 8;
        case FDK_LDS_B64: return 8;
        case FDK_LDS_B128: return 16;
        case FDK_LDS_TAPS_F16: return 8;
        case FDK_LDS_TAPS_F32: return 16;
        case FDK_LDS_B64_ASM: return 8;          // 16 reads per iteration in blocks of four
        case FDK_LDS_B64_ASM_DWORD: return 8;
    }
    return 0;
}

}  // namespace
}  // namespace fdk

using namespace fdk;

extern "C" fdk_status fdk_peak_hbm_read(const void* buf, int64_t bytes, int32_t blocks,
                                        uint32_t* sink, void* stream)
{
    if (!buf || !sink) return fail(FDK_E_INVALID, "buffer/sink pointer is NULL");
    if (bytes <= 0 || bytes % 16 != 0) return fail(FDK_E_INVALID, "bytes must be a positive multiple of 16");
    if ((reinterpret_cast<uintptr_t>(buf) & 15) != 0) return fail(FDK_E_INVALID, "buffer not 16-byte aligned");
    if (blocks < 1) return fail(FDK_E_INVALID, "blocks must be positive");
    hipLaunchKernelGGL(hbm_read_kernel, dim3((unsigned)blocks), dim3(kPT), 0, (hipStream_t)stream,
                       (const uint4*)buf, bytes / 16, sink);
    return check_launch("HBM read kernel");
}

extern "C" fdk_status fdk_peak_lds_read(int32_t pattern, int32_t blocks, int32_t iters,
                                        uint32_t* sink, int64_t* bytes_out, void* stream)
{
    if (!sink || !bytes_out) return fail(FDK_E_INVALID, "sink/bytes_out pointer is NULL");
    if (blocks < 1 || iters < 1) return fail(FDK_E_INVALID, "blocks and iters must be positive");
    const int64_t per = lds_bytes_per_lane_step(pattern);
    if (!per) return fail(FDK_E_INVALID, "unknown LDS read pattern");
    hipStream_t st = (hipStream_t)stream;
    // tap patterns: detector rows floor(1.3 + 1.6 k) of the updates k = 0 .. 15
    // of one half of a 32-slice column (1.6 rows per slice)
    LdsSteps S;
    for (int k = 0; k < kReads; ++k) S.off[k] = (13 + 16 * k) / 10;
    switch (pattern) {
#define FDK_LDS(m) case m: hipLaunchKernelGGL(lds_read_kernel<m>, dim3((unsigned)blocks), dim3(kPT), 0, st, iters, S, sink); break;
        FDK_LDS(FDK_LDS_B32) FDK_LDS(FDK_LDS_READ2_B32) FDK_LDS(FDK_LDS_B64)
        FDK_LDS(FDK_LDS_B128) FDK_LDS(FDK_LDS_TAPS_F16) FDK_LDS(FDK_LDS_TAPS_F32)
        FDK_LDS(FDK_LDS_B64_ASM) FDK_LDS(FDK_LDS_B64_ASM_DWORD)
#undef FDK_LDS
    }
    *bytes_out = (int64_t)blocks * kPT * (int64_t)iters * kReads * per;
    return check_launch("LDS read kernel");
}

extern "C" fdk_status fdk_peak_valu_fma(int32_t blocks, int32_t iters, float* sink,
                                        int64_t* ops_out, void* stream)
{
    if (!sink || !ops_out) return fail(FDK_E_INVALID, "sink/ops_out pointer is NULL");
    if (blocks < 1 || iters < 1) return fail(FDK_E_INVALID, "blocks and iters must be positive");
    hipLaunchKernelGGL(valu_fma_kernel, dim3((unsigned)blocks), dim3(kPT), 0, (hipStream_t)stream,
                       iters, sink);
    *ops_out = (int64_t)blocks * kPT * 8 * 16 * (int64_t)iters;
    return check_launch("FMA kernel");
}

extern "C" fdk_status fdk_peak_valu_op(int32_t op, int32_t blocks, int32_t iters, float* sink,
                                       int64_t* ops_out, void* stream)
{
    if (!sink || !ops_out) return fail(FDK_E_INVALID, "sink/ops_out pointer is NULL");
    if (blocks < 1 || iters < 1) return fail(FDK_E_INVALID, "blocks and iters must be positive");
    hipStream_t st = (hipStream_t)stream;
    switch (op) {
#define FDK_OP(m) case m: hipLaunchKernelGGL(valu_op_kernel<m>, dim3((unsigned)blocks), dim3(kPT), 0, st, iters, sink); break;
        FDK_OP(FDK_OP_FMA_F32) FDK_OP(FDK_OP_FMAC_F32) FDK_OP(FDK_OP_SUB_F32)
        FDK_OP(FDK_OP_FRACT_F32) FDK_OP(FDK_OP_CVT_I32_F32) FDK_OP(FDK_OP_MAD_U32_U24)
        FDK_OP(FDK_OP_FMA_MIX_F32) FDK_OP(FDK_OP_CVT_F32_F16) FDK_OP(FDK_OP_DOT2_F32_F16)
        FDK_OP(FDK_OP_PK_FMA_F16) FDK_OP(FDK_OP_ADD_U32) FDK_OP(FDK_OP_FLOOR_F32)
#undef FDK_OP
        default: return fail(FDK_E_INVALID, "unknown VALU instruction");
    }
    *ops_out = (int64_t)blocks * kPT * 8 * 16 * (int64_t)iters;
    return check_launch("VALU instruction kernel");
}
