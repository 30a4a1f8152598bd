// FP16 storage of filtered projections with one power-of-two scale per view.
//
//   m_s = max |p_s|;  scale_s = 1 if m_s == 0, else 2^(ceil(log2 m_s) - 15)
//   h = round-to-nearest-even(p / scale_s) as binary16  (|h| <= 32768)
//
// The paper stores everything in single precision (Section 4.1); halving the
// bytes of the projection stack is an extension.  Division by a power of two
// is exact, so the only rounding is the binary16 conversion, and the result is
// bit-reproducible.  Three passes: clear the per-view maxima (a fill kernel),
// per-view absolute maximum (order-independent atomicMax on the bit pattern of
// non-negative floats), conversion.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace fdk {
namespace {

constexpr int kQThreads = 256;

__global__ void clear_u32(unsigned* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Per-view absolute maximum: a few blocks per view stream the view with
// 16-byte loads (scalar loads for an unaligned view or the tail), reduce in
// the wave and across the block, and post one atomicMax per block.
__global__ __launch_bounds__(kQThreads) void absmax_kernel(const float* __restrict__ in, int64_t npix,
                                                           unsigned* __restrict__ maxbits)
{
    __shared__ float part[kQThreads / 64];
    const int s = blockIdx.y;
    const float* p = in + (size_t)s * npix;
    const int64_t nthreads = (int64_t)gridDim.x * kQThreads;
    const int64_t t0 = (int64_t)blockIdx.x * kQThreads + threadIdx.x;
    float m = 0.f;
    int64_t head = 0;
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0) {
        const float4* p4 = reinterpret_cast<const float4*>(p);
        const int64_t n4 = npix / 4;
        auto absmax4 = [](float4 x) {
            return fmaxf(fmaxf(fabsf(x.x), fabsf(x.y)), fmaxf(fabsf(x.z), fabsf(x.w)));
        };
        int64_t t = t0;
        // four independent loads in flight per thread
        for (; t + 3 * nthreads < n4; t += 4 * nthreads) {
            const float4 x0 = p4[t], x1 = p4[t + nthreads];
            const float4 x2 = p4[t + 2 * nthreads], x3 = p4[t + 3 * nthreads];
            m = fmaxf(m, fmaxf(fmaxf(absmax4(x0), absmax4(x1)), fmaxf(absmax4(x2), absmax4(x3))));
        }
        for (; t < n4; t += nthreads) m = fmaxf(m, absmax4(p4[t]));
        head = n4 * 4;
    }
    for (int64_t t = head + t0; t < npix; t += nthreads) m = fmaxf(m, fabsf(p[t]));
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kQThreads / 64; ++w) m = fmaxf(m, part[w]);
        atomicMax(&maxbits[s], __float_as_uint(m));          // m >= 0: bit order = value order
    }
}

__device__ __forceinline__ float view_scale(float m)
{
    if (!(m > 0.f)) return 1.0f;
    int e;
    const float f = frexpf(m, &e);           // m = f 2^e, f in [0.5, 1)
    return ldexpf(1.0f, f > 0.5f ? e - 15 : e - 16);
}

__global__ __launch_bounds__(kQThreads) void quantize_kernel(const float* __restrict__ in, int64_t npix,
                                                             const unsigned* __restrict__ maxbits,
                                                             uint16_t* __restrict__ out,
                                                             float* __restrict__ scale)
{
    const int s = blockIdx.y;
    const float sc = view_scale(__uint_as_float(maxbits[s]));
    const float inv = 1.0f / sc;             // exact: a power of two
    if (blockIdx.x == 0 && threadIdx.x == 0) scale[s] = sc;
    const float* p = in + (size_t)s * npix;
    uint16_t* o = out + (size_t)s * npix;
    const int64_t t0 = (int64_t)blockIdx.x * kQThreads + threadIdx.x;
    const int64_t nthreads = (int64_t)gridDim.x * kQThreads;
    // product, then v_cvt_f16_f32 (round to nearest even).  The empty asm
    // keeps the two apart: fused into one mixed-precision FMA with a +0
    // addend they would turn a -0 product into +0.
    auto half_bits = [inv](float x) {
        float p = x * inv;
        asm volatile("" : "+v"(p));
        return (unsigned)__builtin_bit_cast(uint16_t, (_Float16)p);
    };
    int64_t head = 0;
    if ((reinterpret_cast<uintptr_t>(p) & 15) == 0 && (reinterpret_cast<uintptr_t>(o) & 15) == 0) {
        // eight pixels per thread: two 16-byte loads, one 16-byte store
        const float4* p4 = reinterpret_cast<const float4*>(p);
        uint4* o8 = reinterpret_cast<uint4*>(o);
        const int64_t n8 = npix / 8;
        for (int64_t t = t0; t < n8; t += nthreads) {
            const float4 a = p4[2 * t], b = p4[2 * t + 1];
            uint4 h;
            h.x = half_bits(a.x) | (half_bits(a.y) << 16);
            h.y = half_bits(a.z) | (half_bits(a.w) << 16);
            h.z = half_bits(b.x) | (half_bits(b.y) << 16);
            h.w = half_bits(b.z) | (half_bits(b.w) << 16);
            o8[t] = h;
        }
        head = n8 * 8;
    }
    for (int64_t t = head + t0; t < npix; t += nthreads) o[t] = (uint16_t)half_bits(p[t]);
}

}  // namespace

fdk_status launch_clear_u32(unsigned* p, int32_t n, void* stream)
{
    if (n <= 0) return FDK_OK;
    hipLaunchKernelGGL(clear_u32, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, p, n);
    return check_launch("clear kernel");
}

fdk_status launch_quantize_with_max(int32_t np, int64_t npix, const float* in,
                                    const unsigned* maxbits, uint16_t* out, float* scale,
                                    void* stream)
{
    // enough blocks to fill the GPU, each streaming a large contiguous share
    int64_t bx = (npix + kQThreads * 32 - 1) / (kQThreads * 32);
    if (bx > 1024) bx = 1024;
    if (bx < 1) bx = 1;
    hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)bx, (unsigned)np), dim3(kQThreads), 0,
                       (hipStream_t)stream, in, npix, maxbits, out, scale);
    return check_launch("quantize kernel");
}

fdk_status launch_quantize_f16(int32_t np, int64_t npix, const float* in, uint16_t* out,
                               float* scale, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    void* d_max = nullptr;
    fdk_status s = device_alloc_async((size_t)np * sizeof(unsigned), stream, &d_max);
    if (s != FDK_OK) return s;
    unsigned* mx = (unsigned*)d_max;
    s = launch_clear_u32(mx, np, stream);
    int64_t bmax = (npix + kQThreads * 16 - 1) / (kQThreads * 16);
    if (bmax < 1) bmax = 1;
    const int64_t bm = bmax < 16 ? bmax : 16;
    if (s == FDK_OK) {
        hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)bm, (unsigned)np), dim3(kQThreads), 0, st,
                           in, npix, mx);
        s = check_launch("absmax kernel");
    }
    if (s == FDK_OK) s = launch_quantize_with_max(np, npix, in, mx, out, scale, stream);
    fdk_status s2 = device_free_async(d_max, stream);
    return s != FDK_OK ? s : s2;
}

}  // namespace fdk
