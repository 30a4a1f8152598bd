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
        for (int64_t t = t0; t < n4; t += nthreads) {
            const float4 x = p4[t];
            m = fmaxf(m, fmaxf(fmaxf(fabsf(x.x), fabsf(x.y)), fmaxf(fabsf(x.z), fabsf(x.w))));
        }
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
    for (int64_t t = (int64_t)blockIdx.x * kQThreads + threadIdx.x; t < npix;
         t += (int64_t)gridDim.x * kQThreads) {
        const _Float16 h = (_Float16)(p[t] * inv);   // v_cvt_f16_f32, round to nearest even
        o[t] = __builtin_bit_cast(uint16_t, h);
    }
}

}  // namespace

fdk_status launch_quantize_f16(int32_t np, int64_t npix, const float* in, uint16_t* out,
                               float* scale, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    void* d_max = nullptr;
    fdk_status s = device_alloc_async((size_t)np * sizeof(unsigned), stream, &d_max);
    if (s != FDK_OK) return s;
    unsigned* mx = (unsigned*)d_max;
    hipLaunchKernelGGL(clear_u32, dim3((np + 255) / 256), dim3(256), 0, st, mx, np);
    s = check_launch("clear kernel");
    // enough blocks to fill the GPU, each streaming a large contiguous share
    int64_t bmax = (npix + kQThreads * 16 - 1) / (kQThreads * 16);
    if (bmax < 1) bmax = 1;
    const int64_t bm = bmax < 16 ? bmax : 16;
    int64_t bx = (npix + kQThreads * 8 - 1) / (kQThreads * 8);
    if (bx > 1024) bx = 1024;
    if (bx < 1) bx = 1;
    if (s == FDK_OK) {
        hipLaunchKernelGGL(absmax_kernel, dim3((unsigned)bm, (unsigned)np), dim3(kQThreads), 0, st,
                           in, npix, mx);
        s = check_launch("absmax kernel");
    }
    if (s == FDK_OK) {
        hipLaunchKernelGGL(quantize_kernel, dim3((unsigned)bx, (unsigned)np), dim3(kQThreads), 0,
                           st, in, npix, (const unsigned*)mx, out, scale);
        s = check_launch("quantize kernel");
    }
    fdk_status s2 = device_free_async(d_max, stream);
    return s != FDK_OK ? s : s2;
}

}  // namespace fdk
