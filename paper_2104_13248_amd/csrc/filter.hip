// FDK pre-processing filter (gfx950): cosine weight, Ram-Lak ramp along each
// detector row (linear convolution with zero padding), angular weight.
//
// The paper takes filtered projections as its input and names the filtering
// step without describing it (Sections 2.1.2, 3.1.1).  This is the textbook
// Feldkamp filter: for a row r of view s,
//   q[c]   = raw[c] * sdd / sqrt(sdd^2 + u_mm(c)^2 + v_mm(r)^2)
//   out[c] = tau * arc / (2 np_total) * sum_n h[n] q[c - n]
// with the Ram-Lak kernel h[0] = 1/(4 tau^2), h[odd n] = -1/(pi^2 n^2 tau^2),
// h[even n != 0] = 0 and tau = du sod / sdd.
//
// One block per detector row: the weighted row and the odd-tap coefficients
// live in LDS; each thread produces several outputs, reading each q once per
// pair of symmetric taps (h is even).
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace fdk {
namespace {

constexpr int kFilterThreads = 256;

struct FilterArgs {
    const float* raw;
    float* out;
    int nh, nw;
    float cu, cv, du, dv, sdd2, sdd;
    float h0;          // h[0] * tau * angular weight
    float hscale;      // -1/(pi^2 tau^2) * tau * angular weight
};

__global__ __launch_bounds__(kFilterThreads) void filter_kernel(const FilterArgs A)
{
    extern __shared__ float sm[];
    float* q = sm;                       // [nw] cosine-weighted row
    float* hodd = sm + A.nw;             // [nw/2 + 1] coefficient of tap 2m+1
    const int row = blockIdx.x;          // s * nh + r
    const int r = row % A.nh;
    const float* src = A.raw + (size_t)row * A.nw;
    float* dst = A.out + (size_t)row * A.nw;
    const float vmm = ((float)r - A.cv) * A.dv;
    const float v2 = A.sdd2 + vmm * vmm;
    for (int c = threadIdx.x; c < A.nw; c += kFilterThreads) {
        const float umm = ((float)c - A.cu) * A.du;
        q[c] = src[c] * (A.sdd * rsqrtf(fmaf(umm, umm, v2)));
    }
    const int nodd = (A.nw + 1) / 2;
    for (int m = threadIdx.x; m < nodd; m += kFilterThreads) {
        const float n = (float)(2 * m + 1);
        hodd[m] = A.hscale / (n * n);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < A.nw; c += kFilterThreads) {
        // taps c - n and c + n for odd n; both sides while both exist
        const int both = min(c, A.nw - 1 - c);
        float acc = 0.f;
        int m = 0;
        for (; 2 * m + 1 <= both; ++m) acc = fmaf(hodd[m], q[c - 2 * m - 1] + q[c + 2 * m + 1], acc);
        if (c < A.nw - 1 - c) {
            for (; 2 * m + 1 <= A.nw - 1 - c; ++m) acc = fmaf(hodd[m], q[c + 2 * m + 1], acc);
        } else {
            for (; 2 * m + 1 <= c; ++m) acc = fmaf(hodd[m], q[c - 2 * m - 1], acc);
        }
        dst[c] = fmaf(A.h0, q[c], acc);
    }
}

// Step 1 alone (the input of the learned row filter): q = raw * cosine weight.
__global__ __launch_bounds__(kFilterThreads) void cosine_kernel(const FilterArgs A, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * kFilterThreads + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kFilterThreads) {
        const int64_t row = q / A.nw;
        const int c = (int)(q - row * A.nw);
        const int r = (int)(row % A.nh);
        const float vmm = ((float)r - A.cv) * A.dv;
        const float umm = ((float)c - A.cu) * A.du;
        A.out[q] = A.raw[q] * (A.sdd * rsqrtf(fmaf(umm, umm, A.sdd2 + vmm * vmm)));
    }
}

FilterArgs filter_args(const FilterLaunch& a)
{
    const double tau = a.du * a.sod / a.sdd;
    const double wang = a.arc / (2.0 * (double)a.np_total);
    const double pi = 3.14159265358979323846;
    FilterArgs A;
    A.raw = a.raw;
    A.out = a.out;
    A.nh = a.nh;
    A.nw = a.nw;
    A.cu = (float)(0.5 * (a.nw - 1) + a.u_off);
    A.cv = (float)(0.5 * (a.nh - 1) + a.v_off);
    A.du = (float)a.du;
    A.dv = (float)a.dv;
    A.sdd = (float)a.sdd;
    A.sdd2 = (float)(a.sdd * a.sdd);
    A.h0 = (float)(1.0 / (4.0 * tau * tau) * tau * wang);
    A.hscale = (float)(-1.0 / (pi * pi * tau * tau) * tau * wang);
    return A;
}

}  // namespace

fdk_status launch_cosine_weight(const FilterLaunch& a, void* stream)
{
    const FilterArgs A = filter_args(a);
    const int64_t n = (int64_t)a.np * a.nh * a.nw;
    int64_t blocks = (n + kFilterThreads - 1) / kFilterThreads;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(cosine_kernel, dim3((unsigned)blocks), dim3(kFilterThreads), 0,
                       (hipStream_t)stream, A, n);
    return check_launch("cosine-weight kernel");
}

fdk_status launch_filter(const FilterLaunch& a, void* stream)
{
    const FilterArgs A = filter_args(a);
    const int64_t rows = (int64_t)a.np * a.nh;
    if (rows >= (1ll << 31)) return fail(FDK_E_UNSUPPORTED, "too many detector rows");
    const size_t lds = (size_t)(a.nw + (a.nw + 1) / 2 + 1) * sizeof(float);
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute((const void*)filter_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return fail(FDK_E_DEVICE, "cannot raise the LDS limit of the filter kernel");
    }
    hipLaunchKernelGGL(filter_kernel, dim3((unsigned)rows), dim3(kFilterThreads), lds,
                       (hipStream_t)stream, A);
    return check_launch("filter kernel");
}

}  // namespace fdk
