// Reference kernels for measuring what the paper's CPU optimisations are worth
// on gfx950 (float32 projections only).  Same arithmetic contract as the
// production back-projector: coordinates from the index-space matrix, floor,
// zero outside the detector, weight 1/w^2, FP32 interpolation and accumulation.
//
//   listing1_kernel  Listing 1 as written for a GPU: one voxel per thread (x
//                    fastest), the full projection of every (voxel, view) --
//                    three dot products and a division, no hoisting (Section
//                    3.1.2) -- the four taps read from global memory, and the
//                    volume read and written once per launch of nb views
//                    (Section 3.1.3's batch size nb; the host launches np / nb
//                    times).
//
// (The global-taps variant -- the production structure with Section 3.2's
// local-memory staging removed -- is the production library's own direct
// organisation, bp_direct_kernel, which also serves strongly magnified
// geometries.)
//
// The projection of a voxel is evaluated in FP64 (the MI355X vector FP64 rate
// equals its slow-class FP32 rate) and reduced to FP32 offsets below the
// integer part, so the kernel meets the FP32 tolerance against the oracle.
#include <hip/hip_runtime.h>

#include "fdk_ablation.h"
#include "internal.h"

namespace fdk {
namespace {

struct AblArgs {
    const float* proj;        // [np][nh][nw] float32
    const double* M;          // [np][12] index-space matrices
    float* vol;
    int nx, ny, nz, nh, nw;
    int s0, s1;               // views [s0, s1) of this launch
};

// p[r][c] with zero outside the detector
__device__ __forceinline__ float tap(const float* __restrict__ p, int r, int c, int nh, int nw)
{
    return ((unsigned)r < (unsigned)nh && (unsigned)c < (unsigned)nw) ? p[(size_t)r * nw + c] : 0.f;
}

__device__ __forceinline__ float bilinear(const float* __restrict__ p, int r, int c, float fv,
                                          float fu, int nh, int nw)
{
    const float p00 = tap(p, r, c, nh, nw), p01 = tap(p, r, c + 1, nh, nw);
    const float p10 = tap(p, r + 1, c, nh, nw), p11 = tap(p, r + 1, c + 1, nh, nw);
    const float h0 = fmaf(fu, p01 - p00, p00), h1 = fmaf(fu, p11 - p10, p10);
    return fmaf(fv, h1 - h0, h0);
}

__global__ __launch_bounds__(256) void listing1_kernel(const AblArgs A)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t nvox = (int64_t)A.nx * A.ny * A.nz;
    if (q >= nvox) return;
    const int i = (int)(q % A.nx);
    const int j = (int)((q / A.nx) % A.ny);
    const int k = (int)(q / ((int64_t)A.nx * A.ny));
    const double di = i, dj = j, dk = k;
    float acc = 0.f;
    for (int s = A.s0; s < A.s1; ++s) {
        const double* m = A.M + 12 * (size_t)s;
        const double w = m[8] * di + m[9] * dj + m[10] * dk + m[11];
        const double rw = 1.0 / w;
        const double u = (m[0] * di + m[1] * dj + m[2] * dk + m[3]) * rw;
        const double v = (m[4] * di + m[5] * dj + m[6] * dk + m[7]) * rw;
        const double fu = floor(u), fv = floor(v);
        const float* p = A.proj + (size_t)s * A.nh * A.nw;
        const float val = bilinear(p, (int)fv, (int)fu, (float)(v - fv), (float)(u - fu), A.nh, A.nw);
        acc = fmaf((float)(rw * rw), val, acc);
    }
    A.vol[q] += acc;
}

}  // namespace

fdk_status launch_backproject_variant(int variant, int nb, const float* proj,
                                      const double* mats_index, float* vol, int nx, int ny,
                                      int nz, int np, int nh, int nw, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    AblArgs A;
    A.proj = proj;
    A.M = mats_index;
    A.vol = vol;
    A.nx = nx; A.ny = ny; A.nz = nz; A.nh = nh; A.nw = nw;
    if (variant == FDK_VARIANT_LISTING1) {
        const int64_t nvox = (int64_t)nx * ny * nz;
        const int64_t blocks = (nvox + 255) / 256;
        if (blocks >= (1ll << 31)) return fail(FDK_E_UNSUPPORTED, "volume too large for one launch");
        for (int s0 = 0; s0 < np; s0 += nb) {
            A.s0 = s0;
            A.s1 = s0 + nb < np ? s0 + nb : np;
            hipLaunchKernelGGL(listing1_kernel, dim3((unsigned)blocks), dim3(256), 0, st, A);
            const fdk_status s = check_launch("listing-1 back-projection kernel");
            if (s != FDK_OK) return s;
        }
        return FDK_OK;
    }
    return fail(FDK_E_INVALID, "unknown back-projection variant");
}

}  // namespace fdk
