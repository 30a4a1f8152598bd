// fdk_backproject_noalloc: fdk_backproject without any device or host
// allocation.  The only per-call scratch of the back-projection is the table
// of world matrices and their FP64 compositions with the voxel grid; here it
// lives in a file-scope device array (one copy per GPU, held until the process
// ends), and the world matrices reach it as kernel arguments, 32 views per
// launch, instead of through a pinned staging buffer.  The composition and
// back-projection kernels are the ones fdk_backproject launches, so results
// are bitwise identical.
#include <hip/hip_runtime.h>

#include <mutex>

#include "internal.h"

namespace fdk {
namespace {

constexpr int kMaxDevices = 64;
constexpr int kChunk = 32;                       // world matrices per upload launch

// [0, 12 kNoAllocMaxViews): world matrices; then the composed ones.
static __device__ __align__(256) double scratch[2 * 12 * FDK_NOALLOC_MAX_VIEWS];

std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};             // device address of `scratch` per device

struct MatChunk {
    double m[12 * kChunk];
};

__global__ void put_mats_kernel(const MatChunk c, int n, double* __restrict__ dst)
{
    for (int q = threadIdx.x; q < 12 * n; q += blockDim.x) dst[q] = c.m[q];
}

// Device address of this device's copy of `scratch`, looked up once per device
// with that device current.
fdk_status scratch_address(double** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(FDK_E_DEVICE, "hipGetDevice failed");
    if (dev < 0 || dev >= kMaxDevices) return fail(FDK_E_UNSUPPORTED, "device index out of range");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FDK_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                          hipGetErrorString(e));
        g_scratch[dev] = (double*)p;
    }
    *out = g_scratch[dev];
    return FDK_OK;
}

}  // namespace
}  // namespace fdk

using namespace fdk;

extern "C" fdk_status fdk_backproject_noalloc(const fdk_volume* vg, float* vol,
                                              const fdk_stack* sg, const void* proj,
                                              const float* scale, const double* mats,
                                              void* stream)
{
    fdk_status s = validate_volume(vg);
    if (s != FDK_OK) return s;
    s = validate_stack(sg, true);
    if (s != FDK_OK) return s;
    if (sg->np > FDK_NOALLOC_MAX_VIEWS)
        return fail(FDK_E_UNSUPPORTED, "fdk_backproject_noalloc takes at most " +
                                           std::to_string(FDK_NOALLOC_MAX_VIEWS) +
                                           " views per call (its scratch array is fixed)");
    std::vector<IndexMatrix> M;
    s = validate_geometry(*vg, *sg, mats, &M);
    if (s != FDK_OK) return s;
    if (!vol) return fail(FDK_E_INVALID, "volume pointer is NULL");
    if (!proj) return fail(FDK_E_INVALID, "projection pointer is NULL");
    if (sg->dtype == FDK_F16 && !scale)
        return fail(FDK_E_INVALID, "binary16 projections need a per-view scale array");
    if (sg->dtype == FDK_F32 && scale)
        return fail(FDK_E_INVALID, "a scale array is only accepted with binary16 projections");
    if ((int64_t)sg->nh * sg->nw * (sg->dtype == FDK_F16 ? 2 : 4) >= (1ll << 31))
        return fail(FDK_E_UNSUPPORTED, "one view larger than 2 GiB");
    BpPlan plan;
    s = make_bp_plan(*vg, *sg, M, plan);
    if (s != FDK_OK) return s;

    double* base = nullptr;
    s = scratch_address(&base);
    if (s != FDK_OK) return s;
    double* world = base;
    double* index = base + 12 * (size_t)FDK_NOALLOC_MAX_VIEWS;
    hipStream_t st = (hipStream_t)stream;
    for (int32_t v0 = 0; v0 < sg->np; v0 += kChunk) {
        const int n = sg->np - v0 < kChunk ? sg->np - v0 : kChunk;
        MatChunk c;
        for (int q = 0; q < 12 * n; ++q) c.m[q] = mats[12 * (size_t)v0 + q];
        hipLaunchKernelGGL(put_mats_kernel, dim3(1), dim3(128), 0, st, c, n, world + 12 * (size_t)v0);
        s = check_launch("matrix upload kernel");
        if (s != FDK_OK) return s;
    }
    BpLaunch a;
    a.proj = proj;
    a.scale = scale;
    a.mats_world = world;
    a.mats_index = index;
    a.vol = vol;
    a.nx = vg->nx; a.ny = vg->ny; a.nz = vg->nz;
    a.np = sg->np; a.nh = sg->nh; a.nw = sg->nw;
    a.k_begin = 0;
    a.k_end = vg->nz;
    a.dx = vg->dx; a.dy = vg->dy; a.dz = vg->dz;
    a.ox = vg->cx - 0.5 * (vg->nx - 1) * vg->dx;
    a.oy = vg->cy - 0.5 * (vg->ny - 1) * vg->dy;
    a.oz = vg->cz - 0.5 * (vg->nz - 1) * vg->dz;
    a.f16 = sg->dtype == FDK_F16;
    return launch_backproject(a, plan, stream);
}
