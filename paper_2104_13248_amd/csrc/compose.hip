// FP64 composition of world-mm projection matrices with the voxel grid.
//
// Listing 1 applies the 3x4 matrix to raw voxel indices (i, j, k, 1); the
// library's matrices act on world millimetres, so each view's matrix is
// composed once with the index -> world map of the volume:
//   M = P V,  V = [[dx,0,0,ox],[0,dy,0,oy],[0,0,dz,oz],[0,0,0,1]].
// Done in FP64 on the device, one thread per view.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace fdk {
namespace {

__global__ void compose_kernel(const double* __restrict__ P, double* __restrict__ M, int np,
                               double dx, double dy, double dz, double ox, double oy, double oz)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= np) return;
    const double* p = P + 12 * (size_t)s;
    double* m = M + 12 * (size_t)s;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        m[4 * r + 0] = p[4 * r + 0] * dx;
        m[4 * r + 1] = p[4 * r + 1] * dy;
        m[4 * r + 2] = p[4 * r + 2] * dz;
        m[4 * r + 3] = p[4 * r + 0] * ox + p[4 * r + 1] * oy + p[4 * r + 2] * oz + p[4 * r + 3];
    }
}

}  // namespace

fdk_status launch_compose(const double* P, double* M, int32_t np, double dx, double dy,
                          double dz, double ox, double oy, double oz, void* stream)
{
    hipLaunchKernelGGL(compose_kernel, dim3((np + 63) / 64), dim3(64), 0, (hipStream_t)stream, P,
                       M, np, dx, dy, dz, ox, oy, oz);
    return check_launch("matrix composition kernel");
}

}  // namespace fdk
