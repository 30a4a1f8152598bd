// Forward projection as the exact transpose of the back-projector (gfx950).
//
// The back-projection of Listings 1-2 is a fixed linear map p -> vol: every
// voxel reads the four bilinear taps around its (u, v), weighted by 1/w^2.
// Its transpose scatters each voxel value x, weighted by 1/w^2, into the same
// four taps with the same bilinear weights.  Taps outside the detector are
// dropped (the transpose of zero extension).
//
// Layout mirrors the back-projector: a thread per voxel column keeps its KZ
// voxel values in registers for the whole view loop; per view the block
// accumulates its footprint window in LDS with LDS float atomics, then adds
// the window to the projection with global float atomics.
#include <hip/hip_runtime.h>

#include "footprint.h"
#include "internal.h"

namespace fdk {
namespace {

struct FpArgs {
    const float* vol;
    float* proj;
    const double* M;
    int nx, ny, nz, np, nh, nw;
    int ntx, ntiles, ntiles_pad;
    int rows;
};

template <int KZ, int PITCH>
__global__ __launch_bounds__(kThreads) void fp_kernel(const FpArgs A)
{
    extern __shared__ float smem[];
    float* tile = smem;
    ViewRec* vtab = reinterpret_cast<ViewRec*>(smem + A.rows * PITCH);

    const BlockPos bp = block_position(blockIdx.x, A.ntiles_pad);
    if (bp.tile >= A.ntiles) return;
    const int tx = bp.tile % A.ntx, ty = bp.tile / A.ntx;
    const int kc = bp.chunk_local * KZ;
    const int i0 = tx * kTile, j0 = ty * kTile;
    const int ni = min(kTile, A.nx - i0), nj = min(kTile, A.ny - j0);
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int lx = tid & (kTile - 1), ly = tid >> 4;
    const bool active = lx < ni && ly < nj;
    const float di = (float)min(lx, ni - 1), dj = (float)min(ly, nj - 1);

    // voxel values of this column; idle lanes and slices past nz carry zero
    float x[KZ];
#pragma unroll
    for (int kk = 0; kk < KZ; ++kk) {
        const int k = kc + kk;
        x[kk] = (active && k < A.nz) ? A.vol[((size_t)k * A.ny + j0 + ly) * A.nx + i0 + lx] : 0.f;
    }
    const size_t view_px = (size_t)A.nh * A.nw;

    for (int sb = 0; sb < A.np; sb += kViewBatch) {
        const int nb = min(kViewBatch, A.np - sb);
        __syncthreads();
        if (tid < nb)
            view_record(A.M + 12 * (size_t)(sb + tid), i0, j0, ni, nj, kc, KZ, 1.0f, PITCH, A.rows,
                        false, &vtab[tid]);
        __syncthreads();
        for (int qv = 0; qv < nb; ++qv) {
            const ViewRec rec = vtab[qv];
            // rows of the window to waves, columns to lanes
            for (int rr = wave; rr < rec.R; rr += kThreads / 64)
                for (int cc = lane; cc < rec.C; cc += 64) tile[rr * PITCH + cc] = 0.f;
            __syncthreads();
            const float w = fmaf(rec.d, di, fmaf(rec.e, dj, rec.w0));
            const float F = 1.0f / w;
            const float u = fmaf(rec.a, di, fmaf(rec.b, dj, rec.N0)) * F;
            const float dv = rec.m12 * F;
            const float W = F * F;
            const float fu = __builtin_amdgcn_fractf(u);
            float* T0 = tile + (int)u;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const float v0 = fmaf(rec.half[q].g, di, fmaf(rec.half[q].h, dj, rec.half[q].V0)) * F;
                float* Tq = T0 + rec.half[q].row * PITCH;
#pragma unroll
                for (int t = 0; t < KZ / 2; ++t) {
                    const float v = fmaf((float)t, dv, v0);
                    const float fv = __builtin_amdgcn_fractf(v);
                    float* p = Tq + (int)v * PITCH;
                    const float xw = x[q * (KZ / 2) + t] * W;
                    const float lo = xw * (1.0f - fv), hi = xw * fv;
                    unsafeAtomicAdd(p, lo * (1.0f - fu));
                    unsafeAtomicAdd(p + 1, lo * fu);
                    unsafeAtomicAdd(p + PITCH, hi * (1.0f - fu));
                    unsafeAtomicAdd(p + PITCH + 1, hi * fu);
                }
            }
            __syncthreads();
            float* dst = A.proj + (size_t)(sb + qv) * view_px;
            for (int rr = wave; rr < rec.R; rr += kThreads / 64) {
                const int r = rec.r0 + rr;
                if ((unsigned)r >= (unsigned)A.nh) continue;
                for (int cc = lane; cc < rec.C; cc += 64) {
                    const int c = rec.c0 + cc;
                    const float val = tile[rr * PITCH + cc];
                    if (val != 0.f && (unsigned)c < (unsigned)A.nw)
                        unsafeAtomicAdd(dst + (size_t)r * A.nw + c, val);
                }
            }
            __syncthreads();
        }
    }
}

template <int KZ, int PITCH>
fdk_status launch_fp_kp(const FpArgs& a, size_t lds, unsigned blocks, hipStream_t st)
{
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute((const void*)fp_kernel<KZ, PITCH>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return fail(FDK_E_DEVICE, "cannot raise the LDS limit of the forward-projection kernel");
    }
    hipLaunchKernelGGL((fp_kernel<KZ, PITCH>), dim3(blocks), dim3(kThreads), lds, st, a);
    return check_launch("forward-projection kernel");
}

template <int KZ>
fdk_status launch_fp_k(const FpArgs& a, int pitch, size_t lds, unsigned blocks, hipStream_t st)
{
    switch (pitch) {
        case 40: return launch_fp_kp<KZ, 40>(a, lds, blocks, st);
        case 56: return launch_fp_kp<KZ, 56>(a, lds, blocks, st);
        case 72: return launch_fp_kp<KZ, 72>(a, lds, blocks, st);
        case 88: return launch_fp_kp<KZ, 88>(a, lds, blocks, st);
        case 120: return launch_fp_kp<KZ, 120>(a, lds, blocks, st);
        case 184: return launch_fp_kp<KZ, 184>(a, lds, blocks, st);
        case 248: return launch_fp_kp<KZ, 248>(a, lds, blocks, st);
    }
    return fail(FDK_E_UNSUPPORTED, "no kernel for this LDS pitch");
}

}  // namespace

fdk_status launch_forwardproject(const FpLaunch& a, const BpPlan& plan, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    fdk_status s = launch_compose(a.mats_world, a.mats_index, a.np, a.dx, a.dy, a.dz, a.ox, a.oy,
                                  a.oz, stream);
    if (s != FDK_OK) return s;
    FpArgs A;
    A.vol = a.vol;
    A.proj = a.proj;
    A.M = a.mats_index;
    A.nx = a.nx; A.ny = a.ny; A.nz = a.nz; A.np = a.np; A.nh = a.nh; A.nw = a.nw;
    A.ntx = plan.ntx;
    A.ntiles = plan.ntx * plan.nty;
    A.ntiles_pad = plan.ntiles_pad;
    A.rows = plan.rows_full;
    const int64_t blocks = (int64_t)plan.ntiles_pad * plan.nchunks;
    if (blocks >= (1ll << 31)) return fail(FDK_E_UNSUPPORTED, "grid too large");
    const size_t lds = (size_t)plan.fp_lds_bytes;
    if (lds > 160 * 1024) return fail(FDK_E_UNSUPPORTED, "forward-projection footprint exceeds LDS");
    switch (plan.kz) {
        case 8: return launch_fp_k<8>(A, plan.pitch, lds, (unsigned)blocks, st);
        case 16: return launch_fp_k<16>(A, plan.pitch, lds, (unsigned)blocks, st);
        case 32: return launch_fp_k<32>(A, plan.pitch, lds, (unsigned)blocks, st);
    }
    return fail(FDK_E_UNSUPPORTED, "no kernel for this slice count");
}

}  // namespace fdk
