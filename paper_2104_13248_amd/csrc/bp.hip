// Voxel-driven FDK back-projection for gfx950 (MI355X).
//
// What is computed (Chen et al., ICS'21, Listings 1-2, Algorithm 1):
//   vol[k][j][i] += sum_s scale_s / w^2 * bilinear(p_s, u, v)
// with (u w, v w, w) = M_s (i, j, k, 1) and zero outside the detector.
//
// How (GPU design; the paper's CPU kernels are prior art):
//   * one thread per voxel column (i, j) of a 16 x 16 tile; each thread keeps
//     KZ consecutive slices of its column in registers for the WHOLE view
//     loop, so the volume is read and written once per call (the paper's
//     batching with register accumulation, Section 3.1.3, taken to nb = np);
//   * u and w do not depend on k (Section 3.1.2), so per (column, view) the
//     thread hoists u, the weight, the first v and the step dv; each update
//     is then v = v0 + k dv, one 2x2 gather and three lerps;
//   * per view the detector footprint of the block's voxel box is staged in
//     LDS with zero padding (the local-memory staging of Section 3.2, without
//     a per-update bounds check);
//   * FP64 is used only to compose the index-space matrices and the per-block,
//     per-view bases (coordinates relative to the staged tile), which keeps
//     the FP32 coordinates small and accurate;
//   * block order: z-chunk major so that the resident blocks cover a thin
//     slab and read a narrow band of detector rows; within a chunk each of
//     the 8 XCDs receives a contiguous band of tiles (blocks are dealt to
//     XCDs round-robin by block id), which keeps its L2 footprint small.
#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>

#include "footprint.h"
#include "internal.h"

namespace fdk {
namespace {

// 32-bit LDS addressing (address space 3), so that a row offset and the
// column base combine in a single v_mad_u32_u24.
typedef __attribute__((address_space(3))) const float lds_f32;
__device__ __forceinline__ unsigned lds_addr(const float* p)
{
    return (unsigned)(size_t)(__attribute__((address_space(3))) const float*)p;
}
__device__ __forceinline__ const lds_f32* lds_ptr(unsigned a) { return (const lds_f32*)(size_t)a; }

template <typename T> __device__ __forceinline__ float load_px(const T* p);
template <> __device__ __forceinline__ float load_px<float>(const float* p) { return *p; }
template <> __device__ __forceinline__ float load_px<uint16_t>(const uint16_t* p)
{
    return (float)__builtin_bit_cast(_Float16, *p);
}

struct BpArgs {
    const void* proj;
    const float* scale;
    const double* M;          // [np][12] index-space matrices
    float* vol;               // slab base: slices [k_begin, k_end)
    int nx, ny, nz, np, nh, nw;
    int k_begin, k_end;
    int ntx, ntiles, ntiles_pad, chunk_first;
    int rows;                 // LDS rows allocated
};

template <int KZ, int PITCH, typename T>
__global__ __launch_bounds__(kThreads) void bp_kernel(const BpArgs A)
{
    extern __shared__ float smem[];
    float* tile = smem;                                       // [rows][PITCH]
    ViewRec* vtab = reinterpret_cast<ViewRec*>(smem + A.rows * PITCH);

    // ---- block -> (chunk, tile): z-chunk major, one band of tiles per XCD
    const BlockPos bp = block_position(blockIdx.x, A.ntiles_pad);
    const int t_id = bp.tile, chunk_local = bp.chunk_local;
    if (t_id >= A.ntiles) return;                             // padding block
    const int tx = t_id % A.ntx, ty = t_id / A.ntx;
    const int kc = (A.chunk_first + chunk_local) * KZ;
    const int i0 = tx * kTile, j0 = ty * kTile;
    const int ni = min(kTile, A.nx - i0), nj = min(kTile, A.ny - j0);

    const int tid = threadIdx.x;
    const int lx = tid & (kTile - 1), ly = tid >> 4;
    const bool active = lx < ni && ly < nj;
    // idle lanes of an edge tile shadow a real column so that every LDS read
    // stays inside the staged footprint
    const float di = (float)min(lx, ni - 1), dj = (float)min(ly, nj - 1);

    const T* __restrict__ proj = reinterpret_cast<const T*>(A.proj);
    const size_t view_px = (size_t)A.nh * A.nw;

    float acc[KZ];
#pragma unroll
    for (int kk = 0; kk < KZ; ++kk) acc[kk] = 0.f;

    for (int sb = 0; sb < A.np; sb += kViewBatch) {
        const int nb = min(kViewBatch, A.np - sb);
        __syncthreads();                                      // previous table no longer read
        if (tid < nb) {
            const int s = sb + tid;
            const float sc = A.scale ? A.scale[s] : 1.0f;
            view_record(A.M + 12 * (size_t)s, i0, j0, ni, nj, kc, KZ, sc, PITCH, A.rows, &vtab[tid]);
        }
        __syncthreads();
        for (int qv = 0; qv < nb; ++qv) {
            const ViewRec rec = vtab[qv];
            // ---- stage the footprint of view sb+qv (zero outside the detector)
            {
                const T* src = proj + (size_t)(sb + qv) * view_px;
                const int n = rec.R * rec.C;
                for (int t = tid; t < n; t += kThreads) {
                    const int rr = (int)(((float)t + 0.5f) * rec.invC);
                    const int cc = t - rr * rec.C;
                    const int r = rec.r0 + rr, c = rec.c0 + cc;
                    float val = 0.f;
                    if ((unsigned)r < (unsigned)A.nh && (unsigned)c < (unsigned)A.nw)
                        val = load_px<T>(src + (size_t)r * A.nw + c);
                    tile[rr * PITCH + cc] = val;
                }
            }
            __syncthreads();
            // ---- hoisted per (column, view) quantities
            const float w = fmaf(rec.d, di, fmaf(rec.e, dj, rec.w0));
            const float F = 1.0f / w;
            const float u = fmaf(rec.a, di, fmaf(rec.b, dj, rec.N0)) * F;
            const float v0 = fmaf(rec.g, di, fmaf(rec.h, dj, rec.V0)) * F;
            const float dv = rec.m12 * F;
            const float W = F * F * rec.scale;
            const float fu = __builtin_amdgcn_fractf(u);
            // LDS byte address of column floor(u) of row 0 (u >= 1 inside the tile)
            const unsigned base = lds_addr(tile) + 4u * (unsigned)(int)u;
            // ---- hot loop: KZ updates of this column for this view
#pragma unroll
            for (int kk = 0; kk < KZ; ++kk) {
                const float v = fmaf((float)kk, dv, v0);
                const float fv = __builtin_amdgcn_fractf(v);
                // row floor(v) (v >= 1 inside the tile): one 24-bit multiply-add
                const lds_f32* p = lds_ptr(__umul24((unsigned)(int)v, 4u * PITCH) + base);
                const float p00 = p[0], p01 = p[1], p10 = p[PITCH], p11 = p[PITCH + 1];
                const float h0 = fmaf(fu, p01 - p00, p00);
                const float h1 = fmaf(fu, p11 - p10, p10);
                acc[kk] = fmaf(W, fmaf(fv, h1 - h0, h0), acc[kk]);
            }
            __syncthreads();                                  // tile is overwritten next
        }
    }

    // ---- one read-modify-write of the volume per call
    if (active) {
        const int i = i0 + lx, j = j0 + ly;
#pragma unroll
        for (int kk = 0; kk < KZ; ++kk) {
            const int k = kc + kk;
            if (k >= A.k_begin && k < A.k_end) {
                float* dst = A.vol + ((size_t)(k - A.k_begin) * A.ny + j) * A.nx + i;
                *dst += acc[kk];
            }
        }
    }
}

template <int KZ, int PITCH>
fdk_status launch_kz_pitch(const BpArgs& a, bool f16, size_t lds, unsigned blocks, hipStream_t st)
{
    const void* fn = f16 ? (const void*)bp_kernel<KZ, PITCH, uint16_t>
                         : (const void*)bp_kernel<KZ, PITCH, float>;
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return fail(FDK_E_DEVICE, "cannot raise the LDS limit of the back-projection kernel");
    }
    if (f16)
        hipLaunchKernelGGL((bp_kernel<KZ, PITCH, uint16_t>), dim3(blocks), dim3(kThreads), lds, st, a);
    else
        hipLaunchKernelGGL((bp_kernel<KZ, PITCH, float>), dim3(blocks), dim3(kThreads), lds, st, a);
    return check_launch("back-projection kernel");
}

template <int KZ>
fdk_status launch_kz(const BpArgs& a, int pitch, bool f16, size_t lds, unsigned blocks, hipStream_t st)
{
    switch (pitch) {
        case 48: return launch_kz_pitch<KZ, 48>(a, f16, lds, blocks, st);
        case 80: return launch_kz_pitch<KZ, 80>(a, f16, lds, blocks, st);
        case 112: return launch_kz_pitch<KZ, 112>(a, f16, lds, blocks, st);
        case 144: return launch_kz_pitch<KZ, 144>(a, f16, lds, blocks, st);
        case 176: return launch_kz_pitch<KZ, 176>(a, f16, lds, blocks, st);
        case 208: return launch_kz_pitch<KZ, 208>(a, f16, lds, blocks, st);
        case 240: return launch_kz_pitch<KZ, 240>(a, f16, lds, blocks, st);
    }
    return fail(FDK_E_UNSUPPORTED, "no kernel for this LDS pitch");
}

}  // namespace

fdk_status launch_backproject(const BpLaunch& a, const BpPlan& plan, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    fdk_status s = launch_compose(a.mats_world, a.mats_index, a.np, a.dx, a.dy, a.dz, a.ox, a.oy,
                                  a.oz, stream);
    if (s != FDK_OK) return s;

    const int chunk_first = a.k_begin / plan.kz;
    const int chunk_last = (a.k_end - 1) / plan.kz;
    const int nch = chunk_last - chunk_first + 1;
    BpArgs A;
    A.proj = a.proj;
    A.scale = a.scale;
    A.M = a.mats_index;
    A.vol = a.vol;
    A.nx = a.nx; A.ny = a.ny; A.nz = a.nz; A.np = a.np; A.nh = a.nh; A.nw = a.nw;
    A.k_begin = a.k_begin;
    A.k_end = a.k_end;
    A.ntx = plan.ntx;
    A.ntiles = plan.ntx * plan.nty;
    A.ntiles_pad = plan.ntiles_pad;
    A.chunk_first = chunk_first;
    A.rows = plan.rows;
    const size_t lds = (size_t)plan.lds_bytes;
    const int64_t blocks = (int64_t)plan.ntiles_pad * nch;
    if (blocks >= (1ll << 31)) return fail(FDK_E_UNSUPPORTED, "grid too large");
    switch (plan.kz) {
        case 8: return launch_kz<8>(A, plan.pitch, a.f16, lds, (unsigned)blocks, st);
        case 16: return launch_kz<16>(A, plan.pitch, a.f16, lds, (unsigned)blocks, st);
        case 32: return launch_kz<32>(A, plan.pitch, a.f16, lds, (unsigned)blocks, st);
    }
    return fail(FDK_E_UNSUPPORTED, "no kernel for this slice count");
}

}  // namespace fdk
