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
//     a per-update bounds check).  Each wave stages whole detector rows:
//     float32 rows go straight from memory into LDS (buffer loads with the
//     LDS-direct bit, no VGPR round trip); a buffer descriptor per row makes
//     columns and rows outside the detector read as zero;
//   * binary16 stacks are staged as (p[c], p[c+1]) pairs in one LDS word (the
//     right neighbour arrives by a DPP lane shift), so one LDS read yields
//     both horizontal taps and the lerps run as mixed-precision FMAs on the
//     binary16 halves: FP32 arithmetic, half the LDS bytes per update;
//   * FP64 is used only to compose the index-space matrices and the per-block,
//     per-view bases (coordinates relative to the staged tile), which keeps
//     the FP32 coordinates small and accurate;
//   * block order: z-chunk major so that the resident blocks cover a thin
//     slab and read a narrow band of detector rows; within a chunk each of
//     the 8 XCDs receives a contiguous band of tiles (blocks are dealt to
//     XCDs round-robin by block id), which keeps its L2 footprint small.
#include <hip/hip_runtime.h>

#include "footprint.h"
#include "internal.h"

namespace fdk {
namespace {

// Raw buffer descriptor word 3 for gfx9-family targets (32-bit untyped data).
constexpr int kBufferFlags = 0x00020000;

typedef __attribute__((address_space(3))) const float lds_f32;
typedef __attribute__((address_space(3))) const unsigned lds_u32;
typedef __attribute__((address_space(3))) void lds_void;

// 32-bit LDS byte address of a generic pointer into dynamic shared memory.
__device__ __forceinline__ unsigned lds_addr(const void* p)
{
    return (unsigned)(size_t)(__attribute__((address_space(3))) const char*)p;
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uniform(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}

// p[c] + fu (p[c+1] - p[c]) for a word holding binary16 p[c] (low half) and
// p[c+1] (high half), evaluated in FP32 by mixed-precision FMAs.
__device__ __forceinline__ float lerp_pair_f16(unsigned x, float fu)
{
    float d, h;
    asm("v_fma_mix_f32 %0, %1, 1.0, -%1 op_sel:[1,0,0] op_sel_hi:[1,0,1]" : "=v"(d) : "v"(x));
    asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[0,0,1]" : "=v"(h) : "v"(fu), "v"(d), "v"(x));
    return h;
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

// Stage rows [r0, r0+R) x columns [c0, c0+C) of one view into the LDS tile
// (row pitch PITCH words), zero outside the detector.  Wave w stages rows
// w, w+4, ...; lanes run along the row.
template <int PITCH, bool F16>
__device__ __forceinline__ void stage_view(float* tile, const char* vbase, int nh, int nw,
                                           int r0, int c0, int R, int C, int wave, int lane)
{
    const unsigned row_bytes = (unsigned)nw * (F16 ? 2u : 4u);
    if (!F16) {
        for (int rr = wave; rr < R; rr += kThreads / 64) {
            const int r = r0 + rr;
            const bool ok = (unsigned)r < (unsigned)nh;
            const char* rb = vbase + (ok ? (size_t)r * row_bytes : 0);
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc((void*)rb, 0, ok ? (int)row_bytes : 0, kBufferFlags);
            for (int g = 0; g * 64 < C; ++g) {
                if (g * 64 + lane < C) {
                    // columns left of the detector wrap to huge unsigned
                    // offsets and read as zero like those on the right
                    const unsigned voff = (unsigned)(c0 + g * 64 + lane) * 4u;
                    lds_void* dst = (lds_void*)(size_t)lds_addr(tile + rr * PITCH + g * 64);
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, dst, 4, voff, 0, 0, 0);
                }
            }
        }
    } else {
        // groups of 63 pairs: lane 63 only supplies the right neighbour of lane 62
        for (int rr = wave; rr < R; rr += kThreads / 64) {
            const int r = r0 + rr;
            const bool ok = (unsigned)r < (unsigned)nh;
            const char* rb = vbase + (ok ? (size_t)r * row_bytes : 0);
            const __amdgpu_buffer_rsrc_t rs =
                __builtin_amdgcn_make_buffer_rsrc((void*)rb, 0, ok ? (int)row_bytes : 0, kBufferFlags);
            for (int g = 0; g * 63 < C; ++g) {
                const int cc = g * 63 + lane;
                const unsigned voff = (unsigned)(c0 + cc) * 2u;
                const unsigned lo = __builtin_amdgcn_raw_buffer_load_b16(rs, voff, 0, 0);
                // DPP wave shift left by one lane: lane i receives (lane i+1) << 16
                const unsigned pair =
                    __builtin_amdgcn_update_dpp(0u, lo << 16, 0x130, 0xf, 0xf, false) | lo;
                if (lane < 63 && cc < C)
                    reinterpret_cast<unsigned*>(tile)[rr * PITCH + cc] = pair;
            }
        }
    }
}

template <int KZ, int PITCH, bool F16>
__global__ __launch_bounds__(kThreads) void bp_kernel(const BpArgs A)
{
    extern __shared__ float smem[];
    float* tile = smem;                                       // [rows][PITCH] words
    ViewRec* vtab = reinterpret_cast<ViewRec*>(smem + A.rows * PITCH);

    const BlockPos bp = block_position(blockIdx.x, A.ntiles_pad);
    const int t_id = bp.tile, chunk_local = bp.chunk_local;
    if (t_id >= A.ntiles) return;                             // padding block
    const int tx = t_id % A.ntx, ty = t_id / A.ntx;
    const int kc = (A.chunk_first + chunk_local) * KZ;
    const int i0 = tx * kTile, j0 = ty * kTile;
    const int ni = min(kTile, A.nx - i0), nj = min(kTile, A.ny - j0);

    const int tid = threadIdx.x;
    const int wave = uniform(tid >> 6), lane = tid & 63;
    const int lx = tid & (kTile - 1), ly = tid >> 4;
    const bool active = lx < ni && ly < nj;
    // idle lanes of an edge tile shadow a real column so that every LDS read
    // stays inside the staged footprint
    const float di = (float)min(lx, ni - 1), dj = (float)min(ly, nj - 1);

    const char* proj = reinterpret_cast<const char*>(A.proj);
    const size_t view_bytes = (size_t)A.nh * A.nw * (F16 ? 2 : 4);
    const unsigned tile_base = lds_addr(tile);

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
            const ViewRec& rv = vtab[qv];
            const int c0 = uniform(rv.c0), r0 = uniform(rv.r0);
            const int C = uniform(rv.C), R = uniform(rv.R);
            // ---- stage the footprint of view sb+qv (zero outside the detector)
            stage_view<PITCH, F16>(tile, proj + (size_t)(sb + qv) * view_bytes, A.nh, A.nw, r0, c0,
                                   R, C, wave, lane);
            __builtin_amdgcn_s_waitcnt(0);                    // this wave's LDS writes landed
            __syncthreads();
            // ---- hoisted per (column, view) quantities
            const float w = fmaf(uniform(rv.d), di, fmaf(uniform(rv.e), dj, uniform(rv.w0)));
            float F = __builtin_amdgcn_rcpf(w);
            F = F * fmaf(-w, F, 2.0f);                        // one Newton step
            const float u = fmaf(uniform(rv.a), di, fmaf(uniform(rv.b), dj, uniform(rv.N0))) * F;
            const float v0 = fmaf(uniform(rv.g), di, fmaf(uniform(rv.h), dj, uniform(rv.V0))) * F;
            const float dv = uniform(rv.m12) * F;
            const float W = F * F * uniform(rv.scale);
            const float fu = __builtin_amdgcn_fractf(u);
            // LDS byte address of column floor(u) of row 0 (u >= 1 inside the tile)
            const unsigned base = tile_base + 4u * (unsigned)(int)u;
            // ---- hot loop: KZ updates of this column for this view
#pragma unroll
            for (int kk = 0; kk < KZ; ++kk) {
                const float v = fmaf((float)kk, dv, v0);
                const float fv = __builtin_amdgcn_fractf(v);
                // row floor(v) (v >= 1 inside the tile): one 24-bit multiply-add
                const unsigned at = __umul24((unsigned)(int)v, 4u * PITCH) + base;
                float h0, h1;
                if (F16) {
                    const lds_u32* p = (const lds_u32*)(size_t)at;
                    h0 = lerp_pair_f16(p[0], fu);
                    h1 = lerp_pair_f16(p[PITCH], fu);
                } else {
                    const lds_f32* p = (const lds_f32*)(size_t)at;
                    const float p00 = p[0], p01 = p[1], p10 = p[PITCH], p11 = p[PITCH + 1];
                    h0 = fmaf(fu, p01 - p00, p00);
                    h1 = fmaf(fu, p11 - p10, p10);
                }
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
    const void* fn = f16 ? (const void*)bp_kernel<KZ, PITCH, true>
                         : (const void*)bp_kernel<KZ, PITCH, false>;
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return fail(FDK_E_DEVICE, "cannot raise the LDS limit of the back-projection kernel");
    }
    if (f16)
        hipLaunchKernelGGL((bp_kernel<KZ, PITCH, true>), dim3(blocks), dim3(kThreads), lds, st, a);
    else
        hipLaunchKernelGGL((bp_kernel<KZ, PITCH, false>), dim3(blocks), dim3(kThreads), lds, st, a);
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
