// Forward projection as the exact transpose of the back-projector (gfx950).
//
// The back-projection of Listings 1-2 is a fixed linear map p -> vol: every
// voxel reads the four bilinear taps around its (u, v), weighted by 1/w^2.
// Its transpose scatters each voxel value x, weighted by 1/w^2, into the same
// four taps with the same bilinear weights.  Taps outside the detector are
// dropped (the transpose of zero extension).
//
// Ownership by detector pixels: a block owns one band of `rb` detector rows
// of one view, and each of its threads owns whole detector columns of that
// band, so every projection sample is accumulated by exactly one thread and
// no atomics are needed.  With the hoisting of Section 3.1.2 (u and w do not
// depend on k), the voxels whose left or right u-tap is column c form, in
// each volume row, an interval of the lane axis found in closed form (u is a
// Moebius function of the index), and the slices whose v-taps fall in the
// band form one interval of k.  The thread adds each such voxel, weighted by
// its 1/w^2 and bilinear weights, into its column of an LDS window of the band
// (rows r0-1 .. r0+rb); the block then adds rows r0 .. r0+rb-1 of the window
// to the projection.  Blocks of the same band are scheduled side by side and
// read the same slab of the volume.
//
// The lane axis is the volume axis whose step moves u the most (so that each
// column's interval holds one or two voxels); when that axis is y the kernel
// reads a transposed copy of the volume (x and y swapped), which keeps the
// loads of neighbouring columns in the same cache lines.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>

#include "internal.h"

namespace fdk {
namespace {

struct FpArgs {
    const float* vol;        // [nz][ny][nx]
    const float* volT;       // [nz][nx][ny] (x and y swapped), or nullptr if no view needs it
    float* proj;             // [np][nh][nw]
    const double* M;         // [np][12] index-space matrices
    const int* swap;         // [np] 1: lanes along y (read volT)
    int nx, ny, nz, np, nh, nw;
    int rb, pitch;           // band rows; LDS row pitch (columns per chunk + 2)
    int ncb;                 // column chunks of kThreads columns
};

__global__ __launch_bounds__(kThreads) void fp_kernel(const FpArgs A)
{
    extern __shared__ float win[];   // (rb + 2) x pitch
    // blocks of one band (all column chunks, all views) are consecutive
    const int s = blockIdx.x % A.np;
    const int rest = blockIdx.x / A.np;
    const int chunk = rest % A.ncb, band = rest / A.ncb;
    const int r0 = band * A.rb;
    const int cbase = chunk * kThreads;
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int wrows = A.rb + 2;
    for (int q = tid; q < wrows * A.pitch; q += kThreads) win[q] = 0.f;
    __syncthreads();

    const double* m = A.M + 12 * (size_t)s;
    const bool sw = A.swap[s] != 0;
    const float* src = sw ? A.volT : A.vol;
    const int na = sw ? A.ny : A.nx;   // lane axis
    const int nb = sw ? A.nx : A.ny;
    const double ua = sw ? m[1] : m[0], ub = sw ? m[0] : m[1], u3 = m[3];
    const double va = sw ? m[5] : m[4], vb_ = sw ? m[4] : m[5], v3 = m[7], v2 = m[6];
    const double wa = sw ? m[9] : m[8], wb = sw ? m[8] : m[9], w3 = m[11];
    const double inv_v2 = v2 != 0.0 ? 1.0 / v2 : 0.0;
    const double vshift = (double)(r0 - 1);
    const double top = (double)(A.rb + 1);
    const float topf = (float)(A.rb + 1);
    const double kmax = (double)A.nz;
    const size_t slice = (size_t)na * nb;

    const int c = cbase + tid;
    if (c < A.nw) {
        // this thread owns detector column c of the band: window column tid + 1
        float* wc = win + (tid + 1);
        // voxels with floor(u) in {c - 1, c}: u(a) = (ua a + urow) / (wa a + wrow) is a
        // Moebius function of a, monotone across the volume (w > 0), so they form an
        // interval of a per volume row b, bounded by the solutions of u(a) = c -/+ 1
        const double tl = (double)c - 1.0, th = (double)c + 1.0;
        const double dl = ua - tl * wa, dh = ua - th * wa;
        const bool solvable = dl != 0.0 && dh != 0.0;
        const double il = solvable ? 1.0 / dl : 0.0, ih = solvable ? 1.0 / dh : 0.0;
        for (int b = 0; b < nb; ++b) {
            const double db = (double)b;
            const double wrow = fma(wb, db, w3), urow = fma(ub, db, u3), vrow = fma(vb_, db, v3);
            double alo = 0.0, ahi = (double)(na - 1);
            if (solvable) {
                const double x1 = (tl * wrow - urow) * il, x2 = (th * wrow - urow) * ih;
                alo = fmin(x1, x2);
                ahi = fmax(x1, x2);
            }
            const int a0 = (int)floor(fmin(fmax(alo, 0.0), (double)na));
            const int a1 = (int)ceil(fmax(fmin(ahi, (double)(na - 1)), -1.0));
            for (int a = a0; a <= a1; ++a) {
                const double da = (double)a;
                const double w = fma(wa, da, wrow);
                const double F = 1.0 / w;
                const double u = fma(ua, da, urow) * F;
                const double fl = floor(u);
                // bilinear weight of this column: 1 - fu for the left tap, fu for the right
                double wu;
                if (fl == (double)c) wu = 1.0 - (u - fl);
                else if (fl == tl) wu = u - fl;
                else continue;
                // v relative to row r0 - 1 at k = 0, and its step per slice
                const double v0 = fma(va, da, vrow) * F - vshift;
                const double dv = v2 * F;
                // slices with 0 <= v0 + k dv < rb + 1 (taps in window rows 0 .. rb + 1)
                double klo, khi;
                if (dv != 0.0) {
                    const double inv = w * inv_v2;             // 1 / dv
                    const double ka = -v0 * inv, kb = (top - v0) * inv;
                    klo = fmin(ka, kb);
                    khi = fmax(ka, kb);
                } else {
                    if (!(v0 >= 0.0 && v0 < top)) continue;
                    klo = 0.0;
                    khi = kmax;
                }
                // clamped in floating point first, so the conversions stay in range
                const int k0 = (int)floor(fmin(fmax(klo, 0.0), kmax));
                const int k1 = (int)ceil(fmax(fmin(khi, kmax - 1.0), -1.0));
                if (k0 > k1) continue;
                const float Wu = (float)(F * F * wu);
                const float vk0 = (float)fma(dv, (double)k0, v0);
                const float dvf = (float)dv;
                const float* p = src + (size_t)k0 * slice + (size_t)b * na + a;
#pragma unroll 4
                for (int k = k0; k <= k1; ++k, p += slice) {
                    const float x = *p;    // in bounds for every k of the range
                    const float v = fmaf((float)(k - k0), dvf, vk0);
                    if (v >= 0.0f && v < topf) {
                        const int r = (int)v;
                        const float fv = v - (float)r;
                        const float xw = x * Wu;
                        float* q = wc + r * A.pitch;
                        q[0] += xw * (1.0f - fv);
                        q[A.pitch] += xw * fv;
                    }
                }
            }
        }
    }
    __syncthreads();
    // window rows 1 .. rb are detector rows r0 .. r0 + rb - 1; columns 1 .. kThreads
    float* dst = A.proj + (size_t)s * A.nh * A.nw + cbase;
    const int ncol = min(kThreads, A.nw - cbase);
    for (int rr = wave; rr < A.rb; rr += kThreads / 64) {
        const int r = r0 + rr;
        if (r >= A.nh) break;
        const float* wrow_l = win + (rr + 1) * A.pitch + 1;
        float* drow = dst + (size_t)r * A.nw;
        for (int cc = lane; cc < ncol; cc += 64) drow[cc] += wrow_l[cc];
    }
}

// volT[k][i][j] = vol[k][j][i] through a 32 x 33 LDS tile.
__global__ __launch_bounds__(256) void transpose_xy_kernel(const float* __restrict__ vol,
                                                           float* __restrict__ volT, int nx,
                                                           int ny, int tiles_x)
{
    __shared__ float t[32][33];
    const int k = blockIdx.y;
    const int ti = blockIdx.x % tiles_x, tj = blockIdx.x / tiles_x;
    const int i0 = ti * 32, j0 = tj * 32;
    const int lx = threadIdx.x & 31, ly = threadIdx.x >> 5;   // 32 x 8
    const size_t sl = (size_t)nx * ny * k;
    for (int y = ly; y < 32; y += 8) {
        const int i = i0 + lx, j = j0 + y;
        t[y][lx] = (i < nx && j < ny) ? vol[sl + (size_t)j * nx + i] : 0.f;
    }
    __syncthreads();
    for (int y = ly; y < 32; y += 8) {
        const int j = j0 + lx, i = i0 + y;
        if (i < nx && j < ny) volT[sl + (size_t)i * ny + j] = t[lx][y];
    }
}

}  // namespace

int64_t fp_lds_bytes(int rb, int nw) { return (int64_t)(rb + 2) * (std::min(nw, kThreads) + 2) * 4; }

fdk_status make_fp_plan(const fdk_volume& vg, const fdk_stack& sg, FpPlan& plan)
{
    (void)vg;
    // small windows: occupancy (many resident blocks) matters more than the
    // per-column set-up that taller bands would amortise
    int64_t budget = 16 * 1024;
    if (const char* e = std::getenv("FDK_FP_LDS_BUDGET")) budget = std::atoll(e);
    const int pitch = std::min(sg.nw, kThreads) + 2;
    int rb = (int)(budget / (4 * (int64_t)pitch)) - 2;
    if (rb > 64) rb = 64;
    if (rb < 1) rb = 1;
    if (rb > sg.nh) rb = sg.nh;
    if (fp_lds_bytes(rb, sg.nw) > 150 * 1024)
        return fail(FDK_E_UNSUPPORTED, "detector rows too long for the forward projector's LDS window");
    plan.rb = rb;
    plan.pitch = pitch;
    plan.nbands = (sg.nh + rb - 1) / rb;
    plan.ncb = (sg.nw + kThreads - 1) / kThreads;
    plan.lds_bytes = fp_lds_bytes(rb, sg.nw);
    plan.blocks = (int64_t)plan.nbands * plan.ncb * sg.np;
    return FDK_OK;
}

fdk_status launch_forwardproject(const FpLaunch& a, const FpPlan& plan, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (plan.blocks >= (1ll << 31)) return fail(FDK_E_UNSUPPORTED, "grid too large");
    fdk_status s = launch_compose(a.mats_world, a.mats_index, a.np, a.dx, a.dy, a.dz, a.ox, a.oy,
                                  a.oz, stream);
    if (s != FDK_OK) return s;
    if (a.volT) {
        const int tx = (a.nx + 31) / 32, ty = (a.ny + 31) / 32;
        if ((int64_t)tx * ty >= (1ll << 31) || a.nz > 65535)
            return fail(FDK_E_UNSUPPORTED, "volume too large for the transpose kernel");
        hipLaunchKernelGGL(transpose_xy_kernel, dim3((unsigned)(tx * ty), (unsigned)a.nz),
                           dim3(256), 0, st, a.vol, a.volT, a.nx, a.ny, tx);
        s = check_launch("transpose kernel");
        if (s != FDK_OK) return s;
    }
    FpArgs A;
    A.vol = a.vol;
    A.volT = a.volT;
    A.proj = a.proj;
    A.M = a.mats_index;
    A.swap = a.swap;
    A.nx = a.nx; A.ny = a.ny; A.nz = a.nz; A.np = a.np; A.nh = a.nh; A.nw = a.nw;
    A.rb = plan.rb;
    A.pitch = plan.pitch;
    A.ncb = plan.ncb;
    const size_t lds = (size_t)plan.lds_bytes;
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute((const void*)fp_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return fail(FDK_E_DEVICE, "cannot raise the LDS limit of the forward-projection kernel");
    }
    hipLaunchKernelGGL(fp_kernel, dim3((unsigned)plan.blocks), dim3(kThreads), lds, st, A);
    return check_launch("forward-projection kernel");
}

}  // namespace fdk
