// Forward projection as the exact transpose of the back-projector (gfx950).
//
// The back-projection of Listings 1-2 is a fixed linear map p -> vol: every
// voxel reads the four bilinear taps around its (u, v), weighted by 1/w^2.
// Its transpose scatters each voxel value x, weighted by 1/w^2, into the same
// four taps with the same bilinear weights.  Taps outside the detector are
// dropped (the transpose of zero extension).
//
// Both organisations below accumulate one (band of detector rows, chunk of
// columns, view) in an LDS window and add it to the projection once, so every
// projection sample is written by exactly one block, without atomics, and the
// result does not depend on scheduling.  Both use the hoisting of Section
// 3.1.2: u and w do not depend on k, so the voxels whose u-taps fall in given
// columns form, in each volume row, an interval of the lane axis found in
// closed form (u is a Moebius function of the index), and the slices whose
// v-taps fall in the band form one interval of k.
//
// fp_voxel_kernel (the default): lanes own voxels; see its comment.
// fp_kernel (the fallback when the voxel kernel's 31-bit load offsets would
// not cover a tile): each thread owns one detector column of the band and adds
// every voxel that touches it.
//
// The lane axis is the volume axis whose step moves u the most; when that
// axis is y the kernels read a transposed copy of the volume (x and y
// swapped), which keeps the loads of neighbouring lanes in the same lines.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <string>

#include "internal.h"

namespace fdk {
namespace {

// LDS window pitches (words) of the voxel-driven kernel's instantiations.
constexpr int kFpPitches[] = {36, 68, 132, 196, 244};
// Buffer resource word 3 of gfx950 (32-bit format, no swizzle).
constexpr int kBufferFlags = 0x00020000;

struct FpArgs {
    const float* vol;        // [nz][ny][nx]
    const float* volT;       // [nz][nx][ny] (x and y swapped), or nullptr if no view needs it
    float* proj;             // [np][nh][nw]
    const double* M;         // [np][12] index-space matrices
    const int* lanes;        // [np] (S << 1) | swap; swap 1: lanes along y (read volT);
                             // S bounds the voxel kernel's lane stride over the volume
    int nx, ny, nz, np, nh, nw;
    int rb, pitch;           // band rows; LDS row pitch (words)
    int cw, ncb;             // columns per chunk; column chunks
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
    const bool sw = (A.lanes[s] & 1) != 0;
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
        // both ends on one branch of the Moebius function (its asymptote u = ua / wa
        // outside [tl, th]); otherwise the interval is the whole row
        const bool solvable = dl != 0.0 && dh != 0.0 && (dl > 0.0) == (dh > 0.0);
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

// Four slices of one voxel column: x at byte offsets aoff + (k0 + j) sb of
// the segment (slice indices clamped to kl, the segment's last).
__device__ __forceinline__ void load4(__amdgpu_buffer_rsrc_t rs, int aoff, int sb, int k0, int kl,
                                      float x[4])
{
#pragma unroll
    for (int j = 0; j < 4; ++j)
        x[j] = __uint_as_float(
            __builtin_amdgcn_raw_buffer_load_b32(rs, aoff, min(k0 + j, kl) * sb, 0));
}

// Adds four slices of one voxel into its column pair of the window: slice j
// (j <= last) has v = kf dv + v_j; only lanes whose v lies in [0, top) take
// part (window rows floor(v) and floor(v) + 1 <= rb + 1).
template <int P>
__device__ __forceinline__ void add4(float* win, int col, const float x[4], const float vj[4],
                                     float kf, float dvf, float topf, float WL, float WR, int last)
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float v = fmaf(kf, dvf, vj[j]);
        if (j <= last && v >= 0.0f && v < topf) {
            const int r = (int)v;
            const float fv = __builtin_amdgcn_fractf(v), gv = 1.0f - fv;
            float* q = win + (__mul24(r, P) + col);
            const float xl = x[j] * WL, xr = x[j] * WR;
            const float q0 = q[0], q1 = q[1], q2 = q[P], q3 = q[P + 1];
            q[0] = fmaf(xl, gv, q0);
            q[1] = fmaf(xr, gv, q1);
            q[P] = fmaf(xl, fv, q2);
            q[P + 1] = fmaf(xr, fv, q3);
        }
    }
}

// Voxel-driven organisation.  A block is one wave and owns an LDS window of
// rb + 2 rows (band rows r0 - 1 .. r0 + rb) by the columns c0 - 1 .. c0 + cw
// plus two spare columns.  For each volume row b, the voxels whose left u-tap
// lies in columns c0 - 1 .. c0 + cw - 1 form an interval of the lane axis
// (Moebius solve), which the wave covers in passes of 64 voxels spaced S
// apart.  S is chosen per row so that u moves by at least two columns between
// the lanes of a pass; their column pairs {floor(u), floor(u) + 1} are then
// disjoint and stay so for every slice (u does not depend on k), so the lanes'
// read-modify-writes of the window never collide.  Each voxel's set-up (1/w,
// u, its two column weights, v and dv) is done once per band, against once per
// column and band in fp_kernel.
//
// Lanes take part in a slice's update only while their v lies in the band's
// window (lanes without a voxel keep v < 0), so idle lanes cost no LDS
// bandwidth.  P, the window pitch, is a compile-time constant >= cw + 4 (two
// spare columns, where a lane without a voxel points) so that a voxel's four
// taps are one address plus the constant offsets 0, 1, P, P + 1.
template <int P>
__global__ __launch_bounds__(64) void fp_voxel_kernel(const FpArgs A)
{
    extern __shared__ float win[];   // (rb + 2) x P
    const int s = blockIdx.x % A.np;
    const int rest = blockIdx.x / A.np;
    const int chunk = rest % A.ncb, band = rest / A.ncb;
    const int r0 = band * A.rb;
    const int c0 = chunk * A.cw;
    const int cw = min(A.cw, A.nw - c0);
    const int lane = threadIdx.x;
    for (int q = lane; q < (A.rb + 2) * P; q += 64) win[q] = 0.f;
    __syncthreads();

    const double* m = A.M + 12 * (size_t)s;
    const int info = A.lanes[s];
    const bool sw = (info & 1) != 0;
    const int Sv = info >> 1;
    const float* src = sw ? A.volT : A.vol;
    const int na = sw ? A.ny : A.nx;
    const int nb = sw ? A.nx : A.ny;
    const double ua = sw ? m[1] : m[0], ub = sw ? m[0] : m[1], u3 = m[3];
    const double va = sw ? m[5] : m[4], vb_ = sw ? m[4] : m[5], v3 = m[7], v2 = m[6];
    const double wa = sw ? m[9] : m[8], wb = sw ? m[8] : m[9], w3 = m[11];
    const double vshift = (double)(r0 - 1);
    const double top = (double)(A.rb + 1);
    const float topf = (float)(A.rb + 1);
    const double iv2 = v2 != 0.0 ? 1.0 / v2 : 0.0;
    const size_t slice_bytes = (size_t)na * nb * sizeof(float);
    // left taps in window columns 0 .. cw: u in [c0 - 1, c0 + cw)
    const double tl = (double)c0 - 1.0, th = (double)(c0 + cw);
    const double dl = ua - tl * wa, dh = ua - th * wa;
    // both ends on one branch of the Moebius function (its asymptote u = ua / wa
    // outside [tl, th]); otherwise the interval is the whole row
    const bool solvable = dl != 0.0 && dh != 0.0 && (dl > 0.0) == (dh > 0.0);
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
        const int a0 = __builtin_amdgcn_readfirstlane((int)floor(fmin(fmax(alo, 0.0), (double)na)));
        const int a1 = __builtin_amdgcn_readfirstlane((int)ceil(fmax(fmin(ahi, (double)(na - 1)), -1.0)));
        const char* rowp = (const char*)(src + (size_t)b * na);
        // lane stride of this row: |du/da| = |N| / w^2 with N = ua W(b) - wa U(b)
        // and w largest at an end of [a0, a1] (w is affine in a), so S voxels
        // apart u moves by at least 2.0001 columns anywhere in the row; the
        // view's stride, valid for the whole volume, bounds it
        int S = Sv;
        {
            const double nrow = fabs(ua * wrow - wa * urow);
            const double wm = fmax(fma(wa, (double)a0, wrow), fma(wa, (double)a1, wrow));
            if (nrow > 0.0) S = (int)fmin(ceil(2.0001 * wm * wm / nrow), (double)Sv);
            S = __builtin_amdgcn_readfirstlane(max(S, 1));
        }
        const int span = 64 * S;
        for (int t0 = a0; t0 <= a1; t0 += span) {
            // Each lane runs over its own slices, the ones with v in [0, top)
            // (window rows 0 .. rb + 1), starting at its own first slice klb;
            // n, the largest count in the tile, bounds the slice loop.  Over
            // the tile, the count top w / |v2| is largest at its deeper end
            // and the first slice, (vshift w - (va a + vrow)) / v2 or the same
            // with vshift + top, is affine in a: the tile's end voxels bound
            // both (one slice of margin).  The lanes' loads are then the
            // buffer at slice kbase plus a per-lane offset (klb - kbase) sb + 4a
            // plus the slice step t sb (wave-uniform).
            const double as = (double)t0, ae = (double)min(t0 + span - 1, a1);
            const double wS = fma(wa, as, wrow), wE = fma(wa, ae, wrow);
            int n = A.nz, kbase = 0;
            if (v2 != 0.0) {
                const double cnt = top * fmax(wS, wE) * fabs(iv2) + 2.0;
                n = (int)fmin(cnt, (double)A.nz);
                const double nS = fma(va, as, vrow), nE = fma(va, ae, vrow);
                const double k1 = (vshift * wS - nS) * iv2, k2 = ((vshift + top) * wS - nS) * iv2;
                const double k3 = (vshift * wE - nE) * iv2, k4 = ((vshift + top) * wE - nE) * iv2;
                const double klo = fmin(fmin(k1, k2), fmin(k3, k4)) - 1.0;
                kbase = (int)floor(fmin(fmax(klo, 0.0), (double)(A.nz - n)));
            }
            n = __builtin_amdgcn_readfirstlane(n);
            kbase = __builtin_amdgcn_readfirstlane(kbase);
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(rowp + (size_t)kbase * slice_bytes), 0, 0x7fffffff, kBufferFlags);
            const int sb = (int)slice_bytes;
            for (int p = 0; p < S && t0 + p <= a1; ++p) {
                const int a = t0 + p + S * lane;
                // per-voxel set-up; lanes without a voxel in the chunk keep v < 0
                // and load slices kbase .. kbase + n - 1 of voxel t0
                float vb = -1.0f, dvf = 0.0f, WL = 0.0f, WR = 0.0f;
                int col = cw + 2, vo = t0 * 4;
                if (a <= a1) {
                    const double da = (double)a;
                    const double w = fma(wa, da, wrow);
                    const double F = 1.0 / w;
                    const double u = fma(ua, da, urow) * F;
                    const double fl = floor(u);
                    const double v0 = fma(va, da, vrow) * F - vshift;
                    const double dv = v2 * F;
                    // slices with 0 <= v0 + k dv < top, clamped in floating point
                    // first so that the conversions stay in range
                    double klo = 0.0, khi = (double)(A.nz - 1);
                    bool any = true;
                    if (dv != 0.0) {
                        const double inv = w * iv2;   // 1 / dv
                        const double ka = -v0 * inv, kb = (top - v0) * inv;
                        klo = fmin(ka, kb);
                        khi = fmax(ka, kb);
                    } else {
                        any = v0 >= 0.0 && v0 < top;
                    }
                    const int k0 = (int)floor(fmin(fmax(klo, 0.0), (double)A.nz));
                    const int k1 = (int)ceil(fmax(fmin(khi, (double)(A.nz - 1)), -1.0));
                    if (fl >= tl && fl < th && any && k0 <= k1) {
                        col = (int)(fl - tl);
                        const double fu = u - fl, W = F * F;
                        WL = (float)(W * (1.0 - fu));
                        WR = (float)(W * fu);
                        const int klb = max(kbase, min(k0, A.nz - n));
                        vb = (float)fma(dv, (double)klb, v0);
                        dvf = (float)dv;
                        vo = (klb - kbase) * sb + a * 4;
                    }
                }
                // groups of four slices, the loads of the next group in flight
                // while one group is added (two register sets used in turn; the
                // empty asm statements keep each group's loads where they are
                // issued: the compiler would otherwise sink them below the
                // additions to their first use)
                float vj[4];   // v at slices klb + j
#pragma unroll
                for (int j = 0; j < 4; ++j) vj[j] = fmaf((float)j, dvf, vb);
                const int last = n - 1;
                float xa[4], xb[4];
                load4(rs, vo, sb, 0, last, xa);
                for (int t = 0; t <= last; t += 8) {
                    load4(rs, vo, sb, t + 4, last, xb);
                    asm volatile("" ::: "memory");
                    add4<P>(win, col, xa, vj, (float)t, dvf, topf, WL, WR, last - t);
                    if (t + 4 > last) break;
                    load4(rs, vo, sb, t + 8, last, xa);
                    asm volatile("" ::: "memory");
                    add4<P>(win, col, xb, vj, (float)(t + 4), dvf, topf, WL, WR, last - t - 4);
                }
                // the next pass gives the lanes other columns
                asm volatile("" ::: "memory");
            }
        }
    }
    __syncthreads();
    float* dst = A.proj + (size_t)s * A.nh * A.nw + c0;
    for (int rr = 0; rr < A.rb; ++rr) {
        const int r = r0 + rr;
        if (r >= A.nh) break;
        const float* wr = win + (rr + 1) * P + 1;
        float* drow = dst + (size_t)r * A.nw;
        for (int cc = lane; cc < cw; cc += 64) drow[cc] += wr[cc];
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

namespace {

// Window geometry of one organisation: rb rows of a band from the LDS budget.
fdk_status fp_layout(const fdk_stack& sg, bool voxel, FpPlan& plan)
{
    int64_t budget = voxel ? 10 * 1024 : 16 * 1024;
    if (const char* e = std::getenv("FDK_FP_LDS_BUDGET")) budget = std::atoll(e);
    int cw, ncb, pitch = 0;
    if (voxel) {
        // chunks of at most 128 columns (measured best: a row's voxels in a
        // chunk then fill about one tile, and the 10 KB window leaves room for
        // ~15 waves per CU); the pitch, a template constant of at least cw + 4,
        // keeps a voxel's taps (0, 1, pitch, pitch + 1 words) within the
        // offsets of one LDS instruction pair
        int cmax = 128;
        if (const char* e = std::getenv("FDK_FP_CHUNK")) cmax = std::max(16, std::min(240, std::atoi(e)));
        ncb = (sg.nw + cmax - 1) / cmax;
        cw = (sg.nw + ncb - 1) / ncb;
        for (int p : kFpPitches)
            if (pitch == 0 && p >= cw + 4) pitch = p;
    } else {
        cw = std::min(sg.nw, kThreads);
        ncb = (sg.nw + kThreads - 1) / kThreads;
        pitch = cw + 2;
    }
    int rb = (int)(budget / (4 * (int64_t)pitch)) - 2;
    if (rb > 64) rb = 64;
    if (rb < 1) rb = 1;
    if (rb > sg.nh) rb = sg.nh;
    const int64_t lds = (int64_t)(rb + 2) * pitch * 4;
    if (lds > 150 * 1024)
        return fail(FDK_E_UNSUPPORTED, "detector rows too long for the forward projector's LDS window");
    plan.voxel = voxel;
    plan.rb = rb;
    plan.cw = cw;
    plan.pitch = pitch;
    plan.nbands = (sg.nh + rb - 1) / rb;
    plan.ncb = ncb;
    plan.lds_bytes = lds;
    plan.blocks = (int64_t)plan.nbands * plan.ncb * sg.np;
    return FDK_OK;
}

// Whether the voxel-driven kernel's load offsets stay below 2^31 bytes for
// every view: a tile of 64 S voxels reads slices kbase .. kbase + spread + n,
// spread bounded by the slope of the first slice along the lane axis,
// |vshift wa - va| / |v2| per voxel (vshift from -1 to nh + rb), n by
// (rb + 1) wmax / |v2| + 2.
bool fp_voxel_offsets_fit(const fdk_volume& vg, const fdk_stack& sg,
                          const std::vector<IndexMatrix>& M, const std::vector<int32_t>& lanes,
                          int rb)
{
    const double sb = (double)vg.nx * vg.ny * 4.0;
    for (size_t s = 0; s < M.size(); ++s) {
        const double* m = M[s].m;
        const int sw = lanes[s] & 1;
        const double S = (double)(lanes[s] >> 1);
        const double va = sw ? m[5] : m[4], wa = sw ? m[9] : m[8], wb = sw ? m[8] : m[9];
        const int na = sw ? vg.ny : vg.nx, nb = sw ? vg.nx : vg.ny;
        double wmax = 0.0;
        for (double a : {0.0, (double)(na - 1)})
            for (double b : {0.0, (double)(nb - 1)}) wmax = std::max(wmax, wa * a + wb * b + m[11]);
        double slices;
        if (m[6] == 0.0) {
            slices = (double)vg.nz;
        } else {
            const double iv = 1.0 / std::fabs(m[6]);
            const double slope = std::max(std::fabs(-wa - va), std::fabs((sg.nh + rb) * wa - va)) * iv;
            slices = 64.0 * S * slope + 4.0 + (rb + 1) * wmax * iv + 3.0;
        }
        if (std::min(slices, (double)vg.nz + 1.0) * sb + 4.0 * na >= 2147483647.0) return false;
    }
    return true;
}

}  // namespace

fdk_status make_fp_plan(const fdk_volume& vg, const fdk_stack& sg, const std::vector<IndexMatrix>& M,
                        std::vector<int32_t>& lanes, FpPlan& plan)
{
    fp_view_lanes(vg, M, lanes);
    const char* algo = std::getenv("FDK_FP_ALGO");
    const bool voxel = !(algo && std::string(algo) == "gather");
    fdk_status s = fp_layout(sg, voxel, plan);
    if (s != FDK_OK || !voxel) return s;
    if (!fp_voxel_offsets_fit(vg, sg, M, lanes, plan.rb)) return fp_layout(sg, false, plan);
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
    A.lanes = a.lanes;
    A.nx = a.nx; A.ny = a.ny; A.nz = a.nz; A.np = a.np; A.nh = a.nh; A.nw = a.nw;
    A.rb = plan.rb;
    A.pitch = plan.pitch;
    A.cw = plan.cw;
    A.ncb = plan.ncb;
    const size_t lds = (size_t)plan.lds_bytes;
    const void* fn = (const void*)fp_kernel;
    if (plan.voxel) {
        switch (plan.pitch) {
        case kFpPitches[0]: fn = (const void*)fp_voxel_kernel<kFpPitches[0]>; break;
        case kFpPitches[1]: fn = (const void*)fp_voxel_kernel<kFpPitches[1]>; break;
        case kFpPitches[2]: fn = (const void*)fp_voxel_kernel<kFpPitches[2]>; break;
        case kFpPitches[3]: fn = (const void*)fp_voxel_kernel<kFpPitches[3]>; break;
        case kFpPitches[4]: fn = (const void*)fp_voxel_kernel<kFpPitches[4]>; break;
        default: return fail(FDK_E_UNSUPPORTED, "forward-projector pitch without a kernel");
        }
    }
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
            hipSuccess)
            return fail(FDK_E_DEVICE, "cannot raise the LDS limit of the forward-projection kernel");
    }
    void* args[] = {&A};
    if (hipLaunchKernel(fn, dim3((unsigned)plan.blocks), dim3(plan.voxel ? 64 : kThreads), args,
                        lds, st) != hipSuccess)
        return fail(FDK_E_DEVICE, "forward-projection kernel launch failed");
    return check_launch("forward-projection kernel");
}

}  // namespace fdk
