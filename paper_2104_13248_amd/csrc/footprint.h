// Per-(block, view) footprint record shared by the back- and forward
// projectors: which detector window a 16 x 16 x KZ voxel box projects to, and
// FP32 bases of the column coordinates relative to that window, derived in
// FP64 from the index-space matrix.
#pragma once

#include <hip/hip_runtime.h>

namespace fdk {

// Per (block, view) record in LDS, 24 words.  The slices of a chunk are
// processed in two halves; each half has its own row origin so that its FP32
// row coordinates stay below the height of half a footprint.
struct HalfBase {
    float g, h, V0;           // v_loc w = V0 + g di + h dj + m12 t, t = slice - first slice of the half
    int row;                  // LDS tile row of the half's origin
};
struct ViewRec {
    int c0, C;                // staged columns [c0, c0 + C)
    int r0, R;                // rows [r0, r0 + R) staged first
    float d, e, w0;           // w  = w0 + d di + e dj
    float a, b, N0;           // u_loc w = N0 + a di + b dj   (u_loc = u - c0)
    HalfBase half[2];
    float m12;
    float scale;              // dequantisation scale of the view (1 for float32)
    int split;                // 1: the second half's rows [r1, r1 + R1) are staged separately
    int r1, R1;
    int pad;
};
static_assert(sizeof(ViewRec) == 24 * 4, "view record is 24 words");

// The corner loops below are kept rolled: this FP64 code runs once per view
// and block, and unrolling it would raise the register count of the whole
// kernel (and so lower its occupancy).
//
// Rows [first, first + count) that slices ka..kb of the tile reach: the
// projective image of the voxel box is the hull of its corner images, so the
// four corner columns at the two end slices bound it; one row of margin on
// each side absorbs FP32 rounding of the per-thread coordinates.
__device__ inline void footprint_rows(const double* __restrict__ m, const double* ii,
                                      const double* jj, double ka, double kb, int* first, int* count)
{
    double vmin = 0.0, vmax = 0.0;       // seeded by the first corner
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        const int a = q & 1, b = q >> 1;
        const double rw = 1.0 / (m[8] * ii[a] + m[9] * jj[b] + m[11]);
        const double A = m[4] * ii[a] + m[5] * jj[b] + m[7];
        const double v0 = (A + m[6] * ka) * rw;
        const double v1 = (A + m[6] * kb) * rw;
        const double lo = fmin(v0, v1), hi = fmax(v0, v1);
        vmin = q ? fmin(vmin, lo) : lo;
        vmax = q ? fmax(vmax, hi) : hi;
    }
    const double f0 = floor(vmin), f1 = floor(vmax);
    *first = (int)f0 - 1;
    *count = (int)(f1 - f0) + 4;
}

// FP64 bases of one view for one block (tile origin (i0, j0), ni x nj real
// columns, slices kc .. kc + kz - 1).  The window is the footprint of the
// whole chunk when it has at most rows_max rows (or `allow_split` is false);
// otherwise the first half's rows are staged first and the second half's
// separately (each half fits rows_max by construction of the launch plan).
__device__ inline void view_record(const double* __restrict__ m, int i0, int j0, int ni, int nj,
                                   int kc, int kz, float scale, int pitch_max, int rows_max,
                                   bool allow_split, ViewRec* out)
{
    const double ii[2] = {(double)i0, (double)(i0 + ni - 1)};
    const double jj[2] = {(double)j0, (double)(j0 + nj - 1)};
    double umin = 0.0, umax = 0.0;       // seeded by the first corner
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        const int a = q & 1, b = q >> 1;
        const double u = (m[0] * ii[a] + m[1] * jj[b] + m[3]) / (m[8] * ii[a] + m[9] * jj[b] + m[11]);
        umin = q ? fmin(umin, u) : u;
        umax = q ? fmax(umax, u) : u;
    }
    const double fu0 = floor(umin), fu1 = floor(umax);
    const int c0 = (int)fu0 - 1;
    int C = (int)(fu1 - fu0) + 4;
    C = C < pitch_max ? C : pitch_max;     // the launch plan bounds C; clamp for safety
    const int h2 = kz / 2;
    int rf, Rf, ra, Ra, rb, Rb;
    footprint_rows(m, ii, jj, (double)kc, (double)(kc + kz - 1), &rf, &Rf);
    footprint_rows(m, ii, jj, (double)kc, (double)(kc + h2 - 1), &ra, &Ra);
    footprint_rows(m, ii, jj, (double)(kc + h2), (double)(kc + kz - 1), &rb, &Rb);
    const bool split = Rf > rows_max && allow_split;
    const double w0 = m[8] * i0 + m[9] * j0 + m[11];
    out->c0 = c0;
    out->C = C;
    out->d = (float)m[8];
    out->e = (float)m[9];
    out->w0 = (float)w0;
    out->a = (float)(m[0] - c0 * m[8]);
    out->b = (float)(m[1] - c0 * m[9]);
    out->N0 = (float)((m[0] * i0 + m[1] * j0 + m[3]) - c0 * w0);
    const int org[2] = {ra, rb};
    const int ks[2] = {kc, kc + h2};
    for (int q = 0; q < 2; ++q) {
        out->half[q].g = (float)(m[4] - org[q] * m[8]);
        out->half[q].h = (float)(m[5] - org[q] * m[9]);
        out->half[q].V0 = (float)((m[4] * i0 + m[5] * j0 + m[6] * (double)ks[q] + m[7]) - org[q] * w0);
    }
    if (split) {
        out->r0 = ra;
        out->R = Ra < rows_max ? Ra : rows_max;
        out->half[0].row = 0;
        out->half[1].row = 0;
        out->split = 1;
        out->r1 = rb;
        out->R1 = Rb < rows_max ? Rb : rows_max;
    } else {
        // both halves' windows lie inside the whole-chunk window
        out->r0 = rf;
        out->R = Rf < rows_max ? Rf : rows_max;
        out->half[0].row = ra - rf;
        out->half[1].row = rb - rf;
        out->split = 0;
        out->r1 = rb;
        out->R1 = 0;
    }
    out->m12 = (float)m[6];
    out->scale = scale;
    out->pad = 0;
}

// Record of the symmetric variant (Section 3.1.2): the block's kz / 2 direct
// slices kc .. kc + kz/2 - 1 and their mirrors nz - 1 - k.  With v(nz-1-k) =
// nh - 1 - v(k) the mirrored slices read the mirror image of the direct
// window, rows nh - 1 - r0 - q for q = 0 .. R - 1, which the kernel stages in
// that (descending) order, so a mirrored update uses the same window-relative
// row and weight as its direct partner.  `split` is set when the window is
// taller than one of the two LDS regions (region_rows): the two windows are
// then staged one after the other over the whole tile.  half[1] and r1, R1
// are unused.
__device__ inline void view_record_sym(const double* __restrict__ m, int i0, int j0, int ni,
                                       int nj, int kc, int kz, float scale, int pitch_max,
                                       int region_rows, ViewRec* out)
{
    const double ii[2] = {(double)i0, (double)(i0 + ni - 1)};
    const double jj[2] = {(double)j0, (double)(j0 + nj - 1)};
    double umin = 0.0, umax = 0.0;       // seeded by the first corner
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
        const int a = q & 1, b = q >> 1;
        const double u = (m[0] * ii[a] + m[1] * jj[b] + m[3]) / (m[8] * ii[a] + m[9] * jj[b] + m[11]);
        umin = q ? fmin(umin, u) : u;
        umax = q ? fmax(umax, u) : u;
    }
    const double fu0 = floor(umin), fu1 = floor(umax);
    const int c0 = (int)fu0 - 1;
    int C = (int)(fu1 - fu0) + 4;
    C = C < pitch_max ? C : pitch_max;
    const int h2 = kz / 2;
    int ra, Ra;
    footprint_rows(m, ii, jj, (double)kc, (double)(kc + h2 - 1), &ra, &Ra);
    const double w0 = m[8] * i0 + m[9] * j0 + m[11];
    out->c0 = c0;
    out->C = C;
    out->d = (float)m[8];
    out->e = (float)m[9];
    out->w0 = (float)w0;
    out->a = (float)(m[0] - c0 * m[8]);
    out->b = (float)(m[1] - c0 * m[9]);
    out->N0 = (float)((m[0] * i0 + m[1] * j0 + m[3]) - c0 * w0);
    out->half[0].g = (float)(m[4] - ra * m[8]);
    out->half[0].h = (float)(m[5] - ra * m[9]);
    out->half[0].V0 = (float)((m[4] * i0 + m[5] * j0 + m[6] * (double)kc + m[7]) - ra * w0);
    out->half[0].row = 0;
    out->half[1] = out->half[0];
    const int rmax = 2 * region_rows;
    out->r0 = ra;
    out->R = Ra < rmax ? Ra : rmax;
    out->split = Ra > region_rows ? 1 : 0;
    out->r1 = 0;
    out->R1 = 0;
    out->m12 = (float)m[6];
    out->scale = scale;
    out->pad = 0;
}

// Block id -> (chunk, tile).  Chunk-major so that resident blocks cover a thin
// z-slab; blocks are dealt to the 8 XCDs round-robin by id, so XCD x gets the
// contiguous band of tiles [x per, (x+1) per) of every chunk.
struct BlockPos {
    int tile, chunk_local;
};
__device__ __forceinline__ BlockPos block_position(int bid, int ntiles_pad)
{
    const int xcd = bid & 7;
    const int q = bid >> 3;
    const int per = ntiles_pad >> 3;
    BlockPos p;
    p.chunk_local = q / per;
    p.tile = xcd * per + (q - p.chunk_local * per);
    return p;
}

}  // namespace fdk
