// Per-(block, view) footprint record shared by the back- and forward
// projectors: which detector window a 16 x 16 x KZ voxel box projects to, and
// FP32 bases of the column coordinates relative to that window, derived in
// FP64 from the index-space matrix.
#pragma once

#include <hip/hip_runtime.h>

namespace fdk {

// Per (block, view) record in LDS, 16 words.
struct ViewRec {
    int c0, r0, C, R;         // staged footprint: columns [c0, c0+C), rows [r0, r0+R)
    float d, e, w0;           // w  = w0 + d di + e dj
    float a, b, N0;           // u_loc w = N0 + a di + b dj   (u_loc = u - c0)
    float g, h, V0;           // v_loc w = V0 + g di + h dj + m12 kk (v_loc = v - r0)
    float m12;
    float scale;              // dequantisation scale of the view (1 for float32)
    float invC;               // 1 / C, for the staging index split
};
static_assert(sizeof(ViewRec) == 16 * 4, "view record is 16 words");

// FP64 bases of one view for one block.  Footprint from the four corner
// columns of the tile and the two end slices of the chunk (the projective
// image of the voxel box is the hull of its corner images), with one pixel of
// margin on each side for FP32 rounding of the per-thread coordinates.
__device__ inline void view_record(const double* __restrict__ m, int i0, int j0, int ni, int nj, int kc,
                            int kz, float scale, int pitch_max, int rows_max, ViewRec* out)
{
    const double ii[2] = {(double)i0, (double)(i0 + ni - 1)};
    const double jj[2] = {(double)j0, (double)(j0 + nj - 1)};
    double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const double w = m[8] * ii[a] + m[9] * jj[b] + m[11];
            const double rw = 1.0 / w;
            const double u = (m[0] * ii[a] + m[1] * jj[b] + m[3]) * rw;
            const double A = m[4] * ii[a] + m[5] * jj[b] + m[7];
            const double v0 = (A + m[6] * (double)kc) * rw;
            const double v1 = (A + m[6] * (double)(kc + kz - 1)) * rw;
            umin = fmin(umin, u);
            umax = fmax(umax, u);
            vmin = fmin(vmin, fmin(v0, v1));
            vmax = fmax(vmax, fmax(v0, v1));
        }
    const double fu0 = floor(umin), fu1 = floor(umax), fv0 = floor(vmin), fv1 = floor(vmax);
    const int c0 = (int)fu0 - 1;
    const int r0 = (int)fv0 - 1;
    int C = (int)(fu1 - fu0) + 4;
    int R = (int)(fv1 - fv0) + 4;
    C = C < pitch_max ? C : pitch_max;     // the launch plan bounds both; clamp for safety
    R = R < rows_max ? R : rows_max;
    const double w0 = m[8] * i0 + m[9] * j0 + m[11];
    out->c0 = c0;
    out->r0 = r0;
    out->C = C;
    out->R = R;
    out->d = (float)m[8];
    out->e = (float)m[9];
    out->w0 = (float)w0;
    out->a = (float)(m[0] - c0 * m[8]);
    out->b = (float)(m[1] - c0 * m[9]);
    out->N0 = (float)((m[0] * i0 + m[1] * j0 + m[3]) - c0 * w0);
    out->g = (float)(m[4] - r0 * m[8]);
    out->h = (float)(m[5] - r0 * m[9]);
    out->V0 = (float)((m[4] * i0 + m[5] * j0 + m[6] * (double)kc + m[7]) - r0 * w0);
    out->m12 = (float)m[6];
    out->scale = scale;
    out->invC = 1.0f / (float)C;
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
