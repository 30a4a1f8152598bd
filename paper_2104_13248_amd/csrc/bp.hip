// Voxel-driven FDK back-projection for gfx950 (MI355X).
//
// What is computed (Chen et al., ICS'21, Listings 1-2, Algorithm 1):
//   vol[k][j][i] += sum_s scale_s / w^2 * bilinear(p_s, u, v)
// with (u w, v w, w) = M_s (i, j, k, 1) and zero outside the detector.
//
// How (GPU design; the paper's CPU kernels are prior art):
//   * one thread per voxel column (i, j) of a 16 x 16 tile, each wave an 8 x 8
//     quarter of it; each thread keeps
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
//     LDS-direct bit, no VGPR round trip); the buffer's range check makes
//     rows and columns outside the detector read as zero;
//   * the LDS tile is sized for nearly every (block, view) footprint; the
//     rare taller ones (blocks near the source at a large cone angle) are
//     staged and consumed in two half-chunks of slices, which keeps the LDS
//     per block small and the occupancy high;
//   * binary16 stacks are staged as (p[c], p[c+1]) pairs in one LDS word, in
//     two regions (pairs at even and at odd offsets, the second loaded 2
//     bytes further), so one LDS read yields both horizontal taps and the
//     lerps run as mixed-precision FMAs on the binary16 halves: FP32
//     arithmetic, half the LDS bytes per update;
//   * FP64 composes the index-space matrices and the per-block, per-view
//     bases (coordinates relative to the staged tile, which keeps the FP32
//     coordinates small and accurate); launches with windows 120 words wide
//     or more also run each thread's per-view set-up in FP64;
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

// Voxel column (x, y within the 16 x 16 tile) of thread t of bp_kernel: each
// wave takes an 8 x 8 quarter of the tile.  A half-wave's 32 lanes then span
// 8 x 4 columns, whose projections reach fewer detector rows and columns than
// 16 x 2 columns would (the depth, and so v, varies across a row of the
// tile): C3 LDS bank conflicts 34% -> 26% of LDS time (float32 taps), 22% ->
// 15% (binary16), float32 storage 4% faster.
__device__ __forceinline__ int col_x(int t) { return ((t >> 6) & 1) * 8 + (t & 7); }
__device__ __forceinline__ int col_y(int t) { return (t >> 7) * 8 + ((t >> 3) & 7); }
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

// Launch pitches from which the back-projector's per-(column, view) set-up
// runs in FP64 (windows that wide arise only under strong magnification).
constexpr int kPreciseSetupPitch = 120;

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

// Words per LDS row: float32 rows hold PITCH pixels; binary16 rows are two
// regions of pair-word half-rows (even and odd offsets), PITCH / 2 words each.
template <int PITCH, bool F16>
struct TileRow {
    static constexpr int W = F16 ? PITCH / 2 : PITCH;
};

// Stage rows [r0, r0+R) x columns [c0, c0+C) of one view into the LDS tile,
// zero outside the detector (REV: rows r0, r0 - 1, .., r0 - R + 1, tile row rr
// holding detector row r0 - rr).  One buffer descriptor covers the view; an
// out-of-range offset reads as zero.  The tile has `ralloc` rows of
// TileRow::W words (float32), or two such regions (binary16: even-offset
// pairs, then odd-offset pairs).
//
// A window inside the detector's columns is staged by 16-byte loads straight
// into LDS, whole rows at a time: a row of W words takes W / 4 lanes, so one
// instruction stages 64 / (W / 4) rows and the lanes of a row land side by
// side.  Other windows are staged by 4-byte loads: lanes along a row, wave w
// taking rows w, w + 4, ...
template <int PITCH, bool F16, bool REV = false>
__device__ __forceinline__ void stage_rows(float* tile, int ralloc, const __amdgpu_buffer_rsrc_t& rs,
                                           int nh, unsigned row_bytes, int nw, int r0, int c0, int R,
                                           int C, int wave, int lane)
{
    constexpr int kWaves = kThreads / 64;
    constexpr unsigned kOut = 0x80000000u;   // beyond any view: the load returns zero
    constexpr int RW = TileRow<PITCH, F16>::W;
    constexpr int SEG = RW / 4;               // 16-byte lanes per row
    constexpr int RPI = 64 / SEG;             // rows per instruction
    static_assert(RW % 4 == 0 && RPI >= 1, "row width");
    unsigned* wtile = reinterpret_cast<unsigned*>(tile);
    {
        const int cs = F16 ? (c0 & ~1) : c0;                  // first staged pixel
        const int span = F16 ? 8 * SEG + 1 : 4 * SEG;         // pixels a row's loads read
        if (cs >= 0 && cs + span <= nw) {
            // The descriptor's range check zeroes the rows outside the
            // detector: a row above it has a negative offset (>= 2^31 as
            // unsigned), a row below it an offset >= the view's bytes (< 2^31).
            // The odd-offset pairs of binary16 rows are the same loads 2 bytes
            // further (the instruction's immediate offset).
            // A window wholly above or below the detector is zero wherever it
            // starts: clamping its first row to [-R, nh] (descending: [-1,
            // nh + R - 1]) keeps every offset within +-(nh + R) rows, which
            // the launch plan bounds below 2^31 bytes.
            const int r0c = REV ? min(max(r0, -1), nh + R - 1) : min(max(r0, -R), nh);
            const int rsub = lane / SEG, sg = lane - rsub * SEG;
            const int colb = cs * (F16 ? 2 : 4) + 16 * sg;
            const int rstep = kWaves * RPI;
            const int ostep = (REV ? -rstep : rstep) * (int)row_bytes;
            int vo = (REV ? r0c - (wave * RPI + rsub) : r0c + wave * RPI + rsub) * (int)row_bytes + colb;
            for (int rr0 = wave * RPI; rr0 < R; rr0 += rstep, vo += ostep) {
                if (rsub < RPI && rr0 + rsub < R) {
                    lds_void* d = (lds_void*)(size_t)lds_addr(tile + rr0 * RW);
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, d, 16, (unsigned)vo, 0, 0, 0);
                    if (F16) {
                        lds_void* d2 = (lds_void*)(size_t)lds_addr(tile + (ralloc + rr0) * RW);
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, d2, 16, (unsigned)vo, 0, 2, 0);
                    }
                }
            }
            return;
        }
    }
    if (!F16) {
        for (int g = 0; g * 64 < C; ++g) {
            const int cc = g * 64 + lane;
            const int c = c0 + cc;
            const unsigned voff = (unsigned)c < (unsigned)nw ? (unsigned)c * 4u : kOut;
            const bool keep = cc < C;
            for (int rr = wave; rr < R; rr += kWaves) {
                const int r = REV ? r0 - rr : r0 + rr;
                if ((unsigned)r < (unsigned)nh) {
                    if (keep) {
                        lds_void* dst = (lds_void*)(size_t)lds_addr(tile + rr * PITCH + g * 64);
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, dst, 4, voff,
                                                                 (unsigned)r * row_bytes, 0, 0);
                    }
                } else if (keep) {
                    wtile[rr * PITCH + cc] = 0u;
                }
            }
        }
    } else {
        // Binary16 rows are staged as pair words by asynchronous dword loads
        // straight into LDS: EV[m] holds pixels (ce+2m, ce+2m+1) (aligned
        // loads) and OD[m] pixels (ce+2m+1, ce+2m+2) (2-byte aligned loads),
        // ce = c0 rounded down to even, in two regions of half-rows.  The pair
        // (p[c], p[c+1]) of column c is EV[(c-ce)/2] or OD[(c-ce-1)/2].  A word
        // with one pixel outside the detector is rewritten afterwards from a
        // 16-bit load of its valid pixel.
        constexpr int HP = PITCH / 2;
        const int ce = c0 & ~1;
        int NE = (C + (c0 - ce) + 1) >> 1;
        NE = NE < HP ? NE : HP;
        for (int g = 0; g * 64 < NE; ++g) {
            const int mm = g * 64 + lane;
            const int pe = ce + 2 * mm, po = pe + 1;
            const unsigned voe = (unsigned)pe < (unsigned)nw ? (unsigned)pe * 2u : kOut;
            const unsigned voo = (unsigned)po < (unsigned)nw ? (unsigned)po * 2u : kOut;
            const bool keep = mm < NE;
            for (int rr = wave; rr < R; rr += kWaves) {
                const int r = REV ? r0 - rr : r0 + rr;
                if ((unsigned)r < (unsigned)nh) {
                    if (keep) {
                        lds_void* de = (lds_void*)(size_t)lds_addr(tile + rr * HP + g * 64);
                        lds_void* dd = (lds_void*)(size_t)lds_addr(tile + (ralloc + rr) * HP + g * 64);
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, de, 4, voe, (unsigned)r * row_bytes, 0, 0);
                        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, dd, 4, voo, (unsigned)r * row_bytes, 0, 0);
                    }
                } else if (keep) {
                    wtile[rr * HP + mm] = 0u;
                    wtile[(ralloc + rr) * HP + mm] = 0u;
                }
            }
        }
        // words straddling the detector edges (uniform test: the window
        // reaches column -1 or column nw)
        const int mleft = (-2 - ce) >> 1;                       // OD word (p[-1], p[0])
        const int jr = nw - 1 - ce;                             // word starting at p[nw-1]
        const int mright = jr >> 1, right_od = jr & 1;
        const bool fix_left = ce <= -2 && mleft < NE;
        const bool fix_right = jr >= 0 && mright < NE;
        if (fix_left || fix_right) {
            __builtin_amdgcn_s_waitcnt(0);                    // this wave's row loads landed
            for (int rr = wave; rr < R; rr += kWaves) {
                const int r = REV ? r0 - rr : r0 + rr;
                if ((unsigned)r >= (unsigned)nh) continue;
                if (fix_left && lane == 0) {
                    const unsigned p0 = __builtin_amdgcn_raw_buffer_load_b16(rs, 0u, (unsigned)r * row_bytes, 0);
                    wtile[(ralloc + rr) * HP + mleft] = p0 << 16;
                }
                if (fix_right && lane == 1) {
                    const unsigned pl = __builtin_amdgcn_raw_buffer_load_b16(
                        rs, (unsigned)(nw - 1) * 2u, (unsigned)r * row_bytes, 0);
                    wtile[((right_od ? ralloc : 0) + rr) * HP + mright] = pl;
                }
            }
        }
    }
}

// Taps of update kk of a column for one view: the two pair words (binary16)
// or four words (float32) around row floor(v), column floor(u); v >= 1 inside
// the tile.
template <int PITCH, bool F16>
__device__ __forceinline__ void load_taps(unsigned base, float v, unsigned (&t)[4], float& fv)
{
    constexpr int RW = TileRow<PITCH, F16>::W;
    fv = __builtin_amdgcn_fractf(v);
    const lds_u32* p = (const lds_u32*)(size_t)(__umul24((unsigned)(int)v, 4u * RW) + base);
    t[0] = p[0];
    t[2] = p[RW];
    if (!F16) {
        t[1] = p[1];
        t[3] = p[RW + 1];
    }
}

// Bilinear value at (floor(u) + fu, floor(v) + fv) from the taps of load_taps
// (Listing 2: horizontal lerps of the two rows, then the vertical one).
template <bool F16>
__device__ __forceinline__ float bilinear(const unsigned (&t)[4], float fu, float fv)
{
    float h0, h1;
    if (F16) {
        // lerp_pair_f16 of both rows, the two rows' differences first: no
        // instruction then reads the result of the one just before it (a
        // hazard wait after each mixed-precision FMA otherwise)
        float d0, d1;
        asm("v_fma_mix_f32 %0, %1, 1.0, -%1 op_sel:[1,0,0] op_sel_hi:[1,0,1]" : "=v"(d0) : "v"(t[0]));
        asm("v_fma_mix_f32 %0, %1, 1.0, -%1 op_sel:[1,0,0] op_sel_hi:[1,0,1]" : "=v"(d1) : "v"(t[2]));
        asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[0,0,1]" : "=v"(h0) : "v"(fu), "v"(d0), "v"(t[0]));
        asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel_hi:[0,0,1]" : "=v"(h1) : "v"(fu), "v"(d1), "v"(t[2]));
    } else {
        const float p00 = __builtin_bit_cast(float, t[0]), p01 = __builtin_bit_cast(float, t[1]);
        const float p10 = __builtin_bit_cast(float, t[2]), p11 = __builtin_bit_cast(float, t[3]);
        h0 = fmaf(fu, p01 - p00, p00);
        h1 = fmaf(fu, p11 - p10, p10);
    }
    return fmaf(fv, h1 - h0, h0);
}

// KZ/2 consecutive updates kk = k0 + t, t = 0 .. KZ/2 - 1, of one column for
// one view; v = v0 + t dv (v0 itself at t = 0: the compiler cannot drop an FMA
// by zero) is the row coordinate relative to the half's origin,
// whose LDS row address (plus the column) is `base`.  Tap loads run
// kPrefetch updates ahead of their use.
template <int KZ, int PITCH, bool F16>
__device__ __forceinline__ void update_half(float (&acc)[KZ], int k0, unsigned base, float v0,
                                            float dv, float fu, float W)
{
    constexpr int kPrefetch = KZ / 2 < 8 ? KZ / 2 : 8;
#pragma unroll
    for (int g0 = 0; g0 < KZ / 2; g0 += kPrefetch) {
        float fv[kPrefetch];
        unsigned t[kPrefetch][4];
#pragma unroll
        for (int q = 0; q < kPrefetch; ++q)
            load_taps<PITCH, F16>(base, g0 + q == 0 ? v0 : fmaf((float)(g0 + q), dv, v0), t[q], fv[q]);
#pragma unroll
        for (int q = 0; q < kPrefetch; ++q)
            acc[k0 + g0 + q] = fmaf(W, bilinear<F16>(t[q], fu, fv[q]), acc[k0 + g0 + q]);
    }
}

// All KZ updates of one column for one view, in groups of two whose tap
// loads are issued one group ahead: the two halves (row origins base0 /
// base1, v origins v00 / v01) form one sequence.  When the footprint is
// staged per half (`split`), `restage` replaces the window between the
// halves and the second half's first loads wait for it; otherwise they are
// in flight while the first half's last group is added.  A scheduling
// barrier separates each group's loads from the previous group's arithmetic:
// the scheduler would otherwise either hoist all loads (and run out of
// registers) or sink them to their first use.
template <int KZ, int PITCH, bool F16, typename Restage>
__device__ __forceinline__ void update_column(float (&acc)[KZ], unsigned base0, unsigned base1,
                                              float v00, float v01, float dv, float fu, float W,
                                              bool split, Restage restage)
{
    constexpr int H = KZ / 2;
    constexpr int G = 2;
    constexpr int NG = KZ / G;
    static_assert(H % G == 0, "groups do not straddle the halves");
    unsigned t[2][G][4];
    float fv[2][G];
    auto load_group = [&](int g) {
        const int k = g * G;
        const unsigned b = k < H ? base0 : base1;
        const float v0 = k < H ? v00 : v01;
        const int t0 = k < H ? k : k - H;
#pragma unroll
        for (int q = 0; q < G; ++q)
            load_taps<PITCH, F16>(b, t0 + q == 0 ? v0 : fmaf((float)(t0 + q), dv, v0), t[g & 1][q],
                                  fv[g & 1][q]);
    };
    load_group(0);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if (g + 1 < NG && (g + 1 != NG / 2 || !split)) load_group(g + 1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int q = 0; q < G; ++q)
            acc[g * G + q] = fmaf(W, bilinear<F16>(t[g & 1][q], fu, fv[g & 1][q]), acc[g * G + q]);
        if (g + 1 == NG / 2 && split) {
            restage();
            load_group(g + 1);
        }
    }
}

// Symmetric variant (Section 3.1.2): KZ/2 direct slices kk = t and their
// mirrors kk = KZ/2 + t.  The mirrored window is staged in descending row
// order `moff` bytes after the direct one, so a mirrored update reads the same
// window-relative rows with the same weights: v, its row and fraction, and the
// LDS address are computed once for both updates.
template <int KZ, int PITCH, bool F16>
__device__ __forceinline__ void update_pair(float (&acc)[KZ], unsigned base, unsigned moff, float v0,
                                            float dv, float fu, float W)
{
    constexpr int H = KZ / 2;
    constexpr int kPrefetch = H < 4 ? H : 4;
    constexpr int RW = TileRow<PITCH, F16>::W;
#pragma unroll
    for (int g0 = 0; g0 < H; g0 += kPrefetch) {
        float fv[kPrefetch];
        unsigned t[kPrefetch][4], tm[kPrefetch][4];
#pragma unroll
        for (int q = 0; q < kPrefetch; ++q) {
            const float v = fmaf((float)(g0 + q), dv, v0);
            fv[q] = __builtin_amdgcn_fractf(v);
            const unsigned addr = __umul24((unsigned)(int)v, 4u * RW) + base;
            const lds_u32* p = (const lds_u32*)(size_t)addr;
            const lds_u32* pm = (const lds_u32*)(size_t)(addr + moff);
            t[q][0] = p[0];
            t[q][2] = p[RW];
            tm[q][0] = pm[0];
            tm[q][2] = pm[RW];
            if (!F16) {
                t[q][1] = p[1];
                t[q][3] = p[RW + 1];
                tm[q][1] = pm[1];
                tm[q][3] = pm[RW + 1];
            }
        }
#pragma unroll
        for (int q = 0; q < kPrefetch; ++q) {
            float h0, h1, m0, m1;
            if (F16) {
                h0 = lerp_pair_f16(t[q][0], fu);
                h1 = lerp_pair_f16(t[q][2], fu);
                m0 = lerp_pair_f16(tm[q][0], fu);
                m1 = lerp_pair_f16(tm[q][2], fu);
            } else {
                const float p00 = __builtin_bit_cast(float, t[q][0]), p01 = __builtin_bit_cast(float, t[q][1]);
                const float p10 = __builtin_bit_cast(float, t[q][2]), p11 = __builtin_bit_cast(float, t[q][3]);
                const float q00 = __builtin_bit_cast(float, tm[q][0]), q01 = __builtin_bit_cast(float, tm[q][1]);
                const float q10 = __builtin_bit_cast(float, tm[q][2]), q11 = __builtin_bit_cast(float, tm[q][3]);
                h0 = fmaf(fu, p01 - p00, p00);
                h1 = fmaf(fu, p11 - p10, p10);
                m0 = fmaf(fu, q01 - q00, q00);
                m1 = fmaf(fu, q11 - q10, q10);
            }
            acc[g0 + q] = fmaf(W, fmaf(fv[q], h1 - h0, h0), acc[g0 + q]);
            acc[H + g0 + q] = fmaf(W, fmaf(fv[q], m1 - m0, m0), acc[H + g0 + q]);
        }
    }
}

// Symmetric variant of the back-projector (Section 3.1.2) for geometries with
// v(nz - 1 - k) = nh - 1 - v(k) (circular orbit, detector row centre at the
// orbit plane, volume centred on it): a block owns KZ/2 slices of the lower
// half of the volume and their mirrors.  Per view it stages the direct window
// (rows r0 ..) in LDS region 0 and the mirrored one (rows nh - 1 - r0, nh -
// 2 - r0, ..) in region 1, then runs the paired updates; a window taller than
// one region is staged alone over the whole tile, direct then mirrored.
template <int KZ, int PITCH, bool F16>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void bp_sym_kernel(const BpArgs A)
{
    static_assert(KZ % 2 == 0, "slices are paired");
    constexpr int H = KZ / 2;
    constexpr int RW = TileRow<PITCH, F16>::W;
    extern __shared__ float smem[];
    float* tile = smem;                                       // [rows][PITCH] words
    ViewRec* vtab = reinterpret_cast<ViewRec*>(smem + A.rows * PITCH);

    const BlockPos bp = block_position(blockIdx.x, A.ntiles_pad);
    const int t_id = bp.tile, chunk_local = bp.chunk_local;
    if (t_id >= A.ntiles) return;                             // padding block
    const int tx = t_id % A.ntx, ty = t_id / A.ntx;
    const int kc = chunk_local * H;                           // first direct slice
    const int i0 = tx * kTile, j0 = ty * kTile;
    const int ni = min(kTile, A.nx - i0), nj = min(kTile, A.ny - j0);

    const int tid = threadIdx.x;
    const int wave = uniform(tid >> 6), lane = tid & 63;
    const int lx = tid & (kTile - 1), ly = tid >> 4;
    const bool active = lx < ni && ly < nj;
    const float di = (float)min(lx, ni - 1), dj = (float)min(ly, nj - 1);

    const char* proj = reinterpret_cast<const char*>(A.proj);
    const unsigned row_bytes = (unsigned)A.nw * (F16 ? 2u : 4u);
    const unsigned view_bytes = row_bytes * (unsigned)A.nh;
    const unsigned tile_base = lds_addr(tile);
    const int rr = A.rows / 2;                                // rows per region
    float* mtile = tile + rr * RW;                            // region 1
    const unsigned moff = 4u * (unsigned)(rr * RW);

    float acc[KZ];
#pragma unroll
    for (int kk = 0; kk < KZ; ++kk) acc[kk] = 0.f;

    for (int sb = 0; sb < A.np; sb += kViewBatch) {
        const int nb = min(kViewBatch, A.np - sb);
        __syncthreads();
        if (tid < nb) {
            const int s = sb + tid;
            const float sc = A.scale ? A.scale[s] : 1.0f;
            view_record_sym(A.M + 12 * (size_t)s, i0, j0, ni, nj, kc, KZ, sc, PITCH, rr, &vtab[tid]);
        }
        __syncthreads();
        for (int qv = 0; qv < nb; ++qv) {
            const ViewRec& rv = vtab[qv];
            const int c0 = uniform(rv.c0), C = uniform(rv.C);
            const int r0 = uniform(rv.r0), R = uniform(rv.R);
            const bool split = uniform(rv.split) != 0;
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(proj + (size_t)(sb + qv) * view_bytes), 0, (int)view_bytes, kBufferFlags);
            stage_rows<PITCH, F16>(tile, A.rows, rs, A.nh, row_bytes, A.nw, r0, c0, R, C, wave, lane);
            if (!split)
                stage_rows<PITCH, F16, true>(mtile, A.rows, rs, A.nh, row_bytes, A.nw, A.nh - 1 - r0, c0,
                                             R, C, wave, lane);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            const float w = fmaf(uniform(rv.d), di, fmaf(uniform(rv.e), dj, uniform(rv.w0)));
            float F = __builtin_amdgcn_rcpf(w);
            F = F * fmaf(-w, F, 2.0f);                        // one Newton step
            const float u = fmaf(uniform(rv.a), di, fmaf(uniform(rv.b), dj, uniform(rv.N0))) * F;
            const float dv = uniform(rv.m12) * F;
            const float W = F * F * uniform(rv.scale);
            const float fu = __builtin_amdgcn_fractf(u);
            unsigned base;
            if (F16) {
                const int j = (int)u + (c0 & 1);
                base = tile_base + 4u * (unsigned)((j >> 1) + ((j & 1) ? A.rows * (PITCH / 2) : 0));
            } else {
                base = tile_base + 4u * (unsigned)(int)u;
            }
            const HalfBase& hb = rv.half[0];
            const float v0 = fmaf(uniform(hb.g), di, fmaf(uniform(hb.h), dj, uniform(hb.V0))) * F;
            if (!split) {
                update_pair<KZ, PITCH, F16>(acc, base, moff, v0, dv, fu, W);
            } else {
                update_half<KZ, PITCH, F16>(acc, 0, base, v0, dv, fu, W);
                __syncthreads();
                stage_rows<PITCH, F16, true>(tile, A.rows, rs, A.nh, row_bytes, A.nw, A.nh - 1 - r0, c0,
                                             R, C, wave, lane);
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
                update_half<KZ, PITCH, F16>(acc, H, base, v0, dv, fu, W);
            }
            __syncthreads();                                  // tile is overwritten next
        }
    }

    // ---- one read-modify-write per direct slice and per mirror
    if (active) {
        const int i = i0 + lx, j = j0 + ly;
#pragma unroll
        for (int t = 0; t < H; ++t) {
            const int kd = kc + t, km = A.nz - 1 - kd;
            if (kd <= km) {
                float* dst = A.vol + ((size_t)kd * A.ny + j) * A.nx + i;
                *dst += acc[t];
            }
            if (km > kd) {
                float* dst = A.vol + ((size_t)km * A.ny + j) * A.nx + i;
                *dst += acc[H + t];
            }
        }
    }
}

// Sub-line variant (Section 3.1.5 and Algorithm 1's sub-line step): per
// (column, view) the detector columns floor(u) and floor(u) + 1 are blended
// once, with the column's weight fu, along every row its KZ slices reach,
// into a line in LDS; each update is then one 1-D interpolation along that
// line.  Lines are stored row-major with the thread index fastest
// ([line_rows][256] words): a lane reads and writes only its own column of
// them, so the lanes of a wave meet in distinct banks whatever their rows and
// no barrier is needed between blending and use.  The window holds every
// whole-chunk footprint (the plan sizes it so); float32 stacks only.
template <int KZ, int PITCH>
__global__ __launch_bounds__(kThreads) void bp_subline_kernel(const BpArgs A, int line_rows)
{
    extern __shared__ float smem[];
    float* tile = smem;                                       // [rows][PITCH] words
    float* lines = smem + A.rows * PITCH;                     // [line_rows][kThreads]
    ViewRec* vtab = reinterpret_cast<ViewRec*>(lines + line_rows * kThreads);

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
    const float di = (float)min(lx, ni - 1), dj = (float)min(ly, nj - 1);

    const char* proj = reinterpret_cast<const char*>(A.proj);
    const unsigned row_bytes = (unsigned)A.nw * 4u;
    const unsigned view_bytes = row_bytes * (unsigned)A.nh;
    float* myline = lines + tid;

    float acc[KZ];
#pragma unroll
    for (int kk = 0; kk < KZ; ++kk) acc[kk] = 0.f;

    for (int sb = 0; sb < A.np; sb += kViewBatch) {
        const int nb = min(kViewBatch, A.np - sb);
        __syncthreads();
        if (tid < nb) {
            const int s = sb + tid;
            view_record(A.M + 12 * (size_t)s, i0, j0, ni, nj, kc, KZ, 1.0f, PITCH, A.rows, false,
                        &vtab[tid]);
        }
        __syncthreads();
        for (int qv = 0; qv < nb; ++qv) {
            const ViewRec& rv = vtab[qv];
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(proj + (size_t)(sb + qv) * view_bytes), 0, (int)view_bytes, kBufferFlags);
            stage_rows<PITCH, false>(tile, A.rows, rs, A.nh, row_bytes, A.nw, uniform(rv.r0),
                                     uniform(rv.c0), uniform(rv.R), uniform(rv.C), wave, lane);
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            const float w = fmaf(uniform(rv.d), di, fmaf(uniform(rv.e), dj, uniform(rv.w0)));
            float F = __builtin_amdgcn_rcpf(w);
            F = F * fmaf(-w, F, 2.0f);                        // one Newton step
            const float u = fmaf(uniform(rv.a), di, fmaf(uniform(rv.b), dj, uniform(rv.N0))) * F;
            const float dv = uniform(rv.m12) * F;
            const float W = F * F;
            const float fu = __builtin_amdgcn_fractf(u);
            const HalfBase& hb = rv.half[0];
            // v of slice kc relative to window row 0
            const float v0 = fmaf(fmaf(uniform(hb.g), di, fmaf(uniform(hb.h), dj, uniform(hb.V0))), F,
                                  (float)uniform(hb.row));
            // first line row one below the lowest row reached (>= 0: the window
            // starts a row below every footprint), so that v - m0 >= 1 - rounding
            // and (int) is the floor for every slice
            const float vlo = fminf(v0, fmaf((float)(KZ - 1), dv, v0));
            const int m0 = (int)vlo - 1;
            // ---- the column's line: columns floor(u), floor(u) + 1 blended with fu
            const float* col = tile + (int)u;
            for (int m = 0; m < line_rows; ++m) {
                const int r = min(m0 + m, A.rows - 1);
                const float p0 = col[r * PITCH], p1 = col[r * PITCH + 1];
                myline[m * kThreads] = fmaf(fu, p1 - p0, p0);
            }
            // ---- updates: one 1-D interpolation along the line each
            const float vb = v0 - (float)m0;
#pragma unroll
            for (int t = 0; t < KZ; ++t) {
                const float v = fmaf((float)t, dv, vb);
                const int r = (int)v;
                const float fv = __builtin_amdgcn_fractf(v);
                const float l0 = myline[r * kThreads], l1 = myline[(r + 1) * kThreads];
                acc[t] = fmaf(W, fmaf(fv, l1 - l0, l0), acc[t]);
            }
            __syncthreads();                                  // tile is overwritten next
        }
    }

    if (active) {
        const int i = i0 + lx, j = j0 + ly;
#pragma unroll
        for (int kk = 0; kk < KZ; ++kk) {
            const int k = kc + kk;
            if (k < A.nz) {
                float* dst = A.vol + ((size_t)k * A.ny + j) * A.nx + i;
                *dst += acc[kk];
            }
        }
    }
}

// Direct organisation, for geometries whose block footprint does not fit an
// LDS tile (strong magnification: beyond ~15 detector pixels per voxel, a
// 16 x 16 x 8 block reaches more pixels than the widest tile holds): the same
// blocks, hoisting and register accumulation, with the four taps read from
// the projection in memory through the caches.  Per (column, view) the
// projection of the column is evaluated in FP64 and reduced to an integer
// row/column origin plus FP32 offsets below one pixel; the row step per
// slice is split into its integer part (added as an integer) and its
// fraction (accumulated in FP32), so that at tens of rows per slice the FP32
// row coordinate of the last slice is still accurate to ~1e-6 of a pixel.
// Taps outside the detector read as zero.
template <bool F16>
__device__ __forceinline__ float direct_tap(const void* view, int r, int c, int nh, int nw)
{
    if ((unsigned)r >= (unsigned)nh || (unsigned)c >= (unsigned)nw) return 0.f;
    const size_t q = (size_t)r * nw + c;
    if (F16) return (float)__builtin_bit_cast(_Float16, reinterpret_cast<const uint16_t*>(view)[q]);
    return reinterpret_cast<const float*>(view)[q];
}

template <int KZ, bool F16>
__global__ __launch_bounds__(kThreads) void bp_direct_kernel(const BpArgs A)
{
    const BlockPos bp = block_position(blockIdx.x, A.ntiles_pad);
    const int t_id = bp.tile;
    if (t_id >= A.ntiles) return;                             // padding block (no barriers here)
    const int tx = t_id % A.ntx, ty = t_id / A.ntx;
    const int kc = (A.chunk_first + bp.chunk_local) * KZ;
    const int i = tx * kTile + (threadIdx.x & (kTile - 1));
    const int j = ty * kTile + (threadIdx.x >> 4);
    if (i >= A.nx || j >= A.ny) return;
    const double di = i, dj = j;
    const size_t view_elems = (size_t)A.nh * A.nw;
    const char* proj = reinterpret_cast<const char*>(A.proj);
    // pixel offsets are clamped to this range before conversion: everything
    // beyond it is off any detector of fewer than 2^24 rows or columns
    constexpr double kFar = 16777216.0;

    float acc[KZ];
#pragma unroll
    for (int t = 0; t < KZ; ++t) acc[t] = 0.f;
    for (int s = 0; s < A.np; ++s) {
        const double* m = A.M + 12 * (size_t)s;
        const double rw = 1.0 / (m[8] * di + m[9] * dj + m[11]);
        const double u = (m[0] * di + m[1] * dj + m[3]) * rw;
        const double v0 = (m[4] * di + m[5] * dj + m[6] * (double)kc + m[7]) * rw;
        const double cu = fmin(fmax(floor(u), -kFar), kFar);
        const double r0d = fmin(fmax(floor(v0), -kFar), kFar);
        const float fu = (float)(u - floor(u));
        const float vl = (float)(v0 - r0d);                   // v of slice kc relative to row r0
        const double dvd = m[6] * rw;                         // rows per slice
        const double dvi_d = fmin(fmax(floor(dvd), -1048576.0), 1048576.0);
        const float dvf = (float)(dvd - floor(dvd));          // its fraction, in [0, 1)
        const int dvi = (int)dvi_d;                           // and its integer part
        const float W = (float)(rw * rw) * (A.scale ? A.scale[s] : 1.0f);
        const int c = (int)cu, r0 = (int)r0d;
        const void* view = proj + (size_t)s * view_elems * (F16 ? 2 : 4);
#pragma unroll
        for (int t = 0; t < KZ; ++t) {
            const float v = fmaf((float)t, dvf, vl);            // < KZ + 1
            const float fl = floorf(v);
            const float fv = v - fl;
            const int r = r0 + t * dvi + (int)fl;
            const float p00 = direct_tap<F16>(view, r, c, A.nh, A.nw);
            const float p01 = direct_tap<F16>(view, r, c + 1, A.nh, A.nw);
            const float p10 = direct_tap<F16>(view, r + 1, c, A.nh, A.nw);
            const float p11 = direct_tap<F16>(view, r + 1, c + 1, A.nh, A.nw);
            const float h0 = fmaf(fu, p01 - p00, p00), h1 = fmaf(fu, p11 - p10, p10);
            acc[t] = fmaf(W, fmaf(fv, h1 - h0, h0), acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < KZ; ++t) {
        const int k = kc + t;
        if (k >= A.k_begin && k < A.k_end)
            A.vol[((size_t)(k - A.k_begin) * A.ny + j) * A.nx + i] += acc[t];
    }
}

// Four waves per SIMD: the register budget that, with the LDS tile of the
// launch plan, keeps four or more blocks resident per CU.
template <int KZ, int PITCH, bool F16>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(4))) void bp_kernel(const BpArgs A)
{
    static_assert(KZ % 2 == 0, "slices are processed in two halves");
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
    const int lx = col_x(tid), ly = col_y(tid);
    // idle lanes of an edge tile shadow a real column so that every LDS read
    // stays inside the staged footprint
    const float di = (float)min(lx, ni - 1), dj = (float)min(ly, nj - 1);

    const char* proj = reinterpret_cast<const char*>(A.proj);
    const unsigned row_bytes = (unsigned)A.nw * (F16 ? 2u : 4u);
    const unsigned view_bytes = row_bytes * (unsigned)A.nh;   // < 2^31, checked by the host
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
            // opaque copies of the block's tile origin: the FP64 set-up derived
            // from them is recomputed per batch rather than hoisted out of the
            // view loop into registers that the accumulators need
            int bi0 = i0, bj0 = j0, bkc = kc;
            asm volatile("" : "+s"(bi0), "+s"(bj0), "+s"(bkc));
            view_record(A.M + 12 * (size_t)s, bi0, bj0, ni, nj, bkc, KZ, sc, PITCH, A.rows, true,
                        &vtab[tid]);
        }
        __syncthreads();
        for (int qv = 0; qv < nb; ++qv) {
            const ViewRec& rv = vtab[qv];
            const int c0 = uniform(rv.c0), C = uniform(rv.C);
            const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                (void*)(proj + (size_t)(sb + qv) * view_bytes), 0, (int)view_bytes, kBufferFlags);
            // ---- stage the footprint of view sb+qv (zero outside the detector)
            stage_rows<PITCH, F16>(tile, A.rows, rs, A.nh, row_bytes, A.nw, uniform(rv.r0), c0,
                                   uniform(rv.R), C, wave, lane);
            __builtin_amdgcn_s_waitcnt(0);                    // this wave's LDS writes landed
            __syncthreads();
            // ---- hoisted per (column, view) quantities: fu, the weight W,
            // dv, the row origins of the two halves and the LDS address of
            // column floor(u) in tile row 0 (u >= 1 inside the tile)
            float fu, W, dv, v0h[2];
            int iu;
            if constexpr (PITCH >= kPreciseSetupPitch) {
                // Strong magnification: window-relative coordinates reach
                // ~PITCH columns and rows, where FP32 set-up error (~1 ulp of
                // the coordinate) would move the taps by 1e-5 pixels; the
                // set-up runs in FP64 from the view's matrix, and only u's
                // fraction and the row origins are rounded to FP32.
                const double* m = A.M + 12 * (size_t)(sb + qv);
                const double i = (double)i0 + (double)di, j = (double)j0 + (double)dj;
                const double Fd = 1.0 / (m[8] * i + m[9] * j + m[11]);
                const double ud = (m[0] * i + m[1] * j + m[3]) * Fd - (double)c0;
                const double fl = floor(ud);
                fu = (float)(ud - fl);
                iu = (int)fl;
                dv = (float)(m[6] * Fd);
                W = (float)(Fd * Fd) * rv.scale;
                const double vij = m[4] * i + m[5] * j + m[7];
                const int split = uniform(rv.split);
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    // absolute first row of half q's window
                    const int org = ((split && q) ? uniform(rv.r1) : uniform(rv.r0)) +
                                    uniform(rv.half[q].row);
                    v0h[q] = (float)((vij + m[6] * (double)(kc + q * (KZ / 2))) * Fd - (double)org);
                }
            } else {
                // the record's float fields are used as broadcast LDS reads
                // (moving each to a scalar register would cost one more VALU
                // instruction per view)
                const float w = fmaf(rv.d, di, fmaf(rv.e, dj, rv.w0));
                float F = __builtin_amdgcn_rcpf(w);
                F = F * fmaf(-w, F, 2.0f);                    // one Newton step
                const float u = fmaf(rv.a, di, fmaf(rv.b, dj, rv.N0)) * F;
                dv = rv.m12 * F;
                W = F * F * rv.scale;
                fu = __builtin_amdgcn_fractf(u);
                iu = (int)u;
                v0h[0] = v0h[1] = F;                          // origins: see v_origin
            }
            // binary16 tiles hold even- and odd-offset pairs in two regions
            unsigned base;
            if (F16) {
                const int jc = iu + (c0 & 1);
                base = tile_base + 4u * (unsigned)((jc >> 1) + ((jc & 1) ? A.rows * (PITCH / 2) : 0));
            } else {
                base = tile_base + 4u * (unsigned)iu;
            }
            // ---- hot loop: KZ updates of this column for this view, in two
            // halves; a footprint taller than the LDS tile is staged per half
            auto v_origin = [&](int q) {
                if constexpr (PITCH >= kPreciseSetupPitch) {
                    return v0h[q];
                } else {
                    // computed where used (v0h holds 1 / w), which keeps the
                    // second half's origin out of the registers of the first
                    const HalfBase& hb = rv.half[q];
                    return fmaf(hb.g, di, fmaf(hb.h, dj, hb.V0)) * v0h[0];
                }
            };
            auto row_base = [&](int q) {
                return base + (unsigned)(uniform(rv.half[q].row) * 4 * TileRow<PITCH, F16>::W);
            };
            auto restage = [&] {
                __syncthreads();
                stage_rows<PITCH, F16>(tile, A.rows, rs, A.nh, row_bytes, A.nw, uniform(rv.r1), c0,
                                       uniform(rv.R1), C, wave, lane);
                __builtin_amdgcn_s_waitcnt(0);
                __syncthreads();
            };
            if constexpr (F16) {
                // one pipelined sequence over both halves
                update_column<KZ, PITCH, F16>(acc, row_base(0), row_base(1), v_origin(0), v_origin(1),
                                              dv, fu, W, uniform(rv.split) != 0, restage);
            } else {
                // (the float32 taps need twice the registers: the halves stay
                // apart, which keeps the kernel within four waves per SIMD)
                update_half<KZ, PITCH, F16>(acc, 0, row_base(0), v_origin(0), dv, fu, W);
                if (uniform(rv.split)) restage();
                update_half<KZ, PITCH, F16>(acc, KZ / 2, row_base(1), v_origin(1), dv, fu, W);
            }
            __syncthreads();                                  // tile is overwritten next
        }
    }

    // ---- one read-modify-write of the volume per call (the column is
    // re-derived from the thread index, so that it need not stay live
    // through the view loop)
    int tid_end = tid;
    asm volatile("" : "+v"(tid_end));
    if (col_x(tid_end) < ni && col_y(tid_end) < nj) {
        const int i = i0 + col_x(tid_end), j = j0 + col_y(tid_end);
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
fdk_status launch_sym_pitch(const BpArgs& a, bool f16, size_t lds, unsigned blocks, hipStream_t st)
{
    const void* fn = f16 ? (const void*)bp_sym_kernel<KZ, PITCH, true>
                         : (const void*)bp_sym_kernel<KZ, PITCH, false>;
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return fail(FDK_E_DEVICE, "cannot raise the LDS limit of the back-projection kernel");
    }
    if (f16)
        hipLaunchKernelGGL((bp_sym_kernel<KZ, PITCH, true>), dim3(blocks), dim3(kThreads), lds, st, a);
    else
        hipLaunchKernelGGL((bp_sym_kernel<KZ, PITCH, false>), dim3(blocks), dim3(kThreads), lds, st, a);
    return check_launch("symmetric back-projection kernel");
}

template <int KZ>
fdk_status launch_sym_kz(const BpArgs& a, int pitch, bool f16, size_t lds, unsigned blocks, hipStream_t st)
{
    switch (pitch) {
        case 40: return launch_sym_pitch<KZ, 40>(a, f16, lds, blocks, st);
        case 56: return launch_sym_pitch<KZ, 56>(a, f16, lds, blocks, st);
        case 72: return launch_sym_pitch<KZ, 72>(a, f16, lds, blocks, st);
        case 88: return launch_sym_pitch<KZ, 88>(a, f16, lds, blocks, st);
        case 120: return launch_sym_pitch<KZ, 120>(a, f16, lds, blocks, st);
        case 184: return launch_sym_pitch<KZ, 184>(a, f16, lds, blocks, st);
        case 248: return launch_sym_pitch<KZ, 248>(a, f16, lds, blocks, st);
    }
    return fail(FDK_E_UNSUPPORTED, "no kernel for this LDS pitch");
}

template <int KZ, int PITCH>
fdk_status launch_subline_pitch(const BpArgs& a, int line_rows, size_t lds, unsigned blocks,
                                hipStream_t st)
{
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute((const void*)bp_subline_kernel<KZ, PITCH>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
            return fail(FDK_E_DEVICE, "cannot raise the LDS limit of the sub-line kernel");
    }
    hipLaunchKernelGGL((bp_subline_kernel<KZ, PITCH>), dim3(blocks), dim3(kThreads), lds, st, a,
                       line_rows);
    return check_launch("sub-line back-projection kernel");
}

template <int KZ>
fdk_status launch_subline_kz(const BpArgs& a, int pitch, int line_rows, size_t lds,
                             unsigned blocks, hipStream_t st)
{
    switch (pitch) {
        case 40: return launch_subline_pitch<KZ, 40>(a, line_rows, lds, blocks, st);
        case 56: return launch_subline_pitch<KZ, 56>(a, line_rows, lds, blocks, st);
        case 72: return launch_subline_pitch<KZ, 72>(a, line_rows, lds, blocks, st);
        case 88: return launch_subline_pitch<KZ, 88>(a, line_rows, lds, blocks, st);
        case 120: return launch_subline_pitch<KZ, 120>(a, line_rows, lds, blocks, st);
        case 184: return launch_subline_pitch<KZ, 184>(a, line_rows, lds, blocks, st);
        case 248: return launch_subline_pitch<KZ, 248>(a, line_rows, lds, blocks, st);
    }
    return fail(FDK_E_UNSUPPORTED, "no kernel for this LDS pitch");
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
        case 40: return launch_kz_pitch<KZ, 40>(a, f16, lds, blocks, st);
        case 56: return launch_kz_pitch<KZ, 56>(a, f16, lds, blocks, st);
        case 72: return launch_kz_pitch<KZ, 72>(a, f16, lds, blocks, st);
        case 88: return launch_kz_pitch<KZ, 88>(a, f16, lds, blocks, st);
        case 120: return launch_kz_pitch<KZ, 120>(a, f16, lds, blocks, st);
        case 184: return launch_kz_pitch<KZ, 184>(a, f16, lds, blocks, st);
        case 248: return launch_kz_pitch<KZ, 248>(a, f16, lds, blocks, st);
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
    if (plan.direct) {
#define FDK_DIRECT(KZ_)                                                                          \
        if (a.f16)                                                                               \
            hipLaunchKernelGGL((bp_direct_kernel<KZ_, true>), dim3((unsigned)blocks), dim3(kThreads), 0, st, A); \
        else                                                                                     \
            hipLaunchKernelGGL((bp_direct_kernel<KZ_, false>), dim3((unsigned)blocks), dim3(kThreads), 0, st, A); \
        return check_launch("direct back-projection kernel");
        switch (plan.kz) {
            case 8: { FDK_DIRECT(8) }
            case 16: { FDK_DIRECT(16) }
            case 32: { FDK_DIRECT(32) }
        }
#undef FDK_DIRECT
        return fail(FDK_E_UNSUPPORTED, "no kernel for this slice count");
    }
    switch (plan.kz) {
        case 8: return launch_kz<8>(A, plan.pitch, a.f16, lds, (unsigned)blocks, st);
        case 16: return launch_kz<16>(A, plan.pitch, a.f16, lds, (unsigned)blocks, st);
        case 32: return launch_kz<32>(A, plan.pitch, a.f16, lds, (unsigned)blocks, st);
    }
    return fail(FDK_E_UNSUPPORTED, "no kernel for this slice count");
}

fdk_status launch_backproject_sym(const BpLaunch& a, const BpPlan& plan, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    fdk_status s = launch_compose(a.mats_world, a.mats_index, a.np, a.dx, a.dy, a.dz, a.ox, a.oy,
                                  a.oz, stream);
    if (s != FDK_OK) return s;
    const int h = plan.kz / 2;
    const int nch = ((a.nz + 1) / 2 + h - 1) / h;            // chunks of direct slices
    BpArgs A;
    A.proj = a.proj;
    A.scale = a.scale;
    A.M = a.mats_index;
    A.vol = a.vol;
    A.nx = a.nx; A.ny = a.ny; A.nz = a.nz; A.np = a.np; A.nh = a.nh; A.nw = a.nw;
    A.k_begin = 0;
    A.k_end = a.nz;
    A.ntx = plan.ntx;
    A.ntiles = plan.ntx * plan.nty;
    A.ntiles_pad = plan.ntiles_pad;
    A.chunk_first = 0;
    A.rows = plan.rows;
    const size_t lds = (size_t)plan.lds_bytes;
    const int64_t blocks = (int64_t)plan.ntiles_pad * nch;
    if (blocks >= (1ll << 31)) return fail(FDK_E_UNSUPPORTED, "grid too large");
    switch (plan.kz) {
        case 8: return launch_sym_kz<8>(A, plan.pitch, a.f16, lds, (unsigned)blocks, st);
        case 16: return launch_sym_kz<16>(A, plan.pitch, a.f16, lds, (unsigned)blocks, st);
        case 32: return launch_sym_kz<32>(A, plan.pitch, a.f16, lds, (unsigned)blocks, st);
    }
    return fail(FDK_E_UNSUPPORTED, "no kernel for this slice count");
}

fdk_status launch_backproject_subline(const BpLaunch& a, const BpPlan& plan, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    fdk_status s = launch_compose(a.mats_world, a.mats_index, a.np, a.dx, a.dy, a.dz, a.ox, a.oy,
                                  a.oz, stream);
    if (s != FDK_OK) return s;
    BpArgs A;
    A.proj = a.proj;
    A.scale = nullptr;
    A.M = a.mats_index;
    A.vol = a.vol;
    A.nx = a.nx; A.ny = a.ny; A.nz = a.nz; A.np = a.np; A.nh = a.nh; A.nw = a.nw;
    A.k_begin = 0;
    A.k_end = a.nz;
    A.ntx = plan.ntx;
    A.ntiles = plan.ntx * plan.nty;
    A.ntiles_pad = plan.ntiles_pad;
    A.chunk_first = 0;
    A.rows = plan.rows;
    const int64_t blocks = (int64_t)plan.ntiles_pad * plan.nchunks;
    if (blocks >= (1ll << 31)) return fail(FDK_E_UNSUPPORTED, "grid too large");
    const size_t lds = (size_t)plan.lds_bytes;
    switch (plan.kz) {
        case 8: return launch_subline_kz<8>(A, plan.pitch, plan.line_rows, lds, (unsigned)blocks, st);
        case 16: return launch_subline_kz<16>(A, plan.pitch, plan.line_rows, lds, (unsigned)blocks, st);
        case 32: return launch_subline_kz<32>(A, plan.pitch, plan.line_rows, lds, (unsigned)blocks, st);
    }
    return fail(FDK_E_UNSUPPORTED, "no kernel for this slice count");
}

}  // namespace fdk
