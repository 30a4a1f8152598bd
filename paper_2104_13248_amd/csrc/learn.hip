// Kernels of the learned row filter (an extension of the FDK filtering step,
// which the paper takes as given, Sections 2.1.2 and 3.1.1): 1-D convolutions
// along detector rows -- forward, backward with respect to the input, backward
// with respect to the weights -- with a fused ReLU / ReLU-gradient mask and a
// fused residual addend, the squared-error loss of a reconstruction and an
// Adam step.
//
// Tensors are float32 [rows][channels][len] (one detector row per `rows`
// index, its channels contiguous along len).  Weights are [cout][cin][k],
// bias [cout].  Convolution is cross-correlation with zero padding of k/2 on
// both sides ("same" length):
//   out[r][o][x] = bias[o] + sum_i sum_t w[o][i][t] in[r][i][x + t - k/2].
// Instantiated for the filter network's shapes: cin, cout in {1, 32}, k = 9.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace fdk {
namespace {

constexpr int kK = 9;            // taps
constexpr int kHalo = kK / 2;
constexpr int kTo1 = 16;        // positions per thread of the 32 -> 1 layers
constexpr int kCT = 256;         // threads per block

// Launch shape of the layer kernel for COUT output channels: G wave-uniform
// channel groups of COUT / G channels, PPT consecutive positions per thread,
// SEG positions per block, NT threads.
template <int COUT>
struct ConvShape {
    static constexpr int G = COUT >= 4 ? 4 : 1;
    static constexpr int PPT = COUT >= 4 ? 4 : 2;
    static constexpr int NT = COUT >= 4 ? 256 : 128;
    static constexpr int SEG = NT / G * PPT;
};

template <int N>
__device__ __forceinline__ void lds_read(const float* p, float (&v)[N])
{
    // N consecutive floats from an address aligned to 4 (N % 4 == 0) or 2 floats
    if constexpr (N % 4 == 0) {
#pragma unroll
        for (int q = 0; q < N / 4; ++q) {
            const float4 t = reinterpret_cast<const float4*>(p)[q];
            v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < N / 2; ++q) {
            const float2 t = reinterpret_cast<const float2*>(p)[q];
            v[2 * q] = t.x; v[2 * q + 1] = t.y;
        }
    }
}

// Forward convolution, or (TRANS) the backward-data convolution: the
// transpose of a layer with weights w[OUT][IN][k] maps gradients of its
// OUT-channel output back to its IN channels, and is itself a convolution with
// channels swapped and taps mirrored:
//   gin[r][i][x] = sum_o sum_t w[o][i][k-1-t] gout[r][o][x + t - k/2].
// Here CIN/COUT are the channel counts of the convolution computed (for TRANS:
// CIN = layer OUT, COUT = layer IN).
//
// Epilogue: y = bias + conv; ReLU if relu; y = 0 where mask <= 0 (mask is the
// same shape as out); y = alpha y; y += add[...] (same shape as out).
//
// Block: one row segment of SEG positions, all output channels.  Each wave
// owns one group of COUT / G channels, so every weight is a wave-uniform
// (scalar) operand; each lane owns PPT consecutive positions and reads the
// PPT + 8 input samples they need with aligned vector LDS loads, so every
// sample read feeds 9 * PPT / (PPT + 8) multiply-adds per channel.
template <int CIN, int COUT, bool TRANS>
__global__ __launch_bounds__(ConvShape<COUT>::NT) void conv_kernel(
    const float* __restrict__ in, const float* __restrict__ w, const float* __restrict__ bias,
    const float* __restrict__ mask, const float* add, float alpha, int relu, float* out, int len,
    int nseg)
{
    using S = ConvShape<COUT>;
    constexpr int CPT = COUT / S::G;          // output channels per thread
    constexpr int TP = S::SEG + 2 * kHalo;    // staged samples per channel (multiple of 4)
    constexpr int NV = S::PPT + kK - 1;       // samples one lane reads per channel
    static_assert(COUT % S::G == 0 && TP % 4 == 0, "shape");
    __shared__ __attribute__((aligned(16))) float tile[CIN][TP];
    const int r = blockIdx.x / nseg;
    const int x0 = (blockIdx.x - r * nseg) * S::SEG;
    const float* src = in + (size_t)r * CIN * len;
    for (int q = threadIdx.x; q < CIN * TP; q += S::NT) {
        const int ci = q / TP, xx = q - ci * TP;
        const int x = x0 + xx - kHalo;
        tile[ci][xx] = (x >= 0 && x < len) ? src[(size_t)ci * len + x] : 0.f;
    }
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int c0 = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) % S::G * CPT;
    const int xl = (((int)threadIdx.x >> 6) / S::G * 64 + lane) * S::PPT;
    float acc[CPT][S::PPT];
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const float b0 = bias ? bias[c0 + c] : 0.f;
#pragma unroll
        for (int p = 0; p < S::PPT; ++p) acc[c][p] = b0;
    }
    constexpr int UNR = CPT >= 8 ? 1 : 4;     // bounds the weights held in SGPRs
#pragma unroll UNR
    for (int ci = 0; ci < CIN; ++ci) {
        float v[NV];
        lds_read(&tile[ci][xl], v);
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
#pragma unroll
            for (int t = 0; t < kK; ++t) {
                const float wt = TRANS ? w[((size_t)ci * COUT + c0 + c) * kK + (kK - 1 - t)]
                                       : w[((size_t)(c0 + c) * CIN + ci) * kK + t];
#pragma unroll
                for (int p = 0; p < S::PPT; ++p) acc[c][p] = fmaf(wt, v[p + t], acc[c][p]);
            }
        }
    }
    const size_t o = (size_t)r * COUT * len + x0 + xl;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const size_t oc = o + (size_t)(c0 + c) * len;
#pragma unroll
        for (int p = 0; p < S::PPT; ++p) {
            if (x0 + xl + p < len) {
                float y = acc[c][p];
                if (relu) y = fmaxf(y, 0.f);
                if (mask && !(mask[oc + p] > 0.f)) y = 0.f;
                y *= alpha;
                if (add) y += add[oc + p];
                out[oc + p] = y;
            }
        }
    }
}

// Layers with one input or one output channel move 32 channels of
// activations per position against at most 9 x 32 multiply-adds, so they are
// bound by memory, not arithmetic.  Each thread owns consecutive positions
// of one row (4 for the 1 -> 32 layers, kTo1 = 16 for the 32 -> 1 layers,
// whose 32 input channels make the 4-sample halos the larger share of the
// loads) and streams what it needs straight from memory (16-byte loads where
// the row allows; neighbouring threads share the halos through the cache):
// nothing is staged, few registers are live and many waves stay resident to
// cover the memory latency.

// Whether every base pointer allows 16-byte accesses (with len % 4 == 0,
// then so does every row).
__device__ __forceinline__ bool aligned16(const float* a, const float* b, const float* c,
                                          const float* d)
{
    return (((size_t)a | (size_t)b | (size_t)c | (size_t)d) & 15) == 0;
}

// Samples in[x0 - 4 .. x0 + 7] of one channel row, zero outside [0, len).
__device__ __forceinline__ void load12(const float* __restrict__ row, int x0, int len, bool vec,
                                       float (&v)[12])
{
    if (vec) {
        const float4 a = *reinterpret_cast<const float4*>(row + x0 - 4);
        const float4 b = *reinterpret_cast<const float4*>(row + x0);
        const float4 c = *reinterpret_cast<const float4*>(row + x0 + 4);
        v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
        v[4] = b.x; v[5] = b.y; v[6] = b.z; v[7] = b.w;
        v[8] = c.x; v[9] = c.y; v[10] = c.z; v[11] = c.w;
    } else {
#pragma unroll
        for (int e = 0; e < 12; ++e) {
            const int x = x0 - 4 + e;
            v[e] = (x >= 0 && x < len) ? row[x] : 0.f;
        }
    }
}

// Samples in[x0 - 4 .. x0 + N - 5] of one channel row (N a multiple of 4),
// zero outside [0, len).
template <int N>
__device__ __forceinline__ void loadn(const float* __restrict__ row, int x0, int len, bool vec,
                                      float (&v)[N])
{
    if (vec) {
#pragma unroll
        for (int q = 0; q < N / 4; ++q) {
            const float4 a = *reinterpret_cast<const float4*>(row + x0 - 4 + 4 * q);
            v[4 * q] = a.x; v[4 * q + 1] = a.y; v[4 * q + 2] = a.z; v[4 * q + 3] = a.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < N; ++e) {
            const int x = x0 - 4 + e;
            v[e] = (x >= 0 && x < len) ? row[x] : 0.f;
        }
    }
}

// Epilogue of one output channel's 4 positions (the layer kernel's order:
// bias already in acc; ReLU, mask, alpha, residual addend).
__device__ __forceinline__ void store4(float (&acc)[4], size_t oc, int x0, int len, bool vec4,
                                       const float* __restrict__ mask, const float* add, float alpha,
                                       int relu, float* out)
{
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        float y = acc[p];
        if (relu) y = fmaxf(y, 0.f);
        acc[p] = y;
    }
    if (vec4) {
        if (mask) {
            const float4 m = *reinterpret_cast<const float4*>(mask + oc);
            if (!(m.x > 0.f)) acc[0] = 0.f;
            if (!(m.y > 0.f)) acc[1] = 0.f;
            if (!(m.z > 0.f)) acc[2] = 0.f;
            if (!(m.w > 0.f)) acc[3] = 0.f;
        }
        float4 y = make_float4(acc[0] * alpha, acc[1] * alpha, acc[2] * alpha, acc[3] * alpha);
        if (add) {
            const float4 a = *reinterpret_cast<const float4*>(add + oc);
            y.x += a.x; y.y += a.y; y.z += a.z; y.w += a.w;
        }
        *reinterpret_cast<float4*>(out + oc) = y;
    } else {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            if (x0 + p < len) {
                float y = acc[p];
                if (mask && !(mask[oc + p] > 0.f)) y = 0.f;
                y *= alpha;
                if (add) y += add[oc + p];
                out[oc + p] = y;
            }
        }
    }
}

// 32 channels -> 1: the last layer's forward, or (TRANS) the first layer's
// backward-data pass (weights w[32][1][k], taps mirrored).
template <bool TRANS>
__global__ __launch_bounds__(256) void conv_to1_kernel(const float* __restrict__ in,
                                                       const float* __restrict__ w,
                                                       const float* __restrict__ bias,
                                                       const float* __restrict__ mask,
                                                       const float* add, float alpha, int relu,
                                                       float* out, int rows, int len, int nq)
{
    // kTo1 positions per thread: kTo1 + 8 samples per channel (two 4-sample halos)
    constexpr int PP = kTo1, NV = kTo1 + 8;
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)rows * nq) return;
    const int r = (int)(g / nq);
    const int x0 = PP * (int)(g - (int64_t)r * nq);
    const bool al = aligned16(in, out, mask, add) && (len & 3) == 0;
    const bool vec = al && x0 >= 4 && x0 + PP + 4 <= len;
    const float* src = in + (size_t)r * 32 * len;
    float acc[PP];
    const float b0 = bias ? bias[0] : 0.f;
#pragma unroll
    for (int p = 0; p < PP; ++p) acc[p] = b0;
#pragma unroll 2
    for (int i = 0; i < 32; ++i) {
        float v[NV];
        loadn<NV>(src + (size_t)i * len, x0, len, vec, v);
#pragma unroll
        for (int t = 0; t < kK; ++t) {
            const float wt = TRANS ? w[i * kK + (kK - 1 - t)] : w[i * kK + t];
#pragma unroll
            for (int p = 0; p < PP; ++p) acc[p] = fmaf(wt, v[p + t], acc[p]);
        }
    }
#pragma unroll
    for (int q = 0; q < PP / 4; ++q) {
        float a4[4] = {acc[4 * q], acc[4 * q + 1], acc[4 * q + 2], acc[4 * q + 3]};
        const int xq = x0 + 4 * q;
        if (xq < len)
            store4(a4, (size_t)r * len + xq, xq, len, al && xq + 4 <= len, mask, add, alpha, relu,
                   out);
    }
}

// 1 channel -> 32: the first layer's forward, or (TRANS) the last layer's
// backward-data pass (weights w[1][32][k], taps mirrored).
template <bool TRANS>
__global__ __launch_bounds__(256) void conv_from1_kernel(const float* __restrict__ in,
                                                         const float* __restrict__ w,
                                                         const float* __restrict__ bias,
                                                         const float* __restrict__ mask,
                                                         const float* add, float alpha, int relu,
                                                         float* out, int rows, int len, int nq)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= (int64_t)rows * nq) return;
    const int r = (int)(g / nq);
    const int x0 = 4 * (int)(g - (int64_t)r * nq);
    const bool al = aligned16(in, out, mask, add) && (len & 3) == 0;
    const bool vec = al && x0 >= 4 && x0 + 8 <= len;
    const bool vec4 = al && x0 + 4 <= len;
    float v[12];
    load12(in + (size_t)r * len, x0, len, vec, v);
#pragma unroll 2
    for (int o = 0; o < 32; ++o) {
        float acc[4];
        const float b0 = bias ? bias[o] : 0.f;
#pragma unroll
        for (int p = 0; p < 4; ++p) acc[p] = b0;
#pragma unroll
        for (int t = 0; t < kK; ++t) {
            const float wt = TRANS ? w[o * kK + (kK - 1 - t)] : w[o * kK + t];
#pragma unroll
            for (int p = 0; p < 4; ++p) acc[p] = fmaf(wt, v[p + t], acc[p]);
        }
        store4(acc, ((size_t)r * 32 + o) * len + x0, x0, len, vec4, mask, add, alpha, relu, out);
    }
}

// 32 -> 32 channels on the matrix cores (v_mfma_f32_16x16x4f32: FP32
// products, FP32 accumulation).  The layer is a contraction over
// K = 32 channels x 9 taps per output: out[o][x] = sum_k A[o][k] B[k][x], with
// k = 32 t + i so that each 4-wide step of K covers 4 input channels at one
// tap; B[k][x] = in[i][x + t - 4] is then a fixed per-lane LDS offset plus a
// wave-uniform step offset.  Forward: A[o][k] = w[o][i][t]; transposed
// (backward data): A[o][k] = w[i][o][8 - t] (o, i the roles of the computed
// convolution).  The A operands are laid out once per call in the order the
// lanes read them (wa[o-tile][step][lane]), so every block reads them as
// coalesced, cache-resident loads.  Block: one row segment of 256 positions,
// all 32 input channels staged in LDS, 4 waves x 64 positions x 32 output
// channels (2 x 4 tiles of 16 x 16).
constexpr int kMxSeg = 256;                     // positions per block
// LDS pitch of a staged channel: = 16 (mod 64), so the 4 channels x 16
// positions a B operand reads fall in distinct banks
constexpr int kMxTP = kMxSeg + 2 * kHalo + 8;
constexpr int kMxSteps = 32 / 4 * kK;           // K steps (72)

typedef float mx4 __attribute__((ext_vector_type(4)));

// A operands in the order one half of the input channels reads them:
// wa[h][ot][j][l] = A[ot*16 + l%16][k], k = 32 t + 16 h + 4 q + l/16, j = 4 t + q
// (t the tap, q the channel quad within the half).
template <bool TRANS>
__global__ void arrange_a_kernel(const float* __restrict__ w, float* __restrict__ wa)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 2 * kMxSteps * 64) return;
    const int l = idx & 63, j = (idx >> 6) % (kMxSteps / 2);
    const int ot = (idx / (64 * (kMxSteps / 2))) & 1, h = idx / (64 * kMxSteps);
    const int t = j >> 2, q = j & 3;
    const int o = ot * 16 + (l & 15), i = 16 * h + 4 * q + (l >> 4);
    wa[idx] = TRANS ? w[((size_t)i * 32 + o) * kK + (kK - 1 - t)] : w[((size_t)o * 32 + i) * kK + t];
}

typedef __attribute__((address_space(3))) void lds_void_t;

__device__ __forceinline__ lds_void_t* lds_ptr(const void* p)
{
    return (lds_void_t*)(size_t)(unsigned)(size_t)(__attribute__((address_space(3))) const char*)p;
}

// Four blocks per CU (their LDS fits four times in 160 KB): at most 128
// registers per lane.
__global__ __launch_bounds__(256, 4) void conv32_mfma_kernel(const float* __restrict__ in,
                                                        const float* __restrict__ wa,
                                                        const float* __restrict__ bias,
                                                        const float* __restrict__ mask,
                                                        const float* add, float alpha, int relu,
                                                        float* out, int len, int nseg)
{
    // input channels in two halves of 16; each half's A operands (36 steps x 2
    // o-tiles x 64 lanes) are staged in LDS beside its input samples
    __shared__ float tile[16][kMxTP];
    __shared__ float la[2][kMxSteps / 2][64];
    const int r = blockIdx.x / nseg;
    const int x0 = (blockIdx.x - r * nseg) * kMxSeg;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const float* src = in + (size_t)r * 32 * len;
    mx4 acc[2][4];
#pragma unroll
    for (int ot = 0; ot < 2; ++ot)
#pragma unroll
        for (int xt = 0; xt < 4; ++xt) acc[ot][xt] = mx4{0.f, 0.f, 0.f, 0.f};
    // per-lane part of the B address: channel l/16 of the step, position l%16
    const float* tl = &tile[0][0] + (lane >> 4) * kMxTP + wave * 64 + (lane & 15);
    // the block's input rows and the A operands go straight from memory into
    // LDS (asynchronous buffer loads; samples outside the row read as zero)
    const __amdgpu_buffer_rsrc_t rin = __builtin_amdgcn_make_buffer_rsrc(
        (void*)src, 0, (int)(32u * (unsigned)len * 4u), 0x00020000);
    const __amdgpu_buffer_rsrc_t rwa = __builtin_amdgcn_make_buffer_rsrc(
        (void*)wa, 0, 2 * kMxSteps * 64 * 4, 0x00020000);
    constexpr unsigned kOut = 0x80000000u;
    for (int h = 0; h < 2; ++h) {
        __syncthreads();                                   // previous half no longer read
        for (int g = 0; g * 64 < kMxSeg + 2 * kHalo; ++g) {
            const int xx = g * 64 + lane;
            const int x = x0 + xx - kHalo;
            const unsigned vo = (x >= 0 && x < len) ? (unsigned)x * 4u : kOut;
            if (xx < kMxSeg + 2 * kHalo) {                  // lanes past the row write nothing
                for (int ci = wave; ci < 16; ci += 4) {
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(
                        rin, lds_ptr(&tile[ci][g * 64]), 4, vo,
                        (unsigned)(16 * h + ci) * (unsigned)len * 4u, 0, 0);
                }
            }
        }
        for (int q = wave; q * 64 < kMxSteps * 64; q += 4)          // 36 x 2 rows of 64 lanes
            __builtin_amdgcn_raw_ptr_buffer_load_lds(rwa, lds_ptr(&la[0][0][0] + q * 64), 4,
                                                     (unsigned)lane * 4u,
                                                     (unsigned)(h * kMxSteps * 64 + q * 64) * 4u, 0, 0);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
#pragma unroll 4
        for (int j = 0; j < kMxSteps / 2; ++j) {
            const int t = j >> 2, quad = j & 3;
            const float a0 = la[0][j][lane], a1 = la[1][j][lane];
            const float* tb = tl + 4 * quad * kMxTP + t;
#pragma unroll
            for (int xt = 0; xt < 4; ++xt) {
                const float b = tb[16 * xt];
                acc[0][xt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a0, b, acc[0][xt], 0, 0, 0);
                acc[1][xt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a1, b, acc[1][xt], 0, 0, 0);
            }
        }
    }
    // D: lane l, register q -> channel ot*16 + 4 (l/16) + q, position l%16 of
    // the tile.  Per o-tile, the bias, mask and addend of its 16 outputs are
    // loaded before any is used (one wait instead of one per output);
    // positions past the row load from its last position and are not stored.
    const int xl = x0 + wave * 64 + (lane & 15);
    const size_t rb = ((size_t)r * 32 + 4 * (lane >> 4)) * len;       // channel 4 (l/16)
    int xc[4];
#pragma unroll
    for (int xt = 0; xt < 4; ++xt) xc[xt] = min(xl + 16 * xt, len - 1);
#pragma unroll
    for (int ot = 0; ot < 2; ++ot) {
        const size_t ro = rb + (size_t)(ot * 16) * len;
        float bs[4], mk[4][4], ad[4][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) bs[q] = bias ? bias[ot * 16 + 4 * (lane >> 4) + q] : 0.f;
        if (mask) {
#pragma unroll
            for (int xt = 0; xt < 4; ++xt)
#pragma unroll
                for (int q = 0; q < 4; ++q) mk[xt][q] = mask[ro + (size_t)q * len + xc[xt]];
        }
        if (add) {
#pragma unroll
            for (int xt = 0; xt < 4; ++xt)
#pragma unroll
                for (int q = 0; q < 4; ++q) ad[xt][q] = add[ro + (size_t)q * len + xc[xt]];
        }
#pragma unroll
        for (int xt = 0; xt < 4; ++xt) {
            if (xl + 16 * xt < len) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    float y = acc[ot][xt][q] + bs[q];
                    if (relu) y = fmaxf(y, 0.f);
                    if (mask && !(mk[xt][q] > 0.f)) y = 0.f;
                    y *= alpha;
                    if (add) y += ad[xt][q];
                    out[ro + (size_t)q * len + xl + 16 * xt] = y;
                }
            }
        }
    }
}

// grad_w[o][i][t] += sum_{r,x} gout[r][o][x] in[r][i][x + t - k/2]
// grad_b[o]       += sum_{r,x} gout[r][o][x]
// Thread (pair, s) owns NPT (o, i) pairs with their k taps and the s-th of
// SPLIT sub-segments of each staged segment (SPLIT > 1 only when there are
// fewer pairs than threads).  A block walks a run of rows in segments of SEG
// positions staged in LDS (input rows padded to an odd pitch so that the 32
// channels a wave reads fall in distinct banks), reduces the SPLIT partial
// sums in LDS and adds the block's sums with one float atomic per weight.
template <int CIN, int COUT>
struct WgradShape {
    static constexpr int PAIRS = CIN * COUT;
    static constexpr int NPT = (PAIRS + kCT - 1) / kCT;
    static constexpr int SPLIT = PAIRS >= kCT ? 1 : (kCT / PAIRS > 8 ? 8 : kCT / PAIRS);
};

template <int CIN, int COUT>
__global__ __launch_bounds__(kCT) void conv_wgrad_kernel(const float* __restrict__ in,
                                                         const float* __restrict__ go,
                                                         float* __restrict__ gw,
                                                         float* __restrict__ gb, int rows,
                                                         int len, int rows_per_block)
{
    using S = WgradShape<CIN, COUT>;
    constexpr int SEG = 64;
    constexpr int SUB = SEG / S::SPLIT;       // positions per sub-segment
    constexpr int TP = SEG + 2 * kHalo + 1;   // odd pitch
    constexpr int NRED = S::SPLIT > 1 ? S::SPLIT * S::PAIRS * (kK + 1) : 1;
    __shared__ float tin[CIN][TP];
    __shared__ float tgo[COUT][SEG];
    __shared__ float red[NRED];
    const int split = (int)threadIdx.x / (S::SPLIT > 1 ? S::PAIRS : kCT);
    const bool active = split < S::SPLIT;
    float acc[S::NPT][kK];
    float accb[S::NPT];
    int co_[S::NPT], ci_[S::NPT];
#pragma unroll
    for (int q = 0; q < S::NPT; ++q) {
        const int pid = S::SPLIT > 1 ? (int)threadIdx.x % S::PAIRS : (int)threadIdx.x + kCT * q;
        co_[q] = pid < S::PAIRS ? pid / CIN : 0;
        ci_[q] = pid < S::PAIRS ? pid % CIN : 0;
        accb[q] = 0.f;
#pragma unroll
        for (int t = 0; t < kK; ++t) acc[q][t] = 0.f;
    }
    const int r0 = blockIdx.x * rows_per_block;
    const int r1 = min(rows, r0 + rows_per_block);
    for (int r = r0; r < r1; ++r) {
        const float* src = in + (size_t)r * CIN * len;
        const float* g = go + (size_t)r * COUT * len;
        for (int x0 = 0; x0 < len; x0 += SEG) {
            __syncthreads();
            for (int q = threadIdx.x; q < CIN * (SEG + 2 * kHalo); q += kCT) {
                const int ci = q / (SEG + 2 * kHalo), xx = q - ci * (SEG + 2 * kHalo);
                const int x = x0 + xx - kHalo;
                tin[ci][xx] = (x >= 0 && x < len) ? src[(size_t)ci * len + x] : 0.f;
            }
            for (int q = threadIdx.x; q < COUT * SEG; q += kCT) {
                const int co = q / SEG, xx = q - co * SEG;
                const int x = x0 + xx;
                tgo[co][xx] = x < len ? g[(size_t)co * len + x] : 0.f;
            }
            __syncthreads();
            if (!active) continue;
#pragma unroll
            for (int q = 0; q < S::NPT; ++q) {
                const float* ti = &tin[ci_[q]][split * SUB];
                const float* tg = &tgo[co_[q]][split * SUB];
                float win[kK];
#pragma unroll
                for (int t = 0; t < kK - 1; ++t) win[t + 1] = ti[t];
#pragma unroll
                for (int xx = 0; xx < SUB; ++xx) {
#pragma unroll
                    for (int t = 0; t < kK - 1; ++t) win[t] = win[t + 1];
                    win[kK - 1] = ti[xx + kK - 1];
                    const float gv = tg[xx];
                    accb[q] += gv;
#pragma unroll
                    for (int t = 0; t < kK; ++t) acc[q][t] = fmaf(gv, win[t], acc[q][t]);
                }
            }
        }
    }
    if constexpr (S::SPLIT > 1) {
        if (active) {
            const int pid = (int)threadIdx.x % S::PAIRS;
            float* dst = red + ((size_t)split * S::PAIRS + pid) * (kK + 1);
#pragma unroll
            for (int t = 0; t < kK; ++t) dst[t] = acc[0][t];
            dst[kK] = accb[0];
        }
        __syncthreads();
        for (int q = threadIdx.x; q < S::PAIRS * (kK + 1); q += kCT) {
            float sum = 0.f;
#pragma unroll
            for (int s2 = 0; s2 < S::SPLIT; ++s2) sum += red[(size_t)s2 * S::PAIRS * (kK + 1) + q];
            const int pid = q / (kK + 1), t = q - pid * (kK + 1);
            if (t < kK) {
                unsafeAtomicAdd(gw + (size_t)pid * kK + t, sum);
            } else if (gb && pid % CIN == 0) {
                unsafeAtomicAdd(gb + pid / CIN, sum);
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < S::NPT; ++q) {
            const int pid = (int)threadIdx.x + kCT * q;
            if (pid < S::PAIRS) {
#pragma unroll
                for (int t = 0; t < kK; ++t) unsafeAtomicAdd(gw + (size_t)pid * kK + t, acc[q][t]);
                if (gb && ci_[q] == 0) unsafeAtomicAdd(gb + co_[q], accb[q]);
            }
        }
    }
}

// Weight gradient of a 32 -> 32 layer on the matrix cores: for each block's
// run of positions, G[o][n] = sum_x gout[o][x] in[i][x + t - k/2] with
// n = 9 i + t (the column order of w[o][i][t]), i.e. a 32 x 288 contraction
// over positions, 4 positions per v_mfma_f32_16x16x4f32 step.  A block owns
// every 1024th work item (one row segment of 128 positions), staged with
// asynchronous loads straight into LDS; wave w accumulates the 16 x 16 tiles
// (o tile w % 2, n tiles 9 (w / 2) .. 9 (w / 2) + 8) in registers across all
// its items, then writes the block's partial sums (and its bias partial
// sums); a second kernel adds the partials of all blocks in a fixed order, so
// the result does not depend on scheduling.
constexpr int kWgSeg = 128;                       // positions per work item
constexpr int kWgTP = kWgSeg + 2 * kHalo + 4;     // input row pitch (140 = 12 mod 32)
constexpr int kWgGP = kWgSeg + 4;                 // gradient row pitch (132 = 4 mod 32)
constexpr int kWgN = 32 * kK;                     // 288 columns
constexpr int kWgPart = 32 * kWgN + 32;           // floats of one block's partial sums
constexpr int kWgBlocks = 1024;

__global__ __launch_bounds__(256) void wgrad32_mfma_kernel(const float* __restrict__ in,
                                                         const float* __restrict__ go,
                                                         float* __restrict__ part, int rows,
                                                         int len, int nseg)
{
    __shared__ float tin[32][kWgTP];
    __shared__ float tgo[32][kWgGP];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int ot = wave & 1, nt0 = (wave >> 1) * 9;
    // per-lane LDS offsets: A[o][k] = gout[o][x + k], B[k][n] = in[i][x + k + t - k/2]
    const int aoff = (ot * 16 + (lane & 15)) * kWgGP + (lane >> 4);
    int boff[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const int n = 16 * (nt0 + j) + (lane & 15);
        const int i = n / kK, t = n - kK * i;
        boff[j] = i * kWgTP + t + (lane >> 4);
    }
    mx4 acc[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) acc[j] = mx4{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;                             // bias: channel tid % 32, positions tid / 32 + 8 m
    const float* ti = &tin[0][0];
    const float* tg = &tgo[0][0];
    constexpr unsigned kOut = 0x80000000u;
    const int64_t items = (int64_t)rows * nseg;
    for (int64_t it = blockIdx.x; it < items; it += gridDim.x) {
        const int r = (int)(it / nseg);
        const int x0 = (int)(it - (int64_t)r * nseg) * kWgSeg;
        __syncthreads();                                   // previous item no longer read
        const __amdgpu_buffer_rsrc_t rin = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(in + (size_t)r * 32 * len), 0, (int)(32u * (unsigned)len * 4u), 0x00020000);
        const __amdgpu_buffer_rsrc_t rgo = __builtin_amdgcn_make_buffer_rsrc(
            (void*)(go + (size_t)r * 32 * len), 0, (int)(32u * (unsigned)len * 4u), 0x00020000);
        for (int ci = wave; ci < 32; ci += 4) {
            const unsigned rowoff = (unsigned)ci * (unsigned)len * 4u;
            for (int g = 0; g * 64 < kWgSeg + 2 * kHalo; ++g) {
                const int xx = g * 64 + lane;
                const int x = x0 + xx - kHalo;
                const unsigned vo = (x >= 0 && x < len) ? (unsigned)x * 4u : kOut;
                if (xx < kWgSeg + 2 * kHalo)               // lanes past the row write nothing
                    __builtin_amdgcn_raw_ptr_buffer_load_lds(rin, lds_ptr(&tin[ci][g * 64]), 4, vo,
                                                             rowoff, 0, 0);
            }
            for (int g = 0; g * 64 < kWgSeg; ++g) {
                const int x = x0 + g * 64 + lane;
                const unsigned vo = x < len ? (unsigned)x * 4u : kOut;
                __builtin_amdgcn_raw_ptr_buffer_load_lds(rgo, lds_ptr(&tgo[ci][g * 64]), 4, vo,
                                                         rowoff, 0, 0);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        for (int xx = tid >> 5; xx < kWgSeg; xx += 8) bsum += tgo[tid & 31][xx];
#pragma unroll 4
        for (int xs = 0; xs < kWgSeg; xs += 4) {
            const float a = tg[aoff + xs];
#pragma unroll
            for (int j = 0; j < 9; ++j)
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, ti[boff[j] + xs], acc[j], 0, 0, 0);
        }
    }
    // D: lane l, register q -> row o = 16 ot + 4 (l / 16) + q, column n = 16 nt + l % 16
    float* pb = part + (size_t)blockIdx.x * kWgPart;
#pragma unroll
    for (int j = 0; j < 9; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int o = ot * 16 + 4 * (lane >> 4) + q;
            pb[o * kWgN + 16 * (nt0 + j) + (lane & 15)] = acc[j][q];
        }
    __syncthreads();
    float* red = &tgo[0][0];
    red[tid] = bsum;
    __syncthreads();
    if (tid < 32) {
        float sb = 0.f;
#pragma unroll
        for (int st = 0; st < 8; ++st) sb += red[st * 32 + tid];
        pb[32 * kWgN + tid] = sb;
    }
}

// gw[e] += sum_b part[b][e] (e < 32 x 288), gb[o] += sum_b part[b][32 x 288 + o]
__global__ __launch_bounds__(256) void wgrad_reduce_kernel(const float* __restrict__ part, int nblk,
                                                         float* __restrict__ gw,
                                                         float* __restrict__ gb)
{
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= kWgPart) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * kWgPart + e];
    if (e < 32 * kWgN) gw[e] += s;
    else if (gb) gb[e - 32 * kWgN] += s;
}

// Weight gradients of the layers with one input or one output channel
// (32 -> 1 and 1 -> 32; both weight tensors are indexed c k + t with c the
// 32-channel side): memory-bound like their forward passes.  Thread
// (channel group, position stream) owns 4 of the 32 channels with their 9
// taps and bias sums and walks positions 4 at a time across all rows,
// reading the 12 samples of the input side and 4 of the gradient side with
// 16-byte loads where the row allows.  Each block reduces its threads' sums
// (wave shuffles, then LDS) into one partial; a second kernel adds the
// partials in a fixed order.
constexpr int kWsCG = 4;                          // channels per thread
constexpr int kWsBlocks = 128;                    // position streams (blocks) per channel group
constexpr int kWsVals = kWsCG * (kK + 1);         // sums per thread: 9 taps + bias per channel

// gout[x0 .. x0 + 3] of one row, zero at or beyond len.
__device__ __forceinline__ void load4(const float* __restrict__ row, int x0, int len, bool vec4,
                                      float (&g)[4])
{
    if (vec4) {
        const float4 a = *reinterpret_cast<const float4*>(row + x0);
        g[0] = a.x; g[1] = a.y; g[2] = a.z; g[3] = a.w;
    } else {
#pragma unroll
        for (int p = 0; p < 4; ++p) g[p] = x0 + p < len ? row[x0 + p] : 0.f;
    }
}

template <bool TO1>
__global__ __launch_bounds__(256) void wgrad_small_kernel(const float* __restrict__ in,
                                                          const float* __restrict__ go,
                                                          float* __restrict__ part, int rows,
                                                          int len, int nq)
{
    __shared__ float red[4][kWsVals];
    const int cg = blockIdx.x / kWsBlocks, pbk = blockIdx.x - cg * kWsBlocks;
    const int c0 = cg * kWsCG;
    float acc[kWsCG][kK + 1];
#pragma unroll
    for (int c = 0; c < kWsCG; ++c)
#pragma unroll
        for (int t = 0; t <= kK; ++t) acc[c][t] = 0.f;
    const bool al = aligned16(in, go, in, go) && (len & 3) == 0;
    const int64_t items = (int64_t)rows * nq;
    for (int64_t it = (int64_t)pbk * 256 + threadIdx.x; it < items; it += (int64_t)kWsBlocks * 256) {
        const int r = (int)(it / nq);
        const int x0 = 4 * (int)(it - (int64_t)r * nq);
        const bool vec = al && x0 >= 4 && x0 + 8 <= len;
        const bool vec4 = al && x0 + 4 <= len;
        if (TO1) {
            // gw[0][i][t] += sum gout[0][x] in[i][x + t - 4]
            float g[4];
            load4(go + (size_t)r * len, x0, len, vec4, g);
#pragma unroll
            for (int c = 0; c < kWsCG; ++c) {
                float v[12];
                load12(in + ((size_t)r * 32 + c0 + c) * len, x0, len, vec, v);
#pragma unroll
                for (int t = 0; t < kK; ++t)
#pragma unroll
                    for (int p = 0; p < 4; ++p) acc[c][t] = fmaf(g[p], v[p + t], acc[c][t]);
            }
            acc[0][kK] += (g[0] + g[1]) + (g[2] + g[3]);
        } else {
            // gw[o][0][t] += sum gout[o][x] in[0][x + t - 4]
            float v[12];
            load12(in + (size_t)r * len, x0, len, vec, v);
#pragma unroll
            for (int c = 0; c < kWsCG; ++c) {
                float g[4];
                load4(go + ((size_t)r * 32 + c0 + c) * len, x0, len, vec4, g);
#pragma unroll
                for (int t = 0; t < kK; ++t)
#pragma unroll
                    for (int p = 0; p < 4; ++p) acc[c][t] = fmaf(g[p], v[p + t], acc[c][t]);
                acc[c][kK] += (g[0] + g[1]) + (g[2] + g[3]);
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < kWsCG; ++c)
#pragma unroll
        for (int t = 0; t <= kK; ++t) {
            float x = acc[c][t];
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) x += __shfl_xor(x, m, 64);
            if (lane == 0) red[wave][c * (kK + 1) + t] = x;
        }
    __syncthreads();
    if (threadIdx.x < kWsVals) {
        const int q = threadIdx.x;
        part[(size_t)blockIdx.x * kWsVals + q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
    }
}

// gw[c k + t] += sum over streams; bias: gb[c] (1 -> 32) or gb[0] (32 -> 1)
template <bool TO1>
__global__ __launch_bounds__(256) void wgrad_small_reduce_kernel(const float* __restrict__ part,
                                                                 float* __restrict__ gw,
                                                                 float* __restrict__ gb)
{
    const int e = blockIdx.x * 256 + threadIdx.x;    // (channel group, value)
    if (e >= 8 * kWsVals) return;
    const int cg = e / kWsVals, q = e - cg * kWsVals;
    const int c = cg * kWsCG + q / (kK + 1), t = q % (kK + 1);
    float s = 0.f;
    for (int b = 0; b < kWsBlocks; ++b) s += part[((size_t)cg * kWsBlocks + b) * kWsVals + q];
    if (t < kK) gw[c * kK + t] += s;
    else if (gb && (!TO1 || c == 0)) gb[TO1 ? 0 : c] += s;
}

// loss[0] += sum (a - b)^2 ;  grad = scale (a - b)  (scale = 2/n: gradient of the mean)
__global__ __launch_bounds__(256) void sqerr_kernel(const float* __restrict__ a,
                                                    const float* __restrict__ b,
                                                    float* __restrict__ grad, float scale,
                                                    int64_t n, float* __restrict__ loss)
{
    __shared__ float part[4];
    float s = 0.f;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * blockDim.x) {
        const float d = a[q] - b[q];
        s = fmaf(d, d, s);
        if (grad) grad[q] = scale * d;
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) unsafeAtomicAdd(loss, (part[0] + part[1]) + (part[2] + part[3]));
}

// Adam (Kingma and Ba, ICLR 2015, Algorithm 1):
//   m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;
//   p -= lr (m / c1) / (sqrt(v / c2) + eps),  c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int n, float lr,
                            float b1, float b2, float eps, float c1, float c2)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const float gq = g[q];
    const float mq = fmaf(b1, m[q], (1.f - b1) * gq);
    const float vq = fmaf(b2, v[q], (1.f - b2) * gq * gq);
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

template <bool TRANS>
fdk_status conv32(int rows, int len, const float* in, const float* w, const float* b,
                  const float* mask, const float* add, float alpha, int relu, float* out,
                  hipStream_t st)
{
    const int nseg = (len + kMxSeg - 1) / kMxSeg;
    if ((int64_t)nseg * rows >= (1ll << 31) || (int64_t)len * 32 * 4 >= (1ll << 31))
        return fail(FDK_E_UNSUPPORTED, "conv1d tensor too large for one launch");
    void* wa = nullptr;
    constexpr int n = 2 * kMxSteps * 64;
    fdk_status s = device_alloc_async(n * sizeof(float), st, &wa);
    if (s != FDK_OK) return s;
    hipLaunchKernelGGL(arrange_a_kernel<TRANS>, dim3((n + 255) / 256), dim3(256), 0, st, w,
                       (float*)wa);
    s = check_launch("weight layout kernel");
    if (s == FDK_OK) {
        hipLaunchKernelGGL(conv32_mfma_kernel, dim3((unsigned)(nseg * rows)), dim3(256), 0, st, in,
                           (const float*)wa, b, mask, add, alpha, relu, out, len, nseg);
        s = check_launch(TRANS ? "conv1d backward-data kernel" : "conv1d forward kernel");
    }
    const fdk_status s2 = device_free_async(wa, st);
    return s != FDK_OK ? s : s2;
}

// Launch of the streaming kernels (TO1: 32 -> 1, else 1 -> 32).
template <bool TO1, bool TRANS>
fdk_status conv_stream(int rows, int len, const float* in, const float* w, const float* b,
                       const float* mask, const float* add, float alpha, int relu, float* out,
                       hipStream_t st)
{
    const int nq = TO1 ? (len + kTo1 - 1) / kTo1 : (len + 3) / 4;   // threads per row
    const int64_t blocks = ((int64_t)rows * nq + 255) / 256;
    if (blocks >= (1ll << 31)) return fail(FDK_E_UNSUPPORTED, "conv1d tensor too large for one launch");
    if (TO1)
        hipLaunchKernelGGL(conv_to1_kernel<TRANS>, dim3((unsigned)blocks), dim3(256), 0, st, in, w, b,
                           mask, add, alpha, relu, out, rows, len, nq);
    else
        hipLaunchKernelGGL(conv_from1_kernel<TRANS>, dim3((unsigned)blocks), dim3(256), 0, st, in, w,
                           b, mask, add, alpha, relu, out, rows, len, nq);
    return check_launch(TRANS ? "conv1d backward-data kernel" : "conv1d forward kernel");
}

template <int CIN, int COUT, bool TRANS>
fdk_status conv(int rows, int len, const float* in, const float* w, const float* b,
                const float* mask, const float* add, float alpha, int relu, float* out,
                hipStream_t st)
{
    using S = ConvShape<COUT>;
    const int nseg = (len + S::SEG - 1) / S::SEG;
    if ((int64_t)nseg * rows >= (1ll << 31))
        return fail(FDK_E_UNSUPPORTED, "conv1d tensor too large for one launch");
    hipLaunchKernelGGL((conv_kernel<CIN, COUT, TRANS>), dim3((unsigned)(nseg * rows)), dim3(S::NT),
                       0, st, in, w, b, mask, add, alpha, relu, out, len, nseg);
    return check_launch(TRANS ? "conv1d backward-data kernel" : "conv1d forward kernel");
}

template <int CIN, int COUT>
fdk_status wgrad(int rows, int len, const float* in, const float* go, float* gw, float* gb,
                 hipStream_t st)
{
    // about 1024 blocks: enough to fill 256 CUs, few atomics per weight
    int rpb = (rows + 1023) / 1024;
    if (rpb < 1) rpb = 1;
    const int blocks = (rows + rpb - 1) / rpb;
    hipLaunchKernelGGL((conv_wgrad_kernel<CIN, COUT>), dim3((unsigned)blocks), dim3(kCT), 0, st,
                       in, go, gw, gb, rows, len, rpb);
    return check_launch("conv1d weight-gradient kernel");
}

bool supported(int cin, int cout)
{
    return (cin == 1 || cin == 32) && (cout == 1 || cout == 32);
}

}  // namespace

fdk_status launch_conv1d_forward(int cin, int cout, int rows, int len, const float* in,
                                 const float* w, const float* bias, const float* mask,
                                 const float* add, float alpha, int relu, float* out,
                                 void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (!supported(cin, cout))
        return fail(FDK_E_UNSUPPORTED, "conv1d channels must be 1 or 32");
    if (cin == 1 && cout == 32) return conv_stream<false, false>(rows, len, in, w, bias, mask, add, alpha, relu, out, st);
    if (cin == 32 && cout == 32) return conv32<false>(rows, len, in, w, bias, mask, add, alpha, relu, out, st);
    if (cin == 32 && cout == 1) return conv_stream<true, false>(rows, len, in, w, bias, mask, add, alpha, relu, out, st);
    return conv<1, 1, false>(rows, len, in, w, bias, mask, add, alpha, relu, out, st);
}

fdk_status launch_conv1d_backward_data(int cin, int cout, int rows, int len, const float* gout,
                                       const float* w, const float* mask, float* gin, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (!supported(cin, cout))
        return fail(FDK_E_UNSUPPORTED, "conv1d channels must be 1 or 32");
    // the transposed convolution reads `cout` channels and writes `cin`
    if (cin == 1 && cout == 32) return conv_stream<true, true>(rows, len, gout, w, nullptr, mask, nullptr, 1.f, 0, gin, st);
    if (cin == 32 && cout == 32) return conv32<true>(rows, len, gout, w, nullptr, mask, nullptr, 1.f, 0, gin, st);
    if (cin == 32 && cout == 1) return conv_stream<false, true>(rows, len, gout, w, nullptr, mask, nullptr, 1.f, 0, gin, st);
    return conv<1, 1, true>(rows, len, gout, w, nullptr, mask, nullptr, 1.f, 0, gin, st);
}

template <bool TO1>
fdk_status wgrad_small(int rows, int len, const float* in, const float* gout, float* gw,
                       float* gb, hipStream_t st)
{
    const int nq = (len + 3) / 4;
    constexpr int nblk = 8 * kWsBlocks;
    void* part = nullptr;
    fdk_status s = device_alloc_async((size_t)nblk * kWsVals * sizeof(float), st, &part);
    if (s != FDK_OK) return s;
    hipLaunchKernelGGL(wgrad_small_kernel<TO1>, dim3(nblk), dim3(256), 0, st, in, gout,
                       (float*)part, rows, len, nq);
    s = check_launch("conv1d weight-gradient kernel");
    if (s == FDK_OK) {
        hipLaunchKernelGGL(wgrad_small_reduce_kernel<TO1>, dim3((8 * kWsVals + 255) / 256), dim3(256),
                           0, st, (const float*)part, gw, gb);
        s = check_launch("weight-gradient reduction kernel");
    }
    const fdk_status s2 = device_free_async(part, st);
    return s != FDK_OK ? s : s2;
}

fdk_status wgrad32(int rows, int len, const float* in, const float* gout, float* gw, float* gb,
                   hipStream_t st)
{
    const int nseg = (len + kWgSeg - 1) / kWgSeg;
    const int64_t items = (int64_t)rows * nseg;
    if ((int64_t)len * 32 * 4 >= (1ll << 31))
        return fail(FDK_E_UNSUPPORTED, "conv1d rows too long for one launch");
    const int nblk = (int)(items < kWgBlocks ? items : kWgBlocks);
    void* part = nullptr;
    fdk_status s = device_alloc_async((size_t)nblk * kWgPart * sizeof(float), st, &part);
    if (s != FDK_OK) return s;
    hipLaunchKernelGGL(wgrad32_mfma_kernel, dim3((unsigned)nblk), dim3(256), 0, st, in, gout,
                       (float*)part, rows, len, nseg);
    s = check_launch("conv1d weight-gradient kernel");
    if (s == FDK_OK) {
        hipLaunchKernelGGL(wgrad_reduce_kernel, dim3((kWgPart + 255) / 256), dim3(256), 0, st,
                           (const float*)part, nblk, gw, gb);
        s = check_launch("weight-gradient reduction kernel");
    }
    const fdk_status s2 = device_free_async(part, st);
    return s != FDK_OK ? s : s2;
}

fdk_status launch_conv1d_backward_weight(int cin, int cout, int rows, int len, const float* in,
                                         const float* gout, float* gw, float* gb, void* stream)
{
    hipStream_t st = (hipStream_t)stream;
    if (!supported(cin, cout))
        return fail(FDK_E_UNSUPPORTED, "conv1d channels must be 1 or 32");
    if (cin == 1 && cout == 32) return wgrad_small<false>(rows, len, in, gout, gw, gb, st);
    if (cin == 32 && cout == 32) return wgrad32(rows, len, in, gout, gw, gb, st);
    if (cin == 32 && cout == 1) return wgrad_small<true>(rows, len, in, gout, gw, gb, st);
    return wgrad<1, 1>(rows, len, in, gout, gw, gb, st);
}

fdk_status launch_sqerr(int64_t n, const float* a, const float* b, float* grad, float scale,
                        float* loss, void* stream)
{
    int64_t blocks = (n + 255) / 256;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(sqerr_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, a,
                       b, grad, scale, n, loss);
    return check_launch("squared-error kernel");
}

fdk_status launch_adam(int n, float* p, const float* g, float* m, float* v, float lr, float b1,
                       float b2, float eps, int step, void* stream)
{
    const float c1 = (float)(1.0 - std::pow((double)b1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)b2, (double)step));
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                       (hipStream_t)stream, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return check_launch("adam kernel");
}

}  // namespace fdk
