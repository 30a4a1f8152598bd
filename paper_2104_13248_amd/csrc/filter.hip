// FDK pre-processing filter (gfx950): cosine weight, Ram-Lak ramp along each
// detector row (linear convolution with zero padding), angular weight.
//
// The paper takes filtered projections as its input and names the filtering
// step without describing it (Sections 2.1.2, 3.1.1).  This is the textbook
// Feldkamp filter: for a row r of view s,
//   q[c]   = raw[c] * sdd / sqrt(sdd^2 + u_mm(c)^2 + v_mm(r)^2)
//   out[c] = tau * arc / (2 np_total) * sum_n h[n] q[c - n]
// with the Ram-Lak kernel h[0] = 1/(4 tau^2), h[odd n] = -1/(pi^2 n^2 tau^2),
// h[even n != 0] = 0 and tau = du sod / sdd.
//
// Rows up to 2048 pixels are filtered through the Fourier domain: h is even,
// so its length-M transform H (M the power of two >= 2 nw - 1, which keeps the
// circular convolution free of wrap-around over the nw outputs) is real, and
// two weighted rows a, b packed as z = a + i b give z * h = (a * h) + i (b * h)
// from one forward transform, a multiplication by H and one inverse transform.
// A block owns such a pair of rows; the transforms are Stockham radix-16/8/4/2
// passes in LDS (natural order in and out), the inverse taken as
// conj(FFT(conj(.))) with 1/M and the FDK constants folded into H, its radices
// in the reverse order so that the forward's last pass, the product with H and
// the inverse's first pass run in registers as one step.  H and the
// twiddle factors are built per call in FP64.  Longer rows use a direct
// convolution: one block per row, the weighted row and the odd-tap
// coefficients in LDS, each q read once per pair of symmetric taps.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.h"

namespace fdk {
namespace {

constexpr int kFilterThreads = 256;
constexpr int kFftMaxRow = 2048;   // rows up to this length are filtered through the Fourier domain

struct FilterArgs {
    const float* raw;
    float* out;
    int nh, nw;
    float cu, cv, du, dv, sdd2, sdd;
    float h0;          // h[0] * tau * angular weight
    float hscale;      // -1/(pi^2 tau^2) * tau * angular weight
    unsigned* maxbits; // per-view |out| maxima (float bits, atomicMax) or nullptr
};

// Maximum over the block of a non-negative per-thread value, posted with one
// atomicMax to the bit pattern of maxbits[view] (bit order = value order for
// non-negative floats, so the result does not depend on the order).  `part`
// holds one word per wave.  Every thread of the block must call it.
__device__ __forceinline__ void post_block_max(float m, float* part, unsigned* maxbits, int64_t view)
{
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    const int nwaves = (blockDim.x + 63) >> 6;
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < nwaves; ++w) m = fmaxf(m, part[w]);
        atomicMax(&maxbits[view], __float_as_uint(m));
    }
}

__global__ __launch_bounds__(kFilterThreads) void filter_kernel(const FilterArgs A)
{
    extern __shared__ float sm[];
    float* q = sm;                       // [nw] cosine-weighted row
    float* hodd = sm + A.nw;             // [nw/2 + 1] coefficient of tap 2m+1
    const int row = blockIdx.x;          // s * nh + r
    const int r = row % A.nh;
    const float* src = A.raw + (size_t)row * A.nw;
    float* dst = A.out + (size_t)row * A.nw;
    const float vmm = ((float)r - A.cv) * A.dv;
    const float v2 = A.sdd2 + vmm * vmm;
    for (int c = threadIdx.x; c < A.nw; c += kFilterThreads) {
        const float umm = ((float)c - A.cu) * A.du;
        q[c] = src[c] * (A.sdd * rsqrtf(fmaf(umm, umm, v2)));
    }
    const int nodd = (A.nw + 1) / 2;
    for (int m = threadIdx.x; m < nodd; m += kFilterThreads) {
        const float n = (float)(2 * m + 1);
        hodd[m] = A.hscale / (n * n);
    }
    __syncthreads();
    float mx = 0.f;
    for (int c = threadIdx.x; c < A.nw; c += kFilterThreads) {
        // taps c - n and c + n for odd n; both sides while both exist
        const int both = min(c, A.nw - 1 - c);
        float acc = 0.f;
        int m = 0;
        for (; 2 * m + 1 <= both; ++m) acc = fmaf(hodd[m], q[c - 2 * m - 1] + q[c + 2 * m + 1], acc);
        if (c < A.nw - 1 - c) {
            for (; 2 * m + 1 <= A.nw - 1 - c; ++m) acc = fmaf(hodd[m], q[c + 2 * m + 1], acc);
        } else {
            for (; 2 * m + 1 <= c; ++m) acc = fmaf(hodd[m], q[c - 2 * m - 1], acc);
        }
        const float y = fmaf(A.h0, q[c], acc);
        dst[c] = y;
        mx = fmaxf(mx, fabsf(y));
    }
    if (A.maxbits) {
        __shared__ float part[kFilterThreads / 64];
        post_block_max(mx, part, A.maxbits, row / A.nh);
    }
}

// ---- Fourier-domain filter

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// In-place forward DFT of R = 2, 4, 8 or 16 points (kernel e^{-2 pi i n k / R}).
// HALF: v[R/2 ..] are zero on entry (the zero-padded half of a row), so the
// first radix-2 stage of the even/odd split reduces to copies.
template <int R, bool HALF = false>
__device__ __forceinline__ void dft(float2 (&v)[R])
{
    if constexpr (HALF && R == 2) {
        v[1] = v[0];
    } else if constexpr (HALF && R == 4) {
        // (a, b, 0, 0) -> (a + b, a - i b, a - b, a + i b)
        const float2 a = v[0], b = v[1];
        v[0] = make_float2(a.x + b.x, a.y + b.y);
        v[2] = make_float2(a.x - b.x, a.y - b.y);
        v[1] = make_float2(a.x + b.y, a.y - b.x);
        v[3] = make_float2(a.x - b.y, a.y + b.x);
    } else if constexpr (R == 2) {
        const float2 a = v[0], b = v[1];
        v[0] = make_float2(a.x + b.x, a.y + b.y);
        v[1] = make_float2(a.x - b.x, a.y - b.y);
    } else if constexpr (R == 4) {
        const float2 t0 = make_float2(v[0].x + v[2].x, v[0].y + v[2].y);
        const float2 t1 = make_float2(v[0].x - v[2].x, v[0].y - v[2].y);
        const float2 t2 = make_float2(v[1].x + v[3].x, v[1].y + v[3].y);
        const float2 t3 = make_float2(v[1].y - v[3].y, v[3].x - v[1].x);   // -i (v1 - v3)
        v[0] = make_float2(t0.x + t2.x, t0.y + t2.y);
        v[2] = make_float2(t0.x - t2.x, t0.y - t2.y);
        v[1] = make_float2(t1.x + t3.x, t1.y + t3.y);
        v[3] = make_float2(t1.x - t3.x, t1.y - t3.y);
    } else if constexpr (R == 16) {
        // X[k] = E[k] + W16^k O[k], X[k + 8] = E[k] - W16^k O[k]
        float2 e[8], o[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            e[r] = v[2 * r];
            o[r] = v[2 * r + 1];
        }
        dft<8, HALF>(e);
        dft<8, HALF>(o);
        constexpr float c1 = 0.92387953251128676f, s1 = 0.38268343236508977f;
        constexpr float h = 0.70710678118654752f;
        const float2 w16[8] = {make_float2(1.f, 0.f), make_float2(c1, -s1), make_float2(h, -h),
                               make_float2(s1, -c1), make_float2(0.f, -1.f), make_float2(-s1, -c1),
                               make_float2(-h, -h), make_float2(-c1, -s1)};
#pragma unroll
        for (int k = 1; k < 8; ++k) o[k] = cmul(o[k], w16[k]);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            v[k] = make_float2(e[k].x + o[k].x, e[k].y + o[k].y);
            v[k + 8] = make_float2(e[k].x - o[k].x, e[k].y - o[k].y);
        }
    } else {
        // X[k] = E[k] + W8^k O[k], X[k + 4] = E[k] - W8^k O[k]
        float2 e[4] = {v[0], v[2], v[4], v[6]};
        float2 o[4] = {v[1], v[3], v[5], v[7]};
        dft<4, HALF>(e);
        dft<4, HALF>(o);
        constexpr float h = 0.70710678118654752f;
        o[1] = make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));     // * (h, -h)
        o[2] = make_float2(o[2].y, -o[2].x);                                   // * -i
        o[3] = make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));    // * (-h, -h)
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k] = make_float2(e[k].x + o[k].x, e[k].y + o[k].y);
            v[k + 4] = make_float2(e[k].x - o[k].x, e[k].y - o[k].y);
        }
    }
}

// LDS index of element e: one pad word pair per 32 elements breaks the
// power-of-two strides of the passes' writes across the banks.
__device__ __forceinline__ int fpad(int e) { return e + (e >> 5); }

// Twiddles w[r] = W^r, r = 1 .. R - 1, of one butterfly from one table entry
// W: the others by at most four complex products (W^2 = W W, W^4 = W^2 W^2,
// W^8 = W^4 W^4, W^3 = W^2 W, W^5 = W^4 W, W^6 = W^4 W^2, W^7 = W^4 W^3,
// W^(8+r) = W^8 W^r).
template <int R>
__device__ __forceinline__ void twiddles(float2 W, float2 (&w)[R])
{
    w[1] = W;
    if constexpr (R >= 4) {
        w[2] = cmul(W, W);
        w[3] = cmul(w[2], W);
    }
    if constexpr (R >= 8) {
        w[4] = cmul(w[2], w[2]);
        w[5] = cmul(w[4], W);
        w[6] = cmul(w[4], w[2]);
        w[7] = cmul(w[4], w[3]);
    }
    if constexpr (R == 16) {
        w[8] = cmul(w[4], w[4]);
#pragma unroll
        for (int r = 9; r < 16; ++r) w[r] = cmul(w[8], w[r - 8]);
    }
}

// Radix of the pass after sub-transforms of length NS: 16 while at least 16
// remain, then the rest.
__host__ __device__ constexpr int fft_radix(int M, int NS) { return M / NS >= 16 ? 16 : M / NS; }

// Sub-transform length before the forward transform's last pass.
__host__ __device__ constexpr int last_pass_ns(int M)
{
    int ns = 1;
    while (ns * 16 < M) ns *= 16;
    return ns;
}

// Stockham passes of a length-M forward DFT (natural order in and out), from
// sub-transform length NS on.  Pass of radix R after sub-transforms of length
// NS: butterfly j reads elements j + r M/R, twiddles them by
// W_{NS R}^{(j mod NS) r}, and writes (j / NS) NS R + (j mod NS) + r NS.  The
// first pass reads through first(e) and the last writes through last(e, v)
// (FIRST_LDS / LAST_LDS: whether those touch the LDS buffer, which decides the
// barriers); the passes in between use the buffer.  The passes stop at
// sub-transform length NS_END.
// HALF_IN: the input's upper half is zero (the first pass reads none of it);
// HALF_OUT: only the output's lower half is used (the last pass neither
// computes nor stores the rest).
template <int M, int T, int NS, int NS_END, bool FIRST_LDS, bool LAST_LDS, bool HALF_IN,
          bool HALF_OUT, class First, class Last>
__device__ __forceinline__ void fft_passes(float2* buf, const float2* __restrict__ tw, int tid,
                                           First first, Last last)
{
    if constexpr (NS < NS_END) {
        constexpr int R = fft_radix(M, NS);
        constexpr bool is_first = NS == 1, is_last = NS * R == NS_END;
        constexpr bool load_lds = !is_first || FIRST_LDS;
        constexpr bool store_lds = !is_last || LAST_LDS;
        constexpr int B = M / R;
        constexpr int J = (B + T - 1) / T;
        float2 v[J][R];
#pragma unroll
        for (int q = 0; q < J; ++q) {
            const int j = tid + T * q;
            if (j < B) {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if constexpr (is_first) {
                        v[q][r] = !HALF_IN || 2 * r < R ? first(j + r * B) : make_float2(0.f, 0.f);
                    } else {
                        v[q][r] = buf[fpad(j + r * B)];
                    }
                }
                if constexpr (NS > 1) {
                    float2 w[R];
                    twiddles<R>(tw[(j % NS) * (M / (NS * R))], w);
#pragma unroll
                    for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], w[r]);
                }
                dft<R, is_first && HALF_IN>(v[q]);
            }
        }
        if constexpr (load_lds && store_lds) __syncthreads();   // in place: all reads first
#pragma unroll
        for (int q = 0; q < J; ++q) {
            const int j = tid + T * q;
            if (j < B) {
                const int d = (j / NS) * NS * R + j % NS;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if constexpr (is_last) {
                        if (!HALF_OUT || 2 * r < R) last(d + r * NS, v[q][r]);
                    } else {
                        buf[fpad(d + r * NS)] = v[q][r];
                    }
                }
            }
        }
        if constexpr (store_lds) __syncthreads();
        fft_passes<M, T, NS * R, NS_END, FIRST_LDS, LAST_LDS, HALF_IN, HALF_OUT>(buf, tw, tid,
                                                                                first, last);
    }
}

// The forward transform's last pass and the inverse's first, fused in
// registers: with the inverse's radices taken in the reverse order, both
// passes read elements j + r NS_LAST for butterfly j (R = M / NS_LAST), so
// each thread twiddles and transforms its elements, multiplies them by H
// (real) and conjugates them (the inverse as conj(FFT(conj(.)))), transforms
// them again as the inverse's first pass (no twiddles after sub-transforms of
// length 1) and stores them to where that pass writes, element j R + r.
template <int M, int T>
__device__ __forceinline__ void fft_middle(float2* buf, const float2* __restrict__ tw,
                                           const float* __restrict__ H, int tid)
{
    constexpr int NS = last_pass_ns(M);
    constexpr int R = M / NS;
    constexpr int B = NS;                          // butterflies of either pass
    constexpr int J = (B + T - 1) / T;
    float2 v[J][R];
#pragma unroll
    for (int q = 0; q < J; ++q) {
        const int j = tid + T * q;
        if (j < B) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[q][r] = buf[fpad(j + r * B)];
            if constexpr (NS > 1) {
                float2 w[R];
                twiddles<R>(tw[j], w);
#pragma unroll
                for (int r = 1; r < R; ++r) v[q][r] = cmul(v[q][r], w[r]);
            }
            dft<R>(v[q]);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const float h = H[j + r * NS];
                v[q][r] = make_float2(v[q][r].x * h, -v[q][r].y * h);
            }
            dft<R>(v[q]);
        }
    }
    __syncthreads();                               // in place: all reads first
#pragma unroll
    for (int q = 0; q < J; ++q) {
        const int j = tid + T * q;
        if (j < B) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[fpad(j * R + r)] = v[q][r];
        }
    }
    __syncthreads();
}

// Threads of the Fourier-domain filter's block: one per radix-16 butterfly.
template <int M>
constexpr int fft_threads() { return M / 16 < 64 ? 64 : (M / 16 > 256 ? 256 : M / 16); }

// MAXB: also post the |output| maxima of each view to A.maxbits.  H holds
// the factor sdd of the cosine weight besides 1/M and the FDK constants.
template <int M, bool MAXB>
__global__ __launch_bounds__(fft_threads<M>()) void filter_fft_kernel(const FilterArgs A,
                                                                    const float* __restrict__ H,
                                                                    const float2* __restrict__ tw,
                                                                    int64_t nrows)
{
    __shared__ float2 buf[M + M / 32];
    const int tid = threadIdx.x;
    const int64_t row0 = 2 * (int64_t)blockIdx.x;
    const bool two = row0 + 1 < nrows;
    const float* s0 = A.raw + row0 * A.nw;
    const float* s1 = s0 + A.nw;
    const int64_t view0 = row0 / A.nh;             // view and detector row of row0
    const int r0 = (int)(row0 - view0 * A.nh);
    const bool wrap = r0 + 1 == A.nh;              // row0 + 1 starts the next view
    const float v0 = ((float)r0 - A.cv) * A.dv;
    const float v1 = ((float)(wrap ? 0 : r0 + 1) - A.cv) * A.dv;
    const float w0 = A.sdd2 + v0 * v0, w1 = A.sdd2 + v1 * v1;
    // forward transform of z = a + i b, the two cosine-weighted rows (zero
    // beyond nw), read straight from the stack by the first pass
    auto weighted = [&](int c) {
        float a = 0.f, b = 0.f;
        if (c < A.nw) {
            const float umm = ((float)c - A.cu) * A.du;
            a = s0[c] * rsqrtf(fmaf(umm, umm, w0));
            if (two) b = s1[c] * rsqrtf(fmaf(umm, umm, w1));
        }
        return make_float2(a, b);
    };
    auto to_buf = [&](int e, float2 v) { buf[fpad(e)] = v; };
    constexpr int T = fft_threads<M>();
    // inverse transform as conj(FFT(conj(Z H))) (H is real and holds 1/M);
    // its last pass writes row a = Re, row b = -Im of the first nw outputs
    // straight to the stack.  conj_zh reads conj(Z H) for a separate first
    // inverse pass (M = 16); longer transforms apply H in fft_middle.
    auto conj_zh = [&](int k) {
        const float2 z = buf[fpad(k)];
        const float h = H[k];
        return make_float2(z.x * h, -z.y * h);
    };
    float* d0 = A.out + row0 * A.nw;
    float m0 = 0.f, m1 = 0.f;                     // |output| maxima of the two rows
    auto to_rows = [&](int c, float2 y) {
        if (c < A.nw) {
            d0[c] = y.x;
            if constexpr (MAXB) m0 = fmaxf(m0, fabsf(y.x));
            if (two) {
                d0[A.nw + c] = -y.y;
                if constexpr (MAXB) m1 = fmaxf(m1, fabsf(y.y));
            }
        }
    };
    // M >= 2 nw (M is even and at least 2 nw - 1): the forward input's upper
    // half is padding and the inverse output's upper half is not stored
    constexpr int NSL = last_pass_ns(M);
    if constexpr (NSL > 1) {
        // forward passes up to the last, the fused middle, then the inverse
        // passes after its first (radix M / NSL)
        fft_passes<M, T, 1, NSL, false, true, true, false>(buf, tw, tid, weighted, to_buf);
        fft_middle<M, T>(buf, tw, H, tid);
        fft_passes<M, T, M / NSL, M, true, false, false, true>(buf, tw, tid, conj_zh, to_rows);
    } else {
        // one pass each way
        fft_passes<M, T, 1, M, false, true, true, false>(buf, tw, tid, weighted, to_buf);
        fft_passes<M, T, 1, M, true, false, false, true>(buf, tw, tid, conj_zh, to_rows);
    }
    if constexpr (MAXB) {
        __shared__ float part[2][4];
        if (!two || !wrap) {
            post_block_max(fmaxf(m0, m1), part[0], A.maxbits, view0);
        } else {
            post_block_max(m0, part[0], A.maxbits, view0);
            post_block_max(m1, part[1], A.maxbits, view0 + 1);
        }
    }
}

// tw[e] = exp(-2 pi i e / M); H[k] = (1/M) (h0 + 2 sum_{odd n < nw} hs / n^2
// cos(2 pi k n / M)), the transform of the wrapped, even kernel; FP64.  One
// wave per k: lanes split the sum over n, then a shuffle reduction.
__global__ __launch_bounds__(64) void filter_tables_kernel(int M, int nw, double h0, double hs,
                                                          float2* __restrict__ tw,
                                                          float* __restrict__ H)
{
    const int k = blockIdx.x, lane = threadIdx.x;
    double acc = 0.0;
    for (int n = 2 * lane + 1; n < nw; n += 128) {
        const int idx = (int)(((int64_t)k * n) % M);
        acc += hs / ((double)n * (double)n) * cospi(2.0 * (double)idx / (double)M);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
    if (lane == 0) {
        double sn, cs;
        sincospi(2.0 * (double)k / (double)M, &sn, &cs);
        tw[k] = make_float2((float)cs, (float)-sn);
        H[k] = (float)((h0 + 2.0 * acc) / (double)M);
    }
}

// Step 1 alone (the input of the learned row filter): q = raw * cosine weight.
__global__ __launch_bounds__(kFilterThreads) void cosine_kernel(const FilterArgs A, int64_t n)
{
    for (int64_t q = (int64_t)blockIdx.x * kFilterThreads + threadIdx.x; q < n;
         q += (int64_t)gridDim.x * kFilterThreads) {
        const int64_t row = q / A.nw;
        const int c = (int)(q - row * A.nw);
        const int r = (int)(row % A.nh);
        const float vmm = ((float)r - A.cv) * A.dv;
        const float umm = ((float)c - A.cu) * A.du;
        A.out[q] = A.raw[q] * (A.sdd * rsqrtf(fmaf(umm, umm, A.sdd2 + vmm * vmm)));
    }
}

FilterArgs filter_args(const FilterLaunch& a)
{
    const double tau = a.du * a.sod / a.sdd;
    const double wang = a.arc / (2.0 * (double)a.np_total);
    const double pi = 3.14159265358979323846;
    FilterArgs A;
    A.raw = a.raw;
    A.out = a.out;
    A.nh = a.nh;
    A.nw = a.nw;
    A.cu = (float)(0.5 * (a.nw - 1) + a.u_off);
    A.cv = (float)(0.5 * (a.nh - 1) + a.v_off);
    A.du = (float)a.du;
    A.dv = (float)a.dv;
    A.sdd = (float)a.sdd;
    A.sdd2 = (float)(a.sdd * a.sdd);
    A.h0 = (float)(1.0 / (4.0 * tau * tau) * tau * wang);
    A.hscale = (float)(-1.0 / (pi * pi * tau * tau) * tau * wang);
    A.maxbits = nullptr;
    return A;
}

}  // namespace

fdk_status launch_cosine_weight(const FilterLaunch& a, void* stream)
{
    const FilterArgs A = filter_args(a);
    const int64_t n = (int64_t)a.np * a.nh * a.nw;
    int64_t blocks = (n + kFilterThreads - 1) / kFilterThreads;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(cosine_kernel, dim3((unsigned)blocks), dim3(kFilterThreads), 0,
                       (hipStream_t)stream, A, n);
    return check_launch("cosine-weight kernel");
}

namespace {

// Filter the rows of A (A.raw, A.out already offset to the first view):
// nviews views of a.nh rows.  tw/H: the Fourier tables (nullptr for rows
// longer than kFftMaxRow); A.maxbits selects the kernels that post maxima.
fdk_status filter_rows(const FilterArgs& A, int32_t nviews, int32_t nh, int32_t nw, int M,
                       const float* H, const float2* tw, hipStream_t st)
{
    const int64_t rows = (int64_t)nviews * nh;
    if (nw <= kFftMaxRow) {
        const dim3 g((unsigned)((rows + 1) / 2));
        switch (M) {
#define FDK_FFT(m)                                                                       \
    case m:                                                                              \
        if (A.maxbits)                                                                   \
            hipLaunchKernelGGL((filter_fft_kernel<m, true>), g, dim3(fft_threads<m>()), 0, \
                               st, A, H, tw, rows);                                      \
        else                                                                             \
            hipLaunchKernelGGL((filter_fft_kernel<m, false>), g, dim3(fft_threads<m>()), 0, \
                               st, A, H, tw, rows);                                      \
        break;
            FDK_FFT(16) FDK_FFT(32) FDK_FFT(64) FDK_FFT(128) FDK_FFT(256) FDK_FFT(512)
            FDK_FFT(1024) FDK_FFT(2048) FDK_FFT(4096)
#undef FDK_FFT
            default: return fail(FDK_E_UNSUPPORTED, "no Fourier filter for this row length");
        }
        return check_launch("filter kernel");
    }
    const size_t lds = (size_t)(nw + (nw + 1) / 2 + 1) * sizeof(float);
    if (lds > 64 * 1024) {
        if (hipFuncSetAttribute((const void*)filter_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)lds) != hipSuccess)
            return fail(FDK_E_DEVICE, "cannot raise the LDS limit of the filter kernel");
    }
    hipLaunchKernelGGL(filter_kernel, dim3((unsigned)rows), dim3(kFilterThreads), lds, st, A);
    return check_launch("filter kernel");
}

// Bytes of float32 workspace per chunk of views of the binary16 output: small
// enough to stay in the last-level cache between the filter and the
// conversion that reads it back.
constexpr int64_t kF16ChunkBytes = 64ll << 20;

}  // namespace

fdk_status launch_filter(const FilterLaunch& a, void* stream)
{
    FilterArgs A = filter_args(a);
    const int64_t rows = (int64_t)a.np * a.nh;
    hipStream_t st = (hipStream_t)stream;
    const bool fft = a.nw <= kFftMaxRow;
    if (fft ? (rows + 1) / 2 >= (1ll << 31) : rows >= (1ll << 31))
        return fail(FDK_E_UNSUPPORTED, "too many detector rows");
    int M = 0;
    void* tab = nullptr;
    float2* tw = nullptr;
    float* H = nullptr;
    fdk_status s = FDK_OK;
    if (fft) {
        M = 16;
        while (M < 2 * a.nw - 1) M *= 2;
        s = device_alloc_async((size_t)M * (sizeof(float) + sizeof(float2)), st, &tab);
        if (s != FDK_OK) return s;
        tw = (float2*)tab;
        H = (float*)(tw + M);
        // H carries the factor sdd of the cosine weight
        const double tau = a.du * a.sod / a.sdd;
        const double wang = a.arc / (2.0 * (double)a.np_total);
        const double pi = 3.14159265358979323846;
        hipLaunchKernelGGL(filter_tables_kernel, dim3(M), dim3(64), 0, st, M, a.nw,
                           1.0 / (4.0 * tau * tau) * tau * wang * a.sdd,
                           -1.0 / (pi * pi * tau * tau) * tau * wang * a.sdd, tw, H);
        s = check_launch("filter table kernel");
    }
    if (s == FDK_OK && !a.out16) {
        s = filter_rows(A, a.np, a.nh, a.nw, M, H, tw, st);
    } else if (s == FDK_OK) {
        // binary16 output: chunks of views through a float32 workspace, the
        // per-view maxima taken by the filter's epilogue
        const int64_t npix = (int64_t)a.nh * a.nw;
        int64_t chunk = kF16ChunkBytes / (npix * (int64_t)sizeof(float));
        if (chunk < 1) chunk = 1;
        if (chunk > a.np) chunk = a.np;
        void* ws = nullptr;
        void* mx = nullptr;
        s = device_alloc_async((size_t)(chunk * npix) * sizeof(float), st, &ws);
        if (s == FDK_OK) s = device_alloc_async((size_t)a.np * sizeof(unsigned), st, &mx);
        if (s == FDK_OK) s = launch_clear_u32((unsigned*)mx, a.np, stream);
        for (int64_t v0 = 0; s == FDK_OK && v0 < a.np; v0 += chunk) {
            const int32_t nv = (int32_t)(v0 + chunk <= a.np ? chunk : a.np - v0);
            FilterArgs C = A;
            C.raw = a.raw + v0 * npix;
            C.out = (float*)ws;
            C.maxbits = (unsigned*)mx + v0;
            s = filter_rows(C, nv, a.nh, a.nw, M, H, tw, st);
            if (s == FDK_OK)
                s = launch_quantize_with_max(nv, npix, (const float*)ws, (const unsigned*)mx + v0,
                                             a.out16 + v0 * npix, a.scale + v0, stream);
        }
        for (void* d : {mx, ws}) {
            const fdk_status e = device_free_async(d, st);
            if (s == FDK_OK) s = e;
        }
    }
    const fdk_status s2 = device_free_async(tab, st);
    return s != FDK_OK ? s : s2;
}

}  // namespace fdk
