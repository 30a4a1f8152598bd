// Analytic line integrals of ellipsoid phantoms (gfx950, FP64).
//
// Test and training data: the paper back-projects forward projections of the
// RabbitCT volume (Section 4.2) and notes that the arithmetic does not depend
// on the content.  Here the projections are exact: for the ray from the source
// S to a pixel centre P, each ellipsoid is mapped to the unit sphere
// (X -> T (X - c0), T = diag(1/axes) R^T); the ray S' + t d' meets the sphere
// for t between the roots of |S' + t d'|^2 = 1, so the chord is
// 2 sqrt(b^2 - a c) / a in units of t, i.e. times |P - S| in millimetres.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace fdk {
namespace {

constexpr int kPThreads = 256;

struct PhantomArgs {
    const double* ell;     // [n_ell][16]: c0 (3), T row-major (9), rho, 0, 0, 0
    float* proj;
    int n_ell, nh, nw, view_begin;
    double theta0, dtheta, sod, sdd, du, dv, cu, cv;
};

__global__ __launch_bounds__(kPThreads) void phantom_kernel(const PhantomArgs A)
{
    const int s = blockIdx.y;
    const int64_t pix = (int64_t)blockIdx.x * kPThreads + threadIdx.x;
    if (pix >= (int64_t)A.nh * A.nw) return;
    const int r = (int)(pix / A.nw), c = (int)(pix - (int64_t)r * A.nw);
    const double th = A.theta0 + A.dtheta * (double)(A.view_begin + s);
    double sn, cs;
    sincos(th, &sn, &cs);
    const double S[3] = {A.sod * cs, A.sod * sn, 0.0};
    const double um = ((double)c - A.cu) * A.du, vm = ((double)r - A.cv) * A.dv;
    // pixel centre C + um e_u + vm e_v with C = -(sdd - sod)(cos, sin, 0)
    const double P[3] = {-(A.sdd - A.sod) * cs - um * sn, -(A.sdd - A.sod) * sn + um * cs, vm};
    const double d[3] = {P[0] - S[0], P[1] - S[1], P[2] - S[2]};
    const double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double acc = 0.0;
    for (int e = 0; e < A.n_ell; ++e) {
        const double* E = A.ell + 16 * (size_t)e;
        const double o[3] = {S[0] - E[0], S[1] - E[1], S[2] - E[2]};
        double sp[3], dp[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            sp[i] = E[3 + 3 * i] * o[0] + E[4 + 3 * i] * o[1] + E[5 + 3 * i] * o[2];
            dp[i] = E[3 + 3 * i] * d[0] + E[4 + 3 * i] * d[1] + E[5 + 3 * i] * d[2];
        }
        const double a = dp[0] * dp[0] + dp[1] * dp[1] + dp[2] * dp[2];
        const double b = dp[0] * sp[0] + dp[1] * sp[1] + dp[2] * sp[2];
        const double cc = sp[0] * sp[0] + sp[1] * sp[1] + sp[2] * sp[2] - 1.0;
        const double disc = b * b - a * cc;
        if (disc > 0.0) acc += E[12] * (2.0 * sqrt(disc) / a) * dn;
    }
    float* dst = A.proj + (size_t)s * A.nh * A.nw + pix;
    *dst += (float)acc;
}

}  // namespace

fdk_status launch_phantom(const PhantomLaunch& a, void* stream)
{
    PhantomArgs A;
    A.ell = a.ell;
    A.proj = a.proj;
    A.n_ell = a.n_ell;
    A.nh = a.nh;
    A.nw = a.nw;
    A.view_begin = a.view_begin;
    A.theta0 = a.theta0;
    A.dtheta = a.arc / (double)a.np_total;
    A.sod = a.sod;
    A.sdd = a.sdd;
    A.du = a.du;
    A.dv = a.dv;
    A.cu = 0.5 * (a.nw - 1) + a.u_off;
    A.cv = 0.5 * (a.nh - 1) + a.v_off;
    const int64_t px = (int64_t)a.nh * a.nw;
    const int64_t bx = (px + kPThreads - 1) / kPThreads;
    if (bx >= (1ll << 31) || a.np > 65535) return fail(FDK_E_UNSUPPORTED, "stack too large for one launch");
    hipLaunchKernelGGL(phantom_kernel, dim3((unsigned)bx, (unsigned)a.np), dim3(kPThreads), 0,
                       (hipStream_t)stream, A);
    return check_launch("phantom kernel");
}

}  // namespace fdk
