// extern "C" entry points of include/fdk.h: argument validation (host, before
// any HIP call), FP64 geometry checks, scratch management and kernel launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "internal.h"

using namespace fdk;

namespace {

fdk_status common_checks(const fdk_volume* vg, const fdk_stack* sg, bool allow_f16,
                         const double* mats, std::vector<IndexMatrix>* M)
{
    fdk_status s = validate_volume(vg);
    if (s != FDK_OK) return s;
    s = validate_stack(sg, allow_f16);
    if (s != FDK_OK) return s;
    return validate_geometry(*vg, *sg, mats, M);
}

void fill_grid(const fdk_volume& vg, double& ox, double& oy, double& oz)
{
    ox = vg.cx - 0.5 * (vg.nx - 1) * vg.dx;
    oy = vg.cy - 0.5 * (vg.ny - 1) * vg.dy;
    oz = vg.cz - 0.5 * (vg.nz - 1) * vg.dz;
}

}  // namespace

extern "C" fdk_status fdk_bp_plan(const fdk_volume* vg, const fdk_stack* sg, const double* mats,
                                  int64_t* out)
{
    if (!out) return fail(FDK_E_INVALID, "output array is NULL");
    std::vector<IndexMatrix> M;
    fdk_status s = common_checks(vg, sg, true, mats, &M);
    if (s != FDK_OK) return s;
    BpPlan plan;
    s = make_bp_plan(*vg, *sg, M, plan);
    if (s != FDK_OK) return s;
    out[0] = kTile;
    out[1] = kTile;
    out[2] = plan.kz;
    out[3] = plan.pitch;
    out[4] = plan.rows;
    out[5] = plan.lds_bytes;
    out[6] = plan.blocks;
    out[7] = kThreads;
    out[8] = plan.rows_full;
    FpPlan fpp;
    std::vector<int32_t> lanes;
    s = make_fp_plan(*vg, *sg, M, lanes, fpp);
    out[9] = s == FDK_OK ? fpp.lds_bytes : 0;
    out[10] = s == FDK_OK ? fpp.rb : 0;
    out[11] = s == FDK_OK ? fpp.cw : 0;
    return FDK_OK;
}

namespace {

// The back-projection of fdk_backproject_slab; `direct` forces the direct
// organisation (taps from memory) whatever the footprint.
fdk_status backproject_slab(const fdk_volume* vg, int32_t k_begin, int32_t k_count,
                            float* vol_slab, const fdk_stack* sg, const void* proj,
                            const float* scale, const double* mats, void* stream, bool direct)
{
    std::vector<IndexMatrix> M;
    fdk_status s = common_checks(vg, sg, true, mats, &M);
    if (s != FDK_OK) return s;
    if (!vol_slab) return fail(FDK_E_INVALID, "volume pointer is NULL");
    if (!proj) return fail(FDK_E_INVALID, "projection pointer is NULL");
    if (sg->dtype == FDK_F16 && !scale)
        return fail(FDK_E_INVALID, "binary16 projections need a per-view scale array");
    if (sg->dtype == FDK_F32 && scale)
        return fail(FDK_E_INVALID, "a scale array is only accepted with binary16 projections");
    if (k_begin < 0 || k_count <= 0 || (int64_t)k_begin + k_count > vg->nz)
        return fail(FDK_E_INVALID, "slab [k_begin, k_begin + k_count) outside the volume");
    if ((int64_t)sg->nh * sg->nw * (sg->dtype == FDK_F16 ? 2 : 4) >= (1ll << 31))
        return fail(FDK_E_UNSUPPORTED, "one view larger than 2 GiB");
    BpPlan plan;
    s = make_bp_plan(*vg, *sg, M, plan);
    if (s != FDK_OK) return s;
    if (direct && !plan.direct) {
        plan.direct = true;
        plan.kz = 32;
        plan.nchunks = (vg->nz + plan.kz - 1) / plan.kz;
        plan.blocks = (int64_t)plan.ntiles_pad * plan.nchunks;
    }

    const size_t mbytes = (size_t)sg->np * 12 * sizeof(double);
    void* d_world = nullptr;
    void* d_index = nullptr;
    s = upload_async(mats, mbytes, stream, &d_world);
    if (s != FDK_OK) return s;
    s = device_alloc_async(mbytes, stream, &d_index);
    if (s != FDK_OK) {
        device_free_async(d_world, stream);
        return s;
    }
    BpLaunch a;
    a.proj = proj;
    a.scale = scale;
    a.mats_world = (const double*)d_world;
    a.mats_index = (double*)d_index;
    a.vol = vol_slab;
    a.nx = vg->nx; a.ny = vg->ny; a.nz = vg->nz;
    a.np = sg->np; a.nh = sg->nh; a.nw = sg->nw;
    a.k_begin = k_begin;
    a.k_end = k_begin + k_count;
    a.dx = vg->dx; a.dy = vg->dy; a.dz = vg->dz;
    fill_grid(*vg, a.ox, a.oy, a.oz);
    a.f16 = sg->dtype == FDK_F16;
    s = launch_backproject(a, plan, stream);
    fdk_status s2 = device_free_async(d_index, stream);
    fdk_status s3 = device_free_async(d_world, stream);
    if (s != FDK_OK) return s;
    return s2 != FDK_OK ? s2 : s3;
}

}  // namespace

extern "C" fdk_status fdk_backproject_slab(const fdk_volume* vg, int32_t k_begin, int32_t k_count,
                                           float* vol_slab, const fdk_stack* sg, const void* proj,
                                           const float* scale, const double* mats, void* stream)
{
    return backproject_slab(vg, k_begin, k_count, vol_slab, sg, proj, scale, mats, stream, false);
}

extern "C" fdk_status fdk_backproject(const fdk_volume* vg, float* vol, const fdk_stack* sg,
                                      const void* proj, const float* scale, const double* mats,
                                      void* stream)
{
    fdk_status s = validate_volume(vg);
    if (s != FDK_OK) return s;
    return fdk_backproject_slab(vg, 0, vg->nz, vol, sg, proj, scale, mats, stream);
}

extern "C" fdk_status fdk_forwardproject(const fdk_volume* vg, const float* vol,
                                         const fdk_stack* sg, float* proj, const double* mats,
                                         void* stream)
{
    std::vector<IndexMatrix> M;
    fdk_status s = common_checks(vg, sg, false, mats, &M);
    if (s != FDK_OK) return s;
    if (!vol) return fail(FDK_E_INVALID, "volume pointer is NULL");
    if (!proj) return fail(FDK_E_INVALID, "projection pointer is NULL");
    FpPlan plan;
    std::vector<int32_t> lanes;
    s = make_fp_plan(*vg, *sg, M, lanes, plan);
    if (s != FDK_OK) return s;
    bool any_swap = false;
    for (int32_t f : lanes) any_swap = any_swap || (f & 1);
    const size_t mbytes = (size_t)sg->np * 12 * sizeof(double);
    const size_t vbytes = (size_t)vg->nx * vg->ny * vg->nz * sizeof(float);
    void* d_world = nullptr;
    void* d_index = nullptr;
    void* d_lanes = nullptr;
    void* d_volT = nullptr;
    s = upload_async(mats, mbytes, stream, &d_world);
    if (s == FDK_OK) s = upload_async(lanes.data(), lanes.size() * sizeof(int32_t), stream, &d_lanes);
    if (s == FDK_OK) s = device_alloc_async(mbytes, stream, &d_index);
    if (s == FDK_OK && any_swap) s = device_alloc_async(vbytes, stream, &d_volT);
    if (s == FDK_OK) {
        FpLaunch a;
        a.vol = vol;
        a.volT = (float*)d_volT;
        a.lanes = (const int*)d_lanes;
        a.proj = proj;
        a.mats_world = (const double*)d_world;
        a.mats_index = (double*)d_index;
        a.nx = vg->nx; a.ny = vg->ny; a.nz = vg->nz;
        a.np = sg->np; a.nh = sg->nh; a.nw = sg->nw;
        a.dx = vg->dx; a.dy = vg->dy; a.dz = vg->dz;
        fill_grid(*vg, a.ox, a.oy, a.oz);
        s = launch_forwardproject(a, plan, stream);
    }
    fdk_status s2 = FDK_OK;
    for (void* d : {d_volT, d_index, d_lanes, d_world})
        if (d) {
            fdk_status e = device_free_async(d, stream);
            if (s2 == FDK_OK) s2 = e;
        }
    return s != FDK_OK ? s : s2;
}

extern "C" fdk_status fdk_filter(const fdk_stack* sg, const float* raw, int32_t out_dtype,
                                 void* out, float* out_scale, double du, double dv, double sod,
                                 double sdd, double u_off, double v_off, double arc,
                                 int32_t np_total, void* stream)
{
    fdk_status s = validate_stack(sg, false);
    if (s != FDK_OK) return s;
    if (!raw || !out) return fail(FDK_E_INVALID, "raw/out pointer is NULL");
    if (out_dtype != FDK_F32 && out_dtype != FDK_F16)
        return fail(FDK_E_INVALID, "out_dtype must be FDK_F32 or FDK_F16");
    if (out_dtype == FDK_F16 && !out_scale)
        return fail(FDK_E_INVALID, "binary16 output needs a per-view scale array");
    if (out_dtype == FDK_F32 && out_scale)
        return fail(FDK_E_INVALID, "a scale array is only written with binary16 output");
    if ((const void*)raw == out) return fail(FDK_E_INVALID, "raw and out must not overlap");
    if (!(du > 0) || !(dv > 0) || !(sod > 0) || !(sdd > 0) || !std::isfinite(du) ||
        !std::isfinite(dv) || !std::isfinite(sod) || !std::isfinite(sdd) ||
        !std::isfinite(u_off) || !std::isfinite(v_off) || !std::isfinite(arc))
        return fail(FDK_E_INVALID, "pitches and distances must be positive and finite");
    if (np_total <= 0) return fail(FDK_E_INVALID, "np_total must be positive");
    if (sg->nw > 65536) return fail(FDK_E_UNSUPPORTED, "rows longer than 65536 pixels");
    FilterLaunch a;
    a.raw = raw;
    a.out = out_dtype == FDK_F32 ? (float*)out : nullptr;
    a.out16 = out_dtype == FDK_F16 ? (uint16_t*)out : nullptr;
    a.scale = out_scale;
    a.np = sg->np; a.nh = sg->nh; a.nw = sg->nw;
    a.du = du; a.dv = dv; a.sod = sod; a.sdd = sdd; a.u_off = u_off; a.v_off = v_off;
    a.arc = arc;
    a.np_total = np_total;
    return launch_filter(a, stream);
}

extern "C" fdk_status fdk_quantize_f16(int32_t np, int32_t nh, int32_t nw, const float* in,
                                       uint16_t* out, float* scale, void* stream)
{
    if (np <= 0 || nh <= 0 || nw <= 0) return fail(FDK_E_INVALID, "sizes must be positive");
    if (!in || !out || !scale) return fail(FDK_E_INVALID, "in/out/scale pointer is NULL");
    if ((double)np * nh * nw > 9.0e15 / 4) return fail(FDK_E_INVALID, "stack size overflows");
    if (np > 65535) return fail(FDK_E_UNSUPPORTED, "more than 65535 views in one call");
    return launch_quantize_f16(np, (int64_t)nh * nw, in, out, scale, stream);
}

extern "C" fdk_status fdk_phantom_project(const double* ell, int32_t n_ell, const fdk_stack* sg,
                                          float* proj, double arc, double theta0, double sod,
                                          double sdd, double du, double dv, double u_off,
                                          double v_off, int32_t view_begin, int32_t np_total,
                                          void* stream)
{
    fdk_status s = validate_stack(sg, false);
    if (s != FDK_OK) return s;
    if (!proj) return fail(FDK_E_INVALID, "projection pointer is NULL");
    if (n_ell < 0 || (n_ell > 0 && !ell)) return fail(FDK_E_INVALID, "ellipsoid table is NULL");
    if (n_ell > 4096) return fail(FDK_E_UNSUPPORTED, "more than 4096 ellipsoids");
    if (!(du > 0) || !(dv > 0) || !(sod > 0) || !(sdd > 0) || !std::isfinite(arc) ||
        !std::isfinite(theta0) || !std::isfinite(u_off) || !std::isfinite(v_off))
        return fail(FDK_E_INVALID, "pitches and distances must be positive and finite");
    if (np_total <= 0 || view_begin < 0 || (int64_t)view_begin + sg->np > np_total)
        return fail(FDK_E_INVALID, "views outside [0, np_total)");
    for (int64_t q = 0; q < (int64_t)n_ell * 16; ++q)
        if (!std::isfinite(ell[q])) return fail(FDK_E_INVALID, "ellipsoid entries must be finite");
    for (int32_t e = 0; e < n_ell; ++e)
        if (!(ell[16 * e + 3] > 0 && ell[16 * e + 4] > 0 && ell[16 * e + 5] > 0))
            return fail(FDK_E_INVALID, "ellipsoid semi-axes must be positive");
    if (sg->np > 65535) return fail(FDK_E_UNSUPPORTED, "more than 65535 views in one call");
    if (n_ell == 0) return FDK_OK;
    // unit-sphere frame of each ellipsoid: T = diag(1/axes) R^T (rows of T)
    std::vector<double> tab((size_t)n_ell * 16, 0.0);
    for (int32_t e = 0; e < n_ell; ++e) {
        const double* E = ell + 16 * (size_t)e;
        double* t = tab.data() + 16 * (size_t)e;
        t[0] = E[0]; t[1] = E[1]; t[2] = E[2];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) t[3 + 3 * i + j] = E[6 + 3 * j + i] / E[3 + i];
        t[12] = E[15];
    }
    void* d_ell = nullptr;
    s = upload_async(tab.data(), tab.size() * sizeof(double), stream, &d_ell);
    if (s != FDK_OK) return s;
    PhantomLaunch a;
    a.ell = (const double*)d_ell;
    a.n_ell = n_ell;
    a.proj = proj;
    a.np = sg->np; a.nh = sg->nh; a.nw = sg->nw;
    a.view_begin = view_begin;
    a.np_total = np_total;
    a.arc = arc; a.theta0 = theta0; a.sod = sod; a.sdd = sdd; a.du = du; a.dv = dv;
    a.u_off = u_off; a.v_off = v_off;
    s = launch_phantom(a, stream);
    fdk_status s2 = device_free_async(d_ell, stream);
    return s != FDK_OK ? s : s2;
}

// ---------------------------------------------------------------- learned row filter

#include "fdk_learn.h"

namespace {

fdk_status conv_checks(int32_t cin, int32_t cout, int32_t rows, int32_t len)
{
    if (cin <= 0 || cout <= 0 || rows <= 0 || len <= 0)
        return fail(FDK_E_INVALID, "conv1d sizes must be positive");
    if ((cin != 1 && cin != 32) || (cout != 1 && cout != 32))
        return fail(FDK_E_UNSUPPORTED, "conv1d channels must be 1 or 32");
    if ((double)rows * 32.0 * len >= 4.0e18 / 4) return fail(FDK_E_INVALID, "tensor size overflows");
    return FDK_OK;
}

}  // namespace

extern "C" fdk_status fdk_cosine_weight(const fdk_stack* sg, const float* raw, float* out,
                                        double du, double dv, double sdd, double u_off,
                                        double v_off, void* stream)
{
    fdk_status s = validate_stack(sg, false);
    if (s != FDK_OK) return s;
    if (!raw || !out) return fail(FDK_E_INVALID, "raw/out pointer is NULL");
    if (!(du > 0) || !(dv > 0) || !(sdd > 0) || !std::isfinite(du) || !std::isfinite(dv) ||
        !std::isfinite(sdd) || !std::isfinite(u_off) || !std::isfinite(v_off))
        return fail(FDK_E_INVALID, "pitches and distances must be positive and finite");
    FilterLaunch a;
    a.raw = raw;
    a.out = out;
    a.out16 = nullptr;
    a.scale = nullptr;
    a.np = sg->np; a.nh = sg->nh; a.nw = sg->nw;
    a.du = du; a.dv = dv; a.sod = sdd; a.sdd = sdd; a.u_off = u_off; a.v_off = v_off;
    a.arc = 1.0;
    a.np_total = 1;
    return launch_cosine_weight(a, stream);
}

extern "C" fdk_status fdk_conv1d_forward(int32_t cin, int32_t cout, int32_t rows, int32_t len,
                                         const float* in, const float* w, const float* bias,
                                         const float* mask, const float* add, float alpha,
                                         int32_t relu, float* out, void* stream)
{
    fdk_status s = conv_checks(cin, cout, rows, len);
    if (s != FDK_OK) return s;
    if (!in || !w || !out) return fail(FDK_E_INVALID, "in/w/out pointer is NULL");
    if (in == out) return fail(FDK_E_INVALID, "in and out must not overlap");
    if (!std::isfinite(alpha)) return fail(FDK_E_INVALID, "alpha must be finite");
    return launch_conv1d_forward(cin, cout, rows, len, in, w, bias, mask, add, alpha,
                                 relu ? 1 : 0, out, stream);
}

extern "C" fdk_status fdk_conv1d_backward_data(int32_t cin, int32_t cout, int32_t rows,
                                               int32_t len, const float* gout, const float* w,
                                               const float* mask, float* gin, void* stream)
{
    fdk_status s = conv_checks(cin, cout, rows, len);
    if (s != FDK_OK) return s;
    if (!gout || !w || !gin) return fail(FDK_E_INVALID, "gout/w/gin pointer is NULL");
    if (gout == gin) return fail(FDK_E_INVALID, "gout and gin must not overlap");
    return launch_conv1d_backward_data(cin, cout, rows, len, gout, w, mask, gin, stream);
}

extern "C" fdk_status fdk_conv1d_backward_weight(int32_t cin, int32_t cout, int32_t rows,
                                                 int32_t len, const float* in, const float* gout,
                                                 float* gw, float* gb, void* stream)
{
    fdk_status s = conv_checks(cin, cout, rows, len);
    if (s != FDK_OK) return s;
    if (!in || !gout || !gw) return fail(FDK_E_INVALID, "in/gout/gw pointer is NULL");
    return launch_conv1d_backward_weight(cin, cout, rows, len, in, gout, gw, gb, stream);
}

extern "C" fdk_status fdk_sqerr(int64_t n, const float* a, const float* b, float* grad,
                                float grad_scale, float* loss, void* stream)
{
    if (n <= 0) return fail(FDK_E_INVALID, "n must be positive");
    if (!a || !b || !loss) return fail(FDK_E_INVALID, "a/b/loss pointer is NULL");
    if (!std::isfinite(grad_scale)) return fail(FDK_E_INVALID, "grad_scale must be finite");
    return launch_sqerr(n, a, b, grad, grad_scale, loss, stream);
}

extern "C" fdk_status fdk_adam(int32_t n, float* p, const float* g, float* m, float* v, float lr,
                               float beta1, float beta2, float eps, int32_t t, void* stream)
{
    if (n <= 0) return fail(FDK_E_INVALID, "n must be positive");
    if (!p || !g || !m || !v) return fail(FDK_E_INVALID, "p/g/m/v pointer is NULL");
    if (t < 1) return fail(FDK_E_INVALID, "step t starts at 1");
    if (!(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f) ||
        !std::isfinite(lr))
        return fail(FDK_E_INVALID, "Adam needs 0 <= beta < 1, eps > 0, finite lr");
    return launch_adam(n, p, g, m, v, lr, beta1, beta2, eps, t, stream);
}

// ---------------------------------------------------------------- back-projection variants

#include "fdk_ablation.h"

extern "C" fdk_status fdk_backproject_variant(int32_t variant, int32_t nb, const fdk_volume* vg,
                                              float* vol, const fdk_stack* sg, const float* proj,
                                              const double* mats, void* stream)
{
    std::vector<IndexMatrix> M;
    fdk_status s = common_checks(vg, sg, false, mats, &M);
    if (s != FDK_OK) return s;
    if (!vol || !proj) return fail(FDK_E_INVALID, "volume/projection pointer is NULL");
    if (nb < 1) return fail(FDK_E_INVALID, "nb must be at least 1");
    if (variant != FDK_VARIANT_PRODUCTION && variant != FDK_VARIANT_GLOBAL_TAPS &&
        variant != FDK_VARIANT_LISTING1 && variant != FDK_VARIANT_SYMMETRY &&
        variant != FDK_VARIANT_SUBLINE)
        return fail(FDK_E_INVALID, "unknown back-projection variant");
    const int32_t batch = nb < sg->np ? nb : sg->np;
    if (variant == FDK_VARIANT_SYMMETRY || variant == FDK_VARIANT_SUBLINE) {
        const bool sym = variant == FDK_VARIANT_SYMMETRY;
        if (sym && !bp_geometry_symmetric(*vg, *sg, M))
            return fail(FDK_E_GEOMETRY,
                        "the symmetric variant needs v(nz-1-k) = nh-1-v(k) in every view (detector "
                        "centre row on the orbit plane, volume centred on it)");
        if ((int64_t)sg->nh * sg->nw * 4 >= (1ll << 31))
            return fail(FDK_E_UNSUPPORTED, "one view larger than 2 GiB");
        BpPlan plan;
        s = sym ? make_bp_plan_sym(*vg, *sg, M, plan) : make_bp_plan_subline(*vg, *sg, M, plan);
        if (s != FDK_OK) return s;
        const size_t mbytes = (size_t)sg->np * 12 * sizeof(double);
        void* d_world = nullptr;
        void* d_index = nullptr;
        s = upload_async(mats, mbytes, stream, &d_world);
        if (s == FDK_OK) s = device_alloc_async(mbytes, stream, &d_index);
        if (s == FDK_OK) {
            BpLaunch a;
            a.proj = proj;
            a.scale = nullptr;
            a.mats_world = (const double*)d_world;
            a.mats_index = (double*)d_index;
            a.vol = vol;
            a.nx = vg->nx; a.ny = vg->ny; a.nz = vg->nz;
            a.np = sg->np; a.nh = sg->nh; a.nw = sg->nw;
            a.k_begin = 0;
            a.k_end = vg->nz;
            a.dx = vg->dx; a.dy = vg->dy; a.dz = vg->dz;
            fill_grid(*vg, a.ox, a.oy, a.oz);
            a.f16 = 0;
            s = sym ? launch_backproject_sym(a, plan, stream)
                    : launch_backproject_subline(a, plan, stream);
        }
        fdk_status s2 = FDK_OK;
        for (void* d : {d_index, d_world})
            if (d) {
                fdk_status e = device_free_async(d, stream);
                if (s2 == FDK_OK) s2 = e;
            }
        return s != FDK_OK ? s : s2;
    }
    if (variant == FDK_VARIANT_GLOBAL_TAPS)
        return backproject_slab(vg, 0, vg->nz, vol, sg, proj, nullptr, mats, stream, true);
    if (variant == FDK_VARIANT_PRODUCTION) {
        const size_t view = (size_t)sg->nh * sg->nw;
        for (int32_t s0 = 0; s0 < sg->np; s0 += batch) {
            fdk_stack sub = *sg;
            sub.np = s0 + batch < sg->np ? batch : sg->np - s0;
            s = fdk_backproject(vg, vol, &sub, proj + (size_t)s0 * view, nullptr,
                                mats + 12 * (size_t)s0, stream);
            if (s != FDK_OK) return s;
        }
        return FDK_OK;
    }
    const size_t mbytes = (size_t)sg->np * 12 * sizeof(double);
    void* d_world = nullptr;
    void* d_index = nullptr;
    s = upload_async(mats, mbytes, stream, &d_world);
    if (s == FDK_OK) s = device_alloc_async(mbytes, stream, &d_index);
    if (s == FDK_OK) {
        double ox, oy, oz;
        fill_grid(*vg, ox, oy, oz);
        s = launch_compose((const double*)d_world, (double*)d_index, sg->np, vg->dx, vg->dy, vg->dz,
                           ox, oy, oz, stream);
    }
    if (s == FDK_OK)
        s = launch_backproject_variant(variant, batch, proj, (const double*)d_index, vol, vg->nx,
                                       vg->ny, vg->nz, sg->np, sg->nh, sg->nw, stream);
    fdk_status s2 = FDK_OK;
    for (void* d : {d_index, d_world})
        if (d) {
            fdk_status e = device_free_async(d, stream);
            if (s2 == FDK_OK) s2 = e;
        }
    return s != FDK_OK ? s : s2;
}
