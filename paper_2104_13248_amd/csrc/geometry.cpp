// Host-side geometry: validation, FP64 matrix composition, the circular-orbit
// matrix helper and the footprint-driven launch plan of the back-projector.
// No HIP call is made in this file.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <list>
#include <mutex>
#include <sstream>
#include <unordered_map>

#include "internal.h"

namespace fdk {

void compose_index_matrices(const fdk_volume& vg, int32_t np, const double* mats,
                            std::vector<IndexMatrix>& out)
{
    // Voxel (i,j,k) centre = (dx i + ox, dy j + oy, dz k + oz).
    const double ox = vg.cx - 0.5 * (vg.nx - 1) * vg.dx;
    const double oy = vg.cy - 0.5 * (vg.ny - 1) * vg.dy;
    const double oz = vg.cz - 0.5 * (vg.nz - 1) * vg.dz;
    out.resize(np);
    for (int32_t s = 0; s < np; ++s) {
        const double* P = mats + 12 * (size_t)s;
        double* M = out[s].m;
        for (int r = 0; r < 3; ++r) {
            const double* p = P + 4 * r;
            M[4 * r + 0] = p[0] * vg.dx;
            M[4 * r + 1] = p[1] * vg.dy;
            M[4 * r + 2] = p[2] * vg.dz;
            M[4 * r + 3] = p[0] * ox + p[1] * oy + p[2] * oz + p[3];
        }
    }
}

fdk_status validate_volume(const fdk_volume* vg)
{
    if (!vg) return fail(FDK_E_INVALID, "volume geometry is NULL");
    if (vg->nx <= 0 || vg->ny <= 0 || vg->nz <= 0)
        return fail(FDK_E_INVALID, "volume dimensions must be positive");
    if (!(vg->dx > 0 && vg->dy > 0 && vg->dz > 0) || !std::isfinite(vg->dx) ||
        !std::isfinite(vg->dy) || !std::isfinite(vg->dz))
        return fail(FDK_E_INVALID, "voxel pitch must be positive and finite");
    if (!std::isfinite(vg->cx) || !std::isfinite(vg->cy) || !std::isfinite(vg->cz))
        return fail(FDK_E_INVALID, "volume centre must be finite");
    const double n = (double)vg->nx * vg->ny * vg->nz;
    if (n > 9.0e15 / 4) return fail(FDK_E_INVALID, "volume size overflows");
    return FDK_OK;
}

fdk_status validate_stack(const fdk_stack* sg, bool allow_f16)
{
    if (!sg) return fail(FDK_E_INVALID, "stack geometry is NULL");
    if (sg->np <= 0 || sg->nh <= 0 || sg->nw <= 0)
        return fail(FDK_E_INVALID, "stack dimensions must be positive");
    if (sg->dtype != FDK_F32 && sg->dtype != FDK_F16)
        return fail(FDK_E_INVALID, "unknown stack dtype");
    if (sg->dtype == FDK_F16 && !allow_f16)
        return fail(FDK_E_UNSUPPORTED, "binary16 stacks are accepted by the back-projector only");
    if ((double)sg->np * sg->nh * sg->nw > 9.0e15 / 4)
        return fail(FDK_E_INVALID, "stack size overflows");
    if (sg->nh >= (1 << 24) || sg->nw >= (1 << 24))
        return fail(FDK_E_UNSUPPORTED, "detector larger than 2^24 pixels per axis");
    return FDK_OK;
}

fdk_status validate_geometry(const fdk_volume& vg, const fdk_stack& sg, const double* mats,
                             std::vector<IndexMatrix>* composed)
{
    if (!mats) return fail(FDK_E_INVALID, "matrix array is NULL");
    for (int64_t q = 0; q < (int64_t)sg.np * 12; ++q)
        if (!std::isfinite(mats[q])) return fail(FDK_E_INVALID, "matrix entries must be finite");
    std::vector<IndexMatrix> local;
    std::vector<IndexMatrix>& M = composed ? *composed : local;
    compose_index_matrices(vg, sg.np, mats, M);
    const double ci[2] = {0.0, (double)(vg.nx - 1)};
    const double cj[2] = {0.0, (double)(vg.ny - 1)};
    for (int32_t s = 0; s < sg.np; ++s) {
        const double* m = M[s].m;
        // u w and w must not depend on k (detector V-axis parallel to the
        // rotation axis): entries (0,2) and (2,2) vanish.
        const double n0 = std::fabs(m[0]) + std::fabs(m[1]) + std::fabs(m[2]) + std::fabs(m[3]);
        const double n2 = std::fabs(m[8]) + std::fabs(m[9]) + std::fabs(m[10]) + std::fabs(m[11]);
        if (std::fabs(m[2]) > 1e-12 * n0 || std::fabs(m[10]) > 1e-12 * n2) {
            std::ostringstream os;
            os << "view " << s << ": u*w or w depends on the slice index (matrix entries (0,2)/(2,2)"
               << " not zero); the detector V-axis must be parallel to the volume z axis";
            return fail(FDK_E_GEOMETRY, os.str());
        }
        // w is affine in (i, j): positive at the four corner columns means
        // positive over the whole volume (no voxel behind the source).
        for (double i : ci)
            for (double j : cj) {
                const double w = m[8] * i + m[9] * j + m[11];
                if (!(w > 0)) {
                    std::ostringstream os;
                    os << "view " << s << ": depth w <= 0 at volume corner column (" << i << ", "
                       << j << ")";
                    return fail(FDK_E_GEOMETRY, os.str());
                }
                const double u = (m[0] * i + m[1] * j + m[3]) / w;
                const double v0 = (m[4] * i + m[5] * j + m[7]) / w;
                const double v1 = (m[4] * i + m[5] * j + m[6] * (vg.nz - 1) + m[7]) / w;
                if (!(std::fabs(u) < 4.0e6 && std::fabs(v0) < 4.0e6 && std::fabs(v1) < 4.0e6))
                    return fail(FDK_E_UNSUPPORTED,
                                "volume projects more than 4e6 pixels away from the detector");
            }
    }
    return FDK_OK;
}

// ------------------------------------------------------------------ plan

const int kPitches[] = {40, 56, 72, 88, 120, 184, 248};
const int kNumPitches = (int)(sizeof(kPitches) / sizeof(kPitches[0]));

namespace {

struct Extent {
    int cols = 0;        // max over blocks/views of floor(umax) - floor(umin) + 4
    int rows_full = 0;   // bound of the rows of a whole chunk of slices
    int rows_half = 0;   // bound of the rows of half a chunk
    int rows_p95 = 0;    // 95th percentile of the whole-chunk rows
};

// Rows a set of slices needs, as the kernel computes it (four corner columns
// of the tile at the two end slices): floor(vmax) - floor(vmin) + 4.
inline int rows_of(const double* m, const double* ii, const double* jj, const double* rw,
                   double ka, double kb)
{
    double lo = 1e300, hi = -1e300;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const double A = m[4] * ii[a] + m[5] * jj[b] + m[7];
            const double v0 = (A + m[6] * ka) * rw[2 * a + b];
            const double v1 = (A + m[6] * kb) * rw[2 * a + b];
            lo = std::min(lo, std::min(v0, v1));
            hi = std::max(hi, std::max(v0, v1));
        }
    return (int)(std::floor(hi) - std::floor(lo)) + 4;
}

// Footprints of every (xy tile, view) for a given number of slices per block,
// following the kernel's rule.  The width does not depend on the chunk.  The
// height of a set of slices is a convex function of the chunk start (max of
// affine functions minus min of affine functions), so its maximum over all
// chunks is at the first or the last chunk; the floors add at most 1 to
// floor(vmax - vmin) + 4 in between, and one more row/column covers
// host/device rounding.
Extent footprint(const fdk_volume& vg, const std::vector<IndexMatrix>& M, int kz)
{
    Extent e;
    const int ntx = (vg.nx + kTile - 1) / kTile, nty = (vg.ny + kTile - 1) / kTile;
    const int nch = (vg.nz + kz - 1) / kz;
    const double kfirst = 0.0, kmid = (double)((nch / 2) * kz), klast = (double)((nch - 1) * kz);
    std::vector<int> hist(4096, 0);
    int cols = 0, rf = 0, rh = 0;
    int64_t count = 0;
    for (size_t s = 0; s < M.size(); ++s) {
        const double* m = M[s].m;
        for (int ty = 0; ty < nty; ++ty) {
            const int j0 = ty * kTile, nj = std::min(kTile, vg.ny - j0);
            const double jj[2] = {(double)j0, (double)(j0 + nj - 1)};
            for (int tx = 0; tx < ntx; ++tx) {
                const int i0 = tx * kTile, ni = std::min(kTile, vg.nx - i0);
                const double ii[2] = {(double)i0, (double)(i0 + ni - 1)};
                double umin = 1e300, umax = -1e300, rw[4];
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        const double w = m[8] * ii[a] + m[9] * jj[b] + m[11];
                        rw[2 * a + b] = 1.0 / w;
                        const double u = (m[0] * ii[a] + m[1] * jj[b] + m[3]) / w;
                        umin = std::min(umin, u);
                        umax = std::max(umax, u);
                    }
                cols = std::max(cols, (int)(std::floor(umax) - std::floor(umin)) + 4);
                for (double k0 : {kfirst, klast}) {
                    rf = std::max(rf, rows_of(m, ii, jj, rw, k0, k0 + kz - 1));
                    rh = std::max(rh, rows_of(m, ii, jj, rw, k0, k0 + kz / 2 - 1));
                    rh = std::max(rh, rows_of(m, ii, jj, rw, k0 + kz / 2, k0 + kz - 1));
                }
                for (double k0 : {kfirst, kmid, klast}) {
                    const int r = rows_of(m, ii, jj, rw, k0, k0 + kz - 1);
                    hist[std::min(r, 4095)]++;
                    count++;
                }
            }
        }
    }
    int64_t acc = 0;
    int p95 = 0;
    for (int r = 0; r < 4096; ++r) {
        acc += hist[r];
        if (acc * 100 >= count * 95) { p95 = r; break; }
    }
    e.cols = cols + 1;
    e.rows_full = rf + 2;
    e.rows_half = rh + 2;
    e.rows_p95 = p95 + 1;
    return e;
}

uint64_t fnv1a(uint64_t h, const void* p, size_t n)
{
    const unsigned char* b = (const unsigned char*)p;
    for (size_t q = 0; q < n; ++q) {
        h ^= b[q];
        h *= 1099511628211ull;
    }
    return h;
}

std::mutex g_plan_mu;
std::list<std::pair<uint64_t, BpPlan>> g_plans;   // most recent first

// The kernels stage a window of R rows by buffer loads whose byte offsets,
// with the window's first row clamped to [-R, nh] (rows wholly outside the
// detector read as zero either way), lie within +-(nh + R) rows of the view;
// they must stay below 2^31.
bool staging_offsets_fit(const fdk_stack& sg, int rows)
{
    const int64_t rb = (int64_t)sg.nw * (sg.dtype == FDK_F16 ? 2 : 4);
    return ((int64_t)sg.nh + rows + 1) * rb < (1ll << 31);
}

int env_int(const char* name, int dflt)
{
    const char* s = std::getenv(name);
    if (!s || !*s) return dflt;
    return std::atoi(s);
}

}  // namespace

fdk_status make_bp_plan(const fdk_volume& vg, const fdk_stack& sg,
                        const std::vector<IndexMatrix>& M, BpPlan& plan)
{
    const int kz_force = env_int("FDK_BP_KZ", 0);
    const int lds_budget = env_int("FDK_BP_LDS_BUDGET", 32 * 1024);
    const int tile_bytes = env_int("FDK_BP_TILE_BYTES", 39 * 1024);
    const int direct_force = env_int("FDK_BP_DIRECT", 0);
    uint64_t h = 1469598103934665603ull;
    h = fnv1a(h, &vg.nx, sizeof(int32_t) * 3);
    h = fnv1a(h, &sg.np, sizeof(int32_t) * 4);   // np, nh, nw, dtype
    h = fnv1a(h, &kz_force, sizeof(int));
    h = fnv1a(h, &lds_budget, sizeof(int));
    h = fnv1a(h, &tile_bytes, sizeof(int));
    h = fnv1a(h, &direct_force, sizeof(int));
    h = fnv1a(h, M.data(), M.size() * sizeof(IndexMatrix));
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        for (auto it = g_plans.begin(); it != g_plans.end(); ++it)
            if (it->first == h) {
                plan = it->second;
                g_plans.splice(g_plans.begin(), g_plans, it);
                return FDK_OK;
            }
    }
    // LDS rows: enough for every half-chunk and for 95% of the whole-chunk
    // footprints (taller ones are processed per half-chunk).  Largest slice
    // count whose tile fits the budget; otherwise the smallest tile.
    const int cands[3] = {32, 16, 8};
    const int table_bytes = kViewBatch * kViewRec * 4;
    BpPlan best;
    bool found = false;
    int64_t best_bytes = 0;
    for (int q = 0; q < 3; ++q) {
        const int kz = cands[q];
        if (kz_force && kz != kz_force) continue;
        Extent e = footprint(vg, M, kz);
        int pitch = 0;
        for (int p = 0; p < kNumPitches; ++p)
            if (kPitches[p] >= e.cols) { pitch = kPitches[p]; break; }
        if (!pitch) continue;
        const int rows = std::max(e.rows_half, std::min(e.rows_p95, e.rows_full));
        const int64_t bytes = (int64_t)rows * pitch * 4 + table_bytes;
        if (bytes > 150 * 1024) continue;
        if (!found || (best_bytes > lds_budget && bytes < best_bytes)) {
            best.kz = kz;
            best.pitch = pitch;
            best.rows = rows;
            best.rows_full = e.rows_full;
            best.cols = e.cols;
            best.lds_bytes = bytes;
            best_bytes = bytes;
            found = true;
        }
        if (found && best_bytes <= lds_budget) break;
    }
    if (!found || direct_force) {
        // Strong magnification (a 16 x 16 x 8 block's footprint wider than the
        // widest LDS pitch, or taller than 150 KiB of rows): the direct
        // organisation, same blocks and hoisting, taps read from memory.
        best = BpPlan();
        best.kz = kz_force ? kz_force : 32;
        best.direct = true;
    }
    // Rows beyond that cost no occupancy while four blocks (the register
    // limit: four waves per SIMD) still share a CU's 160 KiB of LDS: take as
    // many as fit, so that fewer footprints are staged per half-chunk.  A
    // binary16 tile holds its even- and odd-offset pair words in two regions
    // of rows x PITCH/2 words; rows = 4 (mod 8) puts the second region 16
    // banks (mod 32) after the first for every pitch, so lanes reading
    // neighbouring even and odd pairs do not meet in one bank (an offset of
    // 0 mod 32 measured 4-5% slower).
    if (!best.direct) {
        const int fit = (tile_bytes - table_bytes) / (best.pitch * 4);
        int r = std::min(fit, best.rows_full);
        if (sg.dtype == FDK_F16) {
            const int up = r + (12 - r % 8) % 8;   // smallest >= r that is 4 mod 8
            r = up <= fit ? up : up - 8;
        }
        if (r > best.rows) {
            best.rows = r;
            best.lds_bytes = (int64_t)best.rows * best.pitch * 4 + table_bytes;
        }
        if (!staging_offsets_fit(sg, best.rows)) {
            best = BpPlan();
            best.kz = kz_force ? kz_force : 32;
            best.direct = true;
        }
    }
    best.ntx = (vg.nx + kTile - 1) / kTile;
    best.nty = (vg.ny + kTile - 1) / kTile;
    best.ntiles_pad = ((best.ntx * best.nty + 7) / 8) * 8;
    best.nchunks = (vg.nz + best.kz - 1) / best.kz;
    best.blocks = (int64_t)best.ntiles_pad * best.nchunks;
    plan = best;
    std::lock_guard<std::mutex> lk(g_plan_mu);
    g_plans.emplace_front(h, best);
    if (g_plans.size() > 32) g_plans.pop_back();
    return FDK_OK;
}

// Plan of the symmetric variant: a block owns kz / 2 direct slices and their
// mirrors, and per view stages the direct window and its mirror image in two
// LDS regions of rr rows; two regions must hold every half-chunk window (a
// taller one is staged alone over the whole tile).  Budget 38 KiB (four
// blocks per CU).
fdk_status make_bp_plan_sym(const fdk_volume& vg, const fdk_stack& sg,
                            const std::vector<IndexMatrix>& M, BpPlan& plan)
{
    const int kz_force = env_int("FDK_BP_KZ", 0);
    const int lds_budget = env_int("FDK_BP_SYM_LDS_BUDGET", 38 * 1024);
    const int cands[3] = {32, 16, 8};
    const int table_bytes = kViewBatch * kViewRec * 4;
    BpPlan best;
    bool found = false;
    int64_t best_bytes = 0;
    for (int q = 0; q < 3; ++q) {
        const int kz = cands[q];
        if (kz_force && kz != kz_force) continue;
        Extent e = footprint(vg, M, kz);
        int pitch = 0;
        for (int p = 0; p < kNumPitches; ++p)
            if (kPitches[p] >= e.cols) { pitch = kPitches[p]; break; }
        if (!pitch) continue;
        const int rr_budget = (lds_budget - table_bytes) / (2 * pitch * 4);
        const int rr = std::max((e.rows_half + 1) / 2, std::min(rr_budget, e.rows_half));
        const int64_t bytes = (int64_t)2 * rr * pitch * 4 + table_bytes;
        if (bytes > 150 * 1024) continue;
        if (!found || (best_bytes > lds_budget && bytes < best_bytes)) {
            best.kz = kz;
            best.pitch = pitch;
            best.rows = 2 * rr;
            best.rows_full = e.rows_full;
            best.cols = e.cols;
            best.lds_bytes = bytes;
            best_bytes = bytes;
            found = true;
        }
        if (found && best_bytes <= lds_budget) break;
    }
    if (!found)
        return fail(FDK_E_UNSUPPORTED,
                    "projection footprint of a 16x16x8 voxel block does not fit in LDS "
                    "(magnification too large for the detector pitch)");
    if (!staging_offsets_fit(sg, best.rows))
        return fail(FDK_E_UNSUPPORTED, "views too large for the symmetric variant's staging offsets");
    best.ntx = (vg.nx + kTile - 1) / kTile;
    best.nty = (vg.ny + kTile - 1) / kTile;
    best.ntiles_pad = ((best.ntx * best.nty + 7) / 8) * 8;
    best.nchunks = ((vg.nz + 1) / 2 + best.kz / 2 - 1) / (best.kz / 2);
    best.blocks = (int64_t)best.ntiles_pad * best.nchunks;
    plan = best;
    return FDK_OK;
}

// Plan of the sub-line variant (Section 3.1.5): the window holds every
// whole-chunk footprint (no per-half staging), and each of the 256 threads
// owns a line of line_rows blended values in LDS.  A column's KZ slices reach
// floor(v_max) - floor(v_min) + 2 <= ceil(|dv| (KZ - 1)) + 3 rows, with |dv| =
// |m6| / w largest where w is smallest (at a corner column of the volume, w
// being affine in i and j); one more row absorbs FP32 rounding.  Largest
// slice count within the budget (76 KiB: two blocks per CU).
fdk_status make_bp_plan_subline(const fdk_volume& vg, const fdk_stack& sg,
                                const std::vector<IndexMatrix>& M, BpPlan& plan)
{
    const int kz_force = env_int("FDK_BP_KZ", 0);
    const int lds_budget = env_int("FDK_BP_SUBLINE_LDS_BUDGET", 76 * 1024);
    double dv_max = 0.0;
    for (const IndexMatrix& X : M) {
        const double* m = X.m;
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                const double w = m[8] * (a ? vg.nx - 1 : 0) + m[9] * (b ? vg.ny - 1 : 0) + m[11];
                dv_max = std::max(dv_max, std::fabs(m[6]) / w);
            }
    }
    const int cands[3] = {32, 16, 8};
    const int table_bytes = kViewBatch * kViewRec * 4;
    for (int q = 0; q < 3; ++q) {
        const int kz = cands[q];
        if (kz_force && kz != kz_force) continue;
        Extent e = footprint(vg, M, kz);
        int pitch = 0;
        for (int p = 0; p < kNumPitches; ++p)
            if (kPitches[p] >= e.cols) { pitch = kPitches[p]; break; }
        if (!pitch) continue;
        const int line_rows = (int)std::ceil(dv_max * (kz - 1)) + 4;
        const int64_t bytes = (int64_t)e.rows_full * pitch * 4 + (int64_t)line_rows * kThreads * 4 +
                              table_bytes;
        if (bytes > lds_budget && !(kz_force && bytes <= 150 * 1024)) continue;
        if (!staging_offsets_fit(sg, e.rows_full))
            return fail(FDK_E_UNSUPPORTED, "views too large for the sub-line variant's staging offsets");
        plan.kz = kz;
        plan.pitch = pitch;
        plan.rows = e.rows_full;
        plan.rows_full = e.rows_full;
        plan.cols = e.cols;
        plan.line_rows = line_rows;
        plan.lds_bytes = bytes;
        plan.ntx = (vg.nx + kTile - 1) / kTile;
        plan.nty = (vg.ny + kTile - 1) / kTile;
        plan.ntiles_pad = ((plan.ntx * plan.nty + 7) / 8) * 8;
        plan.nchunks = (vg.nz + kz - 1) / kz;
        plan.blocks = (int64_t)plan.ntiles_pad * plan.nchunks;
        return FDK_OK;
    }
    return fail(FDK_E_UNSUPPORTED,
                "the sub-line variant's window and lines do not fit in LDS for this geometry");
}

// v(i, j, k) + v(i, j, nz - 1 - k) = nh - 1 for all i, j, k iff, with
// v w = m4 i + m5 j + m6 k + m7 and w = m8 i + m9 j + m11 (m10 = 0):
// 2 m4 = (nh - 1) m8, 2 m5 = (nh - 1) m9, 2 m7 + (nz - 1) m6 = (nh - 1) m11.
bool bp_geometry_symmetric(const fdk_volume& vg, const fdk_stack& sg,
                           const std::vector<IndexMatrix>& M)
{
    const double h = (double)(sg.nh - 1), z = (double)(vg.nz - 1);
    auto close = [](double a, double b, double scale) {
        return std::fabs(a - b) <= 1e-10 * scale;
    };
    for (size_t s = 0; s < M.size(); ++s) {
        const double* m = M[s].m;
        const double scale = std::fabs(m[4]) + std::fabs(m[5]) + std::fabs(m[6]) * (z + 1.0) +
                             std::fabs(m[7]) + h * (std::fabs(m[8]) + std::fabs(m[9]) + std::fabs(m[11]));
        if (!close(2.0 * m[4], h * m[8], scale) || !close(2.0 * m[5], h * m[9], scale) ||
            !close(2.0 * m[7] + z * m[6], h * m[11], scale))
            return false;
    }
    return true;
}

void fp_view_lanes(const fdk_volume& vg, const std::vector<IndexMatrix>& M,
                   std::vector<int32_t>& lanes)
{
    const double ic = 0.5 * (vg.nx - 1), jc = 0.5 * (vg.ny - 1);
    lanes.resize(M.size());
    for (size_t s = 0; s < M.size(); ++s) {
        const double* m = M[s].m;
        const double wc = m[8] * ic + m[9] * jc + m[11];
        const double uc = (m[0] * ic + m[1] * jc + m[3]) / wc;
        const double dui = (m[0] - uc * m[8]) / wc, duj = (m[1] - uc * m[9]) / wc;
        const int sw = std::fabs(duj) > std::fabs(dui) ? 1 : 0;
        const double ua = sw ? m[1] : m[0], ub = sw ? m[0] : m[1];
        const double wa = sw ? m[9] : m[8], wb = sw ? m[8] : m[9];
        const int na = sw ? vg.ny : vg.nx, nb = sw ? vg.nx : vg.ny;
        // u = (ua a + U(b)) / (wa a + W(b)): du/da = (ua W(b) - wa U(b)) / w^2
        auto N = [&](double b) { return ua * (wb * b + m[11]) - wa * (ub * b + m[3]); };
        const double n0 = N(0.0), n1 = N((double)(nb - 1));
        double wmax = 0.0;
        for (double a : {0.0, (double)(na - 1)})
            for (double b : {0.0, (double)(nb - 1)}) wmax = std::max(wmax, wa * a + wb * b + m[11]);
        int64_t S = na;   // one voxel per pass: always free of collisions
        if (n0 != 0.0 && n1 != 0.0 && (n0 > 0.0) == (n1 > 0.0)) {
            const double slope = std::min(std::fabs(n0), std::fabs(n1)) / (wmax * wmax);
            const double need = std::ceil(2.0001 / slope);
            if (need < (double)na) S = std::max<int64_t>(1, (int64_t)need);
        }
        lanes[s] = (int32_t)((S << 1) | sw);
    }
}

}  // namespace fdk

// ------------------------------------------------------------------ C ABI

extern "C" fdk_status fdk_circular_matrices(int32_t np, double arc, double theta0, double sod,
                                            double sdd, int32_t nh, int32_t nw, double du,
                                            double dv, double u_off, double v_off,
                                            double* mats_out)
{
    using namespace fdk;
    if (!mats_out) return fail(FDK_E_INVALID, "mats_out is NULL");
    if (np <= 0 || nh <= 0 || nw <= 0) return fail(FDK_E_INVALID, "sizes must be positive");
    if (!(sod > 0) || !(sdd > 0) || !(du > 0) || !(dv > 0) || !std::isfinite(arc) ||
        !std::isfinite(theta0) || !std::isfinite(u_off) || !std::isfinite(v_off) ||
        !std::isfinite(sod) || !std::isfinite(sdd))
        return fail(FDK_E_INVALID, "distances and pitches must be positive and finite");
    // Pinhole camera of a flat detector: project onto the plane at distance
    // sdd from the source along the central ray, in units of pixels, and
    // divide the homogeneous coordinate by sod so that w = 1 on the axis.
    const double mag = sdd / sod;
    const double cu = 0.5 * (nw - 1) + u_off, cv = 0.5 * (nh - 1) + v_off;
    for (int32_t s = 0; s < np; ++s) {
        const double th = theta0 + arc * (double)s / (double)np;
        const double c = std::cos(th), sn = std::sin(th);
        double* m = mats_out + 12 * (size_t)s;
        // depth row: w = (sod - x cos - y sin) / sod
        m[8] = -c / sod;
        m[9] = -sn / sod;
        m[10] = 0.0;
        m[11] = 1.0;
        // u w = mag (-x sin + y cos) / du + cu w
        m[0] = -mag * sn / du + cu * m[8];
        m[1] = mag * c / du + cu * m[9];
        m[2] = 0.0;
        m[3] = cu;
        // v w = mag z / dv + cv w
        m[4] = cv * m[8];
        m[5] = cv * m[9];
        m[6] = mag / dv;
        m[7] = cv;
    }
    return FDK_OK;
}
