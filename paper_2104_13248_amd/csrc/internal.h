// Internal declarations shared by the host library and the kernel launchers.
// Not part of the ABI (the ABI is include/fdk.h).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "fdk.h"

namespace fdk {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
fdk_status fail(fdk_status code, const std::string& msg);

// ---------------------------------------------------------------- geometry
// Index-space matrix of one view: maps (i, j, k, 1) to (u w, v w, w).
struct IndexMatrix {
    double m[12];
};

// Compose world-mm matrices with the voxel grid (FP64): M = P V, where V maps
// voxel indices to the world position of the voxel centre.
void compose_index_matrices(const fdk_volume& vg, int32_t np, const double* mats,
                            std::vector<IndexMatrix>& out);

// Host-side checks shared by every volume<->stack operator.  Returns FDK_OK or
// the error (with the message set).  Makes no HIP call.
fdk_status validate_volume(const fdk_volume* vg);
fdk_status validate_stack(const fdk_stack* sg, bool allow_f16);
fdk_status validate_geometry(const fdk_volume& vg, const fdk_stack& sg, const double* mats,
                             std::vector<IndexMatrix>* composed);

// ---------------------------------------------------------------- BP plan
constexpr int kTile = 16;            // columns per block along x and along y
constexpr int kThreads = kTile * kTile;
constexpr int kViewBatch = 32;       // views whose per-block constants are built at once
constexpr int kViewRec = 24;         // 32-bit words per view record in LDS

struct BpPlan {
    int kz = 0;          // slices per thread (register accumulators)
    int pitch = 0;       // LDS row pitch in floats (compile-time in the kernel)
    int rows = 0;        // LDS rows of the back-projector (taller footprints are split)
    int rows_full = 0;   // bound of every whole-chunk footprint height
    int cols = 0;        // maximum footprint width
    int ntx = 0, nty = 0, ntiles_pad = 0, nchunks = 0;
    int64_t lds_bytes = 0;      // back-projector LDS per block
    int64_t blocks = 0;
    int line_rows = 0;   // sub-line variant: rows of each thread's blended line
    bool direct = false; // taps read from memory (footprint too large for an LDS tile)
};

// Footprint-driven launch plan (cached by a hash of the inputs).
fdk_status make_bp_plan(const fdk_volume& vg, const fdk_stack& sg,
                        const std::vector<IndexMatrix>& M, BpPlan& plan);

// Pitches the kernel is instantiated for (floats per LDS row).
extern const int kPitches[];
extern const int kNumPitches;

// ---------------------------------------------------------------- runtime
// Copy `bytes` of host memory to a new stream-ordered device allocation.
// The host buffer may be reused as soon as the call returns.
fdk_status upload_async(const void* host, size_t bytes, void* stream, void** dev);
fdk_status device_alloc_async(size_t bytes, void* stream, void** dev);
fdk_status device_free_async(void* dev, void* stream);
fdk_status check_launch(const char* what);

// ---------------------------------------------------------------- launchers
// FP64 composition on the device: M_s = P_s V with V the voxel-index -> world
// map (pitch d*, world position o* of voxel (0,0,0)).  P, M: [np][12].
fdk_status launch_compose(const double* P, double* M, int32_t np, double dx, double dy,
                          double dz, double ox, double oy, double oz, void* stream);

struct BpLaunch {
    const void* proj;        // [np][nh][nw] f32 or f16
    const float* scale;      // [np] or nullptr
    const double* mats_world;// device [np][12] world matrices (uploaded)
    double* mats_index;      // device [np][12] scratch for the composed matrices
    float* vol;              // slab base
    int32_t nx, ny, nz, np, nh, nw;
    int32_t k_begin, k_end;  // slab [k_begin, k_end) of the full volume
    double dx, dy, dz, ox, oy, oz;  // voxel pitch and world position of voxel (0,0,0)
    int f16;
};
fdk_status launch_backproject(const BpLaunch& a, const BpPlan& plan, void* stream);
// Symmetric variant (whole volume; geometry checked by the caller with
// bp_geometry_symmetric) and its launch plan.
fdk_status launch_backproject_sym(const BpLaunch& a, const BpPlan& plan, void* stream);
fdk_status make_bp_plan_sym(const fdk_volume& vg, const fdk_stack& sg,
                            const std::vector<IndexMatrix>& M, BpPlan& plan);
// Sub-line variant (whole volume, float32): a window that holds every
// whole-chunk footprint plus one blended line per thread, and its launch.
fdk_status make_bp_plan_subline(const fdk_volume& vg, const fdk_stack& sg,
                                const std::vector<IndexMatrix>& M, BpPlan& plan);
fdk_status launch_backproject_subline(const BpLaunch& a, const BpPlan& plan, void* stream);
// Whether v(i, j, nz-1-k) = nh - 1 - v(i, j, k) for every view (index-space
// matrices, relative tolerance 1e-10).
bool bp_geometry_symmetric(const fdk_volume& vg, const fdk_stack& sg,
                           const std::vector<IndexMatrix>& M);

// Forward projector: a block per (band of rb detector rows, chunk of columns, view).
struct FpPlan {
    bool voxel = true;   // voxel-driven lanes (else one thread per detector column)
    int rb = 0;          // detector rows per band
    int cw = 0;          // detector columns per chunk
    int pitch = 0;       // LDS window pitch (cw + 2)
    int nbands = 0;
    int ncb = 0;         // column chunks
    int64_t lds_bytes = 0;
    int64_t blocks = 0;
};
// Plan of one forward projection; also fills lanes (fp_view_lanes).  The
// voxel-driven organisation unless FDK_FP_ALGO=gather or its load offsets
// would not fit 31 bits for some view.
fdk_status make_fp_plan(const fdk_volume& vg, const fdk_stack& sg, const std::vector<IndexMatrix>& M,
                        std::vector<int32_t>& lanes, FpPlan& plan);

// Per view (S << 1) | swap.  swap: lanes run along y (|du/dj| > |du/di| at the
// volume centre).  S: lane stride of the voxel-driven forward projector, the
// smallest with |u(a + S) - u(a)| >= 2 columns along the lane axis anywhere in
// the volume (|du/da| = |N(b)| / w^2 with N affine in the other index b).
void fp_view_lanes(const fdk_volume& vg, const std::vector<IndexMatrix>& M,
                   std::vector<int32_t>& lanes);

struct FpLaunch {
    const float* vol;
    float* volT;             // scratch [nz][nx][ny] when any view swaps, else nullptr
    const int* lanes;        // device [np], from fp_view_lanes
    float* proj;
    const double* mats_world;
    double* mats_index;
    int32_t nx, ny, nz, np, nh, nw;
    double dx, dy, dz, ox, oy, oz;
};
fdk_status launch_forwardproject(const FpLaunch& a, const FpPlan& plan, void* stream);

struct FilterLaunch {
    const float* raw;
    float* out;              // float32 output (out16 == nullptr)
    uint16_t* out16;         // binary16 output, or nullptr
    float* scale;            // [np] per-view scale of the binary16 output
    int32_t np, nh, nw;
    double du, dv, sod, sdd, u_off, v_off, arc;
    int32_t np_total;
};
// FDK filter into float32 `out`, or (out16 != nullptr) into binary16 codes
// with one power-of-two scale per view (the rule of launch_quantize_f16):
// views are filtered a few at a time into a stream-ordered float32 workspace
// while their maxima are taken in the filter's epilogue, then converted.
fdk_status launch_filter(const FilterLaunch& a, void* stream);
// Cosine weight only (step 1 of the filter); uses raw, out, np, nh, nw, du,
// dv, sdd, u_off, v_off of `a`.
fdk_status launch_cosine_weight(const FilterLaunch& a, void* stream);

// Learned row filter (float32, [rows][channels][len], weights [cout][cin][9]).
fdk_status launch_conv1d_forward(int cin, int cout, int rows, int len, const float* in,
                                 const float* w, const float* bias, const float* mask,
                                 const float* add, float alpha, int relu, float* out,
                                 void* stream);
fdk_status launch_conv1d_backward_data(int cin, int cout, int rows, int len, const float* gout,
                                       const float* w, const float* mask, float* gin,
                                       void* stream);
fdk_status launch_conv1d_backward_weight(int cin, int cout, int rows, int len, const float* in,
                                         const float* gout, float* gw, float* gb, void* stream);
fdk_status launch_sqerr(int64_t n, const float* a, const float* b, float* grad, float scale,
                        float* loss, void* stream);
// Back-projection variants of include/fdk_ablation.h (float32 projections;
// mats_index: device [np][12] composed index-space matrices).
fdk_status launch_backproject_variant(int variant, int nb, const float* proj,
                                      const double* mats_index, float* vol, int nx, int ny,
                                      int nz, int np, int nh, int nw, void* stream);

fdk_status launch_adam(int n, float* p, const float* g, float* m, float* v, float lr, float b1,
                       float b2, float eps, int step, void* stream);

fdk_status launch_quantize_f16(int32_t np, int64_t npix, const float* in, uint16_t* out,
                               float* scale, void* stream);
// Pieces of the FP16 rule for producers that take the per-view maxima
// themselves: zero `n` words (a fill kernel), and convert np views of npix
// float32 values given the bit patterns of their absolute maxima.
fdk_status launch_clear_u32(unsigned* p, int32_t n, void* stream);
fdk_status launch_quantize_with_max(int32_t np, int64_t npix, const float* in,
                                    const unsigned* maxbits, uint16_t* out, float* scale,
                                    void* stream);

struct PhantomLaunch {
    const double* ell;       // device [n_ell][16]
    int32_t n_ell;
    float* proj;
    int32_t np, nh, nw, view_begin, np_total;
    double arc, theta0, sod, sdd, du, dv, u_off, v_off;
};
fdk_status launch_phantom(const PhantomLaunch& a, void* stream);

}  // namespace fdk
