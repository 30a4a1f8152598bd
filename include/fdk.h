/*
 * fdk.h -- C ABI of the MI355X (gfx950) voxel-driven FDK back-projector.
 *
 * The operation is the one of Chen et al., "Performance Portable
 * Back-projection Algorithms on CPUs", ICS'21: the image reconstruction
 * problem nw x nh x np => nx x ny x nz (Section 2.3); for every voxel and every
 * filtered projection, project the voxel centre through the view's 3x4
 * pinhole matrix (Section 2.1.1), bilinearly interpolate the projection at the
 * resulting detector position, weight by 1/w^2 and accumulate into the volume
 * (Listings 1 and 2).
 *
 * Conventions used by every entry point
 *   - volume   float32 vol[nz][ny][nx], x fastest (the layout of Listing 1);
 *              voxel (i,j,k) has its centre at
 *              ((i-(nx-1)/2) dx + cx, (j-(ny-1)/2) dy + cy, (k-(nz-1)/2) dz + cz) mm.
 *   - stack    proj[np][nh][nw] (float32, or binary16 with one float32 scale
 *              per view); pixel (r, c) sits at detector coordinates
 *              (u, v) = (c, r): u along the width nw (fastest), v along nh.
 *   - matrices double mats[np][3][4], row-major, HOST memory, mapping world
 *              millimetres (x, y, z, 1) to (u w, v w, w); the sample weight is
 *              1/w^2 with w as the matrix gives it.
 *   - interpolation: floor of the coordinate; a tap outside
 *              [0, nh-1] x [0, nw-1] contributes zero.
 *   - all device pointers are HIP device memory on the current device, owned
 *     by the caller; the library never frees them.  Work is enqueued on
 *     `stream` (a hipStream_t; NULL = the null stream) and is asynchronous
 *     with respect to the host.  Host inputs are copied before the call
 *     returns and may be reused immediately.
 *   - errors: every entry point returns FDK_OK or a negative fdk_status.
 *     Errors that the host can detect (NULL pointers, sizes, dtypes, geometry)
 *     are returned before any HIP call is made.  A device error surfaces as
 *     FDK_E_DEVICE from the call that hit it; a fault inside a kernel is
 *     reported by the next synchronising HIP call of the caller.
 *     fdk_last_error() returns a message for the calling thread.
 */
#ifndef FDK_H
#define FDK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FDK_OK = 0,
    FDK_E_INVALID = -1,      /* NULL pointer, non-positive or overflowing size, bad dtype/scale */
    FDK_E_GEOMETRY = -2,     /* matrix not of the circular-orbit column form, or w <= 0 */
    FDK_E_UNSUPPORTED = -3,  /* valid request outside what the kernels implement */
    FDK_E_DEVICE = -4,       /* a HIP call failed */
    FDK_E_NOMEM = -5         /* a device or pinned-host allocation failed */
} fdk_status;

typedef enum { FDK_F32 = 0, FDK_F16 = 1 } fdk_dtype;

/* Volume geometry (problem statement nw x nh x np => nx x ny x nz, Section 2.3). */
typedef struct fdk_volume {
    int32_t nx, ny, nz;      /* voxels along x, y, z */
    double dx, dy, dz;       /* voxel pitch in mm, > 0 */
    double cx, cy, cz;       /* world position of the volume centre, mm */
} fdk_volume;

/* Projection stack shape and storage type. */
typedef struct fdk_stack {
    int32_t np, nh, nw;      /* views, detector rows, detector columns */
    int32_t dtype;           /* fdk_dtype of the stored values */
} fdk_stack;

/*
 * fdk_backproject -- vol += BP(proj)   (Listings 1 and 2; Algorithm 1 order)
 *
 *   vol[k][j][i] += sum_s bilinear(proj_s, u_s, v_s) * scale_s / w_s^2
 *
 * vg, sg     volume and stack geometry (host structs).
 * vol        device float32 [nz][ny][nx]; accumulated into, never zeroed.
 * proj       device [np][nh][nw], float32 (sg->dtype == FDK_F32) or
 *            binary16 bit patterns (FDK_F16).
 * scale      device float32 [np] dequantisation scale per view; must be
 *            NULL for FDK_F32 and non-NULL for FDK_F16.
 * mats       host double [np][3][4], world mm -> (u w, v w, w).
 * stream     hipStream_t.
 *
 * Geometry requirement (Section 3.1.2, hoisting): after composing each matrix
 * with the voxel grid, entries (0,2) and (2,2) -- the dependence of u w and w
 * on k -- must vanish (|m| <= 1e-12 of the row norm; a detector whose V-axis
 * is parallel to the rotation axis), and w must be positive over the volume.
 * Otherwise FDK_E_GEOMETRY.  vol and proj must not overlap.
 * The result is deterministic: no atomics, fixed summation order.
 * Each view's detector footprint of a block of voxels is staged in LDS; where
 * it cannot be (strong magnification: roughly beyond 15 detector pixels per
 * voxel) the taps are read from memory instead, with the same result
 * contract (fdk_bp_plan reports lds_pitch = 0 for such launches).
 */
fdk_status fdk_backproject(const fdk_volume* vg, float* vol,
                           const fdk_stack* sg, const void* proj,
                           const float* scale, const double* mats,
                           void* stream);

/*
 * fdk_backproject_slab -- back-projection into a z-slab of a larger volume.
 *
 * Same as fdk_backproject for the volume described by vg, restricted to the
 * slices k_begin .. k_begin + k_count - 1, which vol_slab holds as a
 * contiguous float32 [k_count][ny][nx] array.  Bitwise identical to the same
 * slices of a full-volume fdk_backproject call with the same inputs, so a
 * volume can be split into slabs (e.g. across devices) with no exchange.
 */
fdk_status fdk_backproject_slab(const fdk_volume* vg, int32_t k_begin, int32_t k_count,
                                float* vol_slab, const fdk_stack* sg, const void* proj,
                                const float* scale, const double* mats, void* stream);

/* Views per call of fdk_backproject_noalloc (the size of its fixed scratch array). */
#define FDK_NOALLOC_MAX_VIEWS 16384

/*
 * fdk_backproject_noalloc -- fdk_backproject for callers that cannot allocate
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation.  Same arguments, semantics and errors as fdk_backproject
 * and a bitwise identical result, but the call makes no device, pinned-host or
 * stream-ordered allocation.  Its only scratch -- the world matrices and their
 * FP64 compositions with the voxel grid, 192 bytes per view -- is a fixed
 * device array for FDK_NOALLOC_MAX_VIEWS views (3 MiB), one per GPU, held
 * until the process ends; a stack of more views gives FDK_E_UNSUPPORTED
 * before any HIP call.  The matrices reach that array as kernel arguments (32
 * views per launch), so `mats` may be reused as soon as the call returns.
 * Nothing in the array needs to start at zero: each call writes the entries
 * it reads.  All calls on one GPU share the array: calls that overlap in time
 * on one GPU (on different streams, or from several host threads) race and
 * must be serialised by the caller; calls on one stream are ordered.
 */
fdk_status fdk_backproject_noalloc(const fdk_volume* vg, float* vol,
                                   const fdk_stack* sg, const void* proj,
                                   const float* scale, const double* mats,
                                   void* stream);

/*
 * fdk_forwardproject -- proj += A vol, the exact transpose of the back-projection
 * (the projector of the iterative methods of Section 1: the adjoint pair
 * <BP p, x> = <p, FP x> holds up to rounding).
 *
 * Every voxel value x, weighted by 1/w^2, is split over the four bilinear taps
 * around its (u, v) with the interpolation weights of Listing 2; taps outside
 * the detector are dropped.  vol: device float32 [nz][ny][nx]; proj: device
 * float32 [np][nh][nw] (sg->dtype must be FDK_F32, else FDK_E_UNSUPPORTED),
 * accumulated into.  Each projection sample is summed by one block in a
 * fixed order (no atomics): the result is deterministic.  Where the slices
 * one tile of voxels reads would span 2 GiB or more of the volume (very large
 * slices at steep cone angles), a slower organisation of the same sum is
 * used.  Views whose u
 * changes faster along y than along x read a transposed copy of the volume,
 * a stream-ordered device allocation of the volume's size made by the call.
 * Same geometry requirement as above.
 */
fdk_status fdk_forwardproject(const fdk_volume* vg, const float* vol,
                              const fdk_stack* sg, float* proj,
                              const double* mats, void* stream);

/*
 * fdk_filter -- FDK pre-processing of raw line integrals (the "filtered
 * projections" the paper takes as input, Sections 2.1.2 and 3.1.1):
 *
 *   q = raw * sdd / sqrt(sdd^2 + u_mm^2 + v_mm^2)           cosine weight
 *   q = tau * (h * q)   along each detector row              Ram-Lak ramp
 *   p = q * arc / (2 np_total)                                angular weight
 *
 * with u_mm = (c - (nw-1)/2 - u_off) du, v_mm = (r - (nh-1)/2 - v_off) dv,
 * tau = du sod / sdd, h[0] = 1/(4 tau^2), h[n odd] = -1/(pi^2 n^2 tau^2),
 * h[n even, != 0] = 0, and a linear (zero-padded) convolution over the row.
 *
 * raw        device float32 [np][nh][nw]; sg->dtype must be FDK_F32.
 * out_dtype  FDK_F32: out is device float32 [np][nh][nw] and receives p;
 *            out_scale must be NULL.
 *            FDK_F16: out is device uint16 [np][nh][nw] and receives the
 *            binary16 storage of p with the rule of fdk_quantize_f16 (per-view
 *            power-of-two scale from max |p_s|, round to nearest even), bit
 *            for bit what fdk_quantize_f16 makes of the FDK_F32 output;
 *            out_scale is device float32 [np] and receives the scales.  The
 *            per-view maxima are taken as the filter writes its output (a few
 *            views at a time through a stream-ordered float32 workspace of at
 *            most 64 MiB, or one view if a view is larger), so no separate
 *            pass over a float32 stack is needed.
 * raw and out may not overlap.  Back-projecting the result with the matrices
 * of the same scan (weight 1/w^2, w = 1 at the isocentre) gives the FDK
 * reconstruction.
 */
fdk_status fdk_filter(const fdk_stack* sg, const float* raw, int32_t out_dtype, void* out,
                      float* out_scale, double du, double dv, double sod, double sdd,
                      double u_off, double v_off, double arc, int32_t np_total,
                      void* stream);

/*
 * fdk_quantize_f16 -- FP16 storage of a filtered stack with one scale per view.
 *
 *   m_s = max |p_s|;  scale_s = 1 if m_s == 0, else 2^(ceil(log2 m_s) - 15);
 *   out = round-to-nearest-even(p / scale_s) as binary16   (|out| <= 32768)
 *
 * in: device float32 [np][nh][nw]; out: device uint16 (binary16 bits), same
 * shape; scale: device float32 [np].  Deterministic, bit-exact.
 */
fdk_status fdk_quantize_f16(int32_t np, int32_t nh, int32_t nw, const float* in,
                            uint16_t* out, float* scale, void* stream);

/*
 * fdk_circular_matrices -- host helper: the matrices of a circular orbit about
 * +z (the CBCT geometry of Section 2.1.1; the paper defers the construction
 * to the literature).  View s at theta = theta0 + arc s / np; source at
 * sod (cos, sin, 0); flat detector at distance sdd from the source, axes
 * e_u = (-sin, cos, 0), e_v = (0, 0, 1), pixel pitch du x dv, principal point
 * ((nw-1)/2 + u_off, (nh-1)/2 + v_off); w = depth / sod (1 at the isocentre).
 * mats_out: host double [np][3][4].  No HIP call.
 */
fdk_status fdk_circular_matrices(int32_t np, double arc, double theta0, double sod,
                                 double sdd, int32_t nh, int32_t nw, double du, double dv,
                                 double u_off, double v_off, double* mats_out);

/*
 * fdk_phantom_project -- analytic line integrals of ellipsoids (test data and
 * training data; stands in for the forward-projected RabbitCT data of Section
 * 4.2).  For views view_begin .. view_begin + sg->np - 1 of a circular orbit
 * of np_total views (conventions of fdk_circular_matrices), the ray from the
 * source to every pixel centre is intersected with each ellipsoid and
 * proj += sum_e rho_e * chord_e (mm).
 *
 * ell: host double [n_ell][16] rows (cx, cy, cz, a, b, c, R row-major 3x3
 * whose columns are the semi-axis directions, rho).  proj: device float32
 * [sg->np][nh][nw] (sg->dtype FDK_F32), accumulated into.
 */
fdk_status fdk_phantom_project(const double* ell, int32_t n_ell, const fdk_stack* sg,
                               float* proj, double arc, double theta0, double sod,
                               double sdd, double du, double dv, double u_off,
                               double v_off, int32_t view_begin, int32_t np_total,
                               void* stream);

/*
 * fdk_bp_plan -- host query of the launch the back-projector would use for
 * these inputs: out[0..11] = tile_x, tile_y, kz (slices per thread),
 * lds_pitch (words per LDS row), lds_rows, lds_bytes per block, blocks,
 * threads per block, rows_full (rows of the tallest whole-chunk footprint;
 * taller than lds_rows means such footprints are staged per half-chunk;
 * lds_pitch = lds_rows = lds_bytes = 0: the taps are read from memory),
 * then the forward projector's lds_bytes per block, detector rows per band
 * and detector columns per chunk.  The tile depends on sg->dtype (binary16
 * tiles hold two regions of pair words).  out: host int64 [12].  Validates
 * exactly like fdk_backproject.  No HIP call.
 */
fdk_status fdk_bp_plan(const fdk_volume* vg, const fdk_stack* sg, const double* mats,
                       int64_t* out);

/* Message of the last error on the calling thread ("" if none). */
const char* fdk_last_error(void);

/* Static description of a status code; any value is accepted ("unknown
 * status" for values that are not an fdk_status). */
const char* fdk_status_string(int32_t s);

#ifdef __cplusplus
}
#endif

#endif /* FDK_H */
