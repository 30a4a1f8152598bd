/*
 * fdk_ablation.h -- back-projection variants for measuring the paper's CPU
 * optimisations on the GPU (float32 projections).  Each variant computes the
 * same operation as fdk_backproject (Listings 1 and 2; same conventions,
 * geometry requirement and errors as in fdk.h) with a different kernel
 * organisation:
 *
 *   FDK_VARIANT_PRODUCTION   the production kernel, called once per batch of
 *                            nb views: the volume is read and written np/nb
 *                            times (Section 3.1.3's batching of projections;
 *                            nb = np is the production call).
 *   FDK_VARIANT_GLOBAL_TAPS  production structure (hoisting, register
 *                            accumulation over all views) with the bilinear
 *                            taps read from global memory instead of a
 *                            staged LDS window (Section 3.2 removed): the
 *                            library's direct organisation, which
 *                            fdk_backproject itself uses when a block's
 *                            footprint does not fit an LDS tile; nb is
 *                            ignored.
 *   FDK_VARIANT_LISTING1     Listing 1 on the GPU: a thread per voxel, the
 *                            full projection per (voxel, view) (no hoisting,
 *                            Section 3.1.2 removed), taps from global memory,
 *                            the volume read and written once per batch of nb
 *                            views.
 *   FDK_VARIANT_SYMMETRY     production structure plus the geometric symmetry
 *                            of Section 3.1.2: a thread owns slices k of the
 *                            lower half and their mirrors nz-1-k, whose v is
 *                            nh-1-v(k); the mirrored window is staged in
 *                            descending row order so both updates share v, its
 *                            row, fraction and LDS address.  Needs v(nz-1-k) =
 *                            nh-1-v(k) in every view (a circular orbit with the
 *                            detector's centre row on the orbit plane and the
 *                            volume centred on it), else FDK_E_GEOMETRY; whole
 *                            volume only; nb is ignored.
 *   FDK_VARIANT_SUBLINE      production structure with the sub-line
 *                            interpolation of Section 3.1.5 (Algorithm 1's
 *                            sub-line step): per (column, view) the detector
 *                            columns floor(u) and floor(u) + 1 are blended
 *                            once, along every row the column's slices reach,
 *                            into a line in LDS; each update is one 1-D
 *                            interpolation along that line.  The window holds
 *                            the whole chunk's footprint; whole volume only;
 *                            FDK_E_UNSUPPORTED if window and lines do not fit
 *                            in LDS; nb is ignored.
 *
 * nb: views per batch, 1 <= nb (values above np mean np).  proj: device
 * float32 [np][nh][nw] (sg->dtype must be FDK_F32, else FDK_E_UNSUPPORTED);
 * vol: device float32, accumulated into.
 */
#ifndef FDK_ABLATION_H
#define FDK_ABLATION_H

#include <stdint.h>

#include "fdk.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FDK_VARIANT_PRODUCTION = 0,
    FDK_VARIANT_GLOBAL_TAPS = 1,
    FDK_VARIANT_LISTING1 = 2,
    FDK_VARIANT_SYMMETRY = 3,
    FDK_VARIANT_SUBLINE = 4
} fdk_bp_variant;

fdk_status fdk_backproject_variant(int32_t variant, int32_t nb, const fdk_volume* vg, float* vol,
                                   const fdk_stack* sg, const float* proj, const double* mats,
                                   void* stream);

#ifdef __cplusplus
}
#endif

#endif /* FDK_ABLATION_H */
