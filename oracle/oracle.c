/*
 * FP64 reference ("oracle") for voxel-driven FDK cone-beam back-projection.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP path.
 *
 * What it computes (Chen et al., ICS'21, Section 2.1.2 with the pinhole
 * model of Section 2.1.1): every voxel receives, from every filtered view s,
 * the view's value at the point where the voxel centre X projects, divided
 * by the square of the projective depth:
 *
 *   vol(X) += sum_s  p_s(u_s, v_s) / w_s^2,   (u_s w_s, v_s w_s, w_s) = P_s (X, 1)
 *
 * and the value between pixel centres is bilinear interpolation, written here
 * as the tent-weighted sum it is:
 *
 *   p_s(u, v) = sum_{r, c} p_s[r][c] hat(u - c) hat(v - r),  hat(t) = max(0, 1 - |t|)
 *
 * Only the (at most) four pixels around (u, v) have a non-zero weight; a
 * pixel that does not exist (outside [0,nh-1] x [0,nw-1]) is absent from the
 * sum, i.e. contributes zero.
 *
 * Readings of what the paper leaves open:
 *   - P_s maps world millimetres (voxel centres) to homogeneous pixel
 *     coordinates; voxel (i,j,k) has its centre at
 *     ((i-(nx-1)/2) dx + cx, (j-(ny-1)/2) dy + cy, (k-(nz-1)/2) dz + cz);
 *   - pixel (r, c) of a view sits at (u, v) = (c, r); u runs along the
 *     detector width nw (fastest index), v along the height nh;
 *   - the four pixels are found with the mathematical floor (the paper's
 *     code truncates, which equals floor only for non-negative coordinates);
 *   - the weight is 1/w^2 exactly as the matrix gives w;
 *   - results are added to the caller's volume.
 *
 * Every function works in double precision and takes no shortcut beyond what
 * the definition states.  The projection stack may be given as float32, or as
 * IEEE binary16 bit patterns with a per-view float32 scale (dequantised value
 * = half * scale); both convert exactly to double.  A stack may also hold
 * only a window of each view (rows r0_s .. r0_s + wr - 1, columns
 * c0_s .. c0_s + wc - 1 of the nh x nw detector); a pixel inside the detector
 * but outside its view's window is then reported as a miss (the caller chose
 * too small a window) instead of being silently taken as zero.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <omp.h>

/* ---- the filtered views --------------------------------------------------- */

typedef struct {
    const float *f32;        /* [np][wr][wc] or NULL            */
    const uint16_t *f16;     /* [np][wr][wc] binary16 or NULL   */
    const float *scale;      /* [np] per-view scale for binary16 */
    int64_t nh, nw;          /* detector rows and columns        */
    int64_t wr, wc;          /* stored rows and columns per view */
    const int64_t *origin;   /* [np][2] (r0, c0) of each stored window; NULL: whole views */
    int *miss;               /* set when a needed pixel lies outside its window */
} views_t;

/* IEEE 754 binary16 -> double, decoded from its definition. */
static double half_value(uint16_t h)
{
    int sign = (h >> 15) & 1;
    int expo = (h >> 10) & 0x1f;
    int mant = h & 0x3ff;
    double mag;
    if (expo == 0)
        mag = ldexp((double)mant, -24);              /* subnormal: m * 2^-24 */
    else if (expo == 31)
        mag = mant ? NAN : INFINITY;
    else
        mag = ldexp((double)(mant | 0x400), expo - 25);  /* 1.m * 2^(e-15) */
    return sign ? -mag : mag;
}

/* Pixel value p_s[r][c]; a pixel off the detector does not exist (zero). */
static double pixel(const views_t *V, int64_t s, int64_t r, int64_t c)
{
    if (r < 0 || r >= V->nh || c < 0 || c >= V->nw)
        return 0.0;
    if (V->origin) {
        r -= V->origin[2 * s];
        c -= V->origin[2 * s + 1];
        if (r < 0 || r >= V->wr || c < 0 || c >= V->wc) {
            #pragma omp atomic write
            *V->miss = 1;
            return 0.0;
        }
    }
    int64_t idx = (s * V->wr + r) * V->wc + c;
    if (V->f32)
        return (double)V->f32[idx];
    return half_value(V->f16[idx]) * (double)V->scale[s];
}

/* Tent (hat) function: the weight of a pixel at distance t along one axis. */
static double hat(double t)
{
    double a = 1.0 - fabs(t);
    return a > 0.0 ? a : 0.0;
}

/* Value of view s at detector point (u, v): the tent-weighted sum over the
 * pixels around it.  The weights of pixels farther than one pitch vanish, so
 * only the 2 x 2 pixels starting at (floor(v), floor(u)) are visited.  A
 * point more than one pitch off the detector sees no pixel at all (this also
 * keeps the integer conversion in range). */
static double view_value(const views_t *V, int64_t s, double u, double v)
{
    if (!(u > -1.0 && u < (double)V->nw && v > -1.0 && v < (double)V->nh))
        return 0.0;
    double c_lo = floor(u), r_lo = floor(v);
    double sum = 0.0;
    for (int dr = 0; dr < 2; dr++)
        for (int dc = 0; dc < 2; dc++) {
            double r = r_lo + dr, c = c_lo + dc;
            double wgt = hat(v - r) * hat(u - c);
            if (wgt != 0.0)
                sum += wgt * pixel(V, s, (int64_t)r, (int64_t)c);
        }
    return sum;
}

/* Homogeneous image (u w, v w, w) of the world point X under the 3x4 matrix
 * P (row-major), Section 2.1.1. */
static void image_of(const double *P, const double X[3], double h[3])
{
    for (int row = 0; row < 3; row++) {
        const double *p = P + 4 * row;
        h[row] = p[0] * X[0] + p[1] * X[1] + p[2] * X[2] + p[3];
    }
}

/* What view s adds to the voxel centred at X: p_s(u, v) / w^2. */
static double view_term(const views_t *V, const double *mats, int64_t s, const double X[3])
{
    double h[3];
    image_of(mats + 12 * s, X, h);
    double w = h[2];
    return view_value(V, s, h[0] / w, h[1] / w) / (w * w);
}

/* Sum over the views s = 0 .. np-1, in that order, for the voxel at X. */
static double voxel_sum(const views_t *V, const double *mats, int64_t np, const double X[3])
{
    double acc = 0.0;
    for (int64_t s = 0; s < np; s++)
        acc += view_term(V, mats, s, X);
    return acc;
}

/* ---- the voxel grid ------------------------------------------------------- */

typedef struct {
    int64_t nx, ny, nz;
    double dx, dy, dz, cx, cy, cz;
} grid_t;

/* World position (mm) of the centre of voxel (i, j, k). */
static void voxel_centre(const grid_t *g, int64_t i, int64_t j, int64_t k, double X[3])
{
    X[0] = ((double)i - 0.5 * (double)(g->nx - 1)) * g->dx + g->cx;
    X[1] = ((double)j - 0.5 * (double)(g->ny - 1)) * g->dy + g->cy;
    X[2] = ((double)k - 0.5 * (double)(g->nz - 1)) * g->dz + g->cz;
}

static views_t whole_views(int64_t nh, int64_t nw, const float *p32, const uint16_t *p16,
                           const float *scale)
{
    views_t V = {p32, p16, scale, nh, nw, nh, nw, NULL, NULL};
    return V;
}

/* ---- back-projection of the whole volume --------------------------------- */
/* mats: [np][3][4] world mm -> homogeneous pixel.  vol: [nz][ny][nx] +=.     */
int oracle_bp(int64_t nx, int64_t ny, int64_t nz,
              double dx, double dy, double dz, double cx, double cy, double cz,
              int64_t np, int64_t nh, int64_t nw,
              const float *p32, const uint16_t *p16, const float *scale,
              const double *mats, double *vol, int nthreads)
{
    grid_t g = {nx, ny, nz, dx, dy, dz, cx, cy, cz};
    views_t V = whole_views(nh, nw, p32, p16, scale);
    int64_t n = nx * ny * nz;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; q++) {
        double X[3];
        voxel_centre(&g, q % nx, (q / nx) % ny, q / (nx * ny), X);
        vol[q] += voxel_sum(&V, mats, np, X);
    }
    return 0;
}

/* ---- back-projection of selected voxels ----------------------------------- */
/* ijk: [n][3] voxel indices (i, j, k); out[n] = the sum over all views.      */
int oracle_bp_points(int64_t nx, int64_t ny, int64_t nz,
                     double dx, double dy, double dz, double cx, double cy, double cz,
                     int64_t np, int64_t nh, int64_t nw,
                     const float *p32, const uint16_t *p16, const float *scale,
                     const double *mats, int64_t n, const int64_t *ijk,
                     double *out, int nthreads)
{
    grid_t g = {nx, ny, nz, dx, dy, dz, cx, cy, cz};
    views_t V = whole_views(nh, nw, p32, p16, scale);
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n; q++) {
        double X[3];
        voxel_centre(&g, ijk[3 * q], ijk[3 * q + 1], ijk[3 * q + 2], X);
        out[q] = voxel_sum(&V, mats, np, X);
    }
    return 0;
}

/* ---- back-projection of an axis-aligned sub-block ------------------------- */
/* out: [k1-k0][j1-j0][i1-i0] += the sums over all views.  The stack holds
 * wr x wc pixels per view; with origin != NULL they are the window of view s
 * whose first pixel is detector pixel (origin[s][0], origin[s][1]), else the
 * whole view (wr = nh, wc = nw).  Returns 1 if some voxel needed a detector
 * pixel outside its view's window (the result is then incomplete), else 0.  */
int oracle_bp_block(int64_t nx, int64_t ny, int64_t nz,
                    double dx, double dy, double dz, double cx, double cy, double cz,
                    int64_t np, int64_t nh, int64_t nw, int64_t wr, int64_t wc,
                    const int64_t *origin,
                    const float *p32, const uint16_t *p16, const float *scale,
                    const double *mats,
                    int64_t i0, int64_t i1, int64_t j0, int64_t j1, int64_t k0, int64_t k1,
                    double *out, int nthreads)
{
    grid_t g = {nx, ny, nz, dx, dy, dz, cx, cy, cz};
    int miss = 0;
    views_t V = {p32, p16, scale, nh, nw, wr, wc, origin, &miss};
    int64_t bx = i1 - i0, by = j1 - j0, bz = k1 - k0;
    int64_t n = bx * by * bz;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; q++) {
        double X[3];
        voxel_centre(&g, i0 + q % bx, j0 + (q / bx) % by, k0 + q / (bx * by), X);
        out[q] += voxel_sum(&V, mats, np, X);
    }
    return miss;
}

/* ---- back-projection with u and w computed once per column ---------------- */
/* Section 3.1.2 / Algorithm 1: when neither u w nor w depends on z (the
 * detector's V-axis parallel to the rotation axis, Section 2.1.1), the depth
 * w and the column coordinate u of a voxel column (i, j) are the same for all
 * its slices, and only v changes along k.  This evaluates the sum that way:
 * w and u per (column, view), v per voxel.  It equals oracle_bp in exact
 * arithmetic for such matrices, which the tests check.  Columns are
 * independent; each voxel still sums its views in order s = 0 .. np-1.     */
int oracle_bp_hoisted(int64_t nx, int64_t ny, int64_t nz,
                      double dx, double dy, double dz, double cx, double cy, double cz,
                      int64_t np, int64_t nh, int64_t nw,
                      const float *p32, const uint16_t *p16, const float *scale,
                      const double *mats, double *vol, int nthreads)
{
    grid_t g = {nx, ny, nz, dx, dy, dz, cx, cy, cz};
    views_t V = whole_views(nh, nw, p32, p16, scale);
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for schedule(static)
    for (int64_t col = 0; col < nx * ny; col++) {
        double X[3];
        voxel_centre(&g, col % nx, col / nx, 0, X);
        double base[3];
        for (int64_t s = 0; s < np; s++) {
            const double *P = mats + 12 * s;
            X[2] = 0.0;
            image_of(P, X, base);                      /* (u w, v w, w) at z = 0 */
            double w = base[2];                        /* free of z              */
            double u = base[0] / w;                    /* free of z              */
            for (int64_t k = 0; k < nz; k++) {
                double Z = ((double)k - 0.5 * (double)(nz - 1)) * dz + cz;
                double v = (base[1] + P[6] * Z) / w;
                vol[k * nx * ny + col] += view_value(&V, s, u, v) / (w * w);
            }
        }
    }
    return 0;
}

/* ---- back-projection, geometry mode (no matrices) ------------------------- */
/* Circular source orbit about +z (Section 2.1.1: the detector's V-axis is
 * parallel to the rotation axis).  View s is at angle theta_s =
 * theta0 + arc * s / np.  Source S = sod (cos, sin, 0); detector plane
 * through C = -(sdd - sod)(cos, sin, 0) with in-plane unit axes
 * e_u = (-sin, cos, 0), e_v = (0, 0, 1).  The ray from S through the voxel
 * centre X is intersected with the detector plane; the hit point's
 * coordinates along e_u, e_v (mm) give the pixel position
 *   u = u_mm / du + (nw - 1)/2 + u_off,   v = v_mm / dv + (nh - 1)/2 + v_off,
 * and the depth is the distance from the source to X along the central ray,
 * normalised so that it equals 1 at the isocentre: w = n.(S - X) / sod.      */
static void project_geometry(double th, double sod, double sdd, double du, double dv,
                             double cu, double cv, const double X[3],
                             double *u, double *v, double *w)
{
    double ct = cos(th), st_ = sin(th);
    double S[3] = {sod * ct, sod * st_, 0.0};
    double C[3] = {-(sdd - sod) * ct, -(sdd - sod) * st_, 0.0};
    double n[3] = {ct, st_, 0.0};                 /* unit normal, source side */
    double eu[3] = {-st_, ct, 0.0}, ev[3] = {0.0, 0.0, 1.0};
    double d[3] = {X[0] - S[0], X[1] - S[1], X[2] - S[2]};
    double nd = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
    double ncs = n[0] * (C[0] - S[0]) + n[1] * (C[1] - S[1]) + n[2] * (C[2] - S[2]);
    double lam = ncs / nd;
    double H[3] = {S[0] + lam * d[0] - C[0], S[1] + lam * d[1] - C[1], S[2] + lam * d[2] - C[2]};
    double umm = eu[0] * H[0] + eu[1] * H[1] + eu[2] * H[2];
    double vmm = ev[0] * H[0] + ev[1] * H[1] + ev[2] * H[2];
    *u = umm / du + cu;
    *v = vmm / dv + cv;
    *w = (n[0] * (S[0] - X[0]) + n[1] * (S[1] - X[1]) + n[2] * (S[2] - X[2])) / sod;
}

int oracle_bp_geometry(int64_t nx, int64_t ny, int64_t nz,
                       double dx, double dy, double dz, double cx, double cy, double cz,
                       int64_t np, int64_t nh, int64_t nw,
                       const float *p32, const uint16_t *p16, const float *scale,
                       double arc, double theta0, double sod, double sdd,
                       double du, double dv, double u_off, double v_off,
                       double *vol, int nthreads)
{
    grid_t g = {nx, ny, nz, dx, dy, dz, cx, cy, cz};
    views_t V = whole_views(nh, nw, p32, p16, scale);
    double cu = 0.5 * (double)(nw - 1) + u_off, cv = 0.5 * (double)(nh - 1) + v_off;
    int64_t n = nx * ny * nz;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < n; q++) {
        double X[3];
        voxel_centre(&g, q % nx, (q / nx) % ny, q / (nx * ny), X);
        double acc = 0.0;
        for (int64_t s = 0; s < np; s++) {
            double th = theta0 + arc * (double)s / (double)np;
            double u, v, w;
            project_geometry(th, sod, sdd, du, dv, cu, cv, X, &u, &v, &w);
            acc += view_value(&V, s, u, v) / (w * w);
        }
        vol[q] += acc;
    }
    return 0;
}

/* Geometry-mode projection of points, for checks of matrix builders.
 * xyz: [n][3] world mm; out: [n][3] (u, v, w) for view angle th.            */
int oracle_project_points(double th, double sod, double sdd, double du, double dv,
                          int64_t nh, int64_t nw, double u_off, double v_off,
                          int64_t n, const double *xyz, double *out)
{
    double cu = 0.5 * (double)(nw - 1) + u_off, cv = 0.5 * (double)(nh - 1) + v_off;
    for (int64_t q = 0; q < n; q++)
        project_geometry(th, sod, sdd, du, dv, cu, cv, xyz + 3 * q,
                         &out[3 * q], &out[3 * q + 1], &out[3 * q + 2]);
    return 0;
}

/* ---- forward projection: the exact transpose of oracle_bp ----------------- */
/* Back-projection is linear in the pixels: voxel X receives
 * sum_{s,r,c} p_s[r][c] hat(u_s - c) hat(v_s - r) / w_s^2.  Its transpose
 * therefore gives every existing pixel (r, c) of view s the sum over voxels of
 * x(X) hat(u_s - c) hat(v_s - r) / w_s^2, with the same (u, v, w) and the same
 * pixels (those off the detector do not exist).  One thread owns a view, so
 * no pixel has two writers; voxels are visited in index order.              */
int oracle_fp(int64_t nx, int64_t ny, int64_t nz,
              double dx, double dy, double dz, double cx, double cy, double cz,
              int64_t np, int64_t nh, int64_t nw,
              const double *vol, const double *mats, double *proj, int nthreads)
{
    grid_t g = {nx, ny, nz, dx, dy, dz, cx, cy, cz};
    int64_t n = nx * ny * nz;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < np; s++) {
        double *img = proj + s * nh * nw;
        for (int64_t q = 0; q < n; q++) {
            double X[3], h[3];
            voxel_centre(&g, q % nx, (q / nx) % ny, q / (nx * ny), X);
            image_of(mats + 12 * s, X, h);
            double w = h[2], u = h[0] / w, v = h[1] / w;
            if (!(u > -1.0 && u < (double)nw && v > -1.0 && v < (double)nh))
                continue;
            double x = vol[q] / (w * w);
            double c_lo = floor(u), r_lo = floor(v);
            for (int dr = 0; dr < 2; dr++)
                for (int dc = 0; dc < 2; dc++) {
                    double r = r_lo + dr, c = c_lo + dc;
                    if (r < 0.0 || r >= (double)nh || c < 0.0 || c >= (double)nw)
                        continue;
                    img[(int64_t)r * nw + (int64_t)c] += x * hat(v - r) * hat(u - c);
                }
        }
    }
    return 0;
}

/* ---- FDK pre-processing filter ------------------------------------------ */
/* Feldkamp et al. (1984) as presented in Kak & Slaney, ch. 3: each detector
 * row is (1) multiplied by the cosine weight sdd / sqrt(sdd^2 + u_mm^2 +
 * v_mm^2), (2) linearly convolved (zero padding) with the band-limited ramp
 * (Ram-Lak) kernel sampled at the isocentre pitch tau = du * sod / sdd:
 *   h[0] = 1/(4 tau^2), h[n odd] = -1/(pi^2 n^2 tau^2), h[n even] = 0,
 * times tau (quadrature of the convolution integral), and (3) multiplied by
 * arc / (2 np_total), the angular quadrature weight with the 1/2 of the FDK
 * formula.  The paper only names the filtering step and leaves it out.     */
int oracle_filter(int64_t np, int64_t nh, int64_t nw, const double *raw, double *out,
                  double du, double dv, double sod, double sdd, double u_off, double v_off,
                  double arc, int64_t np_total, int nthreads)
{
    double cu = 0.5 * (double)(nw - 1) + u_off, cv = 0.5 * (double)(nh - 1) + v_off;
    double tau = du * sod / sdd;
    double pi = 3.14159265358979323846;
    double wang = arc / (2.0 * (double)np_total);
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for collapse(2) schedule(static)
    for (int64_t s = 0; s < np; s++)
        for (int64_t r = 0; r < nh; r++) {
            const double *row = raw + (s * nh + r) * nw;
            double *o = out + (s * nh + r) * nw;
            double vmm = ((double)r - cv) * dv;
            double q[nw];                        /* cosine-weighted row (VLA) */
            for (int64_t c = 0; c < nw; c++) {
                double umm = ((double)c - cu) * du;
                q[c] = row[c] * sdd / sqrt(sdd * sdd + umm * umm + vmm * vmm);
            }
            for (int64_t c = 0; c < nw; c++) {
                double acc = 0.0;
                for (int64_t c2 = 0; c2 < nw; c2++) {
                    int64_t n = c - c2;
                    double h;
                    if (n == 0) h = 1.0 / (4.0 * tau * tau);
                    else if (n % 2 == 0) h = 0.0;
                    else h = -1.0 / (pi * pi * (double)n * (double)n * tau * tau);
                    acc += h * q[c2];
                }
                o[c] = acc * tau * wang;
            }
        }
    return 0;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }
