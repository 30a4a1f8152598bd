/*
 * FP64 reference ("oracle") for voxel-driven FDK cone-beam back-projection.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP path.
 *
 * What it computes (Chen et al., ICS'21, Section 2.1.2, Listings 1 and 2):
 *
 *   vol[k][j][i] += sum_s  B_s(u_s, v_s) / w_s^2
 *   (u_s w_s, v_s w_s, w_s) = P_s (X(i), Y(j), Z(k), 1)^T
 *   B_s(u, v) = bilinear interpolation of view s at (u, v), zero outside
 *
 * with the readings that the paper leaves open (they are listed in the
 * design notes of the repository as R1..R20):
 *   - P_s maps world millimetres (voxel centres) to homogeneous pixel
 *     coordinates; voxel (i,j,k) has its centre at
 *     ((i-(nx-1)/2) dx + cx, (j-(ny-1)/2) dy + cy, (k-(nz-1)/2) dz + cz);
 *   - pixel (r, c) of a view sits at (u, v) = (c, r); u runs along the
 *     detector width nw (fastest index), v along the height nh;
 *   - the integer part is the mathematical floor (the listing's (int) cast
 *     truncates, which equals floor only for non-negative coordinates);
 *   - a tap outside [0,nh-1] x [0,nw-1] contributes zero;
 *   - the weight is 1/w^2 exactly as the matrix gives w (Listing 1 squares
 *     f = 1/z);
 *   - accumulation is into the caller's volume (Listing 1 updates with +=).
 *
 * Every function works in double precision and takes no shortcut beyond what
 * the definition states.  The projection stack may be given as float32, or as
 * IEEE binary16 bit patterns with a per-view float32 scale (dequantised value
 * = half * scale); both convert exactly to double.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <omp.h>

/* ---- projection access (exact conversion to double) ------------------- */

typedef struct {
    const float *f32;        /* [np][nh][nw] or NULL           */
    const uint16_t *f16;     /* [np][nh][nw] binary16 or NULL   */
    const float *scale;      /* [np] per-view scale for f16     */
    int64_t nh, nw;
} stack_t_;

/* IEEE 754 binary16 -> double, decoded from its definition. */
static double half_to_double(uint16_t h)
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

/* Pixel (r, c) of view s, zero outside the detector (zero extension). */
static double tap(const stack_t_ *st, int64_t s, int64_t r, int64_t c)
{
    if (r < 0 || r >= st->nh || c < 0 || c >= st->nw)
        return 0.0;
    int64_t idx = (s * st->nh + r) * st->nw + c;
    if (st->f32)
        return (double)st->f32[idx];
    return half_to_double(st->f16[idx]) * (double)st->scale[s];
}

/* mix(x, y, a) = x (1 - a) + y a  (Listing 2) */
static double mix(double x, double y, double a) { return x * (1.0 - a) + y * a; }

/* Bilinear_Interpolate of Listing 2: horizontal blends of rows r and r+1,
 * then a vertical blend; floor instead of truncation, zero outside. */
static double bilinear(const stack_t_ *st, int64_t s, double u, double v)
{
    /* Far outside the detector every tap is zero; this also keeps the
     * integer conversion below in range. */
    if (!(u > -2.0 && u < (double)st->nw + 1.0 && v > -2.0 && v < (double)st->nh + 1.0))
        return 0.0;
    double cf = floor(u), rf = floor(v);
    int64_t c = (int64_t)cf, r = (int64_t)rf;
    double fu = u - cf, fv = v - rf;
    double s0 = mix(tap(st, s, r, c), tap(st, s, r, c + 1), fu);
    double s1 = mix(tap(st, s, r + 1, c), tap(st, s, r + 1, c + 1), fu);
    return mix(s0, s1, fv);
}

/* dot4 of Listing 2 with the homogeneous 1 implicit. */
static double dot4(const double *row, double x, double y, double z)
{
    return row[0] * x + row[1] * y + row[2] * z + row[3];
}

typedef struct {
    int64_t nx, ny, nz;
    double dx, dy, dz, cx, cy, cz;
} volgeom_t;

static double vx(const volgeom_t *g, int64_t i) { return ((double)i - 0.5 * (double)(g->nx - 1)) * g->dx + g->cx; }
static double vy(const volgeom_t *g, int64_t j) { return ((double)j - 0.5 * (double)(g->ny - 1)) * g->dy + g->cy; }
static double vz(const volgeom_t *g, int64_t k) { return ((double)k - 0.5 * (double)(g->nz - 1)) * g->dz + g->cz; }

/* One voxel, one view, matrix mode: the body of Listing 1. */
static double update_matrix(const stack_t_ *st, const double *mat, int64_t s,
                            double X, double Y, double Z)
{
    const double *m = mat + 12 * s;
    double z = dot4(m + 8, X, Y, Z);
    double f = 1.0 / z;
    double x = dot4(m + 0, X, Y, Z) * f;
    double y = dot4(m + 4, X, Y, Z) * f;
    double val = bilinear(st, s, x, y);
    double w = f * f;
    return val * w;
}

static void fill_stack(stack_t_ *st, int64_t nh, int64_t nw, const float *p32,
                       const uint16_t *p16, const float *scale)
{
    st->f32 = p32; st->f16 = p16; st->scale = scale; st->nh = nh; st->nw = nw;
}

/* ---- back-projection, matrix mode, Listing-1 loop order ---------------- */
/* mats: [np][3][4] world-mm -> homogeneous pixel.  vol: [nz][ny][nx] += .   */
int oracle_bp(int64_t nx, int64_t ny, int64_t nz,
              double dx, double dy, double dz, double cx, double cy, double cz,
              int64_t np, int64_t nh, int64_t nw,
              const float *p32, const uint16_t *p16, const float *scale,
              const double *mats, double *vol, int nthreads)
{
    volgeom_t g = {nx, ny, nz, dx, dy, dz, cx, cy, cz};
    stack_t_ st; fill_stack(&st, nh, nw, p32, p16, scale);
    if (nthreads > 0) omp_set_num_threads(nthreads);
    for (int64_t s = 0; s < np; s++) {
        #pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nz; k++)
            for (int64_t j = 0; j < ny; j++)
                for (int64_t i = 0; i < nx; i++)
                    vol[(k * ny + j) * nx + i] +=
                        update_matrix(&st, mats, s, vx(&g, i), vy(&g, j), vz(&g, k));
    }
    return 0;
}

/* ---- back-projection of selected voxels (same arithmetic) -------------- */
/* ijk: [n][3] voxel indices (i, j, k); out[n] = full sum over all views.
 * Views are summed in order s = 0..np-1 for every voxel, as above.          */
int oracle_bp_points(int64_t nx, int64_t ny, int64_t nz,
                     double dx, double dy, double dz, double cx, double cy, double cz,
                     int64_t np, int64_t nh, int64_t nw,
                     const float *p32, const uint16_t *p16, const float *scale,
                     const double *mats, int64_t n, const int64_t *ijk,
                     double *out, int nthreads)
{
    volgeom_t g = {nx, ny, nz, dx, dy, dz, cx, cy, cz};
    stack_t_ st; fill_stack(&st, nh, nw, p32, p16, scale);
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t q = 0; q < n; q++) {
        double X = vx(&g, ijk[3 * q]), Y = vy(&g, ijk[3 * q + 1]), Z = vz(&g, ijk[3 * q + 2]);
        double acc = 0.0;
        for (int64_t s = 0; s < np; s++)
            acc += update_matrix(&st, mats, s, X, Y, Z);
        out[q] = acc;
    }
    return 0;
}

/* ---- back-projection of an axis-aligned sub-block ----------------------- */
/* out: [k1-k0][j1-j0][i1-i0] += contributions of all views.                 */
int oracle_bp_block(int64_t nx, int64_t ny, int64_t nz,
                    double dx, double dy, double dz, double cx, double cy, double cz,
                    int64_t np, int64_t nh, int64_t nw,
                    const float *p32, const uint16_t *p16, const float *scale,
                    const double *mats,
                    int64_t i0, int64_t i1, int64_t j0, int64_t j1, int64_t k0, int64_t k1,
                    double *out, int nthreads)
{
    volgeom_t g = {nx, ny, nz, dx, dy, dz, cx, cy, cz};
    stack_t_ st; fill_stack(&st, nh, nw, p32, p16, scale);
    int64_t bx = i1 - i0, by = j1 - j0;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    for (int64_t s = 0; s < np; s++) {
        #pragma omp parallel for schedule(static)
        for (int64_t k = k0; k < k1; k++)
            for (int64_t j = j0; j < j1; j++)
                for (int64_t i = i0; i < i1; i++)
                    out[((k - k0) * by + (j - j0)) * bx + (i - i0)] +=
                        update_matrix(&st, mats, s, vx(&g, i), vy(&g, j), vz(&g, k));
    }
    return 0;
}

/* ---- back-projection, matrix mode, Algorithm-1 order (hoisted) ---------- */
/* For every column (i, j) and view s the depth w and the detector column u
 * are computed once and shared along k (Section 3.1.2, Algorithm 1); only
 * v is recomputed per k.  The value equals oracle_bp in exact arithmetic
 * provided the matrix has no k-dependence in rows 0 and 2 (the detector's
 * V-axis is parallel to the rotation axis, Section 2.1.1).                  */
int oracle_bp_hoisted(int64_t nx, int64_t ny, int64_t nz,
                      double dx, double dy, double dz, double cx, double cy, double cz,
                      int64_t np, int64_t nh, int64_t nw,
                      const float *p32, const uint16_t *p16, const float *scale,
                      const double *mats, double *vol, int nthreads)
{
    volgeom_t g = {nx, ny, nz, dx, dy, dz, cx, cy, cz};
    stack_t_ st; fill_stack(&st, nh, nw, p32, p16, scale);
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for collapse(2) schedule(static)
    for (int64_t j = 0; j < ny; j++)
        for (int64_t i = 0; i < nx; i++) {
            double X = vx(&g, i), Y = vy(&g, j);
            for (int64_t s = 0; s < np; s++) {
                const double *m = mats + 12 * s;
                double F = 1.0 / dot4(m + 8, X, Y, 0.0);     /* row 2, k-free */
                double W = F * F;
                double U = dot4(m + 0, X, Y, 0.0) * F;       /* row 0, k-free */
                for (int64_t k = 0; k < nz; k++) {
                    double V = dot4(m + 4, X, Y, vz(&g, k)) * F;
                    vol[(k * ny + j) * nx + i] += bilinear(&st, s, U, V) * W;
                }
            }
        }
    return 0;
}

/* ---- back-projection, geometry mode (no matrices) ----------------------- */
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
                             double cu, double cv, double X, double Y, double Z,
                             double *u, double *v, double *w)
{
    double ct = cos(th), st_ = sin(th);
    double S[3] = {sod * ct, sod * st_, 0.0};
    double C[3] = {-(sdd - sod) * ct, -(sdd - sod) * st_, 0.0};
    double n[3] = {ct, st_, 0.0};                 /* unit normal, source side */
    double eu[3] = {-st_, ct, 0.0}, ev[3] = {0.0, 0.0, 1.0};
    double d[3] = {X - S[0], Y - S[1], Z - S[2]};
    double nd = n[0] * d[0] + n[1] * d[1] + n[2] * d[2];
    double ncs = n[0] * (C[0] - S[0]) + n[1] * (C[1] - S[1]) + n[2] * (C[2] - S[2]);
    double lam = ncs / nd;
    double H[3] = {S[0] + lam * d[0] - C[0], S[1] + lam * d[1] - C[1], S[2] + lam * d[2] - C[2]};
    double umm = eu[0] * H[0] + eu[1] * H[1] + eu[2] * H[2];
    double vmm = ev[0] * H[0] + ev[1] * H[1] + ev[2] * H[2];
    *u = umm / du + cu;
    *v = vmm / dv + cv;
    *w = (n[0] * (S[0] - X) + n[1] * (S[1] - Y) + n[2] * (S[2] - Z)) / sod;
}

int oracle_bp_geometry(int64_t nx, int64_t ny, int64_t nz,
                       double dx, double dy, double dz, double cx, double cy, double cz,
                       int64_t np, int64_t nh, int64_t nw,
                       const float *p32, const uint16_t *p16, const float *scale,
                       double arc, double theta0, double sod, double sdd,
                       double du, double dv, double u_off, double v_off,
                       double *vol, int nthreads)
{
    volgeom_t g = {nx, ny, nz, dx, dy, dz, cx, cy, cz};
    stack_t_ st; fill_stack(&st, nh, nw, p32, p16, scale);
    double cu = 0.5 * (double)(nw - 1) + u_off, cv = 0.5 * (double)(nh - 1) + v_off;
    if (nthreads > 0) omp_set_num_threads(nthreads);
    for (int64_t s = 0; s < np; s++) {
        double th = theta0 + arc * (double)s / (double)np;
        #pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < nz; k++)
            for (int64_t j = 0; j < ny; j++)
                for (int64_t i = 0; i < nx; i++) {
                    double u, v, w;
                    project_geometry(th, sod, sdd, du, dv, cu, cv, vx(&g, i), vy(&g, j), vz(&g, k), &u, &v, &w);
                    vol[(k * ny + j) * nx + i] += bilinear(&st, s, u, v) / (w * w);
                }
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
        project_geometry(th, sod, sdd, du, dv, cu, cv, xyz[3 * q], xyz[3 * q + 1], xyz[3 * q + 2],
                         &out[3 * q], &out[3 * q + 1], &out[3 * q + 2]);
    return 0;
}

/* ---- forward projection: the exact transpose of oracle_bp -------------- */
/* proj[s][r][c] += sum over voxels of vol * (1/w^2) * (bilinear weight of
 * tap (r, c) at the voxel's (u, v)); taps outside the detector are dropped,
 * exactly mirroring the zero extension of the back-projection.            */
int oracle_fp(int64_t nx, int64_t ny, int64_t nz,
              double dx, double dy, double dz, double cx, double cy, double cz,
              int64_t np, int64_t nh, int64_t nw,
              const double *vol, const double *mats, double *proj, int nthreads)
{
    volgeom_t g = {nx, ny, nz, dx, dy, dz, cx, cy, cz};
    if (nthreads > 0) omp_set_num_threads(nthreads);
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < np; s++) {
        const double *m = mats + 12 * s;
        double *P = proj + s * nh * nw;
        for (int64_t k = 0; k < nz; k++)
            for (int64_t j = 0; j < ny; j++)
                for (int64_t i = 0; i < nx; i++) {
                    double X = vx(&g, i), Y = vy(&g, j), Z = vz(&g, k);
                    double f = 1.0 / dot4(m + 8, X, Y, Z);
                    double u = dot4(m + 0, X, Y, Z) * f;
                    double v = dot4(m + 4, X, Y, Z) * f;
                    if (!(u > -2.0 && u < (double)nw + 1.0 && v > -2.0 && v < (double)nh + 1.0))
                        continue;
                    double cf = floor(u), rf = floor(v);
                    int64_t c = (int64_t)cf, r = (int64_t)rf;
                    double fu = u - cf, fv = v - rf;
                    double x = vol[(k * ny + j) * nx + i] * f * f;
                    double wt[4] = {(1 - fu) * (1 - fv), fu * (1 - fv), (1 - fu) * fv, fu * fv};
                    int64_t rr[4] = {r, r, r + 1, r + 1}, cc[4] = {c, c + 1, c, c + 1};
                    for (int t = 0; t < 4; t++)
                        if (rr[t] >= 0 && rr[t] < nh && cc[t] >= 0 && cc[t] < nw)
                            P[rr[t] * nw + cc[t]] += x * wt[t];
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
