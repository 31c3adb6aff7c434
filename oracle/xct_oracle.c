/*
 * FP64 CPU oracle for per-slice parallel-beam filtered back-projection.
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct: every function is
 * the definition written out in double precision with plain loops (OpenMP only
 * spreads independent rows / pixels / angles over cores).  It shares no code
 * with the HIP library and is never called by it; only the tests, the smoke
 * check and the benchmark's CPU-baseline leg use it.
 *
 * The paper (Section IV-B; Section V-A c, stage 2) describes FBP only in words:
 * filter every projection row with a ramp-type filter (Kak & Slaney), then
 * back-project the filtered rows into the slice, at cost O(N_p N_x N_y) per
 * slice.  The concrete operator computed here fixes the conventions the paper
 * leaves open:
 *
 *   geometry   x_j = (j - (N_x-1)/2) pix,  y_i = (i - (N_y-1)/2) pix,
 *              u_k(x, y) = (x cos th_k + y sin th_k) / pitch + center   [bins]
 *   hat        K(t) = max(0, 1 - |t|)       (linear detector interpolation)
 *   filter     q[k][n] = (1/pitch) sum_{m=0}^{N_c-1} h_W[n - m] p[k][m]
 *              (linear convolution, row zero outside the detector)
 *   kernels    inverse DTFT of |nu| W(nu) on |nu| <= 1/2:
 *                Ram-Lak      h[0] = 1/4, h[even] = 0, h[odd n] = -1/(pi^2 n^2)
 *                Shepp-Logan  h[n] = 2 / (pi^2 (1 - 4 n^2))        (W = sinc)
 *                Hann         h[n] = h_RL[n]/2 + (h_RL[n-1] + h_RL[n+1])/4
 *   back-proj  f[i][j] = w sum_k sum_n q[k][n] K(u_k(x_j, y_i) - n)
 *   forward    (P x)[k][n] = (pix^2 / pitch) sum_{i,j} x[i][j] K(u_k(x_j, y_i) - n)
 *
 * Because K is a hat, at most two bins n = floor(u), floor(u)+1 carry weight
 * for a given u; the loops below visit exactly those two and skip bins outside
 * [0, N_c) (zero extension, not clamping).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

enum { ORACLE_RAM_LAK = 0, ORACLE_SHEPP_LOGAN = 1, ORACLE_HANN = 2 };

static double ram_lak_tap(long n)
{
    if (n == 0) return 0.25;
    if (n % 2 == 0) return 0.0;
    return -1.0 / (M_PI * M_PI * (double)n * (double)n);
}

/* Tap h_W[n] of the spatial ramp kernel for window W (see header). */
double oracle_kernel_tap(int window, long n)
{
    switch (window) {
    case ORACLE_RAM_LAK:
        return ram_lak_tap(n);
    case ORACLE_SHEPP_LOGAN:
        return 2.0 / (M_PI * M_PI * (1.0 - 4.0 * (double)n * (double)n));
    case ORACLE_HANN:
        return 0.5 * ram_lak_tap(n) + 0.25 * (ram_lak_tap(n - 1) + ram_lak_tap(n + 1));
    default:
        return NAN;
    }
}

/* q = (1/pitch) h_W * p, row by row, direct linear convolution.
 * p, q: (rows, nc) row-major.  Returns 0, or -1 on a bad argument. */
int oracle_filter(const double *p, int64_t rows, int32_t nc, double pitch, int window,
                  double *q)
{
    if (!p || !q || rows < 0 || nc <= 0 || !(pitch > 0) || window < 0 || window > 2)
        return -1;
    double *h = (double *)malloc(sizeof(double) * (size_t)(2 * nc - 1));
    if (!h) return -1;
    for (long d = -(long)(nc - 1); d <= (long)(nc - 1); ++d)
        h[d + nc - 1] = oracle_kernel_tap(window, d);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < rows; ++r) {
        const double *pr = p + r * nc;
        double *qr = q + r * nc;
        for (long n = 0; n < nc; ++n) {
            double s = 0.0;
            for (long m = 0; m < nc; ++m) s += h[n - m + nc - 1] * pr[m];
            qr[n] = s / pitch;
        }
    }
    free(h);
    return 0;
}

/* Linear interpolation of the zero-extended row at detector coordinate u:
 * sum_n row[n] K(u - n) over the two bins with non-zero weight. */
static double row_at(const double *row, int32_t nc, double u)
{
    double fl = floor(u);
    long n0 = (long)fl;
    double t = u - fl;
    double a = (n0 >= 0 && n0 < nc) ? row[n0] : 0.0;
    double b = (n0 + 1 >= 0 && n0 + 1 < nc) ? row[n0 + 1] : 0.0;
    return (1.0 - t) * a + t * b;
}

typedef struct {
    int32_t n_angles, n_det, nx, ny;
    double pitch, pix, center;
    const double *angles;
} ogeom;

static int check_geom(const ogeom *g)
{
    if (!g || g->n_angles <= 0 || g->n_det <= 0 || g->nx <= 0 || g->ny <= 0) return -1;
    if (!(g->pitch > 0) || !(g->pix > 0) || !isfinite(g->center) || !g->angles) return -1;
    return 0;
}

/* f = w * A^T q for one slice; q (N_p, N_c), f (N_y, N_x). */
static void bp_slice(const ogeom *g, const double *q, const double *ct, const double *st,
                     double w, double *f)
{
    const int32_t npr = g->n_angles, nc = g->n_det, nx = g->nx, ny = g->ny;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < ny; ++i) {
        double y = (i - 0.5 * (ny - 1)) * g->pix;
        for (int32_t j = 0; j < nx; ++j) {
            double x = (j - 0.5 * (nx - 1)) * g->pix;
            double s = 0.0;
            for (int32_t k = 0; k < npr; ++k) {
                double u = (x * ct[k] + y * st[k]) / g->pitch + g->center;
                s += row_at(q + (int64_t)k * nc, nc, u);
            }
            f[(int64_t)i * nx + j] = w * s;
        }
    }
}

/* image[s] = w * A^T q[s] for every slice s.  Returns 0 or -1. */
int oracle_backproject(int32_t n_angles, int32_t n_det, int32_t nx, int32_t ny, double pitch,
                       double pix, double center, const double *angles, int32_t n_slices,
                       const double *q, double w, double *image)
{
    ogeom g = {n_angles, n_det, nx, ny, pitch, pix, center, angles};
    if (check_geom(&g) || n_slices < 0 || !q || !image) return -1;
    double *ct = (double *)malloc(sizeof(double) * (size_t)n_angles * 2);
    if (!ct) return -1;
    double *st = ct + n_angles;
    for (int32_t k = 0; k < n_angles; ++k) { ct[k] = cos(angles[k]); st[k] = sin(angles[k]); }
    for (int32_t s = 0; s < n_slices; ++s)
        bp_slice(&g, q + (int64_t)s * n_angles * n_det, ct, st, w, image + (int64_t)s * nx * ny);
    free(ct);
    return 0;
}

/* out[t] = w * (A^T q[slice_t])[row_t][col_t] for a list of pixels given as
 * (slice, row, col) triples.  Returns 0 or -1 (also for an index out of range). */
int oracle_backproject_pixels(int32_t n_angles, int32_t n_det, int32_t nx, int32_t ny,
                              double pitch, double pix, double center, const double *angles,
                              int32_t n_slices, const double *q, const int64_t *pixels,
                              int64_t n_pixels, double w, double *out)
{
    ogeom g = {n_angles, n_det, nx, ny, pitch, pix, center, angles};
    if (check_geom(&g) || n_slices < 0 || !q || !pixels || !out || n_pixels < 0) return -1;
    for (int64_t t = 0; t < n_pixels; ++t) {
        const int64_t *px = pixels + 3 * t;
        if (px[0] < 0 || px[0] >= n_slices || px[1] < 0 || px[1] >= ny || px[2] < 0 || px[2] >= nx)
            return -1;
    }
    double *ct = (double *)malloc(sizeof(double) * (size_t)n_angles * 2);
    if (!ct) return -1;
    double *st = ct + n_angles;
    for (int32_t k = 0; k < n_angles; ++k) { ct[k] = cos(angles[k]); st[k] = sin(angles[k]); }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_pixels; ++t) {
        const int64_t *px = pixels + 3 * t;
        const double *qs = q + px[0] * (int64_t)n_angles * n_det;
        double y = (px[1] - 0.5 * (ny - 1)) * pix;
        double x = (px[2] - 0.5 * (nx - 1)) * pix;
        double s = 0.0;
        for (int32_t k = 0; k < n_angles; ++k) {
            double u = (x * ct[k] + y * st[k]) / pitch + center;
            s += row_at(qs + (int64_t)k * n_det, n_det, u);
        }
        out[t] = w * s;
    }
    free(ct);
    return 0;
}

/* sino[s] = (pix^2/pitch) A image[s]: every pixel spreads its value onto the
 * two bins around u with the hat weights.  Parallel over angles, so each
 * thread owns whole sinogram rows.  Returns 0 or -1. */
int oracle_forward(int32_t n_angles, int32_t n_det, int32_t nx, int32_t ny, double pitch,
                   double pix, double center, const double *angles, int32_t n_slices,
                   const double *image, double *sino)
{
    ogeom g = {n_angles, n_det, nx, ny, pitch, pix, center, angles};
    if (check_geom(&g) || n_slices < 0 || !image || !sino) return -1;
    const double scale = pix * pix / pitch;
    for (int32_t s = 0; s < n_slices; ++s) {
        const double *img = image + (int64_t)s * nx * ny;
        double *sn = sino + (int64_t)s * n_angles * n_det;
#pragma omp parallel for schedule(static)
        for (int32_t k = 0; k < n_angles; ++k) {
            double *row = sn + (int64_t)k * n_det;
            memset(row, 0, sizeof(double) * (size_t)n_det);
            double ct = cos(angles[k]), st = sin(angles[k]);
            for (int32_t i = 0; i < ny; ++i) {
                double y = (i - 0.5 * (ny - 1)) * pix;
                for (int32_t j = 0; j < nx; ++j) {
                    double x = (j - 0.5 * (nx - 1)) * pix;
                    double u = (x * ct + y * st) / pitch + center;
                    double fl = floor(u);
                    long n0 = (long)fl;
                    double t = u - fl;
                    double v = scale * img[(int64_t)i * nx + j];
                    if (n0 >= 0 && n0 < n_det) row[n0] += (1.0 - t) * v;
                    if (n0 + 1 >= 0 && n0 + 1 < n_det) row[n0 + 1] += t * v;
                }
            }
        }
    }
    return 0;
}

int oracle_version(void) { return 1; }

/* Threads the OpenMP loops above use (the CPU baseline reports it). */
int oracle_threads(void)
{
    int n = 1;
#pragma omp parallel
    {
#pragma omp single
        n = omp_get_num_threads();
    }
    return n;
}
