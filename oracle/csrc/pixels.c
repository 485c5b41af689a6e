/* w-stacking dirty image at chosen pixels only -- TEST INFRASTRUCTURE ONLY.
 *
 * Used to check the full-size workloads, where the whole float64 pipeline
 * does not fit a test's time budget.  For a pixel (p, q) the gridded planes,
 * their inverse DFT and the phase screen collapse to one pass over the
 * visibilities, because the kernel is separable:
 *
 *   F_k[q][p] = sum_{j in plane k} A_j  X_j(p) Y_j(q),
 *   X_j(p)    = sum_t g_{s_x}[t] exp(+2 pi i (c_x + t - h - N/2)(p - N/2) / N)
 *   I[q][p]   = n_pq sum_k Re(exp(+2 pi i w_k (n_pq - 1)) F_k[q][p]) / (C_p C_q sum W)
 *
 * which is the same sum as gridding onto the cells, transforming and
 * screening, taken in another order.  The per-visibility position, plane and
 * drop decisions repeat the float64 steps of the Python oracle operation by
 * operation (no contraction, round-half-even, floor division).
 * exp(2 pi i j / N) for integer j is read from a table built with the exact
 * integer residue j mod N.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "decide.h"

/* Returns the number of kept visibilities; acc must hold npix * nw complex
 * (re, im interleaved) and is overwritten; *sum_w receives sum W. */
int64_t oracle_wstack_pixels(
    int64_t nrow, int32_t nchan, const double *uvw, const double *scales /* or NULL */,
    const float *vis /* re,im pairs [nrow][nchan] */, const float *weight /* or NULL */,
    int32_t grid_n, int32_t nw, int32_t support, int32_t oversample, double fov,
    double w_min, double dw, const double *table /* [OS][W] */,
    int64_t npix, const int32_t *pix_p, const int32_t *pix_q,
    double *acc /* [npix][nw][2] */, double *sum_w_out)
{
    const int64_t N = grid_n, OS = oversample, h = (support - 1) / 2;
    const double two_pi = 6.283185307179586476925286766559;
    double *cs = (double *)malloc(sizeof(double) * 2 * N);
    for (int64_t j = 0; j < N; ++j) {
        cs[2 * j] = cos(two_pi * (double)j / (double)N);
        cs[2 * j + 1] = sin(two_pi * (double)j / (double)N);
    }
    /* X_j(p) depends on the pixel column only and Y_j(q) on the row only:
     * they are evaluated once per distinct column and row of the requested
     * pixels (ux[], uy[]), and each pixel multiplies its pair. */
    int32_t *col_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(npix > 0 ? npix : 1));
    int32_t *row_of = (int32_t *)malloc(sizeof(int32_t) * (size_t)(npix > 0 ? npix : 1));
    int64_t *ux = (int64_t *)malloc(sizeof(int64_t) * (size_t)(npix > 0 ? npix : 1));
    int64_t *uy = (int64_t *)malloc(sizeof(int64_t) * (size_t)(npix > 0 ? npix : 1));
    int64_t nux = 0, nuy = 0;
    for (int64_t ip = 0; ip < npix; ++ip) {
        int64_t a = 0, b = 0;
        while (a < nux && ux[a] != pix_p[ip]) ++a;
        if (a == nux) ux[nux++] = pix_p[ip];
        while (b < nuy && uy[b] != pix_q[ip]) ++b;
        if (b == nuy) uy[nuy++] = pix_q[ip];
        col_of[ip] = (int32_t)a;
        row_of[ip] = (int32_t)b;
    }
    memset(acc, 0, sizeof(double) * 2 * npix * nw);
    int64_t kept_total = 0;
    double sumw_total = 0.0;
    #pragma omp parallel
    {
        double *lacc = (double *)calloc((size_t)(2 * npix * nw), sizeof(double));
        double *X = (double *)malloc(sizeof(double) * 2 * (size_t)(nux > 0 ? nux : 1));
        double *Y = (double *)malloc(sizeof(double) * 2 * (size_t)(nuy > 0 ? nuy : 1));
        int64_t kept = 0;
        double sumw = 0.0;
        #pragma omp for schedule(static)
        for (int64_t r = 0; r < nrow; ++r) {
            for (int32_t c = 0; c < nchan; ++c) {
                oracle_vis_t o;
                if (!oracle_decide(r, c, nchan, uvw, scales, vis, weight, N, OS, h, nw, fov, w_min, dw, &o))
                    continue;
                const int64_t cx = o.cx, cy = o.cy, sx = o.sx, sy = o.sy, k = o.k;
                ++kept;
                sumw += o.wt;
                const double ar = o.ar, ai = o.ai;
                const double *gx = table + (sx + OS / 2) * support;
                const double *gy = table + (sy + OS / 2) * support;
                /* residue of (cell - N/2) * (pixel - N/2) modulo N, tap by tap:
                 * the first tap's residue exactly, then + (pixel - N/2) per tap */
                for (int64_t a = 0; a < nux; ++a) {
                    const int64_t pp = ux[a] - N / 2;
                    const int64_t step = ((pp % N) + N) % N;
                    int64_t jx = ((cx - h - N / 2) * pp) % N; if (jx < 0) jx += N;
                    double xr = 0, xi = 0;
                    for (int64_t t = 0; t < support; ++t) {
                        xr += gx[t] * cs[2 * jx]; xi += gx[t] * cs[2 * jx + 1];
                        jx += step; if (jx >= N) jx -= N;
                    }
                    X[2 * a] = xr; X[2 * a + 1] = xi;
                }
                for (int64_t b = 0; b < nuy; ++b) {
                    const int64_t qq = uy[b] - N / 2;
                    const int64_t step = ((qq % N) + N) % N;
                    int64_t jy = ((cy - h - N / 2) * qq) % N; if (jy < 0) jy += N;
                    double yr = 0, yi = 0;
                    for (int64_t t = 0; t < support; ++t) {
                        yr += gy[t] * cs[2 * jy]; yi += gy[t] * cs[2 * jy + 1];
                        jy += step; if (jy >= N) jy -= N;
                    }
                    Y[2 * b] = yr; Y[2 * b + 1] = yi;
                }
                for (int64_t ip = 0; ip < npix; ++ip) {
                    const double xr = X[2 * col_of[ip]], xi = X[2 * col_of[ip] + 1];
                    const double yr = Y[2 * row_of[ip]], yi = Y[2 * row_of[ip] + 1];
                    const double er = xr * yr - xi * yi, ei = xr * yi + xi * yr;
                    double *dst = lacc + 2 * (ip * nw + k);
                    dst[0] += ar * er - ai * ei;
                    dst[1] += ar * ei + ai * er;
                }
            }
        }
        #pragma omp critical
        {
            for (int64_t i = 0; i < 2 * npix * nw; ++i) acc[i] += lacc[i];
            kept_total += kept;
            sumw_total += sumw;
        }
        free(lacc);
        free(X);
        free(Y);
    }
    free(col_of);
    free(row_of);
    free(ux);
    free(uy);
    free(cs);
    *sum_w_out = sumw_total;
    return kept_total;
}
