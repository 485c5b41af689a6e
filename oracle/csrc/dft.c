/* Direct Fourier sum over measured visibilities -- TEST INFRASTRUCTURE ONLY.
 *
 * For every requested sky direction (l, m) with n - 1 = nm1 this computes
 *     D(l, m) = sum_j  A_j * exp(+2 pi i (u_j l + v_j m + w_j nm1))
 * in float64, with A_j = W_j V_j the weighted visibility and (u, v, w) in
 * wavelengths.  This is the imaging relation of Eq. 1 with the integral over
 * (u, v, w) replaced by the sum over the measured samples; the caller turns
 * Re(D) into the dirty image by multiplying by n and dividing by sum W.
 *
 * The phase is formed in turns and reduced by its nearest integer before the
 * trigonometric call.  Pixels are shared out over OpenMP threads; each pixel
 * sums its terms in index order (or reversed, for the order-independence
 * check).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>

void oracle_dft(int64_t nvis, const double *u, const double *v, const double *w,
                const double *are, const double *aim,
                int64_t npix, const double *l, const double *m, const double *nm1,
                int reverse, double *out_re, double *out_im)
{
    const double two_pi = 6.283185307179586476925286766559;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t p = 0; p < npix; ++p) {
        const double lp = l[p], mp = m[p], np1 = nm1[p];
        double sr = 0.0, si = 0.0;
        for (int64_t jj = 0; jj < nvis; ++jj) {
            const int64_t j = reverse ? nvis - 1 - jj : jj;
            double ph = u[j] * lp + v[j] * mp + w[j] * np1;
            ph -= rint(ph);
            const double c = cos(two_pi * ph), s = sin(two_pi * ph);
            sr += are[j] * c - aim[j] * s;
            si += are[j] * s + aim[j] * c;
        }
        out_re[p] = sr;
        out_im[p] = si;
    }
}

/* The same direct sum for visibilities laid out [row][channel] with equally
 * spaced channels, uvw in metres.  Visibility (r, c) sits at
 * (u, v, w) = uvw_r * s_c in wavelengths, s_c = s0 + c ds, so its phase at
 * direction (l, m, nm1) is phi_r s_c with phi_r = uvw_r . (l, m, nm1), and
 *     exp(+2 pi i phi_r s_c) = exp(+2 pi i phi_r s0) * exp(+2 pi i phi_r ds)^c,
 * a geometric progression over the channels of a row (two trigonometric
 * calls per row instead of one per visibility; the rounding it adds grows by
 * about one ulp per channel).  A_rc = W_rc V_rc with V complex64 and W
 * float32 (NULL = 1).  Rows are shared out over OpenMP threads in contiguous
 * ranges; each thread keeps its own partial sum of every pixel and the
 * partial sums are added in thread order.
 */
void oracle_dft_rows(int64_t nrow, int32_t nchan, const double *uvw, double s0, double ds,
                     const float *vis, const float *weight,
                     int64_t npix, const double *l, const double *m, const double *nm1,
                     double *out_re, double *out_im)
{
    const double two_pi = 6.283185307179586476925286766559;
    for (int64_t p = 0; p < npix; ++p) out_re[p] = out_im[p] = 0.0;
    #pragma omp parallel
    {
        double *acc = (double *)calloc((size_t)(2 * npix), sizeof(double));
        #pragma omp for schedule(static)
        for (int64_t r = 0; r < nrow; ++r) {
            const double *x = uvw + 3 * r;
            for (int64_t p = 0; p < npix; ++p) {
                const double phi = x[0] * l[p] + x[1] * m[p] + x[2] * nm1[p];
                double t0 = phi * s0, td = phi * ds;
                t0 -= rint(t0);
                td -= rint(td);
                const double dr = cos(two_pi * td), di = sin(two_pi * td);
                double zr = cos(two_pi * t0), zi = sin(two_pi * t0);
                double sr = 0.0, si = 0.0;
                for (int32_t c = 0; c < nchan; ++c) {
                    const int64_t j = r * nchan + c;
                    const double wt = weight ? (double)weight[j] : 1.0;
                    const double ar = wt * (double)vis[2 * j], ai = wt * (double)vis[2 * j + 1];
                    sr += ar * zr - ai * zi;
                    si += ar * zi + ai * zr;
                    const double nr = zr * dr - zi * di;
                    zi = zr * di + zi * dr;
                    zr = nr;
                }
                acc[2 * p] += sr;
                acc[2 * p + 1] += si;
            }
        }
        #pragma omp for ordered schedule(static, 1)
        for (int t = 0; t < omp_get_num_threads(); ++t) {
            #pragma omp ordered
            for (int64_t p = 0; p < npix; ++p) {
                out_re[p] += acc[2 * p];
                out_im[p] += acc[2 * p + 1];
            }
        }
        free(acc);
    }
}
