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
#include <stdint.h>

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
