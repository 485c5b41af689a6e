/* Whole-input statistics of the oracle's binning -- TEST INFRASTRUCTURE ONLY.
 *
 * For every kept visibility (decisions as in oracle/wstack.py): count one
 * record in the (plane, tile) bin holding the top-left cell (c - h) of its
 * W x W footprint, and add W V to its plane's sum (the sum of a plane's
 * gridded cells equals it, because tap rows sum to 1).  Linear in the number
 * of visibilities, for full-size checks.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "decide.h"

int64_t oracle_bin_stats(int64_t nrow, int32_t nchan, const double *uvw, const double *scales,
                         const float *vis, const float *weight, int32_t grid_n, int32_t nw, int32_t support,
                         int32_t oversample, double fov, double w_min, double dw, int32_t tile,
                         int64_t *counts /* [nw * nt * nt] */, double *plane_sum /* [nw][2] */,
                         double *sum_w_out)
{
    const int64_t N = grid_n, OS = oversample, h = (support - 1) / 2, T = tile, nt = grid_n / tile;
    const int64_t nbins = (int64_t)nw * nt * nt;
    memset(counts, 0, sizeof(int64_t) * nbins);
    memset(plane_sum, 0, sizeof(double) * 2 * nw);
    int64_t kept_total = 0;
    double sumw_total = 0.0;
    #pragma omp parallel
    {
        int64_t *lc = (int64_t *)calloc((size_t)nbins, sizeof(int64_t));
        double *lp = (double *)calloc((size_t)(2 * nw), sizeof(double));
        int64_t kept = 0;
        double sumw = 0.0;
        #pragma omp for schedule(static)
        for (int64_t r = 0; r < nrow; ++r) {
            for (int32_t c = 0; c < nchan; ++c) {
                oracle_vis_t o;
                if (!oracle_decide(r, c, nchan, uvw, scales, vis, weight, N, OS, h, nw, fov, w_min, dw, &o))
                    continue;
                ++kept;
                sumw += o.wt;
                lp[2 * o.k] += o.ar;
                lp[2 * o.k + 1] += o.ai;
                const int64_t tx = (o.cx - h) / T, ty = (o.cy - h) / T;   /* kept: c - h >= 0 */
                lc[(o.k * nt + ty) * nt + tx] += 1;
            }
        }
        #pragma omp critical
        {
            for (int64_t i = 0; i < nbins; ++i) counts[i] += lc[i];
            for (int64_t i = 0; i < 2 * nw; ++i) plane_sum[i] += lp[i];
            kept_total += kept;
            sumw_total += sumw;
        }
        free(lc);
        free(lp);
    }
    *sum_w_out = sumw_total;
    return kept_total;
}
