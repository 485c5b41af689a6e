// w-correction and reduction of the w-planes into the image (Sec. 2.1,
// Eq. 1), fused with the final normalisation:
//   I[q][p] = n_pq sum_k Re(exp(+2 pi i w_k (n_pq - 1)) F_k[q][p]) / (C(l'_p) C(l'_q) sum W)
//
// One thread per pixel walks the planes (each plane read is row-coalesced,
// so the mesh is read exactly once).  n - 1 = -r^2 / (1 + sqrt(1 - r^2)) and
// the phase tau = w_k (n - 1) in turns are formed in float64; tau is reduced
// to tau - rint(tau) in [-1/2, 1/2] before the trigonometric evaluation,
// which then runs in the plane sum's precision (sincospi of 2 tau).  The
// plane sum is plain or compensated (Kahan); normalisation is float64.
#include "rick_internal.h"

namespace rick {

namespace {

constexpr int kScreenBlock = 256;

template <typename real>
struct R2T;
template <>
struct R2T<float> {
    using t = float2;
};
template <>
struct R2T<double> {
    using t = double2;
};

__device__ __forceinline__ void sincospi_r(float x, float *s, float *c) { sincospif(x, s, c); }
__device__ __forceinline__ void sincospi_r(double x, double *s, double *c) { sincospi(x, s, c); }

template <typename real, bool KAHAN>
__global__ __launch_bounds__(kScreenBlock) void k_wscreen(Geom g, const real *__restrict__ mesh,
                                                          const double *__restrict__ corr,
                                                          const Stats *__restrict__ st, real *__restrict__ image) {
    using C = typename R2T<real>::t;
    const int64_t npix = (int64_t)g.N * g.N;
    const int64_t pix = (int64_t)blockIdx.x * kScreenBlock + threadIdx.x;
    if (pix >= npix) return;
    const int q = (int)(pix / g.N), p = (int)(pix % g.N);
    const double dl = g.fov / g.N;
    const double l = (double)(p - g.N / 2) * dl;
    const double m = (double)(q - g.N / 2) * dl;
    const double r2 = l * l + m * m;
    if (!(r2 < 1.0)) {
        image[pix] = 0;
        return;
    }
    const double nm1 = -r2 / (1.0 + sqrt(1.0 - r2));
    const C *f = reinterpret_cast<const C *>(mesh) + pix;
    real sum = 0, comp = 0;
#pragma unroll 4
    for (int k = 0; k < g.Nw; ++k) {
        const C v = f[(int64_t)k * npix];
        const double tau = plane_centre(g, k) * nm1;
        const double tr = tau - rint(tau);
        real sn, cs;
        sincospi_r((real)(2.0 * tr), &sn, &cs);
        const real term = cs * v.x - sn * v.y;
        if (KAHAN) {
            const real y = term - comp;
            const real t = sum + y;
            comp = (t - sum) - y;
            sum = t;
        } else {
            sum += term;
        }
    }
    const double sw = st->sum_w;
    const double val = sw > 0.0 ? (1.0 + nm1) * (double)sum / (taper_at(g, corr, q, p) * sw) : 0.0;
    image[pix] = (real)val;
}

}  // namespace

template <typename real>
hipError_t launch_wscreen(const Geom &g, const real *mesh, const double *corr, const Stats *st, real *image,
                          int kahan, hipStream_t s) {
    const int64_t npix = (int64_t)g.N * g.N;
    const unsigned blocks = (unsigned)((npix + kScreenBlock - 1) / kScreenBlock);
    if (kahan)
        hipLaunchKernelGGL((k_wscreen<real, true>), dim3(blocks), dim3(kScreenBlock), 0, s, g, mesh, corr, st, image);
    else
        hipLaunchKernelGGL((k_wscreen<real, false>), dim3(blocks), dim3(kScreenBlock), 0, s, g, mesh, corr, st,
                           image);
    return hipGetLastError();
}

template hipError_t launch_wscreen<float>(const Geom &, const float *, const double *, const Stats *, float *, int,
                                          hipStream_t);
template hipError_t launch_wscreen<double>(const Geom &, const double *, const double *, const Stats *, double *, int,
                                           hipStream_t);

}  // namespace rick
