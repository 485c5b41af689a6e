// Batched, centred 2-D inverse FFT of every w-plane (the FFT step of
// Sec. 2.1), in place in HBM, in two passes:
//   fft_rows  one block per row (or per few rows for small N): the row is
//             staged in LDS and transformed by Stockham autosort stages,
//   fft_cols  one block per strip of V adjacent columns of one plane: the
//             strip is staged in LDS as [row][V] and transformed likewise.
// Each pass reads and writes the mesh once (two HBM round trips in total).
//
// Stockham stage of radix R over L-point sub-transforms (n = N / R
// butterflies, butterfly b, k = b mod L):
//   a_j = x[b + j n] * w_{L R}^{j k},  A = DFT_R(a),  y[(b / L) L R + k + q L] = A_q
// with w_M = exp(+2 pi i / M); the first stage has radix 2 or 4 when log2 N
// is not a multiple of 3, the rest radix 8.  Twiddles come from a table of
// exp(+2 pi i m / N) computed in float64 on the host and rounded; a radix-8
// butterfly reads w, w^2, w^4 and forms w^3, w^5, w^6, w^7 as one product of
// two table entries each.
//
// Centring: for N divisible by 4,
//   sum_i x_i exp(+2 pi i (i - N/2)(p - N/2) / N) = (-1)^p sum_i (-1)^i x_i exp(+2 pi i i p / N),
// so each pass flips signs on load and on store.
//
// LDS element e is stored at e + e / 8, which keeps the stride-R writes of the
// early stages on distinct banks.
#include "rick_internal.h"

namespace rick {

namespace {

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

template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
template <typename C>
__device__ __forceinline__ C cmul(C a, C b) { return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
template <typename C>
__device__ __forceinline__ C mul_pi(C a) { return C{-a.y, a.x}; }   // * (+i)
template <typename C>
__device__ __forceinline__ C cneg_if(C a, bool n) { return n ? C{-a.x, -a.y} : a; }

// inverse DFT of size 2, 4, 8 in place (positive exponent), natural order out
template <typename C>
__device__ __forceinline__ void dft2(C &a0, C &a1) {
    const C t = a0;
    a0 = cadd(t, a1);
    a1 = csub(t, a1);
}
template <typename C>
__device__ __forceinline__ void dft4(C &a0, C &a1, C &a2, C &a3) {
    const C s02 = cadd(a0, a2), d02 = csub(a0, a2);
    const C s13 = cadd(a1, a3), d13 = mul_pi(csub(a1, a3));
    a0 = cadd(s02, s13);
    a2 = csub(s02, s13);
    a1 = cadd(d02, d13);
    a3 = csub(d02, d13);
}
template <typename C>
__device__ __forceinline__ void dft8(C *a) {
    using real = decltype(a[0].x);
    C e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
    C o0 = a[1], o1 = a[3], o2 = a[5], o3 = a[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    const real r = (real)0.70710678118654752440;
    // w8 = (1 + i)/sqrt2, w8^2 = i, w8^3 = (-1 + i)/sqrt2
    const C t1 = C{(o1.x - o1.y) * r, (o1.x + o1.y) * r};
    const C t2 = mul_pi(o2);
    const C t3 = C{(-o3.x - o3.y) * r, (o3.x - o3.y) * r};
    a[0] = cadd(e0, o0);
    a[4] = csub(e0, o0);
    a[1] = cadd(e1, t1);
    a[5] = csub(e1, t1);
    a[2] = cadd(e2, t2);
    a[6] = csub(e2, t2);
    a[3] = cadd(e3, t3);
    a[7] = csub(e3, t3);
}

template <int R, typename C>
__device__ __forceinline__ void dftR(C *a) {
    if constexpr (R == 2) dft2(a[0], a[1]);
    else if constexpr (R == 4) dft4(a[0], a[1], a[2], a[3]);
    else dft8(a);
}

__device__ __forceinline__ int padi(int e) { return e + (e >> 3); }

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

// One Stockham stage over V interleaved transforms held in LDS as
// buf[padi(e) * V + v].  Thread handles butterflies b = tb + i * NT for the
// vector lanes v in [v0, v0 + VC).
template <int N, int R, int V, int VC, int NT, typename C>
__device__ __forceinline__ void stage(C *buf, int L, int tb, int v0, const C *__restrict__ tw) {
    constexpr int NB = N / R;         // butterflies per transform
    constexpr int PER = NB / NT;      // butterflies per thread
    C a[PER][VC][R];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = tb + i * NT;
#pragma unroll
        for (int j = 0; j < R; ++j) {
#pragma unroll
            for (int v = 0; v < VC; ++v) a[i][v][j] = buf[padi(b + j * NB) * V + v0 + v];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int b = tb + i * NT;
        const int k = b & (L - 1);
        if (L > 1) {
            // w^j for j < R: w, w^2, w^4 from the table, the rest as one product
            // of two table entries each
            const int step = k * (N / (L * R));
            C wj[R];
            wj[1] = tw[step];
            if constexpr (R >= 4) {
                wj[2] = tw[2 * step];
                wj[3] = cmul(wj[1], wj[2]);
            }
            if constexpr (R == 8) {
                wj[4] = tw[4 * step];
                wj[5] = cmul(wj[1], wj[4]);
                wj[6] = cmul(wj[2], wj[4]);
                wj[7] = cmul(wj[3], wj[4]);
            }
#pragma unroll
            for (int j = 1; j < R; ++j) {
#pragma unroll
                for (int v = 0; v < VC; ++v) a[i][v][j] = cmul(a[i][v][j], wj[j]);
            }
        }
#pragma unroll
        for (int v = 0; v < VC; ++v) dftR<R>(a[i][v]);
        const int base = (b / L) * L * R + k;
#pragma unroll
        for (int q = 0; q < R; ++q) {
#pragma unroll
            for (int v = 0; v < VC; ++v) buf[padi(base + q * L) * V + v0 + v] = a[i][v][q];
        }
    }
    __syncthreads();
}

template <int N, int V, int VC, int NT, typename C>
__device__ __forceinline__ void fft_lds(C *buf, int tb, int v0, const C *__restrict__ tw) {
    constexpr int LG = ilog2c(N);
    constexpr int R0 = (LG % 3 == 0) ? 8 : (LG % 3 == 1 ? 2 : 4);
    int L = 1;
    stage<N, R0, V, VC, NT>(buf, L, tb, v0, tw);
    L *= R0;
#pragma unroll 1
    for (; L < N; L *= 8) stage<N, 8, V, VC, NT>(buf, L, tb, v0, tw);
}

// ---- rows: B rows per block, NT = N/8 threads per row ----
template <typename real, int N, int B>
__global__ __launch_bounds__((N / 8) * B) void k_fft_rows(real *__restrict__ mesh, const real *__restrict__ twr,
                                                         int64_t nrows) {
    using C = typename R2T<real>::t;
    constexpr int NT = N / 8;
    constexpr int PADN = N + N / 8;
    extern __shared__ __align__(16) unsigned char smem[];
    C *lds = reinterpret_cast<C *>(smem);
    const C *tw = reinterpret_cast<const C *>(twr);
    const int rb = threadIdx.x / NT, tb = threadIdx.x % NT;
    const int64_t row = (int64_t)blockIdx.x * B + rb;
    C *buf = lds + rb * PADN;
    C *g = reinterpret_cast<C *>(mesh) + row * N;
    const bool live = row < nrows;
    if (live) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = tb + i * NT;
            buf[padi(e)] = cneg_if(g[e], e & 1);
        }
    }
    __syncthreads();
    fft_lds<N, 1, 1, NT>(buf, tb, 0, tw);
    if (live) {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int e = tb + i * NT;
            g[e] = cneg_if(buf[padi(e)], e & 1);
        }
    }
}

// ---- columns: one block per (plane, strip of V columns); NT threads per column group ----
template <typename real, int N, int V, int VC>
__global__ __launch_bounds__((N / 8) * (V / VC)) void k_fft_cols(real *__restrict__ mesh,
                                                                 const real *__restrict__ twr, int32_t nw) {
    using C = typename R2T<real>::t;
    constexpr int NT = N / 8;
    constexpr int NTH = NT * (V / VC);
    constexpr int NSTRIP = N / V;
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);
    const C *tw = reinterpret_cast<const C *>(twr);
    // XCD-aware order: blocks are dealt to the 8 XCDs round-robin; give the
    // blocks that share an XCD adjacent strips so that they share L2 lines.
    const int64_t nblk = (int64_t)nw * NSTRIP;
    int64_t logical = blockIdx.x;
    if ((nblk & 7) == 0) logical = (int64_t)(blockIdx.x & 7) * (nblk >> 3) + (blockIdx.x >> 3);
    const int64_t plane = logical / NSTRIP;
    const int c0 = (int)(logical % NSTRIP) * V;
    C *g = reinterpret_cast<C *>(mesh) + plane * (int64_t)N * N + c0;
    for (int idx = threadIdx.x; idx < N * V; idx += NTH) {
        const int e = idx / V, v = idx % V;
        buf[padi(e) * V + v] = cneg_if(g[(int64_t)e * N + v], e & 1);
    }
    __syncthreads();
    const int tb = threadIdx.x % NT, v0 = (threadIdx.x / NT) * VC;
    fft_lds<N, V, VC, NT>(buf, tb, v0, tw);
    for (int idx = threadIdx.x; idx < N * V; idx += NTH) {
        const int e = idx / V, v = idx % V;
        g[(int64_t)e * N + v] = cneg_if(buf[padi(e) * V + v], e & 1);
    }
}

__device__ __forceinline__ void sincospi_r(float x, float *s, float *c) { sincospif(x, s, c); }
__device__ __forceinline__ void sincospi_r(double x, double *s, double *c) { sincospi(x, s, c); }

// ---- columns fused with the w-correction and the plane sum ----
// One block per strip of V columns loops over all planes: the strip of plane
// k (already transformed along rows) is staged in LDS and transformed along
// columns, and each thread adds Re(exp(+2 pi i w_k (n - 1)) F_k) for the
// pixels it owns; plane k + 1 is fetched into registers meanwhile.  The
// transformed planes are never written back, and the image is written once.
// Phase in float64 turns, reduced to [-1/2, 1/2] before sincospi, as in the
// stand-alone screen.
template <typename real, int N, int V, int VC, bool KAHAN>
__global__ __launch_bounds__((N / 8) * (V / VC)) void k_fft_cols_screen(Geom g, const real *__restrict__ mesh,
                                                                        const real *__restrict__ twr,
                                                                        const double *__restrict__ wk,
                                                                        const double *__restrict__ corr,
                                                                        const Stats *__restrict__ st,
                                                                        real *__restrict__ image) {
    using C = typename R2T<real>::t;
    constexpr int NT = N / 8;
    constexpr int NTH = NT * (V / VC);
    constexpr int NSTRIP = N / V;
    constexpr int PPT = N * V / NTH;   // pixels per thread
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);
    const C *tw = reinterpret_cast<const C *>(twr);
    int strip = blockIdx.x;
    if ((NSTRIP & 7) == 0) strip = (blockIdx.x & 7) * (NSTRIP >> 3) + (blockIdx.x >> 3);
    const int c0 = strip * V;
    const C *g0 = reinterpret_cast<const C *>(mesh) + c0;
    const int64_t plane_stride = (int64_t)N * N;
    const double dl = g.fov / N;
    // n - 1 of the strip's pixels, float64, in LDS after the strip buffer
    double *s_nm1 = reinterpret_cast<double *>(buf + (N + N / 8) * V);
    real acc[PPT], comp[PPT];
    C pre[PPT];
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int idx = threadIdx.x + NTH * i;
        const int e = idx / V, v = idx % V;
        const double l = (double)(c0 + v - N / 2) * dl, m = (double)(e - N / 2) * dl;
        const double r2 = l * l + m * m;
        s_nm1[idx] = r2 < 1.0 ? -r2 / (1.0 + sqrt(1.0 - r2)) : 0.0;
        acc[i] = 0;
        comp[i] = 0;
        pre[i] = g0[(int64_t)e * N + v];
    }
    const int tb = threadIdx.x % NT, v0 = (threadIdx.x / NT) * VC;
    for (int k = 0; k < g.Nw; ++k) {
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int idx = threadIdx.x + NTH * i;
            const int e = idx / V, v = idx % V;
            buf[padi(e) * V + v] = cneg_if(pre[i], e & 1);
        }
        __syncthreads();
        if (k + 1 < g.Nw) {
            const C *gk = g0 + (int64_t)(k + 1) * plane_stride;
#pragma unroll
            for (int i = 0; i < PPT; ++i) {
                const int idx = threadIdx.x + NTH * i;
                const int e = idx / V, v = idx % V;
                pre[i] = gk[(int64_t)e * N + v];
            }
        }
        fft_lds<N, V, VC, NT>(buf, tb, v0, tw);
        const double w = wk[k];
#pragma unroll
        for (int i = 0; i < PPT; ++i) {
            const int idx = threadIdx.x + NTH * i;
            const int e = idx / V, v = idx % V;
            const C f = cneg_if(buf[padi(e) * V + v], e & 1);
            const double tau = w * s_nm1[idx];
            const double tr = tau - rint(tau);
            real sn, cs;
            sincospi_r((real)(2.0 * tr), &sn, &cs);
            const real term = cs * f.x - sn * f.y;
            if (KAHAN) {
                const real y = term - comp[i];
                const real t = acc[i] + y;
                comp[i] = (t - acc[i]) - y;
                acc[i] = t;
            } else {
                acc[i] += term;
            }
        }
        __syncthreads();
    }
    const double sw = st->sum_w;
#pragma unroll
    for (int i = 0; i < PPT; ++i) {
        const int idx = threadIdx.x + NTH * i;
        const int e = idx / V, v = idx % V;
        const int p = c0 + v, q = e;
        const double l = (double)(p - N / 2) * dl, m = (double)(q - N / 2) * dl;
        const bool in_sky = l * l + m * m < 1.0;
        const double val =
            (sw > 0.0 && in_sky) ? (1.0 + s_nm1[idx]) * (double)acc[i] / (corr[p] * corr[q] * sw) : 0.0;
        image[(int64_t)q * N + p] = (real)val;
    }
}

template <typename real, int N>
hipError_t rows_n(const Geom &g, real *mesh, const real *tw, hipStream_t s) {
    using C = typename R2T<real>::t;
    constexpr int NT = N / 8;
    constexpr int B = NT >= 256 ? 1 : 256 / NT;
    const int64_t nrows = (int64_t)g.Nw * N;
    const size_t lds = size_t(B) * (N + N / 8) * sizeof(C);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_fft_rows<real, N, B>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
        attr = true;
    }
    hipLaunchKernelGGL((k_fft_rows<real, N, B>), dim3((unsigned)((nrows + B - 1) / B)), dim3(NT * B), lds, s, mesh,
                       tw, nrows);
    return hipGetLastError();
}

template <typename real, int N>
hipError_t cols_n(const Geom &g, real *mesh, const real *tw, hipStream_t s) {
    using C = typename R2T<real>::t;
    // V columns per block: the strip fills about 74 KB of LDS, so that two
    // blocks share a CU and one loads while the other computes (16 for small N)
    constexpr int VRAW = (8192 * 8 / (int)sizeof(C)) / N;
    constexpr int V = VRAW < 1 ? 1 : (VRAW > 16 ? 16 : VRAW);
    constexpr int NT = N / 8;
    constexpr int VC = (NT * V > 1024) ? (NT * V) / 1024 : 1;
    const size_t lds = size_t(N + N / 8) * V * sizeof(C);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_fft_cols<real, N, V, VC>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr = true;
    }
    const int64_t nblk = (int64_t)g.Nw * (N / V);
    hipLaunchKernelGGL((k_fft_cols<real, N, V, VC>), dim3((unsigned)nblk), dim3(NT * (V / VC)), lds, s, mesh, tw,
                       g.Nw);
    return hipGetLastError();
}

template <typename real, int N>
hipError_t cols_screen_n(const Geom &g, const real *mesh, const real *tw, const double *wk, const double *corr,
                         const Stats *st, real *image, int kahan, hipStream_t s) {
    using C = typename R2T<real>::t;
    // two columns per strip for N >= 4096 (one in float64 at 8192): a 74 KB strip
    // and eight pixels per thread of plane-sum state
    constexpr int VRAW = (8192 * 8 / (int)sizeof(C)) / N;
    constexpr int V = VRAW < 1 ? 1 : (VRAW > 16 ? 16 : VRAW);
    constexpr int NT = N / 8;
    constexpr int VC = (NT * V > 1024) ? (NT * V) / 1024 : 1;
    const size_t lds = size_t(N + N / 8) * V * sizeof(C) + size_t(N) * V * sizeof(double);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_fft_cols_screen<real, N, V, VC, false>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipFuncSetAttribute((const void *)k_fft_cols_screen<real, N, V, VC, true>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        attr = true;
    }
    if (kahan)
        hipLaunchKernelGGL((k_fft_cols_screen<real, N, V, VC, true>), dim3(N / V), dim3(NT * (V / VC)), lds, s, g,
                           mesh, tw, wk, corr, st, image);
    else
        hipLaunchKernelGGL((k_fft_cols_screen<real, N, V, VC, false>), dim3(N / V), dim3(NT * (V / VC)), lds, s, g,
                           mesh, tw, wk, corr, st, image);
    return hipGetLastError();
}

}  // namespace

bool fft_supported(int N) { return N >= 64 && N <= 8192 && (N & (N - 1)) == 0; }

size_t fused_screen_lds_bytes(int N, size_t real_bytes) {
    const int cbytes = (int)(2 * real_bytes);
    int v = (8192 * 8 / cbytes) / N;
    v = v < 1 ? 1 : (v > 16 ? 16 : v);
    return size_t(N + N / 8) * v * cbytes + size_t(N) * v * sizeof(double);
}

template <typename real>
hipError_t launch_fft_cols_screen(const Geom &g, const real *mesh, const real *tw, const double *wk,
                                  const double *corr, const Stats *st, real *image, int kahan, hipStream_t s) {
    switch (g.N) {
#define CASE(n) \
    case n: return cols_screen_n<real, n>(g, mesh, tw, wk, corr, st, image, kahan, s);
        CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096) CASE(8192)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_fft_cols_screen<float>(const Geom &, const float *, const float *, const double *,
                                                  const double *, const Stats *, float *, int, hipStream_t);
template hipError_t launch_fft_cols_screen<double>(const Geom &, const double *, const double *, const double *,
                                                   const double *, const Stats *, double *, int, hipStream_t);

template <typename real>
hipError_t launch_fft_rows(const Geom &g, real *mesh, const real *tw, hipStream_t s) {
    switch (g.N) {
        case 64: return rows_n<real, 64>(g, mesh, tw, s);
        case 128: return rows_n<real, 128>(g, mesh, tw, s);
        case 256: return rows_n<real, 256>(g, mesh, tw, s);
        case 512: return rows_n<real, 512>(g, mesh, tw, s);
        case 1024: return rows_n<real, 1024>(g, mesh, tw, s);
        case 2048: return rows_n<real, 2048>(g, mesh, tw, s);
        case 4096: return rows_n<real, 4096>(g, mesh, tw, s);
        case 8192: return rows_n<real, 8192>(g, mesh, tw, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename real>
hipError_t launch_fft_cols(const Geom &g, real *mesh, const real *tw, hipStream_t s) {
    switch (g.N) {
        case 64: return cols_n<real, 64>(g, mesh, tw, s);
        case 128: return cols_n<real, 128>(g, mesh, tw, s);
        case 256: return cols_n<real, 256>(g, mesh, tw, s);
        case 512: return cols_n<real, 512>(g, mesh, tw, s);
        case 1024: return cols_n<real, 1024>(g, mesh, tw, s);
        case 2048: return cols_n<real, 2048>(g, mesh, tw, s);
        case 4096: return cols_n<real, 4096>(g, mesh, tw, s);
        case 8192: return cols_n<real, 8192>(g, mesh, tw, s);
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_fft_rows<float>(const Geom &, float *, const float *, hipStream_t);
template hipError_t launch_fft_rows<double>(const Geom &, double *, const double *, hipStream_t);
template hipError_t launch_fft_cols<float>(const Geom &, float *, const float *, hipStream_t);
template hipError_t launch_fft_cols<double>(const Geom &, double *, const double *, hipStream_t);

}  // namespace rick
