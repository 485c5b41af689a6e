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
// exp(+2 pi i m / N) computed in float64 on the host and rounded.
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
            const int step = k * (N / (L * R));
#pragma unroll
            for (int j = 1; j < R; ++j) {
                const C w = tw[j * step];
#pragma unroll
                for (int v = 0; v < VC; ++v) a[i][v][j] = cmul(a[i][v][j], w);
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
    // V columns per block: the strip fills about 128 KB of LDS (16 for small N)
    constexpr int VRAW = (16384 * 8 / (int)sizeof(C)) / N;
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

}  // namespace

bool fft_supported(int N) { return N >= 64 && N <= 8192 && (N & (N - 1)) == 0; }

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
