// Prediction (degridding): visibilities of a model sky image by the
// w-stacking discretisation of Sec. 2.1 run the other way, i.e. Eq. 2
// evaluated plane by plane:
//   plane images   P_k[q][p] = M[q][p] exp(-2 pi i w_k (n_pq - 1)) / (n_pq C(l'_p) C(l'_q))
//   forward DFT    H_k[j][i] = sum_{q,p} P_k[q][p] exp(-2 pi i ((i-N/2)(p-N/2) + (j-N/2)(q-N/2)) / N)
//   interpolation  V = sum_{t_y,t_x} g_{s_y}[t_y] g_{s_x}[t_x] H_k[c_y + t_y - h][c_x + t_x - h]
// with the visibility's cell, sub-cell offset, plane and drop decision taken
// exactly as imaging takes them (quant.h), so that prediction is the adjoint
// of the imaging steps.
//
// The forward DFT runs through the library's centred inverse FFT: the screen
// kernel writes the complex conjugate of P_k, the inverse transform of
// conj(P_k) is conj(H_k), and the interpolation conjugates what it reads.
#include <utility>

#include "rick_internal.h"
#include "quant.h"

namespace rick {

namespace {

constexpr int kPredBlock = 256;
constexpr int kDegridBlock = 256;

template <typename real>
struct Cplx;
template <>
struct Cplx<float> {
    using t = float2;
};
template <>
struct Cplx<double> {
    using t = double2;
};

__device__ __forceinline__ void sincospi_p(float x, float *s, float *c) { sincospif(x, s, c); }
__device__ __forceinline__ void sincospi_p(double x, double *s, double *c) { sincospi(x, s, c); }

// conj(P_k) for every plane, one thread per pixel (each plane's write is
// row-coalesced).  n - 1 and the phase w_k (n - 1) in turns are formed in
// float64 and reduced to [-1/2, 1/2] before the trigonometric evaluation, as
// in imaging; pixels outside the unit circle are zero.
template <typename real>
__global__ __launch_bounds__(kPredBlock) void k_predict_screen(Geom g, const real *__restrict__ model,
                                                               const double *__restrict__ corr,
                                                               real *__restrict__ mesh) {
    using C = typename Cplx<real>::t;
    const int64_t npix = (int64_t)g.N * g.N;
    const int64_t pix = (int64_t)blockIdx.x * kPredBlock + threadIdx.x;
    if (pix >= npix) return;
    const int q = (int)(pix / g.N), p = (int)(pix % g.N);
    const double dl = g.fov / g.N;
    const double l = (double)(p - g.N / 2) * dl;
    const double m = (double)(q - g.N / 2) * dl;
    const double r2 = l * l + m * m;
    const bool inside = r2 < 1.0;
    const double nm1 = inside ? -r2 / (1.0 + sqrt(1.0 - r2)) : 0.0;
    const real base = inside ? (real)((double)model[pix] / ((1.0 + nm1) * corr[p] * corr[q])) : (real)0;
    C *out = reinterpret_cast<C *>(mesh) + pix;
    for (int k = 0; k < g.Nw; ++k) {
        const double tau = plane_centre(g, k) * nm1;
        const double tr = tau - rint(tau);
        real sn, cs;
        sincospi_p((real)(2.0 * tr), &sn, &cs);
        C v;
        v.x = base * cs;   // conj(exp(-2 pi i tau)) = exp(+2 pi i tau)
        v.y = base * sn;
        out[(int64_t)k * npix] = v;
    }
}

// Every tile and tile row of every plane marked as holding values (the FFT
// then reads the whole of each plane).
__global__ void k_fill_bits(Geom g, uint64_t *__restrict__ tile_bits, uint64_t *__restrict__ row_bits) {
    const int64_t n_tile_words = (int64_t)g.Nw * g.nt * g.occw;
    const int64_t n_row_words = (int64_t)g.Nw * g.occw;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_tile_words + n_row_words; i += stride) {
        const int32_t word = (int32_t)((i < n_tile_words ? i : i - n_tile_words) % g.occw);
        const int32_t left = g.nt - 64 * word;   // tiles (or tile rows) covered by this word
        const uint64_t bits = left >= 64 ? ~0ull : ((1ull << left) - 1ull);
        if (i < n_tile_words) tile_bits[i] = bits;
        else row_bits[i - n_tile_words] = bits;
    }
}

// Element (row j, column i) of a plane: row order (j N + i), or column-panel
// order ((i / PW) N PW + j PW + i % PW, PW = 2^log2pw) when PANEL.
template <bool PANEL>
struct PlaneLayout {
    int32_t N, log2pw;
    __device__ __forceinline__ int64_t at(int32_t j, int32_t i) const {
        if (PANEL)
            return (((int64_t)(i >> log2pw) * N + j) << log2pw) + (i & ((1 << log2pw) - 1));
        return (int64_t)j * N + i;
    }
};

// The W x W taps of a footprint with origin cell (x0, y0) read from one
// plane, conjugated, weighted by tap-table rows gx, gy; one complex result.
template <typename real, int W, bool PANEL>
__device__ __forceinline__ void interp(const typename Cplx<real>::t *__restrict__ plane, PlaneLayout<PANEL> L,
                                       int32_t x0, int32_t y0, const real *gx, const real *gy, real &vr,
                                       real &vi) {
    using C = typename Cplx<real>::t;
    real ar = 0, ai = 0;
#pragma unroll
    for (int ty = 0; ty < W; ++ty) {
        real rr = 0, ri = 0;
#pragma unroll
        for (int tx = 0; tx < W; ++tx) {
            const C h = plane[L.at(y0 + ty, x0 + tx)];
            rr += gx[tx] * h.x;
            ri += gx[tx] * h.y;
        }
        ar += gy[ty] * rr;
        ai += gy[ty] * ri;
    }
    vr = ar;
    vi = -ai;   // the plane holds conj(H_k)
}

// One thread per visibility (row r, channel c at index r * nchan + c): the
// position, plane and drop decision of imaging, then the footprint read from
// the plane.  Dropped visibilities are predicted as 0.
template <typename real, int W, bool PANEL>
__global__ __launch_bounds__(kDegridBlock) void k_degrid(Geom g, const double *__restrict__ uvw,
                                                         const double *__restrict__ scales, int64_t nrow,
                                                         int32_t nchan, const real *__restrict__ lut,
                                                         const real *__restrict__ mesh, int32_t log2pw,
                                                         real *__restrict__ out) {
    using C = typename Cplx<real>::t;
    extern __shared__ __align__(16) unsigned char smem[];
    real *s_lut = reinterpret_cast<real *>(smem);
    for (int i = threadIdx.x; i < g.OS * W; i += kDegridBlock) s_lut[i] = lut[i];
    __syncthreads();
    const int64_t nvis = nrow * nchan;
    const int64_t npix = (int64_t)g.N * g.N;
    const PlaneLayout<PANEL> L{g.N, log2pw};
    const C *planes = reinterpret_cast<const C *>(mesh);
    C *vout = reinterpret_cast<C *>(out);
    const int64_t stride = (int64_t)gridDim.x * kDegridBlock;
    for (int64_t i = (int64_t)blockIdx.x * kDegridBlock + threadIdx.x; i < nvis; i += stride) {
        const int64_t r = i / nchan;
        const int32_t c = (int32_t)(i - r * nchan);
        double u, v, w;
        {
#pragma clang fp contract(off)
            const double sc = scales[c];
            u = uvw[3 * r] * sc;
            v = uvw[3 * r + 1] * sc;
            w = uvw[3 * r + 2] * sc;
        }
        Quant qq;
        const bool keep = quantise<real>(g, u, v, w, (real)0, (real)0, 1.0f, qq);
        C o;
        o.x = 0;
        o.y = 0;
        if (keep)
            interp<real, W, PANEL>(planes + (int64_t)qq.k * npix, L, qq.cx - g.h, qq.cy - g.h,
                                   s_lut + (qq.sx + (g.OS >> 1)) * W, s_lut + (qq.sy + (g.OS >> 1)) * W, o.x, o.y);
        vout[i] = o;
    }
}

// Sort order for repeated prediction at fixed positions: per visibility a
// key, the offset of its footprint origin in the planes' layout (k N^2 plus
// the row-order or column-panel offset of (x0, y0)), all ones for a dropped
// one (sorted last), and a value (index | sub-cell x << 32 | sub-cell y << 40,
// sub-cells as s + OS/2).
template <typename real>
__global__ __launch_bounds__(kDegridBlock) void k_order_keys(Geom g, const double *__restrict__ uvw,
                                                             const double *__restrict__ scales, int64_t nrow,
                                                             int32_t nchan, int32_t log2pw,
                                                             uint64_t *__restrict__ keys,
                                                             uint64_t *__restrict__ vals) {
    const int64_t nvis = nrow * nchan;
    const int64_t stride = (int64_t)gridDim.x * kDegridBlock;
    for (int64_t i = (int64_t)blockIdx.x * kDegridBlock + threadIdx.x; i < nvis; i += stride) {
        const int64_t r = i / nchan;
        const int32_t c = (int32_t)(i - r * nchan);
        double u, v, w;
        {
#pragma clang fp contract(off)
            const double sc = scales[c];
            u = uvw[3 * r] * sc;
            v = uvw[3 * r + 1] * sc;
            w = uvw[3 * r + 2] * sc;
        }
        Quant qq;
        const bool keep = quantise<real>(g, u, v, w, (real)0, (real)0, 1.0f, qq);
        const int32_t x0 = qq.cx - g.h, y0 = qq.cy - g.h;
        const int64_t off = log2pw > 0 ? PlaneLayout<true>{g.N, log2pw}.at(y0, x0)
                                       : PlaneLayout<false>{g.N, 0}.at(y0, x0);
        keys[i] = keep ? (uint64_t)qq.k * (uint64_t)g.N * (uint64_t)g.N + (uint64_t)off : ~0ull;
        vals[i] = (uint64_t)i | (uint64_t)(qq.sx + (g.OS >> 1)) << 32 | (uint64_t)(qq.sy + (g.OS >> 1)) << 40;
    }
}

// Interpolation in sorted order: neighbouring threads read neighbouring
// footprints, so a wave's loads share cache lines; results are written to
// each visibility's own index.  The key is the footprint origin's offset in
// the planes' layout (N and PW powers of two).
template <typename real, int W, bool PANEL>
__global__ __launch_bounds__(kDegridBlock) void k_degrid_sorted(Geom g, const uint64_t *__restrict__ keys,
                                                                const uint64_t *__restrict__ vals, int64_t nvis,
                                                                const real *__restrict__ lut,
                                                                const real *__restrict__ mesh, int32_t log2pw,
                                                                real *__restrict__ out) {
    using C = typename Cplx<real>::t;
    extern __shared__ __align__(16) unsigned char smem[];
    real *s_lut = reinterpret_cast<real *>(smem);
    for (int i = threadIdx.x; i < g.OS * W; i += kDegridBlock) s_lut[i] = lut[i];
    __syncthreads();
    const int log2n = __builtin_ctz((unsigned)g.N);
    const PlaneLayout<PANEL> L{g.N, log2pw};
    const C *planes = reinterpret_cast<const C *>(mesh);
    C *vout = reinterpret_cast<C *>(out);
    const int64_t stride = (int64_t)gridDim.x * kDegridBlock;
    for (int64_t j = (int64_t)blockIdx.x * kDegridBlock + threadIdx.x; j < nvis; j += stride) {
        const uint64_t key = keys[j], val = vals[j];
        const int64_t i = (int64_t)(val & 0xffffffffull);
        C o;
        o.x = 0;
        o.y = 0;
        if (key != ~0ull) {
            const int32_t sx = (int32_t)((val >> 32) & 0xffu), sy = (int32_t)((val >> 40) & 0xffu);
            const int64_t k = (int64_t)(key >> (2 * log2n));
            const uint64_t off = key & (((uint64_t)1 << (2 * log2n)) - 1);
            int32_t x0, y0;
            if (PANEL) {
                y0 = (int32_t)((off >> log2pw) & (uint64_t)(g.N - 1));
                x0 = (int32_t)(((off >> (log2n + log2pw)) << log2pw) | (off & (((uint64_t)1 << log2pw) - 1)));
            } else {
                y0 = (int32_t)(off >> log2n);
                x0 = (int32_t)(off & (uint64_t)(g.N - 1));
            }
            interp<real, W, PANEL>(planes + (k << (2 * log2n)), L, x0, y0, s_lut + sx * W, s_lut + sy * W, o.x,
                                   o.y);
        }
        vout[i] = o;
    }
}

template <typename real, int W>
hipError_t degrid_w(const Geom &g, const double *uvw, const double *scales, int64_t nrow, int32_t nchan,
                    const real *lut, const real *mesh, int32_t panel, real *out, hipStream_t s) {
    const int64_t nvis = nrow * nchan;
    if (nvis == 0) return hipSuccess;
    int64_t blocks = (nvis + kDegridBlock - 1) / kDegridBlock;
    if (blocks > 65536) blocks = 65536;
    const size_t lds = (size_t)g.OS * W * sizeof(real);
    const int32_t log2pw = panel > 0 ? __builtin_ctz((unsigned)panel) : 0;
    if (panel > 0)
        hipLaunchKernelGGL((k_degrid<real, W, true>), dim3((unsigned)blocks), dim3(kDegridBlock), lds, s, g, uvw,
                           scales, nrow, nchan, lut, mesh, log2pw, out);
    else
        hipLaunchKernelGGL((k_degrid<real, W, false>), dim3((unsigned)blocks), dim3(kDegridBlock), lds, s, g, uvw,
                           scales, nrow, nchan, lut, mesh, log2pw, out);
    return hipGetLastError();
}

template <typename real, int W>
hipError_t degrid_sorted_w(const Geom &g, const uint64_t *keys, const uint64_t *vals, int64_t nvis, const real *lut,
                           const real *mesh, int32_t panel, real *out, hipStream_t s) {
    if (nvis == 0) return hipSuccess;
    int64_t blocks = (nvis + kDegridBlock - 1) / kDegridBlock;
    if (blocks > 65536) blocks = 65536;
    const size_t lds = (size_t)g.OS * W * sizeof(real);
    const int32_t log2pw = panel > 0 ? __builtin_ctz((unsigned)panel) : 0;
    if (panel > 0)
        hipLaunchKernelGGL((k_degrid_sorted<real, W, true>), dim3((unsigned)blocks), dim3(kDegridBlock), lds, s, g,
                           keys, vals, nvis, lut, mesh, log2pw, out);
    else
        hipLaunchKernelGGL((k_degrid_sorted<real, W, false>), dim3((unsigned)blocks), dim3(kDegridBlock), lds, s, g,
                           keys, vals, nvis, lut, mesh, log2pw, out);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fill_bits(const Geom &g, uint64_t *tile_bits, uint64_t *row_bits, hipStream_t s) {
    const int64_t words = (int64_t)g.Nw * (g.nt + 1) * g.occw;
    const unsigned fb = (unsigned)((words + 255) / 256 < 4096 ? (words + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_fill_bits, dim3(fb), dim3(256), 0, s, g, tile_bits, row_bits);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_predict_screen(const Geom &g, const real *model, const double *corr, real *mesh,
                                 uint64_t *tile_bits, uint64_t *row_bits, hipStream_t s) {
    const int64_t npix = (int64_t)g.N * g.N;
    const unsigned blocks = (unsigned)((npix + kPredBlock - 1) / kPredBlock);
    hipLaunchKernelGGL((k_predict_screen<real>), dim3(blocks), dim3(kPredBlock), 0, s, g, model, corr, mesh);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t words = (int64_t)g.Nw * (g.nt + 1) * g.occw;
    const unsigned fb = (unsigned)((words + 255) / 256 < 4096 ? (words + 255) / 256 : 4096);
    hipLaunchKernelGGL(k_fill_bits, dim3(fb), dim3(256), 0, s, g, tile_bits, row_bits);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_degrid(const Geom &g, const double *uvw, const double *scales, int64_t nrow, int32_t nchan,
                         const real *lut, const real *mesh, int32_t panel, real *out, hipStream_t s) {
    switch (g.W) {
#define RICK_DEGRID_W(w) \
    case w: return degrid_w<real, w>(g, uvw, scales, nrow, nchan, lut, mesh, panel, out, s);
        RICK_DEGRID_W(1)
        RICK_DEGRID_W(3)
        RICK_DEGRID_W(5)
        RICK_DEGRID_W(7)
        RICK_DEGRID_W(9)
        RICK_DEGRID_W(11)
        RICK_DEGRID_W(13)
        RICK_DEGRID_W(15)
#undef RICK_DEGRID_W
        default: return hipErrorInvalidValue;
    }
}

template <typename real>
hipError_t launch_order_keys(const Geom &g, const double *uvw, const double *scales, int64_t nrow, int32_t nchan,
                             int32_t panel, uint64_t *keys, uint64_t *vals, hipStream_t s) {
    const int64_t nvis = nrow * nchan;
    if (nvis == 0) return hipSuccess;
    int64_t blocks = (nvis + kDegridBlock - 1) / kDegridBlock;
    if (blocks > 65536) blocks = 65536;
    const int32_t log2pw = panel > 0 ? __builtin_ctz((unsigned)panel) : 0;
    hipLaunchKernelGGL((k_order_keys<real>), dim3((unsigned)blocks), dim3(kDegridBlock), 0, s, g, uvw, scales, nrow,
                       nchan, log2pw, keys, vals);
    return hipGetLastError();
}

// Stable LSD radix sort of (key, value) pairs, 8 bits per pass.  A block
// takes a tile of kSortTile consecutive items; per pass a histogram kernel
// counts the tile's digits in LDS and writes them digit-major into a
// (digit, block) table, a flat exclusive scan of that table gives every
// (digit, block) its first output slot, and a scatter kernel walks the tile
// again in order, one item per thread per round: each wave finds the lanes
// sharing an item's digit with eight ballots, the rank among them, and the
// counts of earlier waves of the round come through LDS, so equal digits keep
// their input order.
constexpr int kSortThreads = 256;   // = the radix
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kSortWaves = kSortThreads / 64;

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                            int32_t nblk, int32_t *__restrict__ counts) {
    __shared__ int32_t h[kSortThreads];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
    for (int j = 0; j < kSortItems; ++j) {
        const int64_t i = base + j * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(int)((keys[i] >> shift) & 0xffu)], 1);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(const uint64_t *__restrict__ kin,
                                                               const uint64_t *__restrict__ vin, int64_t n, int shift,
                                                               int32_t nblk, const int32_t *__restrict__ first,
                                                               uint64_t *__restrict__ kout,
                                                               uint64_t *__restrict__ vout) {
    __shared__ int32_t s_next[kSortThreads];             // next output slot of each digit
    __shared__ int32_t s_wc[kSortWaves][kSortThreads];   // per-wave digit counts of the round
    const int t = (int)threadIdx.x, lane = t & 63, wid = t >> 6;
    s_next[t] = first[(int64_t)t * nblk + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int j = 0; j < kSortItems; ++j) {
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) s_wc[w][t] = 0;
        __syncthreads();
        const int64_t i = base + j * kSortThreads + t;
        const bool valid = i < n;
        const uint64_t key = valid ? kin[i] : 0ull, val = valid ? vin[i] : 0ull;
        const int d = (int)((key >> shift) & 0xffu);
        // lanes of this wave holding an item with the same digit
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1;
            const uint64_t b = __ballot(on);
            peers &= on ? b : ~b;
        }
        const uint64_t below = peers & ((1ull << lane) - 1ull);
        if (valid && below == 0ull) s_wc[wid][d] = __popcll(peers);   // the group's first lane
        __syncthreads();
        if (valid) {
            int32_t pos = s_next[d] + __popcll(below);
            for (int w = 0; w < wid; ++w) pos += s_wc[w][d];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        int32_t add = 0;
#pragma unroll
        for (int w = 0; w < kSortWaves; ++w) add += s_wc[w][t];
        s_next[t] += add;
        __syncthreads();
    }
}

hipError_t sort_order(void *temp, size_t &temp_bytes, uint64_t *keys_in, uint64_t *keys_out, uint64_t *vals_in,
                      uint64_t *vals_out, int64_t n, int begin_bit, int end_bit, hipStream_t s) {
    const int64_t nblk = (n + kSortTile - 1) / kSortTile;
    const int64_t ncount = (int64_t)kSortThreads * nblk;
    const size_t count_bytes = ((size_t)(ncount + 1) * sizeof(int32_t) + 255) & ~size_t(255);
    const size_t need = count_bytes + (size_t)flat_scan_partials(ncount) * sizeof(int32_t);
    if (!temp) {
        temp_bytes = need;
        return hipSuccess;
    }
    if (temp_bytes < need || n <= 0 || n >= (int64_t(1) << 31)) return hipErrorInvalidValue;
    int32_t *counts = static_cast<int32_t *>(temp);
    int32_t *bsum = reinterpret_cast<int32_t *>(static_cast<unsigned char *>(temp) + count_bytes);
    const int passes = (end_bit - begin_bit + 7) / 8;
    // pass p reads from one buffer pair and writes the other; an odd count
    // of passes ends in the output pair, an even one is copied there
    uint64_t *ks = keys_in, *vs = vals_in, *kd = keys_out, *vd = vals_out;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = begin_bit + 8 * pass;
        hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nblk), dim3(kSortThreads), 0, s, ks, n, shift, (int32_t)nblk,
                           counts);
        hipError_t e = launch_flat_scan(counts, ncount, bsum, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nblk), dim3(kSortThreads), 0, s, ks, vs, n, shift,
                           (int32_t)nblk, counts, kd, vd);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        std::swap(ks, kd);
        std::swap(vs, vd);
    }
    if (ks != keys_out) {
        hipError_t e = hipMemcpyAsync(keys_out, ks, (size_t)n * 8, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(vals_out, vs, (size_t)n * 8, hipMemcpyDeviceToDevice, s);
        return e;
    }
    return hipSuccess;
}

template <typename real>
hipError_t launch_degrid_sorted(const Geom &g, const uint64_t *keys, const uint64_t *vals, int64_t nvis,
                                const real *lut, const real *mesh, int32_t panel, real *out, hipStream_t s) {
    switch (g.W) {
#define RICK_DEGRID_SW(w) \
    case w: return degrid_sorted_w<real, w>(g, keys, vals, nvis, lut, mesh, panel, out, s);
        RICK_DEGRID_SW(1)
        RICK_DEGRID_SW(3)
        RICK_DEGRID_SW(5)
        RICK_DEGRID_SW(7)
        RICK_DEGRID_SW(9)
        RICK_DEGRID_SW(11)
        RICK_DEGRID_SW(13)
        RICK_DEGRID_SW(15)
#undef RICK_DEGRID_SW
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_order_keys<float>(const Geom &, const double *, const double *, int64_t, int32_t,
                                             int32_t, uint64_t *, uint64_t *, hipStream_t);
template hipError_t launch_order_keys<double>(const Geom &, const double *, const double *, int64_t, int32_t,
                                              int32_t, uint64_t *, uint64_t *, hipStream_t);
template hipError_t launch_degrid_sorted<float>(const Geom &, const uint64_t *, const uint64_t *, int64_t,
                                                const float *, const float *, int32_t, float *, hipStream_t);
template hipError_t launch_degrid_sorted<double>(const Geom &, const uint64_t *, const uint64_t *, int64_t,
                                                 const double *, const double *, int32_t, double *, hipStream_t);
template hipError_t launch_predict_screen<float>(const Geom &, const float *, const double *, float *, uint64_t *,
                                                 uint64_t *, hipStream_t);
template hipError_t launch_predict_screen<double>(const Geom &, const double *, const double *, double *,
                                                  uint64_t *, uint64_t *, hipStream_t);
template hipError_t launch_degrid<float>(const Geom &, const double *, const double *, int64_t, int32_t,
                                         const float *, const float *, int32_t, float *, hipStream_t);
template hipError_t launch_degrid<double>(const Geom &, const double *, const double *, int64_t, int32_t,
                                          const double *, const double *, int32_t, double *, hipStream_t);

}  // namespace rick
