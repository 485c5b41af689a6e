// LDS-tiled convolutional gridding (Sec. 2.1, Eq. 3) of binned records onto
// the w-plane stack.
//
// One block takes one work item: a chunk of at most CH records of one
// (plane, tile) bin.  The tile's T x T accumulator (re and im planes) lives in
// LDS; each wave takes one record at a time with one lane per kernel tap
// (lane t < W*W is tap (t / W, t % W)), so one record costs two LDS atomic
// adds and no lane pair of an instruction shares an address.  Records arrive
// 64 at a time in one coalesced load and are broadcast across the wave with
// readlane.  The LDS row pitch is congruent to W modulo 32 elements.  Every
// 4 x 64 records per wave the LDS tile is folded into float64 registers
// (each thread owns T^2/256 cells) and cleared: dense cells collect
// thousands of terms, and float32 accumulation of all of them would cost
// about 1e-5 of image RMS.  Taps outside the tile are skipped: a record whose
// footprint straddles tile edges was binned into every tile it touches.
//
// After the records, the tile is written to HBM once, row-coalesced:
//   - bins with a single chunk own their tile and store it (empty bins store
//     zeros, so the mesh needs no clearing);
//   - bins split over several chunks (the dense uv centre) add their partial
//     tiles with float atomics onto a tile zeroed beforehand.
// On a rick_grid that accumulates onto an earlier one, every tile is added.
#include "rick_internal.h"

namespace rick {

namespace {

constexpr int kGridBlock = 256;

template <typename real>
struct real2_t;
template <>
struct real2_t<float> {
    using type = float2;
};
template <>
struct real2_t<double> {
    using type = double2;
};

__device__ __forceinline__ float bcast(float v, int j) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), j));
}
__device__ __forceinline__ double bcast(double v, int j) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffll), j);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), j);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ void atomic_add_real(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_real(double *p, double v) { unsafeAtomicAdd(p, v); }

// Heavy bins (several chunks) are zeroed before gridding; the scan lists them.
template <typename real>
__global__ __launch_bounds__(kGridBlock) void k_zero_heavy(Geom g, const int32_t *__restrict__ heavy_bins,
                                                           const Stats *__restrict__ st, real *__restrict__ mesh) {
    using r2 = typename real2_t<real>::type;
    r2 *m = reinterpret_cast<r2 *>(mesh);
    const int32_t nheavy = (int32_t)st->n_heavy;
    for (int32_t h = blockIdx.x; h < nheavy; h += gridDim.x) {
        const int32_t b = heavy_bins[h];
        const int32_t k = b / (g.nt * g.nt);
        const int32_t rem = b - k * g.nt * g.nt;
        const int32_t y0 = (rem / g.nt) << g.log2T, x0 = (rem % g.nt) << g.log2T;
        for (int32_t c = threadIdx.x; c < g.T * g.T; c += kGridBlock) {
            const int32_t y = c >> g.log2T, x = c & (g.T - 1);
            m[((int64_t)k * g.N + y0 + y) * g.N + x0 + x] = r2{0, 0};
        }
    }
}

// acc_t: LDS accumulator type (float in the float32 modes, double in float64
// mode).  The LDS tile is folded into float64 registers every kRound records
// per block, so a float accumulator only ever sums a few terms per cell.
constexpr int kBatchesPerRound = 4;                       // per wave
constexpr int kMaxCellsPerThread = 16;                    // T <= 64

template <typename real, typename acc_t, int W>
__global__ __launch_bounds__(kGridBlock) void k_grid(Geom g, const BinScan *__restrict__ scan,
                                                     const int32_t *__restrict__ item_bin,
                                                     const uint32_t *__restrict__ rec_pos,
                                                     const real *__restrict__ rec_vis, const real *__restrict__ lut,
                                                     real *__restrict__ mesh, int accumulate) {
    constexpr int W2 = W * W;
    constexpr int NG = (W2 + 63) / 64;   // groups of 64 taps
    constexpr int H = (W - 1) / 2;
    constexpr int nwave = kGridBlock / 64;
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t total = scan[g.nbins].item;
    const int32_t item = blockIdx.x;
    if (item >= total) return;
    const int32_t b = item_bin[item];
    const int32_t first = scan[b].item;
    const int32_t nchunk = scan[b + 1].item - first;
    const int32_t chunk = item - first;
    const int32_t r_begin = scan[b].rec + chunk * g.CH;
    int32_t r_end = r_begin + g.CH;
    if (r_end > scan[b + 1].rec) r_end = scan[b + 1].rec;
    const int32_t n = r_end - r_begin;

    const int32_t T = g.T, P = g.pitch;
    acc_t *acc_re = reinterpret_cast<acc_t *>(smem);
    acc_t *acc_im = acc_re + T * P;
    real *s_lut = reinterpret_cast<real *>(acc_im + T * P);
    // cells owned by this thread for the register fold and the final store
    const int cpt = (T * T) / kGridBlock;
    double fre[kMaxCellsPerThread], fim[kMaxCellsPerThread];
#pragma unroll
    for (int i = 0; i < kMaxCellsPerThread; ++i) {
        fre[i] = 0.0;
        fim[i] = 0.0;
    }
    if (n > 0) {
        for (int i = threadIdx.x; i < T * P; i += kGridBlock) {
            acc_re[i] = 0;
            acc_im[i] = 0;
        }
        for (int i = threadIdx.x; i < g.OS * W; i += kGridBlock) s_lut[i] = lut[i];
        __syncthreads();

        const int lane = __lane_id();
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        // per-lane taps: lane + 64 gi -> (ty, tx)
        int tap_ty[NG], tap_tx[NG], tap_off[NG];
        bool tap_on[NG];
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            const int t = lane + 64 * gi;
            tap_on[gi] = t < W2;
            tap_ty[gi] = tap_on[gi] ? t / W : 0;
            tap_tx[gi] = tap_on[gi] ? t - tap_ty[gi] * W : 0;
            tap_off[gi] = tap_ty[gi] * P + tap_tx[gi];
        }
        const int32_t nbatch = (n + 63) >> 6;
        const int32_t per_round = nwave * kBatchesPerRound;
        const int32_t nround = (nbatch + per_round - 1) / per_round;
        for (int32_t rd = 0; rd < nround; ++rd) {
            // records in batches of 64: one coalesced load per batch, broadcast by readlane
            for (int f = 0; f < kBatchesPerRound; ++f) {
                const int32_t bt = rd * per_round + f * nwave + wave;
                if (bt >= nbatch) break;
                const int32_t r0 = r_begin + (bt << 6);
                const int32_t cnt = min(64, r_end - r0);
                uint32_t vpos = 0;
                real vre = 0, vim = 0;
                if (lane < cnt) {
                    vpos = rec_pos[r0 + lane];
                    vre = rec_vis[2 * (int64_t)(r0 + lane)];
                    vim = rec_vis[2 * (int64_t)(r0 + lane) + 1];
                }
                for (int j = 0; j < cnt; ++j) {
                    const uint32_t pos = __builtin_amdgcn_readlane(vpos, j);
                    const real vr = bcast(vre, j);
                    const real vi = bcast(vim, j);
                    const int ox = (int)(pos & 0xffu) - 2 * H;
                    const int oy = (int)((pos >> 8) & 0xffu) - 2 * H;
                    const int lx = (int)((pos >> 16) & 0xffu) * W;
                    const int ly = (int)(pos >> 24) * W;
                    const int base = oy * P + ox;
                    const bool inside = ox >= 0 && oy >= 0 && ox + W <= T && oy + W <= T;
#pragma unroll
                    for (int gi = 0; gi < NG; ++gi) {
                        bool on = tap_on[gi];
                        if (!inside) {
                            const int x = ox + tap_tx[gi], y = oy + tap_ty[gi];
                            on = on && x >= 0 && x < T && y >= 0 && y < T;
                        }
                        if (on) {
                            const real wgt = s_lut[ly + tap_ty[gi]] * s_lut[lx + tap_tx[gi]];
                            atomicAdd(&acc_re[base + tap_off[gi]], (acc_t)(wgt * vr));
                            atomicAdd(&acc_im[base + tap_off[gi]], (acc_t)(wgt * vi));
                        }
                    }
                }
            }
            __syncthreads();
            // fold the LDS tile into float64 registers and clear it
#pragma unroll
            for (int i = 0; i < kMaxCellsPerThread; ++i) {
                if (i < cpt) {
                    const int c = threadIdx.x + i * kGridBlock;
                    const int idx = (c >> g.log2T) * P + (c & (T - 1));
                    fre[i] += (double)acc_re[idx];
                    fim[i] += (double)acc_im[idx];
                    acc_re[idx] = 0;
                    acc_im[idx] = 0;
                }
            }
            __syncthreads();
        }
    }

    const int32_t k = b / (g.nt * g.nt);
    const int32_t rem = b - k * g.nt * g.nt;
    const int32_t y0 = (rem / g.nt) << g.log2T, x0 = (rem % g.nt) << g.log2T;
    using r2 = typename real2_t<real>::type;
    r2 *m = reinterpret_cast<r2 *>(mesh);
    const bool shared_tile = nchunk > 1;
#pragma unroll
    for (int i = 0; i < kMaxCellsPerThread; ++i) {
        if (i < cpt) {
            const int32_t c = threadIdx.x + i * kGridBlock;
            const int32_t y = c >> g.log2T, x = c & (T - 1);
            const real re = (real)fre[i], im = (real)fim[i];
            r2 *dst = m + ((int64_t)k * g.N + y0 + y) * g.N + x0 + x;
            if (shared_tile) {
                if (re != 0) atomic_add_real(&dst->x, re);
                if (im != 0) atomic_add_real(&dst->y, im);
            } else if (accumulate) {
                const r2 old = *dst;
                *dst = r2{old.x + re, old.y + im};
            } else {
                *dst = r2{re, im};
            }
        }
    }
}

template <typename real>
__global__ void k_zero_mesh(real *__restrict__ a, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = 0;
}

}  // namespace

template <typename real>
hipError_t launch_zero_mesh(real *mesh, int64_t n_real, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_mesh<real>, dim3(8192), dim3(256), 0, s, mesh, n_real);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_zero_heavy(const Geom &g, const int32_t *heavy_bins, const Stats *st, real *mesh, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_heavy<real>, dim3(1024), dim3(kGridBlock), 0, s, g, heavy_bins, st, mesh);
    return hipGetLastError();
}

template <typename real, typename acc_t, int W>
hipError_t grid_w(const Geom &g, const BinScan *scan, const int32_t *item_bin, const uint32_t *rec_pos,
                  const real *rec_vis, const real *lut, real *mesh, int accumulate, int32_t max_items,
                  hipStream_t s) {
    const size_t lds = size_t(2) * g.T * g.pitch * sizeof(acc_t) + size_t(g.OS) * g.W * sizeof(real);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_grid<real, acc_t, W>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(160 * 1024));
        attr = true;
    }
    hipLaunchKernelGGL((k_grid<real, acc_t, W>), dim3(max_items), dim3(kGridBlock), lds, s, g, scan, item_bin,
                       rec_pos, rec_vis, lut, mesh, accumulate);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_grid(const Geom &g, const BinScan *scan, const int32_t *item_bin, const uint32_t *rec_pos,
                       const real *rec_vis, const real *lut, real *mesh, int accumulate, int32_t max_items,
                       hipStream_t s) {
    using acc_t = real;   // float LDS atomics for float32, double for float64 (both folded into float64)
    switch (g.W) {
#define CASE(w) \
    case w: return grid_w<real, acc_t, w>(g, scan, item_bin, rec_pos, rec_vis, lut, mesh, accumulate, max_items, s);
        CASE(1) CASE(3) CASE(5) CASE(7) CASE(9) CASE(11) CASE(13) CASE(15)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_zero_mesh<float>(float *, int64_t, hipStream_t);
template hipError_t launch_zero_mesh<double>(double *, int64_t, hipStream_t);
template hipError_t launch_zero_heavy<float>(const Geom &, const int32_t *, const Stats *, float *, hipStream_t);
template hipError_t launch_zero_heavy<double>(const Geom &, const int32_t *, const Stats *, double *, hipStream_t);
template hipError_t launch_grid<float>(const Geom &, const BinScan *, const int32_t *, const uint32_t *,
                                       const float *, const float *, float *, int, int32_t, hipStream_t);
template hipError_t launch_grid<double>(const Geom &, const BinScan *, const int32_t *, const uint32_t *,
                                        const double *, const double *, double *, int, int32_t, hipStream_t);

}  // namespace rick
