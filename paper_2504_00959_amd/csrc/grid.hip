// LDS-tiled convolutional gridding (Sec. 2.1, Eq. 3) of binned records onto
// the w-plane stack.
//
// One block takes one work item: a chunk of at most CH records of one
// (plane, tile) bin.  The tile's T x T accumulator (float64 re and im planes)
// lives in LDS; each wave takes one record at a time with one lane per kernel
// tap (lane t < W*W is tap (t / W, t % W)), so one record costs two LDS
// atomic adds and no lane pair of an instruction shares an address.  The LDS
// row pitch is congruent to W modulo 32 elements, which spreads the W x W
// footprint over the banks.
//
// Accumulators are float64 in every precision mode: float64 LDS atomic adds
// run at the rate of plain LDS traffic on gfx950, float32 ones several times
// slower, and dense cells collect thousands of terms, which float32
// accumulation would round to ~1e-5 of image RMS.
//
// Records arrive 64 at a time in one coalesced load; each lane decodes the
// record it loaded (footprint origin, tap-table rows, whether the footprint
// lies inside the tile), and the decoded fields are broadcast with readlane,
// four records per step whose tap-table reads are issued together.  Taps outside
// the tile are skipped: a record whose footprint straddles tile edges was
// binned into every tile it touches.
//
// After the records the tile is written to HBM once, row-coalesced:
//   - bins with a single chunk own their tile and store it (empty bins store
//     zeros, so the mesh needs no clearing);
//   - bins split over several chunks (the dense uv centre) add their partial
//     tiles with atomics onto a tile zeroed beforehand.
// On a rick_grid that accumulates onto an earlier one, every tile is added.
#include "rick_internal.h"

namespace rick {

namespace {

constexpr int kGridBlock = 512;   // 8 waves share one tile
constexpr int kGroup = 4;         // records whose tap-table reads are issued together
constexpr int kZeroBlock = 256;

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

__device__ __forceinline__ int32_t bcast(int32_t v, int j) { return __builtin_amdgcn_readlane(v, j); }
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
__global__ __launch_bounds__(kZeroBlock) void k_zero_heavy(Geom g, const int32_t *__restrict__ heavy_bins,
                                                           const Stats *__restrict__ st, real *__restrict__ mesh) {
    using r2 = typename real2_t<real>::type;
    r2 *m = reinterpret_cast<r2 *>(mesh);
    const int32_t nheavy = (int32_t)st->n_heavy;
    for (int32_t hb = blockIdx.x; hb < nheavy; hb += gridDim.x) {
        const int32_t b = heavy_bins[hb];
        const int32_t k = b / (g.nt * g.nt);
        const int32_t rem = b - k * g.nt * g.nt;
        const int32_t y0 = (rem / g.nt) << g.log2T, x0 = (rem % g.nt) << g.log2T;
        for (int32_t c = threadIdx.x; c < g.T * g.T; c += kZeroBlock) {
            const int32_t y = c >> g.log2T, x = c & (g.T - 1);
            m[((int64_t)k * g.N + y0 + y) * g.N + x0 + x] = r2{0, 0};
        }
    }
}

// One decoded record, as broadcast to the wave.
template <typename real>
struct Rec {
    int32_t base;   // LDS index of the footprint's first tap (may be < 0 for straddling records)
    int32_t lxy;    // tap-table row offsets: (s_x row * W) | (s_y row * W) << 16
    int32_t oxy;    // footprint origin in tile cells, (ox + 64) | (oy + 64) << 8, bit 31: fully inside
    real vr, vi;
};

// Adds G records: all tap-table reads first, then all atomics, so the wave
// waits for LDS once per group (LDS operations retire in order, and a wait
// for a table read also waits for every earlier atomic).
template <typename real, int W, int NG, int G>
__device__ __forceinline__ void add_records(const Rec<real> (&r)[G], int valid, const int (&tap_ty)[NG],
                                            const int (&tap_tx)[NG], const int (&tap_off)[NG],
                                            const bool (&tap_on)[NG], int T, const real *__restrict__ s_lut,
                                            double *acc_re, double *acc_im) {
    real gy[G][NG], gx[G][NG];
    bool on[G][NG];
#pragma unroll
    for (int q = 0; q < G; ++q) {
        const bool inside = r[q].oxy < 0;
        const int ox = (r[q].oxy & 0xff) - 64, oy = ((r[q].oxy >> 8) & 0xff) - 64;
        const int lx = r[q].lxy & 0xffff, ly = r[q].lxy >> 16;
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            bool o = tap_on[gi] && q < valid;
            if (!inside) {
                const int x = ox + tap_tx[gi], y = oy + tap_ty[gi];
                o = o && x >= 0 && x < T && y >= 0 && y < T;
            }
            on[q][gi] = o;
            gy[q][gi] = s_lut[ly + tap_ty[gi]];
            gx[q][gi] = s_lut[lx + tap_tx[gi]];
        }
    }
#pragma unroll
    for (int q = 0; q < G; ++q) {
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) {
            if (on[q][gi]) {
                const real wgt = gy[q][gi] * gx[q][gi];
                atomicAdd(&acc_re[r[q].base + tap_off[gi]], (double)(wgt * r[q].vr));
                atomicAdd(&acc_im[r[q].base + tap_off[gi]], (double)(wgt * r[q].vi));
            }
        }
    }
}

template <typename real, int W>
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
    const int32_t k = b / (g.nt * g.nt);
    const int32_t rem = b - k * g.nt * g.nt;
    const int32_t y0 = (rem / g.nt) << g.log2T, x0 = (rem % g.nt) << g.log2T;
    using r2 = typename real2_t<real>::type;
    r2 *m = reinterpret_cast<r2 *>(mesh);
    if (n == 0) {
        // empty bin: a single chunk that owns its tile; store zeros unless accumulating
        if (!accumulate) {
            for (int32_t c = threadIdx.x; c < T * T; c += kGridBlock) {
                const int32_t y = c >> g.log2T, x = c & (T - 1);
                m[((int64_t)k * g.N + y0 + y) * g.N + x0 + x] = r2{0, 0};
            }
        }
        return;
    }
    double *acc_re = reinterpret_cast<double *>(smem);
    double *acc_im = acc_re + T * P;
    real *s_lut = reinterpret_cast<real *>(acc_im + T * P);
    for (int i = threadIdx.x; i < T * P; i += kGridBlock) {
        acc_re[i] = 0.0;
        acc_im[i] = 0.0;
    }
    {
        for (int i = threadIdx.x; i < g.OS * W; i += kGridBlock) s_lut[i] = lut[i];
        __syncthreads();

        const int lane = __lane_id();
        const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
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
        for (int32_t bt = wave; bt < nbatch; bt += nwave) {
            const int32_t r0 = r_begin + (bt << 6);
            const int32_t cnt = min(64, r_end - r0);
            // lane j loads and decodes record r0 + j
            Rec<real> mine{0, 0, 0, 0, 0};
            if (lane < cnt) {
                const uint32_t pos = rec_pos[r0 + lane];
                mine.vr = rec_vis[2 * (int64_t)(r0 + lane)];
                mine.vi = rec_vis[2 * (int64_t)(r0 + lane) + 1];
                const int ox = (int)(pos & 0xffu) - 2 * H;
                const int oy = (int)((pos >> 8) & 0xffu) - 2 * H;
                mine.base = oy * P + ox;
                mine.lxy = (int)((pos >> 16) & 0xffu) * W | ((int)(pos >> 24) * W) << 16;
                const bool inside = ox >= 0 && oy >= 0 && ox + W <= T && oy + W <= T;
                mine.oxy = (ox + 64) | (oy + 64) << 8 | (inside ? (int)0x80000000 : 0);
            }
            // groups of kGroup records (the last group is partial); lanes past
            // cnt decoded a zero record whose taps are all switched off
            for (int j = 0; j < cnt; j += kGroup) {
                Rec<real> rg[kGroup];
#pragma unroll
                for (int q = 0; q < kGroup; ++q) {
                    const int jj = (j + q) & 63;
                    rg[q] = Rec<real>{bcast(mine.base, jj), bcast(mine.lxy, jj), bcast(mine.oxy, jj),
                                      bcast(mine.vr, jj), bcast(mine.vi, jj)};
                }
                add_records<real, W, NG, kGroup>(rg, cnt - j, tap_ty, tap_tx, tap_off, tap_on, T, s_lut, acc_re,
                                                 acc_im);
            }
        }
    }
    __syncthreads();

    const bool shared_tile = nchunk > 1;
    for (int32_t c = threadIdx.x; c < T * T; c += kGridBlock) {
        const int32_t y = c >> g.log2T, x = c & (T - 1);
        const real re = (real)acc_re[y * P + x], im = (real)acc_im[y * P + x];
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

template <typename real>
__global__ void k_zero_mesh(real *__restrict__ a, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = 0;
}

template <typename real, int W>
hipError_t grid_w(const Geom &g, const BinScan *scan, const int32_t *item_bin, const uint32_t *rec_pos,
                  const real *rec_vis, const real *lut, real *mesh, int accumulate, int32_t max_items,
                  hipStream_t s) {
    const size_t lds = size_t(2) * g.T * g.pitch * sizeof(double) + size_t(g.OS) * g.W * sizeof(real);
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_grid<real, W>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(160 * 1024));
        attr = true;
    }
    hipLaunchKernelGGL((k_grid<real, W>), dim3(max_items), dim3(kGridBlock), lds, s, g, scan, item_bin, rec_pos,
                       rec_vis, lut, mesh, accumulate);
    return hipGetLastError();
}

}  // namespace

size_t grid_lds_bytes(const Geom &g, size_t real_bytes) {
    return size_t(2) * g.T * g.pitch * sizeof(double) + size_t(g.OS) * g.W * real_bytes;
}

template <typename real>
hipError_t launch_zero_mesh(real *mesh, int64_t n_real, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_mesh<real>, dim3(8192), dim3(256), 0, s, mesh, n_real);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_zero_heavy(const Geom &g, const int32_t *heavy_bins, const Stats *st, real *mesh, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_heavy<real>, dim3(1024), dim3(kZeroBlock), 0, s, g, heavy_bins, st, mesh);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_grid(const Geom &g, const BinScan *scan, const int32_t *item_bin, const uint32_t *rec_pos,
                       const real *rec_vis, const real *lut, real *mesh, int accumulate, int32_t max_items,
                       hipStream_t s) {
    switch (g.W) {
#define CASE(w) \
    case w: return grid_w<real, w>(g, scan, item_bin, rec_pos, rec_vis, lut, mesh, accumulate, max_items, s);
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
