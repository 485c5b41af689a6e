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
// Records arrive 64 at a time in one coalesced load (the next 64 are loaded
// while these are gridded); each lane decodes the record it loaded (footprint
// origin, tap-table rows), and the decoded fields are broadcast with readlane.
// Per record and lane the work is two table reads, three multiplies, two
// conversions, a three-instruction in-tile test and two atomics; the table
// reads of the next four records are issued before the atomics of the current
// four.  Taps outside the tile are skipped: a record whose footprint straddles
// tile edges was binned into every tile it touches.
//
// After the records the tile is written to HBM once, row-coalesced:
//   - bins with a single chunk own their tile and store it, or add it to the
//     tile's contents if an earlier rick_grid since the reset wrote that tile;
//   - bins split over several chunks (the dense uv centre) add their partial
//     tiles with atomics onto a tile zeroed beforehand (unless an earlier
//     rick_grid wrote it).
// Empty bins have no work item and write nothing: a bitmap of written tiles
// (set after gridding, cleared by rick_reset) tells the FFT which tiles hold
// values; the others stand for zeros and are never read.
#include "rick_internal.h"

namespace rick {

namespace {

constexpr int kGridBlock = 512;   // 8 waves share one tile
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

// Heavy bins (several chunks) are zeroed before gridding, unless an earlier
// rick_grid wrote the tile; the scan lists them.
template <typename real>
__global__ __launch_bounds__(kZeroBlock) void k_zero_heavy(Geom g, const int32_t *__restrict__ heavy_bins,
                                                           const Stats *__restrict__ st,
                                                           const uint64_t *__restrict__ tile_bits,
                                                           real *__restrict__ mesh) {
    using r2 = typename real2_t<real>::type;
    r2 *m = reinterpret_cast<r2 *>(mesh);
    const int32_t nheavy = (int32_t)st->n_heavy;
    for (int32_t hb = blockIdx.x; hb < nheavy; hb += gridDim.x) {
        const int32_t b = heavy_bins[hb];
        const int32_t k = b / (g.nt * g.nt);
        const int32_t rem = b - k * g.nt * g.nt;
        if (tile_set(tile_bits, g, k, rem / g.nt, rem % g.nt)) continue;
        const int32_t y0 = (rem / g.nt) << g.log2T, x0 = (rem % g.nt) << g.log2T;
        for (int32_t c = threadIdx.x; c < g.T * g.T; c += kZeroBlock) {
            const int32_t y = c >> g.log2T, x = c & (g.T - 1);
            m[((int64_t)k * g.N + y0 + y) * g.N + x0 + x] = r2{0, 0};
        }
    }
}

// Offset (in doubles) of the imaginary accumulator plane from the real one:
// the size of a 64-row plane, a compile-time constant so that the second
// atomic of a tap reuses the first one's address register with an immediate
// offset.  It is a multiple of 32 doubles, so both planes map a footprint to
// the same LDS banks.
template <int W>
constexpr int im_plane_offset() { return 64 * (64 + W % 32); }

// Records per group.  The tap-table reads of the next group are issued before
// the atomics of this one, so a wait for table values never waits for the
// atomics just issued (LDS operations complete in order).
constexpr int kGroup = 4;

template <typename real, int W>
__global__ __launch_bounds__(kGridBlock) void k_grid(Geom g, const BinScan *__restrict__ scan,
                                                     const int32_t *__restrict__ item_bin,
                                                     const uint32_t *__restrict__ rec_pos,
                                                     const real *__restrict__ rec_vis, const real *__restrict__ lut,
                                                     real *__restrict__ mesh, const uint64_t *__restrict__ tile_bits) {
    constexpr int W2 = W * W;
    constexpr int NG = (W2 + 63) / 64;   // groups of 64 taps
    constexpr int H = (W - 1) / 2;
    constexpr int nwave = kGridBlock / 64;
    constexpr int KOFF = im_plane_offset<W>();
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
    if (n <= 0) return;   // (empty bins have no work item)
    // LDS: real plane at byte 0, imaginary plane KOFF doubles further, then the tap table
    double *acc_re = reinterpret_cast<double *>(smem);
    double *acc_im = acc_re + KOFF;
    const int32_t lut_byte = (KOFF + T * P) * (int32_t)sizeof(double);
    real *s_lut = reinterpret_cast<real *>(smem + lut_byte);
    for (int i = threadIdx.x; i < T * P; i += kGridBlock) {
        acc_re[i] = 0.0;
        acc_im[i] = 0.0;
    }
    for (int i = threadIdx.x; i < g.OS * W; i += kGridBlock) s_lut[i] = lut[i];
    __syncthreads();

    const int lane = __lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // Per-lane tap constants: LDS byte offset of the tap from the footprint
    // origin, and the byte addresses of its tap-table columns.
    int tap_off8[NG], lut_x[NG], lut_y[NG];
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
        const int t = lane + 64 * gi;
        const bool on = t < W2;
        const int ty = on ? t / W : 0, tx = on ? t - (t / W) * W : 0;
        tap_off8[gi] = (ty * P + tx) * (int)sizeof(double);
        lut_x[gi] = lut_byte + tx * (int)sizeof(real);
        lut_y[gi] = lut_byte + ty * (int)sizeof(real);
    }

    // this wave's batches of 64 records, one record per lane; the next
    // batch's raw fields are loaded while the current one is gridded
    const int32_t nbatch = (n + 63) >> 6;
    int32_t bt = wave;
    uint32_t raw_pos = 0;
    real raw_vr = 0, raw_vi = 0;
    auto fetch = [&](int32_t bi) {
        const int32_t r = r_begin + (bi << 6) + lane;
        if (r < r_end) {
            raw_pos = rec_pos[r];
            raw_vr = rec_vis[2 * (int64_t)r];
            raw_vi = rec_vis[2 * (int64_t)r + 1];
        }
    };
    if (bt < nbatch) fetch(bt);
    for (; bt < nbatch; bt += nwave) {
        const int32_t cnt = min(64, r_end - (r_begin + (bt << 6)));
        // decode this lane's record: byte offset of the footprint origin in
        // the real plane (negative for origins left of or above the tile),
        // tap-table row byte offsets, visibility, and the mask of its taps
        // that fall inside the tile (bit t of group t / 64 for tap t =
        // ty W + tx: the rectangle of tx, ty with ox + tx, oy + ty in [0, T))
        int32_t d_base8 = 0, d_lxy = 0;
        real d_vr = 0, d_vi = 0;
        uint64_t d_mask[NG];
#pragma unroll
        for (int gi = 0; gi < NG; ++gi) d_mask[gi] = 0;
        if (lane < cnt) {
            const int ox = (int)(raw_pos & 0xffu) - 2 * H;
            const int oy = (int)((raw_pos >> 8) & 0xffu) - 2 * H;
            const int sx = (int)((raw_pos >> 16) & 0xffu), sy = (int)(raw_pos >> 24);
            d_base8 = (oy * P + ox) * (int)sizeof(double);
            d_lxy = (sx * W * (int)sizeof(real)) | (sy * W * (int)sizeof(real)) << 16;
            d_vr = raw_vr;
            d_vi = raw_vi;
            const int tx_lo = ox < 0 ? -ox : 0, tx_hi = T - 1 - ox < W - 1 ? T - 1 - ox : W - 1;
            const int ty_lo = oy < 0 ? -oy : 0, ty_hi = T - 1 - oy < W - 1 ? T - 1 - oy : W - 1;
            const uint64_t row = ((2ull << tx_hi) - 1) & ~((1ull << tx_lo) - 1);
#pragma unroll
            for (int ty = 0; ty < W; ++ty) {
                if (ty >= ty_lo && ty <= ty_hi) {
#pragma unroll
                    for (int gi = 0; gi < NG; ++gi) {
                        const int rel = ty * W - 64 * gi;   // bit of the row's first tap in group gi
                        if (rel >= 0 && rel < 64) d_mask[gi] |= row << rel;
                        else if (rel < 0 && rel > -W) d_mask[gi] |= row >> (-rel);
                    }
                }
            }
        }
        if (bt + nwave < nbatch) fetch(bt + nwave);

        // tap-table values of one group of records (indices past the batch
        // wrap to lanes holding a switched-off record: the reads stay in the
        // table and their values go unused)
        auto lut_reads = [&](int j, real (&gy)[kGroup][NG], real (&gx)[kGroup][NG]) {
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                const int32_t lxy = bcast(d_lxy, (j + q) & 63);
                const int32_t lx = lxy & 0xffff, ly = lxy >> 16;
#pragma unroll
                for (int gi = 0; gi < NG; ++gi) {
                    gy[q][gi] = *reinterpret_cast<const real *>(smem + (lut_y[gi] + ly));
                    gx[q][gi] = *reinterpret_cast<const real *>(smem + (lut_x[gi] + lx));
                }
            }
        };
        auto add_group = [&](int j, const real (&gy)[kGroup][NG], const real (&gx)[kGroup][NG]) {
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                const int32_t base8 = bcast(d_base8, (j + q) & 63);
                const real vr = bcast(d_vr, (j + q) & 63), vi = bcast(d_vi, (j + q) & 63);
#pragma unroll
                for (int gi = 0; gi < NG; ++gi) {
                    const uint64_t m = (uint64_t)(uint32_t)bcast((int32_t)(d_mask[gi] >> 32), (j + q) & 63) << 32 |
                                       (uint32_t)bcast((int32_t)d_mask[gi], (j + q) & 63);
                    // the products are formed outside the branch, so the wait
                    // for the table values is the same on every path
                    const real wgt = gy[q][gi] * gx[q][gi];
                    double tr = (double)(wgt * vr), ti = (double)(wgt * vi);
                    __asm__ volatile("" : "+v"(tr), "+v"(ti));   // keeps them here (emits nothing)
                    // lanes whose tap of this record lies in the tile (the mask
                    // is wave-uniform and becomes the execution mask directly)
                    if (__builtin_amdgcn_inverse_ballot_w64(m)) {
                        double *a = reinterpret_cast<double *>(smem + (base8 + tap_off8[gi]));
                        atomicAdd(a, tr);
                        atomicAdd(a + KOFF, ti);
                    }
                }
            }
        };
        // two table buffers used in turn: the reads for group j + kGroup are
        // issued before the atomics of group j, and no value is copied
        real ay[kGroup][NG], ax[kGroup][NG], by[kGroup][NG], bx[kGroup][NG];
        lut_reads(0, ay, ax);
#pragma unroll
        for (int j = 0; j < 64; j += 2 * kGroup) {
            lut_reads(j + kGroup, by, bx);
            add_group(j, ay, ax);
            if (j + kGroup >= cnt) break;
            lut_reads(j + 2 * kGroup, ay, ax);
            add_group(j + kGroup, by, bx);
            if (j + 2 * kGroup >= cnt) break;
        }
    }
    __syncthreads();

    const bool shared_tile = nchunk > 1;
    const bool accumulate = tile_set(tile_bits, g, k, rem / g.nt, rem % g.nt);
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

// After gridding: one block per plane, one wave per tile row at a time.
// Lane l of a wave takes tiles l, l + 64, ... of its row; a tile is set if it
// was set before or received records now (the ballot is the bitmap word).
// The row bits are rebuilt from the tile bits, in LDS.
constexpr int kMarkBlock = 256;
constexpr int kMaxOccWords = 8;   // tiles per axis <= 512
__global__ __launch_bounds__(kMarkBlock) void k_mark_tiles(Geom g, const BinScan *__restrict__ scan,
                                                           uint64_t *__restrict__ tile_bits,
                                                           uint64_t *__restrict__ row_bits) {
    __shared__ unsigned long long s_row[kMaxOccWords];
    const int32_t k = blockIdx.x;
    const int lane = __lane_id(), wave = threadIdx.x >> 6;
    if (threadIdx.x < kMaxOccWords) s_row[threadIdx.x] = 0;
    __syncthreads();
    for (int32_t ty = wave; ty < g.nt; ty += kMarkBlock / 64) {
        bool any = false;
        for (int32_t j = 0; j < g.occw; ++j) {
            const int32_t tx = lane + 64 * j;
            bool got = false;
            if (tx < g.nt) {
                const int64_t b = ((int64_t)k * g.nt + ty) * g.nt + tx;
                got = scan[b + 1].rec > scan[b].rec;
            }
            const int64_t wi = ((int64_t)k * g.nt + ty) * g.occw + j;
            const uint64_t word = tile_bits[wi] | __ballot(got);
            if (lane == 0) tile_bits[wi] = word;
            any = any || word != 0;
        }
        if (lane == 0 && any) atomicOr(&s_row[ty >> 6], 1ull << (ty & 63));
    }
    __syncthreads();
    if (threadIdx.x < g.occw) row_bits[(int64_t)k * g.occw + threadIdx.x] = s_row[threadIdx.x];
}

__global__ void k_clear_bits(uint64_t *__restrict__ tile_bits, int64_t n_tile, uint64_t *__restrict__ row_bits,
                             int64_t n_row) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_tile + n_row; i += stride) {
        if (i < n_tile) tile_bits[i] = 0;
        else row_bits[i - n_tile] = 0;
    }
}

template <typename real, int W>
hipError_t grid_w(const Geom &g, const BinScan *scan, const int32_t *item_bin, const uint32_t *rec_pos,
                  const real *rec_vis, const real *lut, real *mesh, const uint64_t *tile_bits, int32_t max_items,
                  hipStream_t s) {
    const size_t lds = grid_lds_bytes(g, sizeof(real));
    static bool attr = false;
    if (!attr) {
        (void)hipFuncSetAttribute((const void *)k_grid<real, W>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(160 * 1024));
        attr = true;
    }
    hipLaunchKernelGGL((k_grid<real, W>), dim3(max_items), dim3(kGridBlock), lds, s, g, scan, item_bin, rec_pos,
                       rec_vis, lut, mesh, tile_bits);
    return hipGetLastError();
}

}  // namespace

size_t grid_lds_bytes(const Geom &g, size_t real_bytes) {
    // the imaginary plane starts 64 (64 + W % 32) doubles after the real one
    const size_t koff = size_t(64) * (64 + g.W % 32);
    return (koff + size_t(g.T) * g.pitch) * sizeof(double) + size_t(g.OS) * g.W * real_bytes;
}

template <typename real>
hipError_t launch_zero_mesh(real *mesh, int64_t n_real, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_mesh<real>, dim3(8192), dim3(256), 0, s, mesh, n_real);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_zero_heavy(const Geom &g, const int32_t *heavy_bins, const Stats *st, const uint64_t *tile_bits,
                             real *mesh, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_heavy<real>, dim3(1024), dim3(kZeroBlock), 0, s, g, heavy_bins, st, tile_bits, mesh);
    return hipGetLastError();
}

hipError_t launch_mark_tiles(const Geom &g, const BinScan *scan, uint64_t *tile_bits, uint64_t *row_bits,
                             hipStream_t s) {
    if (g.occw > kMaxOccWords) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mark_tiles, dim3(g.Nw), dim3(kMarkBlock), 0, s, g, scan, tile_bits, row_bits);
    return hipGetLastError();
}

hipError_t launch_clear_bits(const Geom &g, uint64_t *tile_bits, uint64_t *row_bits, hipStream_t s) {
    const int64_t n_row = (int64_t)g.Nw * g.occw, n_tile = n_row * g.nt;
    const int64_t blocks = (n_tile + n_row + 255) / 256;
    hipLaunchKernelGGL(k_clear_bits, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, tile_bits,
                       n_tile, row_bits, n_row);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_grid(const Geom &g, const BinScan *scan, const int32_t *item_bin, const uint32_t *rec_pos,
                       const real *rec_vis, const real *lut, real *mesh, const uint64_t *tile_bits,
                       int32_t max_items, hipStream_t s) {
    switch (g.W) {
#define CASE(w) \
    case w: return grid_w<real, w>(g, scan, item_bin, rec_pos, rec_vis, lut, mesh, tile_bits, max_items, s);
        CASE(1) CASE(3) CASE(5) CASE(7) CASE(9) CASE(11) CASE(13) CASE(15)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_zero_mesh<float>(float *, int64_t, hipStream_t);
template hipError_t launch_zero_mesh<double>(double *, int64_t, hipStream_t);
template hipError_t launch_zero_heavy<float>(const Geom &, const int32_t *, const Stats *, const uint64_t *, float *,
                                             hipStream_t);
template hipError_t launch_zero_heavy<double>(const Geom &, const int32_t *, const Stats *, const uint64_t *,
                                              double *, hipStream_t);
template hipError_t launch_grid<float>(const Geom &, const BinScan *, const int32_t *, const uint32_t *,
                                       const float *, const float *, float *, const uint64_t *, int32_t,
                                       hipStream_t);
template hipError_t launch_grid<double>(const Geom &, const BinScan *, const int32_t *, const uint32_t *,
                                        const double *, const double *, double *, const uint64_t *, int32_t,
                                        hipStream_t);

}  // namespace rick
