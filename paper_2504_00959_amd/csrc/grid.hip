// LDS-tiled convolutional gridding (Sec. 2.1, Eq. 3) of binned records onto
// the w-plane stack.
//
// One block takes one work item: a chunk of at most CH records of one
// (plane, tile) bin.  A record is binned into the tile holding its
// footprint's top-left cell, so the block's accumulator (float64 re and im
// planes in LDS) covers the tile plus a margin of W - 1 cells right and below:
// (T + W - 1)^2 cells, and every footprint lies inside it.  Each wave takes
// one record at a time with one lane per kernel tap (lane t < W*W is tap
// (t / W, t % W)), so one record costs two LDS atomic adds and no lane pair
// of an instruction shares an address.  The LDS row pitch is congruent to W
// modulo 32 elements, which spreads the W x W footprint over the banks.
//
// Accumulators are 64-bit: float32 LDS atomic adds are many times slower than
// 64-bit ones on gfx950, and dense cells collect thousands of terms, which
// float32 accumulation would round to ~1e-5 of image RMS.  In float64 mode
// they are float64 (re and im planes).  In the float32 modes a cell is one
// 64-bit word holding re and im as two 32-bit fixed-point halves (below):
// each term W V g_y g_x is scaled by a power of two 2^s chosen per bin from
// the largest |W V| of the bin (found by the binning) and the largest tap,
// rounded to an integer below 2^21, and both halves are added with one
// integer atomic; integer sums do not depend on the order of the adds.
// Records arrive 64 at a time in one coalesced load (the next 64 are loaded
// while these are gridded); each lane decodes the record it loaded (footprint
// origin, tap-table rows), and the decoded fields are broadcast with readlane.
// Per record and lane the work is two table reads, three multiplies, two
// conversions and two atomics; the table reads of the next four records are
// issued before the atomics of the current four.
//
// After the records the tile is written to HBM once, row-coalesced:
//   - bins with a single chunk own their tile and store it, or add it to the
//     tile's contents if an earlier rick_grid since the reset wrote that tile;
//   - bins split over several chunks (the dense uv centre) add their partial
//     tiles with atomics onto a tile zeroed beforehand (unless an earlier
//     rick_grid wrote it).
// The margins (a strip W - 1 wide right of the tile, including the corner,
// and one W - 1 high below it) go to a per-bin margin buffer, stored (or added
// with atomics for split bins); a merge kernel then adds them to the
// neighbouring tiles, one block per tile row, each target tile written by one
// block.  Empty bins have no work item and write nothing: a bitmap of tiles
// holding values (set by the merge, cleared by rick_reset) tells the FFT which
// tiles to read; the others stand for zeros and are never read.
#include <type_traits>

#include "rick_internal.h"

namespace rick {

namespace {

// Threads of a gridding block: 16 waves share a 64-cell tile (its 80 KB of
// accumulators allow two blocks per CU), 8 waves a smaller one (more blocks fit).
constexpr int grid_threads(int T) { return T >= 64 ? 1024 : 512; }
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

// Margin buffer of a bin, in complex values: the right strip, rows
// 0 .. T + W - 2 by columns T .. T + W - 2 (row-major, W - 1 per row), then
// the bottom strip, rows T .. T + W - 2 by columns 0 .. T - 1.
__host__ __device__ inline int64_t margin_len(int32_t T, int32_t W) {
    return (int64_t)(T + W - 1) * (W - 1) + (int64_t)(W - 1) * T;
}

// Heavy bins (several chunks) are zeroed before gridding, unless an earlier
// rick_grid wrote the tile; the scan lists them.  Also zeroes the gridder's
// work-item counter.
template <typename real>
__global__ __launch_bounds__(kZeroBlock) void k_zero_heavy(Geom g, const int32_t *__restrict__ heavy_bins,
                                                           Stats *__restrict__ st,
                                                           const uint64_t *__restrict__ tile_bits,
                                                           const int32_t *__restrict__ plane_tr,
                                                           real *__restrict__ mesh, real *__restrict__ margin) {
    using r2 = typename real2_t<real>::type;
    r2 *m = reinterpret_cast<r2 *>(mesh);
    const int32_t nheavy = (int32_t)st->n_heavy;
    if (blockIdx.x == 0 && threadIdx.x == 0) st->grid_next = 0;
    const int64_t mlen = margin_len(g.T, g.W);
    for (int32_t hb = blockIdx.x; hb < nheavy; hb += gridDim.x) {
        const int32_t b = heavy_bins[hb];
        // the margin buffer is filled anew by every rick_grid
        r2 *mb = reinterpret_cast<r2 *>(margin) + (int64_t)b * mlen;
        for (int64_t c = threadIdx.x; c < mlen; c += kZeroBlock) mb[c] = r2{0, 0};
        const int32_t k = b / (g.nt * g.nt);
        const int32_t rem = b - k * g.nt * g.nt;
        // the tile in the stored orientation of its plane
        const bool tr = plane_transposed(plane_tr, k);
        const int32_t sty = tr ? rem % g.nt : rem / g.nt, stx = tr ? rem / g.nt : rem % g.nt;
        if (tile_set(tile_bits, g, k, sty, stx)) continue;
        const int32_t y0 = sty << g.log2T, x0 = stx << g.log2T;
        for (int32_t c = threadIdx.x; c < g.T * g.T; c += kZeroBlock) {
            const int32_t y = c >> g.log2T, x = c & (g.T - 1);
            m[((int64_t)k * g.N + y0 + y) * g.N + x0 + x] = r2{0, 0};
        }
    }
}

// Offset (in doubles) of the imaginary accumulator plane from the real one:
// the size of a plane (T + W - 1 rows of the pitch), a compile-time constant
// (the kernel is instantiated per tile size) so that the second atomic of a
// tap reuses the first one's address register with an immediate offset.  It is a multiple of 32
// doubles, so both planes map a footprint to the same LDS banks.
constexpr int acc_pitch(int T, int W) {
    int p = T + W - 1;   // at least the tile and its margin, congruent to W mod 32
    while ((p - W) % 32 != 0) ++p;
    return p;
}
constexpr int plane_offset(int W, int T) { return ((T + W - 1) * acc_pitch(T, W) + 31) / 32 * 32; }
template <int W, int T>
constexpr int im_plane_offset() { return plane_offset(W, T); }


// Records per group.  The tap-table reads of the next group are issued before
// the atomics of this one, so a wait for table values never waits for the
// atomics just issued (LDS operations complete in order).
constexpr int kGroup = 4;

// Packed float32 accumulation: re and im of a cell share one 64-bit
// LDS word, re in the low and im in the high 32 bits, as the integer
// im 2^32 + re; one ds_add_u64 then adds both.  Each term is rounded to an
// integer below 2^21 (the scale 2^s follows the bin's largest possible
// term), and the block drains the LDS words into 64-bit integer sums held in
// registers (each thread owns a fixed set of cells) after every round of at
// most 1024 records, so a half never sums more than 1024 terms and stays
// inside its signed 32 bits: re is the sign-extended low word, im the rest
// shifted down by 32, exactly.  A term is rounded by one float32 fma against
// 1.5 2^23, which leaves 1.5 2^23 + round(x) with bit pattern
// 0x4B400000 + round(x) for |x| < 2^22; subtracting that constant from both
// halves of the pair at once gives im 2^32 + re.  The precision is that of
// the rounding, 2^-21 of the bin's largest possible term, whatever the
// number of records.
constexpr float kRoundMagic32 = 12582912.0f;   // 1.5 2^23
constexpr unsigned long long kPackBias = 0x4B4000004B400000ull;
constexpr int kPackTermBits = 21;
__device__ __forceinline__ unsigned long long pack_terms(float tr, float ti) {
    return (((unsigned long long)__float_as_uint(ti) << 32) | __float_as_uint(tr)) - kPackBias;
}
__device__ __forceinline__ void unpack_terms(unsigned long long s, long long &re, long long &im) {
    const int32_t lo = (int32_t)(uint32_t)s;
    re = lo;
    im = ((long long)s - (long long)lo) >> 32;
}

// L3: the taps come from a non-separable table in device memory,
// T[iw][s_y][s_x][t_y][t_x] (w-fraction bin iw in bits 6-7 and 14 of the
// packed position), one value per tap instead of the product of two
// separable rows held in LDS; tapmax points at the table's largest |value|.
// float32: packed accumulation (above); float64: float64 re and im planes.

// Per-lane tap constants: LDS byte offset of the tap from the footprint
// origin, and the byte addresses of its tap-table columns (L3: the tap's
// index in a table row; lanes past the footprint read the row's last tap,
// whose values go unused).
template <typename real, int W, bool L3>
__device__ __forceinline__ void tap_constants(int32_t P, int32_t lut_byte, int (&tap_off8)[(W * W + 63) / 64],
                                              int (&lut_x)[(W * W + 63) / 64], int (&lut_y)[(W * W + 63) / 64]) {
    constexpr int W2 = W * W;
    const int lane = __lane_id();
#pragma unroll
    for (int gi = 0; gi < (W2 + 63) / 64; ++gi) {
        const int t = lane + 64 * gi;
        const bool on = t < W2;
        const int ty = on ? t / W : 0, tx = on ? t - (t / W) * W : 0;
        tap_off8[gi] = (ty * P + tx) * (int)sizeof(double);
        lut_x[gi] = lut_byte + tx * (int)sizeof(real);
        lut_y[gi] = L3 ? (on ? t : W2 - 1) : lut_byte + ty * (int)sizeof(real);
    }
}

// LDS byte offset of the separable tap table: after the real plane (and the
// imaginary one in float64 mode), T + W - 1 rows of pitch P each.
template <typename real, int W, int TT>
__device__ __forceinline__ int32_t lut_byte_of(int32_t P) {
    constexpr bool P32 = std::is_same<real, float>::value;
    return ((P32 ? 0 : im_plane_offset<W, TT>()) + (TT + W - 1) * P) * (int32_t)sizeof(double);
}

// One work item (a chunk of at most CH records of one bin) through the
// block: the records accumulated in LDS, then the tile and its margins
// written out.  The separable tap table is in LDS already (written before
// this call; the first barrier here makes it visible).  Ends with the
// accumulators read out but before the block's closing barrier.
template <typename real, int W, int TT, bool L3>
__device__ __forceinline__ void grid_item(const Geom &g, const BinScan *__restrict__ scan,
                                          const int32_t *__restrict__ item_bin, const uint32_t *__restrict__ rec_pos,
                                          const real *__restrict__ rec_vis, const real *__restrict__ lut,
                                          real *__restrict__ mesh, const uint64_t *__restrict__ tile_bits,
                                          real *__restrict__ margin, const uint32_t *__restrict__ bin_vmax,
                                          const float *__restrict__ tapmax, const int32_t *__restrict__ plane_tr,
                                          int32_t item, const int (&tap_off8)[(W * W + 63) / 64],
                                          const int (&lut_x)[(W * W + 63) / 64],
                                          const int (&lut_y)[(W * W + 63) / 64]) {
    constexpr bool P32 = std::is_same<real, float>::value;   // packed fixed point
    constexpr int W2 = W * W;
    constexpr int NG = (W2 + 63) / 64;   // groups of 64 taps
    constexpr int kGridBlock = grid_threads(TT);
    constexpr int nwave = kGridBlock / 64;
    constexpr int KOFF = im_plane_offset<W, TT>();   // TT == g.T
    // packed mode: LDS cells owned per thread (cell i by thread i mod the block size)
    constexpr int CPT = ((TT + W - 1) * acc_pitch(TT, W) + kGridBlock - 1) / kGridBlock;
    static_assert(kGridBlock <= (1 << (31 - kPackTermBits)), "a drain round must stay within 32-bit halves");
    extern __shared__ __align__(16) unsigned char smem[];
    const int32_t T = g.T, P = g.pitch;
    using r2 = typename real2_t<real>::type;
    r2 *m = reinterpret_cast<r2 *>(mesh);
    using acc_t = typename std::conditional<P32, unsigned long long, double>::type;
    using vreg_t = typename std::conditional<P32, float, double>::type;   // W V as the taps multiply it
    // LDS: real plane at byte 0, imaginary plane KOFF doubles further (not
    // with P32), then the tap table; a plane is R = T + W - 1 rows of pitch P
    constexpr int R_PAD = W - 1;
    const int32_t R = T + R_PAD;
    acc_t *acc_re = reinterpret_cast<acc_t *>(smem);
    acc_t *acc_im = acc_re + KOFF;
    const int lane = __lane_id();
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);

    const int32_t b = item_bin[item];
    const int32_t first = scan[b].item;
    const int32_t nchunk = scan[b + 1].item - first;
    const int32_t chunk = item - first;
    const int32_t r_begin = scan[b].rec + chunk * g.CH;
    int32_t r_end = r_begin + g.CH;
    if (r_end > scan[b + 1].rec) r_end = scan[b + 1].rec;
    const int32_t n = r_end - r_begin;   // > 0: empty bins have no work item
    const int32_t k = b / (g.nt * g.nt);
    const int32_t rem = b - k * g.nt * g.nt;
    const int32_t y0 = (rem / g.nt) << g.log2T, x0 = (rem % g.nt) << g.log2T;
    double scale = 1.0, unscale = 1.0;
    if (P32) {
        const double vmax = (double)__uint_as_float(bin_vmax[b]);   // largest |W V| of the bin
        // largest |term|: |W V| times the largest |tap| (the square of the
        // largest separable row value, or the largest entry of the table)
        const double bt = vmax * (L3 ? (double)*tapmax * (1.0 + 1e-6) : (double)g.gmax2);
        if (bt > 0.0 && bt < 1e300) {
            const int et = ilogb(bt) + 1;   // bt < 2^et
            const int sh = min(kPackTermBits - et, 120);   // (2^s stays a normal float32)
            scale = ldexp(1.0, sh);
            unscale = ldexp(1.0, -sh);
        }
    }
    // packed mode: this thread's cells' sums (cell threadIdx.x + j kGridBlock)
    long long own_re[P32 ? CPT : 1], own_im[P32 ? CPT : 1];
#pragma unroll
    for (int j = 0; j < (P32 ? CPT : 1); ++j) own_re[j] = own_im[j] = 0;
    auto drain = [&]() {
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int32_t i = (int32_t)threadIdx.x + j * kGridBlock;
            if (i < R * P) {
                long long re, im;
                unpack_terms(acc_re[i], re, im);
                acc_re[i] = 0;
                own_re[j] += re;
                own_im[j] += im;
            }
        }
    };
    // accumulated value of LDS cell i (packed mode: the float32 pair the
    // owners stored there after the last drain)
    auto cell = [&](int32_t i, real &re, real &im) {
        if constexpr (P32) {
            const float2 v = reinterpret_cast<const float2 *>(acc_re)[i];
            re = v.x;
            im = v.y;
        } else {
            re = (real)acc_re[i];
            im = (real)acc_im[i];
        }
    };
    for (int i = threadIdx.x; i < R * P; i += kGridBlock) {
        acc_re[i] = 0;
        if (!P32) acc_im[i] = 0;
    }
    __syncthreads();

    // this wave's batches of 64 records, one record per lane; the next
    // batch's raw fields are loaded while the current one is gridded
    const int32_t nbatch = (n + 63) >> 6;
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
    if (wave < nbatch) fetch(wave);
    // rounds of one batch per wave (packed mode: drained after each round)
    for (int32_t round0 = 0; round0 < nbatch; round0 += nwave) {
      const int32_t bt = round0 + wave;
      if (bt < nbatch) {
        const int32_t cnt = min(64, r_end - (r_begin + (bt << 6)));
        // decode this lane's record: byte offset of the footprint origin in
        // the real plane, tap-table row byte offsets and visibility (lanes
        // past the batch keep zeros: they add 0 at the region's origin)
        int32_t d_base8 = 0, d_lxy = 0;
        vreg_t d_vr = 0, d_vi = 0;   // W V times 2^s in float32 modes (exact)
        if (lane < cnt) {
            const int sx = (int)((raw_pos >> 16) & 0xffu), sy = (int)(raw_pos >> 24);
            if constexpr (L3) {
                const int ox = (int)(raw_pos & 0x3fu), oy = (int)((raw_pos >> 8) & 0x3fu);   // in [0, T)
                const int iw = (int)((raw_pos >> 6) & 3u) | (int)((raw_pos >> 14) & 1u) << 2;
                d_base8 = (oy * P + ox) * (int)sizeof(double);
                d_lxy = ((iw * g.OS + sy) * g.OS + sx) * W2;   // first entry of the record's table row
            } else {
                const int ox = (int)(raw_pos & 0xffu), oy = (int)((raw_pos >> 8) & 0xffu);   // in [0, T)
                d_base8 = (oy * P + ox) * (int)sizeof(double);
                d_lxy = (sx * W * (int)sizeof(real)) | (sy * W * (int)sizeof(real)) << 16;
            }
            d_vr = (vreg_t)((double)raw_vr * scale);
            d_vi = (vreg_t)((double)raw_vi * scale);
        }
        if (bt + nwave < nbatch) fetch(bt + nwave);

        // tap-table values of one group of records (indices past the batch
        // wrap to lanes holding a switched-off record: the reads stay in the
        // table and their values go unused)
        auto lut_reads = [&](int j, real (&gy)[kGroup][NG], real (&gx)[kGroup][NG]) {
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                const int32_t lxy = bcast(d_lxy, (j + q) & 63);
                if constexpr (L3) {
#pragma unroll
                    for (int gi = 0; gi < NG; ++gi) {
                        gy[q][gi] = lut[lxy + lut_y[gi]];
                        gx[q][gi] = (real)1;
                    }
                } else {
                    const int32_t lx = lxy & 0xffff, ly = lxy >> 16;
#pragma unroll
                    for (int gi = 0; gi < NG; ++gi) {
                        gy[q][gi] = *reinterpret_cast<const real *>(smem + (lut_y[gi] + ly));
                        gx[q][gi] = *reinterpret_cast<const real *>(smem + (lut_x[gi] + lx));
                    }
                }
            }
        };
        auto add_group = [&](int j, const real (&gy)[kGroup][NG], const real (&gx)[kGroup][NG]) {
#pragma unroll
            for (int q = 0; q < kGroup; ++q) {
                const int32_t base8 = bcast(d_base8, (j + q) & 63);
                const vreg_t vr = bcast(d_vr, (j + q) & 63), vi = bcast(d_vi, (j + q) & 63);
#pragma unroll
                for (int gi = 0; gi < NG; ++gi) {
                    // lanes holding a tap of group gi (a compile-time mask)
                    constexpr uint64_t kAll = ~0ull;
                    const uint64_t msk = W2 - 64 * gi >= 64 ? kAll : (1ull << (W2 - 64 * gi)) - 1;
                    // the products are formed outside the branch, so the wait
                    // for the table values is the same on every path
                    const real wgt = gy[q][gi] * gx[q][gi];
                    if constexpr (P32) {
                        // round(g V 2^s) of re and im, then both as one 64-bit word
                        float tr = fmaf(wgt, vr, kRoundMagic32);
                        float ti = fmaf(wgt, vi, kRoundMagic32);
                        __asm__ volatile("" : "+v"(tr), "+v"(ti));   // keeps them here (emits nothing)
                        if (NG == 1 || __builtin_amdgcn_inverse_ballot_w64(msk)) {
                            acc_t *a = reinterpret_cast<acc_t *>(smem + (base8 + tap_off8[gi]));
                            atomicAdd(a, pack_terms(tr, ti));
                        }
                    } else {
                        double tr = wgt * vr, ti = wgt * vi;
                        __asm__ volatile("" : "+v"(tr), "+v"(ti));   // keeps them here (emits nothing)
                        // (with one tap group the whole record loop already runs on the tap lanes)
                        if (NG == 1 || __builtin_amdgcn_inverse_ballot_w64(msk)) {
                            acc_t *a = reinterpret_cast<acc_t *>(smem + (base8 + tap_off8[gi]));
                            atomicAdd(a, tr);
                            atomicAdd(a + KOFF, ti);
                        }
                    }
                }
            }
        };
        // two table buffers used in turn: the reads for group j + kGroup are
        // issued before the atomics of group j, and no value is copied.  With
        // one tap group (W <= 7) the loop runs on the tap lanes only: the
        // execution mask is set once per batch, not per record (readlane
        // reads the records of the other lanes regardless).
        if (NG > 1 || lane < W2) {
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
      }
      if constexpr (P32) {
          __syncthreads();   // the round's atomics are done
          drain();
          __syncthreads();   // the cells are zero again
      }
    }
    if constexpr (P32) {
        // the sums as float32 pairs in the cells, for the row-coalesced flush
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int32_t i = (int32_t)threadIdx.x + j * kGridBlock;
            if (i < R * P)
                reinterpret_cast<float2 *>(acc_re)[i] =
                    float2{(float)((double)own_re[j] * unscale), (float)((double)own_im[j] * unscale)};
        }
    }
    __syncthreads();

    const bool shared_tile = nchunk > 1;
    // a transposed plane: cell (y, x) at row x, column y, and the tile's bit
    // at (tile column, tile row); consecutive threads take consecutive
    // stored columns either way
    const bool tr = plane_transposed(plane_tr, k);
    const bool accumulate =
        tr ? tile_set(tile_bits, g, k, rem % g.nt, rem / g.nt) : tile_set(tile_bits, g, k, rem / g.nt, rem % g.nt);
    for (int32_t c = threadIdx.x; c < T * T; c += kGridBlock) {
        const int32_t hi = c >> g.log2T, lo = c & (T - 1);
        const int32_t y = tr ? lo : hi, x = tr ? hi : lo;
        real re, im;
        cell(y * P + x, re, im);
        r2 *dst = tr ? m + ((int64_t)k * g.N + x0 + x) * g.N + y0 + y : m + ((int64_t)k * g.N + y0 + y) * g.N + x0 + x;
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
    // margins to the bin's margin buffer (the merge adds them to the neighbours)
    if constexpr (R_PAD > 0) {
        r2 *mb = reinterpret_cast<r2 *>(margin) + (int64_t)b * margin_len(T, W);
        const int32_t n_right = R * R_PAD, n_all = n_right + R_PAD * T;
        for (int32_t c = threadIdx.x; c < n_all; c += kGridBlock) {
            int32_t y, x;
            if (c < n_right) {
                y = c / R_PAD;
                x = T + (c - y * R_PAD);
            } else {
                const int32_t d = c - n_right;
                y = T + (d >> g.log2T);
                x = d & (T - 1);
            }
            real re, im;
            cell(y * P + x, re, im);
            if (shared_tile) {
                if (re != 0) atomic_add_real(&mb[c].x, re);
                if (im != 0) atomic_add_real(&mb[c].y, im);
            } else {
                mb[c] = r2{re, im};
            }
        }
    }
}

// Persistent: a block takes work items blockIdx.x, then the next unclaimed
// one from st->grid_next (claimed while the current one is gridded), until
// the device-side item count is reached.
template <typename real, int W, int TT, bool L3>
__global__ __launch_bounds__(grid_threads(TT), W <= 7 ? 8 : 1) void k_grid(Geom g, const BinScan *__restrict__ scan,
                                                     const int32_t *__restrict__ item_bin,
                                                     const uint32_t *__restrict__ rec_pos,
                                                     const real *__restrict__ rec_vis, const real *__restrict__ lut,
                                                     real *__restrict__ mesh, const uint64_t *__restrict__ tile_bits,
                                                     real *__restrict__ margin,
                                                     const uint32_t *__restrict__ bin_vmax,
                                                     const float *__restrict__ tapmax, Stats *__restrict__ st,
                                                     const int32_t *__restrict__ plane_tr) {
    constexpr int NG = (W * W + 63) / 64;
    constexpr int kGridBlock = grid_threads(TT);
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t s_next[2];
    const int32_t total = scan[g.nbins].item;
    if ((int32_t)blockIdx.x >= total) return;
    const int32_t lut_byte = lut_byte_of<real, W, TT>(g.pitch);
    real *s_lut = reinterpret_cast<real *>(smem + lut_byte);
    if (!L3)
        for (int i = threadIdx.x; i < g.OS * W; i += kGridBlock) s_lut[i] = lut[i];
    // (visible after the first item's barrier)
    int tap_off8[NG], lut_x[NG], lut_y[NG];
    tap_constants<real, W, L3>(g.pitch, lut_byte, tap_off8, lut_x, lut_y);

    int32_t item = blockIdx.x;
    for (int it = 0; item < total; ++it) {
        // claim the next item now; it is read after this one's last barrier
        if (threadIdx.x == 0) s_next[it & 1] = (int32_t)gridDim.x + (int32_t)atomicAdd(&st->grid_next, 1ull);
        grid_item<real, W, TT, L3>(g, scan, item_bin, rec_pos, rec_vis, lut, mesh, tile_bits, margin, bin_vmax,
                                   tapmax, plane_tr, item, tap_off8, lut_x, lut_y);
        __syncthreads();   // the accumulators are read out; s_next is written
        item = s_next[it & 1];
    }
}

// Gridding of several jobs (plans) in one persistent launch over a
// device-side queue: the work items of the jobs, in job order, form one
// sequence; a block takes item blockIdx.x, then the next unclaimed one from
// the shared counter, finds its job from the prefix of the jobs' item counts
// (read on the device after their binning) and grids it with that job's
// operands.  Every job of a launch has the same support and tile edge
// (instantiation parameters) and a separable tap table; the table is loaded
// into LDS when a block moves to another job.
typedef __attribute__((address_space(4))) const GridJob const_job;
typedef __attribute__((address_space(4))) const uint32_t const_u32;
// a job's operands, read through the constant address space (the job is the
// same for the whole block: scalar loads into scalar registers)
__device__ __forceinline__ GridJob load_job(const GridJob *p) {
    static_assert(sizeof(GridJob) % 4 == 0, "whole words");
    GridJob v;
    uint32_t *dst = reinterpret_cast<uint32_t *>(&v);
    const const_u32 *src = (const const_u32 *)p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(GridJob) / 4); ++i) dst[i] = src[i];
    return v;
}
template <typename real, int W, int TT>
__global__ __launch_bounds__(grid_threads(TT), W <= 7 ? 8 : 1) void k_grid_jobs(GridJobList list,
                                                                                unsigned long long *__restrict__ next) {
    constexpr int NG = (W * W + 63) / 64;
    constexpr int kGridBlock = grid_threads(TT);
    constexpr int32_t P = acc_pitch(TT, W);   // the pitch of every job of the launch
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int32_t s_next[2];
    __shared__ int32_t s_pre[kMaxGridJobs + 1];   // first item of each job; total at [n]
    const int32_t n = list.n;
    if ((int)threadIdx.x < n) {
        const const_job *J = (const const_job *)list.job[threadIdx.x];
        s_pre[threadIdx.x + 1] = J->scan[J->g.nbins].item;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s_pre[0] = 0;
        for (int32_t j = 0; j < n; ++j) s_pre[j + 1] += s_pre[j];
    }
    __syncthreads();
    const int32_t total = s_pre[n];
    if ((int32_t)blockIdx.x >= total) return;
    const int32_t lut_byte = lut_byte_of<real, W, TT>(P);
    real *s_lut = reinterpret_cast<real *>(smem + lut_byte);
    int tap_off8[NG], lut_x[NG], lut_y[NG];
    tap_constants<real, W, false>(P, lut_byte, tap_off8, lut_x, lut_y);

    int32_t cur = -1;   // the job whose tap table is in LDS
    int32_t item = blockIdx.x;
    for (int it = 0; item < total; ++it) {
        if (threadIdx.x == 0) s_next[it & 1] = (int32_t)gridDim.x + (int32_t)atomicAdd(next, 1ull);
        int32_t j = 0;
        while (j + 1 < n && s_pre[j + 1] <= item) ++j;
        j = __builtin_amdgcn_readfirstlane(j);
        const GridJob J = load_job(list.job[j]);
        const Geom &g = J.g;
        const real *lut = (const real *)J.lut;
        // (the previous item's table reads ended before its last barrier; the
        // first barrier of this item makes the new table visible)
        if (j != cur)
            for (int i = threadIdx.x; i < g.OS * W; i += kGridBlock) s_lut[i] = lut[i];
        cur = j;
        grid_item<real, W, TT, false>(g, J.scan, J.item_bin, J.rec_pos, (const real *)J.rec_vis, lut,
                                      (real *)J.mesh, J.tile_bits, (real *)J.margin, J.bin_vmax, nullptr,
                                      J.plane_tr, item - s_pre[j], tap_off8, lut_x, lut_y);
        __syncthreads();   // the accumulators are read out; s_next is written
        item = s_next[it & 1];
    }
}

template <typename real>
__global__ void k_zero_mesh(real *__restrict__ a, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = 0;
}

// After gridding: one block per tile row (plane k, row ty).  A tile ends up
// set if it was set before, received records now, or receives margins now
// from its left, upper or upper-left neighbour (records in those bins).  Each
// tile receiving margins is written by this block only: cells are read (or
// taken as zero for a tile that held nothing, whose stale contents are
// replaced) and the margin pieces added; the row's bitmap words are then
// written.  The gridder has finished, so every margin buffer is complete.
constexpr int kMergeBlock = 256;
constexpr int kMaxOccWords = 8;   // tiles per axis <= 512
template <typename real>
__global__ __launch_bounds__(kMergeBlock) void k_merge_margins(Geom g, const BinScan *__restrict__ scan,
                                                               const real *__restrict__ margin,
                                                               uint64_t *__restrict__ tile_bits,
                                                               const int32_t *__restrict__ plane_tr,
                                                               real *__restrict__ mesh) {
    using r2 = typename real2_t<real>::type;
    __shared__ unsigned long long s_word[kMaxOccWords];
    __shared__ int32_t s_list[512], s_n;
    const int32_t k = blockIdx.x / g.nt, ty = blockIdx.x % g.nt;
    const int32_t T = g.T, W1 = g.W - 1;
    // a transposed plane keeps cell (y, x) at row x, column y, and the bit of
    // tile (ty, tx) at (tx, ty): bits of other blocks share its words
    const bool tr = plane_transposed(plane_tr, k);
    // the bins of a tile row are consecutive: no record in this tile row or
    // the one above means no tile here changes (no records, no margins)
    const int64_t b_row = ((int64_t)k * g.nt + ty) * g.nt;
    if (!(scan[b_row + g.nt].rec > scan[b_row].rec) && !(ty > 0 && scan[b_row].rec > scan[b_row - g.nt].rec)) return;
    if (threadIdx.x < kMaxOccWords) s_word[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    auto has = [&](int32_t yy, int32_t xx) {
        const int64_t b = ((int64_t)k * g.nt + yy) * g.nt + xx;
        return scan[b + 1].rec > scan[b].rec;
    };
    const int64_t row_w = ((int64_t)k * g.nt + ty) * g.occw;
    for (int32_t tx = threadIdx.x; tx < g.nt; tx += kMergeBlock) {
        const bool old = tr ? tile_set(tile_bits, g, k, tx, ty) : ((tile_bits[row_w + (tx >> 6)] >> (tx & 63)) & 1ull);
        const bool set = old || has(ty, tx);
        const bool l = W1 > 0 && tx > 0 && has(ty, tx - 1);
        const bool u = W1 > 0 && ty > 0 && has(ty - 1, tx);
        const bool ul = W1 > 0 && tx > 0 && ty > 0 && has(ty - 1, tx - 1);
        if (l || u || ul) s_list[atomicAdd(&s_n, 1)] = tx | (int32_t)set << 16 | (int32_t)l << 17 |
                                                         (int32_t)u << 18 | (int32_t)ul << 19;
        if (set || l || u || ul) atomicOr(&s_word[tx >> 6], 1ull << (tx & 63));
    }
    __syncthreads();
    const int64_t mlen = margin_len(T, g.W);
    const int32_t R = T + W1;
    r2 *m = reinterpret_cast<r2 *>(mesh);
    const r2 *mg = reinterpret_cast<const r2 *>(margin);
    for (int32_t i = 0; i < s_n; ++i) {
        const int32_t e = s_list[i];
        const int32_t tx = e & 0xffff;
        const bool set = (e >> 16) & 1, l = (e >> 17) & 1, u = (e >> 18) & 1, ul = (e >> 19) & 1;
        // margin buffers of the left (right strip), upper (bottom strip) and
        // upper-left (corner rows of the right strip) neighbours
        const int32_t txl = l || ul ? tx - 1 : tx, tyu = u || ul ? ty - 1 : ty;
        const r2 *ml = mg + (((int64_t)k * g.nt + ty) * g.nt + txl) * mlen;
        const r2 *mu = mg + (((int64_t)k * g.nt + tyu) * g.nt + tx) * mlen + R * W1;
        const r2 *mul = mg + (((int64_t)k * g.nt + tyu) * g.nt + txl) * mlen;
        for (int32_t c = threadIdx.x; c < T * T; c += kMergeBlock) {
            const int32_t hi = c >> g.log2T, lo = c & (T - 1);
            const int32_t y = tr ? lo : hi, x = tr ? hi : lo;
            const bool hl = l && x < W1, hu = u && y < W1, hul = ul && x < W1 && y < W1;
            if (set && !(hl || hu || hul)) continue;   // a cell no margin reaches keeps its value
            const int64_t gy = ((int64_t)ty << g.log2T) + y, gx = ((int64_t)tx << g.log2T) + x;
            r2 *dst = tr ? m + ((int64_t)k * g.N + gx) * g.N + gy : m + ((int64_t)k * g.N + gy) * g.N + gx;
            r2 v = set ? *dst : r2{0, 0};
            if (hl) {
                const r2 a = ml[y * W1 + x];
                v.x += a.x;
                v.y += a.y;
            }
            if (hu) {
                const r2 a = mu[y * T + x];
                v.x += a.x;
                v.y += a.y;
            }
            if (hul) {
                const r2 a = mul[(T + y) * W1 + x];
                v.x += a.x;
                v.y += a.y;
            }
            *dst = v;
        }
    }
    if (!tr) {
        if (threadIdx.x < g.occw) tile_bits[row_w + threadIdx.x] = s_word[threadIdx.x];
    } else {
        for (int32_t tx = threadIdx.x; tx < g.nt; tx += kMergeBlock)
            if ((s_word[tx >> 6] >> (tx & 63)) & 1ull)
                atomicOr((unsigned long long *)&tile_bits[((int64_t)k * g.nt + tx) * g.occw + (ty >> 6)],
                         1ull << (ty & 63));
    }
}

// Orientation of each plane that holds no set tile: one block per plane
// marks the tile rows and tile columns its records reach (a record's bin and,
// through the margins, the bins right of, below and diagonally below-right of
// it) and stores the plane transposed iff fewer tile columns than tile rows
// are reached.
constexpr int kOrientBlock = 256;
__global__ __launch_bounds__(kOrientBlock) void k_orient(Geom g, const BinScan *__restrict__ scan,
                                                        const uint64_t *__restrict__ row_bits,
                                                        int32_t *__restrict__ plane_tr) {
    __shared__ int32_t s_rows[512], s_cols[512];
    __shared__ int32_t s_nr, s_nc;
    const int32_t k = blockIdx.x;
    bool held = false;
    for (int32_t w = 0; w < g.occw; ++w) held = held || row_bits[(int64_t)k * g.occw + w] != 0;
    if (held) return;   // (uniform) tiles already stored keep their orientation
    for (int32_t i = threadIdx.x; i < g.nt; i += kOrientBlock) s_rows[i] = s_cols[i] = 0;
    if (threadIdx.x == 0) s_nr = s_nc = 0;
    __syncthreads();
    const int32_t spill = g.W > 1 ? 1 : 0;
    for (int32_t t = threadIdx.x; t < g.nt * g.nt; t += kOrientBlock) {
        const int64_t b = (int64_t)k * g.nt * g.nt + t;
        if (scan[b + 1].rec > scan[b].rec) {
            const int32_t ty = t / g.nt, tx = t % g.nt;
            s_rows[ty] = 1;
            s_cols[tx] = 1;
            if (spill && ty + 1 < g.nt) s_rows[ty + 1] = 1;
            if (spill && tx + 1 < g.nt) s_cols[tx + 1] = 1;
        }
    }
    __syncthreads();
    int32_t nr = 0, nc = 0;
    for (int32_t i = threadIdx.x; i < g.nt; i += kOrientBlock) {
        nr += s_rows[i];
        nc += s_cols[i];
    }
    atomicAdd(&s_nr, nr);
    atomicAdd(&s_nc, nc);
    __syncthreads();
    if (threadIdx.x == 0) plane_tr[k] = s_nc < s_nr ? 1 : 0;
}

// Row bitmap from the tile bitmap: one block per plane, one lane per tile row.
__global__ __launch_bounds__(64) void k_row_bits(Geom g, const uint64_t *__restrict__ tile_bits,
                                                 uint64_t *__restrict__ row_bits) {
    const int32_t k = blockIdx.x;
    for (int32_t j = 0; j < g.occw; ++j) {
        const int32_t ty = 64 * j + (int32_t)threadIdx.x;
        bool any = false;
        if (ty < g.nt)
            for (int32_t w = 0; w < g.occw; ++w) any = any || tile_bits[((int64_t)k * g.nt + ty) * g.occw + w] != 0;
        const uint64_t word = __ballot(any);
        if (threadIdx.x == 0) row_bits[(int64_t)k * g.occw + j] = word;
    }
}

__global__ void k_clear_bits(uint64_t *__restrict__ tile_bits, int64_t n_tile, uint64_t *__restrict__ row_bits,
                             int64_t n_row) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_tile + n_row; i += stride) {
        if (i < n_tile) tile_bits[i] = 0;
        else row_bits[i - n_tile] = 0;
    }
}

template <typename real, int W, int TT, bool L3>
hipError_t grid_wt(const Geom &g, const BinScan *scan, const int32_t *item_bin, const uint32_t *rec_pos,
                   const real *rec_vis, const real *lut, real *mesh, const uint64_t *tile_bits, real *margin,
                   const uint32_t *bin_vmax, const float *tapmax, Stats *st, const int32_t *plane_tr,
                   int32_t max_items, hipStream_t s) {
    const size_t lds = grid_lds_bytes(g, sizeof(real));
    static std::once_flag attr_once[kMaxDevices];
    once_per_device(attr_once, [&] {
        // (the kernel's own 8 bytes of static LDS come on top of the dynamic size)
        (void)hipFuncSetAttribute((const void *)k_grid<real, W, TT, L3>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)(160 * 1024 - 64));
    });
    // persistent blocks: as many as the CUs hold at once (LDS and 32 waves per CU)
    int per_cu = int((160 * 1024) / (lds + 64));
    const int by_waves = 2048 / grid_threads(TT);
    per_cu = per_cu < by_waves ? per_cu : by_waves;
    per_cu = per_cu < 1 ? 1 : per_cu;
    const int64_t want = int64_t(device_cus()) * per_cu;
    const int64_t nblk = want < max_items ? want : max_items;
    hipLaunchKernelGGL((k_grid<real, W, TT, L3>), dim3((unsigned)(nblk > 0 ? nblk : 1)), dim3(grid_threads(TT)),
                       lds, s, g, scan, item_bin, rec_pos, rec_vis, lut, mesh, tile_bits, margin, bin_vmax, tapmax,
                       st, plane_tr);
    return hipGetLastError();
}

template <typename real, int W, int TT>
hipError_t grid_jobs_wt(const GridJobList &list, size_t lds, int64_t max_items, unsigned long long *next,
                        hipStream_t s) {
    constexpr size_t kStatic = 512;   // at least the kernel's own LDS (272 bytes with alignment)
    static std::once_flag attr_once[kMaxDevices];
    once_per_device(attr_once, [&] {
        (void)hipFuncSetAttribute((const void *)k_grid_jobs<real, W, TT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)(160 * 1024 - kStatic));
    });
    if (lds + kStatic > 160 * 1024) return hipErrorInvalidValue;
    int per_cu = int((160 * 1024) / (lds + kStatic));
    const int by_waves = 2048 / grid_threads(TT);
    per_cu = per_cu < by_waves ? per_cu : by_waves;
    per_cu = per_cu < 1 ? 1 : per_cu;
    const int64_t want = int64_t(device_cus()) * per_cu;
    const int64_t nblk = want < max_items ? want : max_items;
    hipLaunchKernelGGL((k_grid_jobs<real, W, TT>), dim3((unsigned)(nblk > 0 ? nblk : 1)), dim3(grid_threads(TT)), lds,
                       s, list, next);
    return hipGetLastError();
}

__global__ void k_put_grid_job(GridJob *__restrict__ dst, GridJob v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = v;
}

template <typename real, int W, int TT>
hipError_t grid_wt2(const Geom &g, const BinScan *scan, const int32_t *item_bin, const uint32_t *rec_pos,
                    const real *rec_vis, const real *lut, real *mesh, const uint64_t *tile_bits, real *margin,
                    const uint32_t *bin_vmax, const float *tapmax, Stats *st, const int32_t *plane_tr,
                    int32_t max_items, hipStream_t s) {
#define GRID_WT(L3) \
    grid_wt<real, W, TT, L3>(g, scan, item_bin, rec_pos, rec_vis, lut, mesh, tile_bits, margin, bin_vmax, tapmax, \
                             st, plane_tr, max_items, s)
    return tapmax ? GRID_WT(true) : GRID_WT(false);
#undef GRID_WT
}

template <typename real, int W>
hipError_t grid_w(const Geom &g, const BinScan *scan, const int32_t *item_bin, const uint32_t *rec_pos,
                  const real *rec_vis, const real *lut, real *mesh, const uint64_t *tile_bits, real *margin,
                  const uint32_t *bin_vmax, const float *tapmax, Stats *st, const int32_t *plane_tr,
                  int32_t max_items, hipStream_t s) {
    switch (g.T) {
        case 16:
            return grid_wt2<real, W, 16>(g, scan, item_bin, rec_pos, rec_vis, lut, mesh, tile_bits, margin, bin_vmax,
                                         tapmax, st, plane_tr, max_items, s);
        case 32:
            return grid_wt2<real, W, 32>(g, scan, item_bin, rec_pos, rec_vis, lut, mesh, tile_bits, margin, bin_vmax,
                                         tapmax, st, plane_tr, max_items, s);
        case 64:
            return grid_wt2<real, W, 64>(g, scan, item_bin, rec_pos, rec_vis, lut, mesh, tile_bits, margin, bin_vmax,
                                         tapmax, st, plane_tr, max_items, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

// CUs of the current device (queried once per device)
int device_cus() {
    static int cus[kMaxDevices];
    static std::once_flag once[kMaxDevices];
    once_per_device(once, [&] {
        int dev = 0, n = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
        if (dev >= 0 && dev < kMaxDevices) cus[dev] = n;
    });
    int dev = 0;
    (void)hipGetDevice(&dev);
    return (dev >= 0 && dev < kMaxDevices && cus[dev] > 0) ? cus[dev] : 256;
}

size_t grid_lds_bytes(const Geom &g, size_t real_bytes) {
    // real plane, imaginary plane at plane_offset(W, T) doubles (packed mode:
    // one plane of 64-bit words), each T + W - 1 rows of the pitch; then the tap table
    const size_t koff = real_bytes == 4 ? 0 : size_t(plane_offset(g.W, g.T));
    return (koff + size_t(g.T + g.W - 1) * g.pitch) * sizeof(double) + size_t(g.OS) * g.W * real_bytes;
}

int64_t grid_margin_len(const Geom &g) { return margin_len(g.T, g.W); }

template <typename real>
hipError_t launch_zero_mesh(real *mesh, int64_t n_real, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_mesh<real>, dim3(8192), dim3(256), 0, s, mesh, n_real);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_zero_heavy(const Geom &g, const int32_t *heavy_bins, Stats *st, const uint64_t *tile_bits,
                             const int32_t *plane_tr, real *mesh, real *margin, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_heavy<real>, dim3(1024), dim3(kZeroBlock), 0, s, g, heavy_bins, st, tile_bits, plane_tr,
                       mesh, margin);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_merge_margins(const Geom &g, const BinScan *scan, const real *margin, uint64_t *tile_bits,
                                uint64_t *row_bits, const int32_t *plane_tr, real *mesh, hipStream_t s) {
    if (g.occw > kMaxOccWords || g.nt > 512) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_merge_margins<real>, dim3(g.Nw * g.nt), dim3(kMergeBlock), 0, s, g, scan, margin, tile_bits,
                       plane_tr, mesh);
    hipLaunchKernelGGL(k_row_bits, dim3(g.Nw), dim3(64), 0, s, g, tile_bits, row_bits);
    return hipGetLastError();
}

hipError_t launch_orient(const Geom &g, const BinScan *scan, const uint64_t *row_bits, int32_t *plane_tr,
                         hipStream_t s) {
    if (g.nt > 512) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_orient, dim3(g.Nw), dim3(kOrientBlock), 0, s, g, scan, row_bits, plane_tr);
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
                       const real *rec_vis, const real *lut, real *mesh, const uint64_t *tile_bits, real *margin,
                       const uint32_t *bin_vmax, const float *tapmax, Stats *st, const int32_t *plane_tr,
                       int32_t max_items, hipStream_t s) {
    switch (g.W) {
#define CASE(w) \
    case w: \
        return grid_w<real, w>(g, scan, item_bin, rec_pos, rec_vis, lut, mesh, tile_bits, margin, bin_vmax, \
                               tapmax, st, plane_tr, max_items, s);
        CASE(1) CASE(3) CASE(5) CASE(7) CASE(9) CASE(11) CASE(13) CASE(15)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_put_grid_job(GridJob *dst, const GridJob &v, hipStream_t s) {
    hipLaunchKernelGGL(k_put_grid_job, dim3(1), dim3(64), 0, s, dst, v);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_grid_jobs(const GridJobList &list, int W, int T, size_t lds, int64_t max_items,
                            unsigned long long *next, hipStream_t s) {
    if (list.n < 1 || list.n > kMaxGridJobs) return hipErrorInvalidValue;
#define TCASE(w, t) \
    case t: return grid_jobs_wt<real, w, t>(list, lds, max_items, next, s);
#define WCASE(w) \
    case w: \
        switch (T) { TCASE(w, 16) TCASE(w, 32) TCASE(w, 64) default: return hipErrorInvalidValue; }
    switch (W) {
        WCASE(1) WCASE(3) WCASE(5) WCASE(7) WCASE(9) WCASE(11) WCASE(13) WCASE(15)
        default: return hipErrorInvalidValue;
    }
#undef WCASE
#undef TCASE
}

template hipError_t launch_zero_mesh<float>(float *, int64_t, hipStream_t);
template hipError_t launch_zero_mesh<double>(double *, int64_t, hipStream_t);
template hipError_t launch_zero_heavy<float>(const Geom &, const int32_t *, Stats *, const uint64_t *,
                                             const int32_t *, float *, float *, hipStream_t);
template hipError_t launch_zero_heavy<double>(const Geom &, const int32_t *, Stats *, const uint64_t *,
                                              const int32_t *, double *, double *, hipStream_t);
template hipError_t launch_merge_margins<float>(const Geom &, const BinScan *, const float *, uint64_t *, uint64_t *,
                                                const int32_t *, float *, hipStream_t);
template hipError_t launch_merge_margins<double>(const Geom &, const BinScan *, const double *, uint64_t *,
                                                 uint64_t *, const int32_t *, double *, hipStream_t);
template hipError_t launch_grid<float>(const Geom &, const BinScan *, const int32_t *, const uint32_t *,
                                       const float *, const float *, float *, const uint64_t *, float *,
                                       const uint32_t *, const float *, Stats *, const int32_t *, int32_t,
                                       hipStream_t);
template hipError_t launch_grid<double>(const Geom &, const BinScan *, const int32_t *, const uint32_t *,
                                        const double *, const double *, double *, const uint64_t *, double *,
                                        const uint32_t *, const float *, Stats *, const int32_t *, int32_t,
                                       hipStream_t);
template hipError_t launch_grid_jobs<float>(const GridJobList &, int, int, size_t, int64_t, unsigned long long *,
                                            hipStream_t);
template hipError_t launch_grid_jobs<double>(const GridJobList &, int, int, size_t, int64_t, unsigned long long *,
                                             hipStream_t);

}  // namespace rick
