// Bin-and-sort of visibilities by (w-plane, uv tile): the GPU form of the
// paper's per-sector bucketing of visibilities before convolution
// (Sec. 2.1, "an array is created for each sector").
//
// Three passes over the inputs, all streaming:
//   bin_count   per visibility: position quantised to 1/OS cell, nearest
//               cell, closest w-plane, drop test; one count per (plane, tile)
//               bin the W x W footprint touches (1, 2 or 4 bins);
//               weight sum and gridded/dropped counters.
//   bin_scan    exclusive prefix sums of record counts and gridding chunks;
//               per-copy cursors, the list of gridding work items and the
//               list of bins split over several chunks.
//   bin_scatter repeats the quantisation and writes 12-byte records
//               {packed local position, W V} at cursor-allocated slots.
//
// Counts and slots are taken per run: consecutive visibilities of a wave (the
// channels of a row, in memory order) whose footprints cover the same bins
// form a run, found without loops by comparing each lane's footprint key with
// its left neighbour's; the first lane of a run takes one atomic per bin for
// the whole run, and the others take the slots that follow.
//
// The float64 position arithmetic is written operation by operation with
// contraction off, so that cell, sub-cell offset, plane and drop decisions are
// bit-identical to a plain float64 evaluation of the same steps.
#include "rick_internal.h"

namespace rick {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxBlocks = 8192;   // count and scatter use the same grid: a visibility meets the same counter copy

__global__ void k_zero_stats(Stats *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->n_gridded = 0;
        st->n_dropped = 0;
        st->n_records = 0;
        st->n_heavy = 0;
        st->sum_w = 0.0;
    }
}

// zero the per-copy bin counters and the per-call heavy-bin count
__global__ void k_reset_counts(int32_t *__restrict__ a, int64_t n, Stats *__restrict__ st) {
    if (blockIdx.x == 0 && threadIdx.x == 0) st->n_heavy = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
}

__global__ void k_set_scales(double *__restrict__ dst, ChanScales cs, int32_t n) {
    const int t = threadIdx.x;
    if (t < n) dst[t] = cs.s[t];
}

struct Quant {
    int32_t cx, cy, sx, sy, k;
};

// Position, plane and drop decision of one visibility.
template <typename real>
__device__ __forceinline__ bool quantise(const Geom &g, double u, double v, double w, real vr, real vi, float wt,
                                         Quant &q) {
#pragma clang fp contract(off)
    if (!(isfinite(u) && isfinite(v) && isfinite(w) && isfinite((double)vr) && isfinite((double)vi) &&
          isfinite(wt)))
        return false;
    double xs = u * g.fov;
    xs = xs * (double)g.OS;
    xs = xs + g.half;
    double ys = v * g.fov;
    ys = ys * (double)g.OS;
    ys = ys + g.half;
    if (!(fabs(xs) <= 1073741824.0 && fabs(ys) <= 1073741824.0)) return false;
    const int32_t X = (int32_t)rint(xs);
    const int32_t Y = (int32_t)rint(ys);
    q.cx = (X + (g.OS >> 1)) >> g.log2OS;   // floor division by OS (arithmetic shift)
    q.cy = (Y + (g.OS >> 1)) >> g.log2OS;
    q.sx = X - (q.cx << g.log2OS);
    q.sy = Y - (q.cy << g.log2OS);
    if (!(wt > 0.0f)) return false;
    if (q.cx - g.h < 0 || q.cx + g.h > g.N - 1 || q.cy - g.h < 0 || q.cy + g.h > g.N - 1) return false;
    double kf = floor((w - g.w_min) / g.dw);
    if (isnan(kf)) kf = 0.0;
    kf = kf < 0.0 ? 0.0 : kf;
    kf = kf > (double)(g.Nw - 1) ? (double)(g.Nw - 1) : kf;
    q.k = (int32_t)kf;
    return true;
}

// The bins a footprint touches: its top-left tile (tx0, ty0) and whether it
// also reaches the next tile column (dx) and row (dy).  A tile is at least W
// cells wide, so a footprint touches at most two tiles per axis.  Packed as
// ((plane * nt + ty0) * nt + tx0) * 4 + dx * 2 + dy, the key of the set.
struct Footprint {
    int32_t base;   // bin of the top-left tile
    int32_t dx, dy;
};
__device__ __forceinline__ Footprint footprint(const Geom &g, const Quant &q) {
    const int32_t tx0 = (q.cx - g.h) >> g.log2T, ty0 = (q.cy - g.h) >> g.log2T;
    Footprint f;
    f.dx = ((q.cx + g.h) >> g.log2T) - tx0;
    f.dy = ((q.cy + g.h) >> g.log2T) - ty0;
    f.base = (q.k * g.nt + ty0) * g.nt + tx0;
    return f;
}
// Bin j of the set (j = 0: top-left, 1: right, 2: below, 3: below right), if present.
__device__ __forceinline__ bool has_bin(const Footprint &f, int j) {
    return (j & 1 ? f.dx : 1) && (j & 2 ? f.dy : 1);
}
__device__ __forceinline__ int32_t bin_of(const Geom &g, const Footprint &f, int j) {
    return f.base + (j & 1) + (j >> 1) * g.nt;
}
// The record of a visibility in bin j: footprint origin relative to the tile
// (biased by 2h so that it is non-negative) and sub-cell offsets.
__device__ __forceinline__ uint32_t record_pos(const Geom &g, const Quant &q, int j) {
    const int32_t tx = ((q.cx - g.h) >> g.log2T) + (j & 1), ty = ((q.cy - g.h) >> g.log2T) + (j >> 1);
    const int32_t ox = q.cx - g.h - (tx << g.log2T) + 2 * g.h;   // in [0, T + 2h)
    const int32_t oy = q.cy - g.h - (ty << g.log2T) + 2 * g.h;
    return (uint32_t)ox | (uint32_t)oy << 8 | (uint32_t)(q.sx + (g.OS >> 1)) << 16 |
           (uint32_t)(q.sy + (g.OS >> 1)) << 24;
}

__device__ __forceinline__ void store2(float *p, float a, float b) { *(float2 *)p = make_float2(a, b); }
__device__ __forceinline__ void store2(double *p, double a, double b) { *(double2 *)p = make_double2(a, b); }

// Runs of equal keys along the lanes of a wave.  Must be called by all lanes.
// Lane 0 always starts a run; `leader` is the first lane of this lane's run,
// `len` (meaningful in leaders) the run's length.
struct Run {
    int32_t leader, len;
    bool head;
};
__device__ __forceinline__ Run runs_of(int32_t key) {
    const int lane = (int)__lane_id();
    const int32_t prev = __shfl_up(key, 1);   // key of lane - 1
    Run r;
    r.head = lane == 0 || key != prev;
    const uint64_t heads = __ballot(r.head);
    const uint64_t upto = heads & (~0ull >> (63 - lane));               // heads at lanes <= lane
    const uint64_t after = lane == 63 ? 0ull : heads & (~0ull << (lane + 1));
    r.leader = 63 - __clzll((long long)upto);
    r.len = (after ? __ffsll((long long)after) - 1 : 64) - lane;
    return r;
}

// Grid-stride walk over visibility index i = r * nchan + c with the row r and
// channel c updated incrementally (no division per step; indices fit 32 bits
// because a plan takes fewer than 2^29 visibilities).
struct VisWalk {
    uint32_t i, r, c, di, dr, dc;
    __device__ __forceinline__ VisWalk(uint32_t start, uint32_t stride, uint32_t nchan) {
        i = start;
        r = start / nchan;
        c = start - r * nchan;
        di = stride;
        dr = stride / nchan;
        dc = stride - dr * nchan;
    }
    __device__ __forceinline__ void next(uint32_t nchan) {
        i += di;
        r += dr;
        c += dc;
        if (c >= nchan) {
            c -= nchan;
            ++r;
        }
    }
};

template <typename real>
__device__ __forceinline__ void load_vis(const Geom &g, const double *__restrict__ uvw,
                                         const double *__restrict__ scales, const real *__restrict__ vis,
                                         const float *__restrict__ weight, uint32_t i, uint32_t r, uint32_t c,
                                         double &u, double &v, double &w, real &vr, real &vi, float &wt) {
#pragma clang fp contract(off)
    const double sc = scales[c];
    u = uvw[3 * r] * sc;
    v = uvw[3 * r + 1] * sc;
    w = uvw[3 * r + 2] * sc;
    vr = vis[2 * i];
    vi = vis[2 * i + 1];
    wt = weight ? weight[i] : 1.0f;
}

template <typename real>
__global__ __launch_bounds__(kBlock) void k_bin_count(Geom g, const double *__restrict__ uvw,
                                                      const double *__restrict__ scales,
                                                      const real *__restrict__ vis, const float *__restrict__ weight,
                                                      int64_t nvis, int32_t nchan, int32_t *__restrict__ counts,
                                                      Stats *__restrict__ st) {
    __shared__ double s_w[kBlock / 64];
    __shared__ unsigned long long s_kept[kBlock / 64], s_drop[kBlock / 64];
    double sum_w = 0.0;
    unsigned long long kept = 0, dropped = 0;
    // counters are privatised over kCopies copies (by block), which spreads
    // the atomics on the dense central bins over several cache lines
    int32_t *my_counts = counts + (blockIdx.x % kCopies) * (g.nbins + 1);
    const uint32_t stride = gridDim.x * kBlock;
    // loop bound uniform across the block so that every lane joins the ballots
    const uint32_t iters = (uint32_t)((nvis + stride - 1) / stride);
    VisWalk vw(blockIdx.x * kBlock + threadIdx.x, stride, (uint32_t)nchan);
    for (uint32_t it = 0; it < iters; ++it, vw.next((uint32_t)nchan)) {
        bool keep = false;
        Quant q{};
        if (vw.i < (uint32_t)nvis) {
            double u, v, w;
            real vr, vi;
            float wt;
            load_vis<real>(g, uvw, scales, vis, weight, vw.i, vw.r, vw.c, u, v, w, vr, vi, wt);
            keep = quantise<real>(g, u, v, w, vr, vi, wt, q);
            if (keep) {
                ++kept;
                sum_w += (double)wt;
            } else {
                ++dropped;
            }
        }
        const Footprint f = footprint(g, q);
        const Run run = runs_of(keep ? f.base * 4 + f.dx * 2 + f.dy : -1);
        if (keep && run.head) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (has_bin(f, j)) atomicAdd(&my_counts[bin_of(g, f, j)], run.len);
        }
    }
    // block reduction, one atomic per block and counter
    for (int off = 32; off > 0; off >>= 1) {
        sum_w += __shfl_down(sum_w, off);
        kept += __shfl_down(kept, off);
        dropped += __shfl_down(dropped, off);
    }
    const int wid = threadIdx.x >> 6;
    if (__lane_id() == 0) {
        s_w[wid] = sum_w;
        s_kept[wid] = kept;
        s_drop[wid] = dropped;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tw = 0.0;
        unsigned long long tk = 0, td = 0;
        for (int k = 0; k < kBlock / 64; ++k) {
            tw += s_w[k];
            tk += s_kept[k];
            td += s_drop[k];
        }
        if (tk) {
            atomicAdd(&st->n_gridded, tk);
            unsafeAtomicAdd(&st->sum_w, tw);
        }
        if (td) atomicAdd(&st->n_dropped, td);
    }
}

template <typename real>
__global__ __launch_bounds__(kBlock) void k_bin_scatter(Geom g, const double *__restrict__ uvw,
                                                        const double *__restrict__ scales,
                                                        const real *__restrict__ vis,
                                                        const float *__restrict__ weight, int64_t nvis,
                                                        int32_t nchan, int32_t *__restrict__ cursor,
                                                        uint32_t *__restrict__ rec_pos, real *__restrict__ rec_vis) {
    int32_t *my_cursor = cursor + (blockIdx.x % kCopies) * g.nbins;
    const uint32_t stride = gridDim.x * kBlock;
    const uint32_t iters = (uint32_t)((nvis + stride - 1) / stride);
    VisWalk vw(blockIdx.x * kBlock + threadIdx.x, stride, (uint32_t)nchan);
    for (uint32_t it = 0; it < iters; ++it, vw.next((uint32_t)nchan)) {
        bool keep = false;
        Quant q{};
        real ar = 0, ai = 0;
        if (vw.i < (uint32_t)nvis) {
            double u, v, w;
            real vr, vi;
            float wt;
            load_vis<real>(g, uvw, scales, vis, weight, vw.i, vw.r, vw.c, u, v, w, vr, vi, wt);
            keep = quantise<real>(g, u, v, w, vr, vi, wt, q);
            ar = (real)wt * vr;
            ai = (real)wt * vi;
        }
        const Footprint f = footprint(g, q);
        const Run run = runs_of(keep ? f.base * 4 + f.dx * 2 + f.dy : -1);
        // the run's first lane takes the slots of the whole run in each bin;
        // all atomics are issued before any result is read
        int32_t base[4] = {0, 0, 0, 0};
        if (keep && run.head) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (has_bin(f, j)) base[j] = atomicAdd(&my_cursor[bin_of(g, f, j)], run.len);
        }
        const int32_t rank = (int32_t)__lane_id() - run.leader;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int32_t slot = __shfl(base[j], run.leader) + rank;
            if (keep && has_bin(f, j)) {
                rec_pos[slot] = record_pos(g, q, j);
                store2(rec_vis + 2 * (uint32_t)slot, ar, ai);
            }
        }
    }
}

// ---- scan of per-bin counts ----
constexpr int kScanBlock = 1024;
constexpr int kScanPer = 2;
constexpr int kScanTile = kScanBlock * kScanPer;

__device__ __forceinline__ int32_t chunks_of(int32_t count, int32_t CH) {
    return count <= CH ? 1 : (count + CH - 1) / CH;
}

// block-wide exclusive scan of (a, b) pairs; returns totals through refs
__device__ __forceinline__ void block_scan2(int32_t &a, int32_t &b, int32_t &tot_a, int32_t &tot_b) {
    __shared__ int32_t sa[kScanBlock / 64], sb[kScanBlock / 64];
    const int lane = __lane_id(), wid = threadIdx.x >> 6;
    int32_t xa = a, xb = b;
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t ya = __shfl_up(xa, off), yb = __shfl_up(xb, off);
        if (lane >= off) {
            xa += ya;
            xb += yb;
        }
    }
    if (lane == 63) {
        sa[wid] = xa;
        sb[wid] = xb;
    }
    __syncthreads();
    int32_t pa = 0, pb = 0;
    tot_a = 0;
    tot_b = 0;
    for (int k = 0; k < kScanBlock / 64; ++k) {
        if (k < wid) {
            pa += sa[k];
            pb += sb[k];
        }
        tot_a += sa[k];
        tot_b += sb[k];
    }
    a = pa + xa - a;
    b = pb + xb - b;
    __syncthreads();
}

__device__ __forceinline__ int32_t total_count(const int32_t *__restrict__ counts, int32_t n, int64_t i) {
    int32_t c = 0;
#pragma unroll
    for (int s = 0; s < kCopies; ++s) c += counts[(int64_t)s * (n + 1) + i];
    return c;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_partials(const int32_t *__restrict__ counts, int32_t n,
                                                              int32_t CH, int32_t *__restrict__ bsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanPer;
    int32_t a = 0, b = 0;
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) {
            const int32_t c = total_count(counts, n, base + k);
            a += c;
            b += chunks_of(c, CH);
        }
    }
    int32_t ta, tb;
    block_scan2(a, b, ta, tb);
    if (threadIdx.x == 0) {
        bsum[2 * blockIdx.x] = ta;
        bsum[2 * blockIdx.x + 1] = tb;
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_top(int32_t *__restrict__ bsum, int32_t nblk) {
    int32_t carry_a = 0, carry_b = 0;
    for (int32_t s = 0; s < nblk; s += kScanBlock) {
        const int32_t i = s + threadIdx.x;
        int32_t a = i < nblk ? bsum[2 * i] : 0, b = i < nblk ? bsum[2 * i + 1] : 0;
        int32_t ta, tb;
        block_scan2(a, b, ta, tb);
        if (i < nblk) {
            bsum[2 * i] = a + carry_a;
            bsum[2 * i + 1] = b + carry_b;
        }
        carry_a += ta;
        carry_b += tb;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const int32_t *__restrict__ counts, int32_t n, int32_t CH,
                                                           const int32_t *__restrict__ bsum,
                                                           BinScan *__restrict__ scan, int32_t *__restrict__ cursor,
                                                           int32_t *__restrict__ item_bin,
                                                           int32_t *__restrict__ heavy_bins, Stats *__restrict__ st) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanPer;
    int32_t c[kScanPer], a = 0, b = 0;
    for (int k = 0; k < kScanPer; ++k) {
        c[k] = base + k < n ? total_count(counts, n, base + k) : 0;
        a += c[k];
        b += base + k < n ? chunks_of(c[k], CH) : 0;
    }
    int32_t ta, tb;
    block_scan2(a, b, ta, tb);
    a += bsum[2 * blockIdx.x];
    b += bsum[2 * blockIdx.x + 1];
    for (int k = 0; k < kScanPer; ++k) {
        const int64_t i = base + k;
        if (i < n) {
            scan[i].rec = a;
            scan[i].item = b;
            // each counter copy owns a contiguous sub-range of the bin
            int32_t cur = a;
            for (int s = 0; s < kCopies; ++s) {
                cursor[(int64_t)s * n + i] = cur;
                cur += counts[(int64_t)s * (n + 1) + i];
            }
            const int32_t nch = chunks_of(c[k], CH);
            for (int32_t j = 0; j < nch; ++j) item_bin[b + j] = (int32_t)i;
            if (nch > 1) heavy_bins[atomicAdd(&st->n_heavy, 1ull)] = (int32_t)i;
            a += c[k];
            b += nch;
        } else if (i == n) {
            scan[i].rec = a;
            scan[i].item = b;
            st->n_records = (unsigned long long)a;
        }
    }
}

int grid_blocks(int64_t nvis) {
    int64_t b = (nvis + kBlock - 1) / kBlock;
    if (b < 1) b = 1;
    if (b > kMaxBlocks) b = kMaxBlocks;
    return (int)b;
}

}  // namespace

hipError_t launch_zero_stats(Stats *st, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_stats, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_reset_counts(const Geom &g, int32_t *counts, Stats *st, hipStream_t s) {
    const int64_t n = (int64_t)kCopies * (g.nbins + 1);
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_reset_counts, dim3((unsigned)blocks), dim3(256), 0, s, counts, n, st);
    return hipGetLastError();
}

hipError_t launch_set_scales(double *dst, const double *host_scales, int32_t nchan, hipStream_t s) {
    for (int32_t c0 = 0; c0 < nchan; c0 += kMaxInlineChan) {
        ChanScales cs{};
        const int32_t n = nchan - c0 < kMaxInlineChan ? nchan - c0 : kMaxInlineChan;
        for (int32_t j = 0; j < n; ++j) cs.s[j] = host_scales[c0 + j];
        hipLaunchKernelGGL(k_set_scales, dim3(1), dim3(kMaxInlineChan), 0, s, dst + c0, cs, n);
    }
    return hipGetLastError();
}

template <typename real>
hipError_t launch_bin_count(const Geom &g, const double *uvw, const double *scales_dev, const real *vis,
                            const float *weight, int64_t nrow, int32_t nchan, int32_t *counts, Stats *st,
                            hipStream_t s) {
    const int64_t nvis = nrow * nchan;
    if (nvis == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_bin_count<real>, dim3(grid_blocks(nvis)), dim3(kBlock), 0, s, g, uvw, scales_dev, vis,
                       weight, nvis, nchan, counts, st);
    return hipGetLastError();
}

hipError_t launch_bin_scan(const Geom &g, const int32_t *counts, BinScan *scan, int32_t *block_sums, int32_t *cursor,
                           int32_t *item_bin, int32_t *heavy_bins, Stats *st, hipStream_t s) {
    const int32_t n = g.nbins;
    const int32_t nblk = (n + 1 + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_partials, dim3(nblk), dim3(kScanBlock), 0, s, counts, n, g.CH, block_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, s, block_sums, nblk);
    hipLaunchKernelGGL(k_scan_apply, dim3(nblk), dim3(kScanBlock), 0, s, counts, n, g.CH, block_sums, scan, cursor,
                       item_bin, heavy_bins, st);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_bin_scatter(const Geom &g, const double *uvw, const double *scales_dev, const real *vis,
                              const float *weight, int64_t nrow, int32_t nchan, int32_t *cursor, uint32_t *rec_pos,
                              real *rec_vis, hipStream_t s) {
    const int64_t nvis = nrow * nchan;
    if (nvis == 0) return hipGetLastError();
    hipLaunchKernelGGL(k_bin_scatter<real>, dim3(grid_blocks(nvis)), dim3(kBlock), 0, s, g, uvw, scales_dev, vis,
                       weight, nvis, nchan, cursor, rec_pos, rec_vis);
    return hipGetLastError();
}

template hipError_t launch_bin_count<float>(const Geom &, const double *, const double *, const float *,
                                            const float *, int64_t, int32_t, int32_t *, Stats *, hipStream_t);
template hipError_t launch_bin_count<double>(const Geom &, const double *, const double *, const double *,
                                             const float *, int64_t, int32_t, int32_t *, Stats *, hipStream_t);
template hipError_t launch_bin_scatter<float>(const Geom &, const double *, const double *, const float *,
                                              const float *, int64_t, int32_t, int32_t *, uint32_t *, float *,
                                              hipStream_t);
template hipError_t launch_bin_scatter<double>(const Geom &, const double *, const double *, const double *,
                                               const float *, int64_t, int32_t, int32_t *, uint32_t *, double *,
                                               hipStream_t);

}  // namespace rick
