// Bin-and-sort of visibilities by (w-plane, uv tile): the GPU form of the
// paper's per-sector bucketing of visibilities before convolution
// (Sec. 2.1, "an array is created for each sector").
//
// Two levels, so that no pass needs global atomics (on this part every
// device atomic is executed at the memory side, far slower than LDS):
//   level 1  coarse bins = (plane, coarse tile of C x C tiles), at most 8192.
//     bin_count    each block takes a contiguous range of visibilities:
//                  position quantised to 1/OS cell, nearest cell, closest
//                  w-plane, every drop test but the finiteness of V (so
//                  the visibilities are not read); counts per coarse bin
//                  (that of the footprint's origin) in an LDS histogram;
//                  writes its column of the (coarse bin, block) count table.
//     bin_scan     exclusive scan of that table (coarse-bin major), then the
//                  level-2 chunk list (each coarse bin cut into chunks).
//     bin_scatter  repeats the quantisation; slots from LDS cursors seeded
//                  with the block's scanned offsets; writes the level-1
//                  records as two arrays, positions (4 or 8 bytes, formats
//                  below) and W V; a record whose W V is not finite keeps
//                  its slot, marked dead (W V = NaN); weight sum and counters.
//   level 2  bins = (plane, tile) inside each coarse bin, at most C^2 = 16384.
//     fine_count   one block per chunk: LDS histogram over the tiles of the
//                  coarse tile (that of each record's footprint origin),
//                  from the positions alone (W V too only if a record of
//                  the call is dead).
//     fine_scan    per bin, the total over its coarse bin's chunks; exclusive
//                  scan of records and gridding chunks in bin order (item and
//                  heavy-bin lists); per (chunk, tile) record offsets.
//     fine_scatter one block per chunk: slots from LDS cursors; writes the
//                  12-byte records {packed position in the tile, W V}, and
//                  the largest |W V| per (chunk, tile), then per bin.
//
// A visibility is binned once, into the tile holding the top-left cell
// (c_x - h, c_y - h) of its W x W footprint: the gridder keeps a tile plus a
// (W - 1)-cell margin right and below in LDS, so every footprint of the tile
// lies inside its accumulator (the margins are added to the neighbouring
// tiles after gridding).
//
// Counts and slots in LDS are taken per run: consecutive records of a wave
// whose footprints cover the same bins form a run, found without loops by
// comparing each lane's footprint key with its left neighbour's; the first
// lane of a run takes one LDS atomic per bin for the whole run, and the
// others take the slots that follow.
//
// The float64 position arithmetic is written operation by operation with
// contraction off, so that cell, sub-cell offset, plane and drop decisions are
// bit-identical to a plain float64 evaluation of the same steps.
#include "rick_internal.h"
#include "quant.h"

// Scratch of rick_grid_static: sort buffers of one call, carved per call.
// Each device holds its own copy at its own address; host code never uses
// the array's name as a device address, only the address that
// hipGetSymbolAddress returns on that device (static_scratch below).
static __device__ __align__(256) unsigned char scratch[rick::kStaticScratchBytes];

namespace rick {

namespace {

constexpr int kBlock = 256;
constexpr int kL1Block = 1024;   // threads of a level-1 block (one contiguous range of visibilities)

// Level-1 records: positions in one of two formats, and W V in an array of
// its own (after the positions, 256-byte aligned):
//   full (8 B): cell x | y << 16, sub-cell x | y << 8 | plane << 16;
//   compact (4 B, float32 W V, when 2 (log2(C T) + log2(OS)) <= 32): one word
//     holding the footprint origin inside the coarse tile and the sub-cell
//     indices -- the plane and coarse tile are those of the bin.
// A record whose W V is not finite is dead: counted by bin_count (which
// does not read V) and so given a slot, but skipped by level 2.
template <bool CPT>
struct P1;
template <>
struct P1<false> {
    uint32_t cxy, sub;
};
template <>
struct P1<true> {
    uint32_t pos;
};
__host__ __device__ inline size_t l1_vis_offset(int64_t nrec, bool cpt) {
    return ((size_t)nrec * (cpt ? 4 : 8) + 255) & ~size_t(255);
}

// Footprint origin inside its coarse tile (ox1, oy1, in cells) and sub-cell
// indices s + OS/2 in [0, OS) (sx, sy).
struct Pos1 {
    int32_t ox1, oy1, sx, sy;
    int32_t iw;   // w-fraction bin (full format only; 0 otherwise)
};
__device__ __forceinline__ int32_t coarse_shift(const Geom &g) { return g.log2C + g.log2T; }

__global__ void k_zero_stats(Stats *st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->n_gridded = 0;
        st->n_dropped = 0;
        st->n_records = 0;
        st->n_heavy = 0;
        st->sum_w = 0.0;
    }
}

__global__ void k_set_scales(double *__restrict__ dst, ChanScales cs, int32_t n) {
    const int t = threadIdx.x;
    if (t < n) dst[t] = cs.s[t];
}

__device__ __forceinline__ P1<false> make_p1(const Geom &g, const Quant &q, P1<false> *) {
    // plane in bits 16..28 (< 8192 planes), w-fraction bin in bits 29..31
    return P1<false>{(uint32_t)q.cx | (uint32_t)q.cy << 16,
                     (uint32_t)(q.sx + (g.OS >> 1)) | (uint32_t)(q.sy + (g.OS >> 1)) << 8 | (uint32_t)q.k << 16 |
                         (uint32_t)q.iw << 29};
}
__device__ __forceinline__ P1<true> make_p1(const Geom &g, const Quant &q, P1<true> *) {
    const int32_t lb = coarse_shift(g), m = (1 << lb) - 1;
    const uint32_t ox1 = (uint32_t)((q.cx - g.h) & m), oy1 = (uint32_t)((q.cy - g.h) & m);
    const uint32_t sx = (uint32_t)(q.sx + (g.OS >> 1)), sy = (uint32_t)(q.sy + (g.OS >> 1));
    return P1<true>{ox1 | sx << lb | oy1 << (lb + g.log2OS) | sy << (2 * lb + g.log2OS)};
}
__device__ __forceinline__ Pos1 pos_of(const Geom &g, const P1<false> &r, int32_t ctx, int32_t cty) {
    const int32_t lb = coarse_shift(g);
    const int32_t cx = (int32_t)(r.cxy & 0xffffu), cy = (int32_t)(r.cxy >> 16);
    return Pos1{cx - g.h - (ctx << lb), cy - g.h - (cty << lb), (int32_t)(r.sub & 0xffu),
                (int32_t)((r.sub >> 8) & 0xffu), (int32_t)(r.sub >> 29)};
}
__device__ __forceinline__ Pos1 pos_of(const Geom &g, const P1<true> &r, int32_t, int32_t) {
    const int32_t lb = coarse_shift(g), sb = g.log2OS;
    const uint32_t ml = (1u << lb) - 1, ms = (1u << sb) - 1;
    return Pos1{(int32_t)(r.pos & ml), (int32_t)((r.pos >> (lb + sb)) & ml), (int32_t)((r.pos >> lb) & ms),
                (int32_t)(r.pos >> (2 * lb + sb)), 0};
}

// Tile of edge 2^shift cells holding the footprint origin (c - h) of cell (cx, cy).
struct Span {
    int32_t x0, y0;
};
__device__ __forceinline__ Span span_of(const Quant &q, int32_t h, int32_t shift) {
    return Span{(q.cx - h) >> shift, (q.cy - h) >> shift};
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

// ---- level 1: coarse bins ----

// Level-1 partition: block b takes visibilities [b per, min((b + 1) per, nvis)).
struct L1Part {
    int32_t nb1;
    int32_t per;   // a multiple of kBlock
};

__global__ __launch_bounds__(kL1Block) void k_l1_count(Geom g, const double *__restrict__ uvw,
                                                     const double *__restrict__ scales,
                                                     const float *__restrict__ weight, int64_t nvis, int32_t nchan,
                                                     L1Part part, int32_t *__restrict__ cnt1) {
    extern __shared__ int32_t s_cnt[];   // g.n1 counters
    for (int i = threadIdx.x; i < g.n1; i += kL1Block) s_cnt[i] = 0;
    __syncthreads();
    const int64_t v0 = (int64_t)blockIdx.x * part.per;
    const int64_t v1 = v0 + part.per < nvis ? v0 + part.per : nvis;
    const int32_t cshift = g.log2T + g.log2C;
    VisWalk vw((uint32_t)(v0 + threadIdx.x), kL1Block, (uint32_t)nchan);
    for (int32_t it = 0; it < part.per / kL1Block; ++it, vw.next((uint32_t)nchan)) {
        bool keep = false;
        Quant q{};
        if ((int64_t)vw.i < v1) {
#pragma clang fp contract(off)
            const double sc = scales[vw.c];
            const double u = uvw[3 * vw.r] * sc, v = uvw[3 * vw.r + 1] * sc, w = uvw[3 * vw.r + 2] * sc;
            keep = quantise_pos(g, u, v, w, weight ? weight[vw.i] : 1.0f, q);
        }
        const Span cs = span_of(q, g.h, cshift);
        const int32_t base = (q.k * g.nct + cs.y0) * g.nct + cs.x0;
        const Run run = runs_of(keep ? base : -1);
        if (keep && run.head) atomicAdd(&s_cnt[base], run.len);
    }
    __syncthreads();
    // this block's column of the (coarse bin, block) table
    for (int i = threadIdx.x; i < g.n1; i += kL1Block) cnt1[(int64_t)i * part.nb1 + blockIdx.x] = s_cnt[i];
}

template <typename real, bool CPT>
__global__ __launch_bounds__(kL1Block) void k_l1_scatter(Geom g, const double *__restrict__ uvw,
                                                         const double *__restrict__ scales,
                                                         const real *__restrict__ vis, const float *__restrict__ weight,
                                                         int64_t nvis, int32_t nchan, L1Part part,
                                                         const int32_t *__restrict__ base1, P1<CPT> *__restrict__ pos1,
                                                         real *__restrict__ vis1, Stats *__restrict__ st) {
    extern __shared__ int32_t s_cur[];   // g.n1 cursors
    __shared__ double s_w[kL1Block / 64];
    __shared__ unsigned long long s_kept[kL1Block / 64], s_drop[kL1Block / 64], s_dead[kL1Block / 64];
    for (int i = threadIdx.x; i < g.n1; i += kL1Block) s_cur[i] = base1[(int64_t)i * part.nb1 + blockIdx.x];
    __syncthreads();
    const int64_t v0 = (int64_t)blockIdx.x * part.per;
    const int64_t v1 = v0 + part.per < nvis ? v0 + part.per : nvis;
    const int32_t cshift = g.log2T + g.log2C;
    double sum_w = 0.0;
    unsigned long long kept = 0, dropped = 0, dead = 0;
    VisWalk vw((uint32_t)(v0 + threadIdx.x), kL1Block, (uint32_t)nchan);
    for (int32_t it = 0; it < part.per / kL1Block; ++it, vw.next((uint32_t)nchan)) {
        bool placed = false;   // passed the position tests: counted by bin_count
        Quant q{};
        real ar = 0, ai = 0;
        if ((int64_t)vw.i < v1) {
            double u, v, w;
            real vr, vi;
            float wt;
            load_vis<real>(g, uvw, scales, vis, weight, vw.i, vw.r, vw.c, u, v, w, vr, vi, wt);
            placed = quantise_pos(g, u, v, w, wt, q);
            ar = (real)wt * vr;
            ai = (real)wt * vi;
            // kept: placed with a finite W V; a placed record without one is dead
            const bool live = placed && isfinite((double)ar) && isfinite((double)ai);
            if (live) {
                ++kept;
                sum_w += (double)wt;
            } else {
                ++dropped;
                if (placed) {
                    ++dead;
                    ar = __builtin_nan("");
                    ai = 0;
                }
            }
        }
        const Span cs = span_of(q, g.h, cshift);
        const int32_t base = (q.k * g.nct + cs.y0) * g.nct + cs.x0;
        const Run run = runs_of(placed ? base : -1);
        // the run's first lane takes the slots of the whole run
        int32_t b0 = 0;
        if (placed && run.head) b0 = atomicAdd(&s_cur[base], run.len);
        const int32_t rank = (int32_t)__lane_id() - run.leader;
        const P1<CPT> r1 = make_p1(g, q, (P1<CPT> *)nullptr);
        const int32_t slot = __shfl(b0, run.leader) + rank;
        if (placed) {
            pos1[slot] = r1;
            store2(vis1 + 2 * (int64_t)slot, ar, ai);
        }
    }
    // block reduction of the counters, one atomic per block and counter
    for (int off = 32; off > 0; off >>= 1) {
        sum_w += __shfl_down(sum_w, off);
        kept += __shfl_down(kept, off);
        dropped += __shfl_down(dropped, off);
        dead += __shfl_down(dead, off);
    }
    const int wid = threadIdx.x >> 6;
    if (__lane_id() == 0) {
        s_w[wid] = sum_w;
        s_kept[wid] = kept;
        s_drop[wid] = dropped;
        s_dead[wid] = dead;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tw = 0.0;
        unsigned long long tk = 0, td = 0, tx = 0;
        for (int k = 0; k < kL1Block / 64; ++k) {
            tw += s_w[k];
            tk += s_kept[k];
            td += s_drop[k];
            tx += s_dead[k];
        }
        if (tk) {
            atomicAdd(&st->n_gridded, tk);
            unsafeAtomicAdd(&st->sum_w, tw);
        }
        if (td) atomicAdd(&st->n_dropped, td);
        if (tx) atomicAdd(&st->n_dead, tx);
    }
}

// ---- scans ----
constexpr int kScanBlock = 1024;
constexpr int kScanPer = 2;
constexpr int kScanTile = kScanBlock * kScanPer;

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

// flat exclusive scan of an int32 array, in place; a[n] receives the total
__global__ __launch_bounds__(kScanBlock) void k_flat_partials(const int32_t *__restrict__ a, int64_t n,
                                                              int32_t *__restrict__ bsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanPer;
    int32_t x = 0, y = 0;
    for (int k = 0; k < kScanPer; ++k)
        if (base + k < n) x += a[base + k];
    int32_t tx, ty;
    block_scan2(x, y, tx, ty);
    if (threadIdx.x == 0) bsum[blockIdx.x] = tx;
}

__global__ __launch_bounds__(kScanBlock) void k_flat_top(int32_t *__restrict__ bsum, int32_t nblk) {
    int32_t carry = 0;
    for (int32_t s0 = 0; s0 < nblk; s0 += kScanBlock) {
        const int32_t i = s0 + threadIdx.x;
        int32_t x = i < nblk ? bsum[i] : 0, y = 0;
        int32_t tx, ty;
        block_scan2(x, y, tx, ty);
        if (i < nblk) bsum[i] = x + carry;
        carry += tx;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kScanBlock) void k_flat_apply(int32_t *__restrict__ a, int64_t n,
                                                           const int32_t *__restrict__ bsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanPer;
    int32_t c[kScanPer], x = 0, y = 0;
    for (int k = 0; k < kScanPer; ++k) {
        c[k] = base + k < n ? a[base + k] : 0;
        x += c[k];
    }
    int32_t tx, ty;
    block_scan2(x, y, tx, ty);
    x += bsum[blockIdx.x];
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) a[base + k] = x;
        else if (base + k == n) a[n] = x;
        x += c[k];
    }
}

// Level-2 chunk list: coarse bin c (offsets off(c) = cnt1[c nb1], total at
// cnt1[n1 nb1]) is cut into ceil(n_c / CHK) chunks; key_chunk0[c] is its first
// chunk and chunk_key[] names the coarse bin of each chunk.  One block.
__global__ __launch_bounds__(kScanBlock) void k_l2_chunks(Geom g, const int32_t *__restrict__ base1, int32_t nb1,
                                                          int32_t *__restrict__ key_chunk0,
                                                          int32_t *__restrict__ chunk_key, Stats *__restrict__ st) {
    int32_t carry = 0;
    for (int32_t s0 = 0; s0 < g.n1; s0 += kScanBlock) {
        const int32_t c = s0 + threadIdx.x;
        int32_t nch = 0;
        if (c < g.n1) {
            const int32_t n = base1[(int64_t)(c + 1) * nb1] - base1[(int64_t)c * nb1];
            nch = (n + g.CHK - 1) / g.CHK;
        }
        int32_t x = nch, y = 0, tx, ty;
        block_scan2(x, y, tx, ty);
        if (c < g.n1) {
            key_chunk0[c] = carry + x;
            for (int32_t j = 0; j < nch; ++j) chunk_key[carry + x + j] = c;
        }
        carry += tx;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        key_chunk0[g.n1] = carry;
        st->n_chunks = (unsigned long long)carry;
        st->n_heavy = 0;
        st->n_dead = 0;   // (counted by bin_scatter, which runs next)
    }
}

// ---- level 2: bins inside each coarse bin ----

// Chunk `chunk` of coarse bin `key`: records [r0, r1) of the level-1 array.
struct Chunk {
    int32_t key, r0, r1, ctx, cty;
};
__device__ __forceinline__ Chunk chunk_of(const Geom &g, const int32_t *__restrict__ base1, int32_t nb1,
                                          const int32_t *__restrict__ key_chunk0,
                                          const int32_t *__restrict__ chunk_key, int32_t chunk) {
    Chunk c;
    c.key = chunk_key[chunk];
    const int32_t j = chunk - key_chunk0[c.key];
    const int32_t end = base1[(int64_t)(c.key + 1) * nb1];
    c.r0 = base1[(int64_t)c.key * nb1] + j * g.CHK;
    c.r1 = c.r0 + g.CHK < end ? c.r0 + g.CHK : end;
    const int32_t rem = c.key % (g.nct * g.nct);
    c.cty = rem / g.nct;
    c.ctx = rem % g.nct;
    return c;
}

// Tile of the coarse tile holding a level-1 record's footprint origin: local
// column fx0, row fy0 (in [0, C): the coarse bin is the origin's).
struct Local {
    int32_t fx0, fy0;
};
__device__ __forceinline__ Local local_span(const Geom &g, const Pos1 &p) {
    return Local{p.ox1 >> g.log2T, p.oy1 >> g.log2T};
}

// Per (chunk, tile): live record count, from the positions alone unless a
// record of the call is dead (then W V too).
template <typename real, bool CPT>
__global__ __launch_bounds__(kBlock) void k_l2_count(Geom g, const int32_t *__restrict__ base1, int32_t nb1,
                                                     const int32_t *__restrict__ key_chunk0,
                                                     const int32_t *__restrict__ chunk_key,
                                                     const Stats *__restrict__ st, const P1<CPT> *__restrict__ pos1,
                                                     const real *__restrict__ vis1, int32_t *__restrict__ cnt2) {
    extern __shared__ int32_t s_h[];   // C^2 counters
    const int32_t chunk = blockIdx.x;
    if (chunk >= (int32_t)st->n_chunks) return;
    const int32_t C2 = g.C * g.C;
    const bool any_dead = st->n_dead != 0;
    for (int i = threadIdx.x; i < C2; i += kBlock) s_h[i] = 0;
    __syncthreads();
    const Chunk ck = chunk_of(g, base1, nb1, key_chunk0, chunk_key, chunk);
    for (int32_t r00 = ck.r0; r00 < ck.r1; r00 += kBlock) {
        const int32_t r = r00 + threadIdx.x;
        bool valid = r < ck.r1;
        Local ls{0, 0};
        if (valid) {
            ls = local_span(g, pos_of(g, pos1[r], ck.ctx, ck.cty));
            if (any_dead) valid = !isnan((double)vis1[2 * (int64_t)r]);
        }
        const int32_t f = ls.fy0 * g.C + ls.fx0;
        const Run run = runs_of(valid ? f : -1);
        if (valid && run.head) atomicAdd(&s_h[f], run.len);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < C2; i += kBlock) cnt2[(int64_t)chunk * C2 + i] = s_h[i];
}

// bin b = (plane, tile y, tile x) -> its coarse bin and its index inside it
__device__ __forceinline__ void bin_place(const Geom &g, int32_t b, int32_t &key, int32_t &f) {
    const int32_t k = b / (g.nt * g.nt);
    const int32_t rem = b - k * g.nt * g.nt;
    const int32_t ty = rem / g.nt, tx = rem % g.nt;
    key = (k * g.nct + (ty >> g.log2C)) * g.nct + (tx >> g.log2C);
    f = (ty & (g.C - 1)) * g.C + (tx & (g.C - 1));
}

// records per bin (the sum over its coarse bin's chunks)
__global__ __launch_bounds__(kBlock) void k_l2_totals(Geom g, const int32_t *__restrict__ key_chunk0,
                                                      const int32_t *__restrict__ cnt2, int32_t *__restrict__ counts) {
    const int32_t b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= g.nbins) return;
    int32_t key, f;
    bin_place(g, b, key, f);
    const int64_t C2 = (int64_t)g.C * g.C;
    int32_t t = 0;
    for (int32_t c = key_chunk0[key]; c < key_chunk0[key + 1]; ++c) t += cnt2[c * C2 + f];
    counts[b] = t;
}

// largest |W V| of each bin's records (float32 records: the gridder's
// fixed-point scale), the maximum over its coarse bin's chunks
__global__ __launch_bounds__(kBlock) void k_bin_vmax(Geom g, const int32_t *__restrict__ key_chunk0,
                                                     const uint32_t *__restrict__ vmax2,
                                                     uint32_t *__restrict__ bin_vmax) {
    const int32_t b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= g.nbins) return;
    int32_t key, f;
    bin_place(g, b, key, f);
    const int64_t C2 = (int64_t)g.C * g.C;
    uint32_t m = 0u;
    for (int32_t c = key_chunk0[key]; c < key_chunk0[key + 1]; ++c) m = max(m, vmax2[c * C2 + f]);
    bin_vmax[b] = m;
}

// per (chunk, tile) record offsets, in place over the counts
__global__ __launch_bounds__(kBlock) void k_l2_bases(Geom g, const int32_t *__restrict__ key_chunk0,
                                                     const BinScan *__restrict__ scan, int32_t *__restrict__ cnt2) {
    const int32_t b = blockIdx.x * kBlock + threadIdx.x;
    if (b >= g.nbins) return;
    int32_t key, f;
    bin_place(g, b, key, f);
    const int64_t C2 = (int64_t)g.C * g.C;
    int32_t run = scan[b].rec;
    for (int32_t c = key_chunk0[key]; c < key_chunk0[key + 1]; ++c) {
        const int32_t t = cnt2[c * C2 + f];
        cnt2[c * C2 + f] = run;
        run += t;
    }
}

// Level-2 scatter, staged: the chunk is taken kSub records at a time; slots
// come from the LDS cursors as above, and within a sub-chunk the records of
// one tile have consecutive slots.  They are placed in LDS grouped by tile
// (each tile's group in slot order) and written out from there, so that
// consecutive threads write consecutive slots: whole lines instead of the
// short runs of the load order.
constexpr int kSubPer = 4;                   // records per thread per sub-chunk
constexpr int kSub = kBlock * kSubPer;       // records per sub-chunk

// inclusive scan of a[0..n) in place by one block of kBlock threads; returns the total
__device__ __forceinline__ int32_t block_scan_incl(int32_t *a, int32_t n) {
    __shared__ int32_t s_wave[kBlock / 64];
    const int per = (n + kBlock - 1) / kBlock, lo = threadIdx.x * per;
    int32_t sum = 0;
    for (int i = 0; i < per; ++i)
        if (lo + i < n) sum += a[lo + i];
    const int lane = (int)__lane_id(), wid = threadIdx.x >> 6;
    int32_t x = sum;
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) s_wave[wid] = x;
    __syncthreads();
    int32_t before = 0, total = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
        if (w < wid) before += s_wave[w];
        total += s_wave[w];
    }
    int32_t run = before + x - sum;   // exclusive prefix of this thread's entries
    for (int i = 0; i < per; ++i)
        if (lo + i < n) {
            run += a[lo + i];
            a[lo + i] = run;
        }
    __syncthreads();
    return total;
}

template <typename real, bool CPT>
__global__ __launch_bounds__(kBlock) void k_l2_scatter(Geom g, const int32_t *__restrict__ base1, int32_t nb1,
                                                       const int32_t *__restrict__ key_chunk0,
                                                       const int32_t *__restrict__ chunk_key,
                                                       const Stats *__restrict__ st, const P1<CPT> *__restrict__ pos1,
                                                       const real *__restrict__ vis1,
                                                       const int32_t *__restrict__ base2,
                                                       uint32_t *__restrict__ rec_pos, real *__restrict__ rec_vis,
                                                       uint32_t *__restrict__ vmax2) {
    // C^2 cursors, then C^2 per-tile placement offsets, then (float32) C^2 maxima
    extern __shared__ int32_t s_cur[];
    __shared__ int32_t s_slot[kSub];
    __shared__ uint32_t s_pos[kSub];
    __shared__ real s_v[2 * kSub];
    const int32_t chunk = blockIdx.x;
    if (chunk >= (int32_t)st->n_chunks) return;
    const int32_t C2 = g.C * g.C;
    int32_t *s_adj = s_cur + C2;
    uint32_t *s_m = reinterpret_cast<uint32_t *>(s_cur + 2 * C2);
    constexpr bool VMAX = sizeof(real) == 4;
    for (int i = threadIdx.x; i < C2; i += kBlock) {
        s_cur[i] = base2[(int64_t)chunk * C2 + i];
        if (VMAX) s_m[i] = 0u;
    }
    __syncthreads();
    const Chunk ck = chunk_of(g, base1, nb1, key_chunk0, chunk_key, chunk);
    for (int32_t r0 = ck.r0; r0 < ck.r1; r0 += kSub) {
        for (int i = threadIdx.x; i < C2; i += kBlock) s_adj[i] = s_cur[i];   // cursors at the sub-chunk start
        __syncthreads();
        int32_t slot[kSubPer], tile[kSubPer];
        uint32_t pos[kSubPer];
        real vr[kSubPer], vi[kSubPer];
#pragma unroll
        for (int j = 0; j < kSubPer; ++j) {
            const int32_t r = r0 + j * kBlock + (int32_t)threadIdx.x;
            bool valid = r < ck.r1;
            Pos1 ps{0, 0, 0, 0, 0};
            vr[j] = 0;
            vi[j] = 0;
            if (valid) {
                ps = pos_of(g, pos1[r], ck.ctx, ck.cty);
                vr[j] = vis1[2 * (int64_t)r];
                vi[j] = vis1[2 * (int64_t)r + 1];
                valid = !isnan((double)vr[j]);   // dead records are skipped
            }
            const Local ls = local_span(g, ps);
            const int32_t f = ls.fy0 * g.C + ls.fx0;
            const Run run = runs_of(valid ? f : -1);
            int32_t b0 = 0;
            if (valid && run.head) b0 = atomicAdd(&s_cur[f], run.len);
            if constexpr (VMAX) {
                // largest |W V| per tile (non-negative floats order as their bits)
                const uint32_t mbits = __float_as_uint(fmaxf(fabsf((float)vr[j]), fabsf((float)vi[j])));
                if (valid && mbits) atomicMax(&s_m[f], mbits);
            }
            slot[j] = valid ? __shfl(b0, run.leader) + ((int32_t)__lane_id() - run.leader) : -1;
            tile[j] = f;
            const uint32_t ox = (uint32_t)(ps.ox1 & (g.T - 1)), oy = (uint32_t)(ps.oy1 & (g.T - 1));   // in the tile
            // tile offsets take 6 bits (T <= 64); bits 6-7 and 14 carry the
            // w-fraction bin of a non-separable table
            const uint32_t iw = (uint32_t)ps.iw;
            pos[j] = ox | (iw & 3u) << 6 | oy << 8 | (iw >> 2) << 14 | (uint32_t)ps.sx << 16 | (uint32_t)ps.sy << 24;
        }
        __syncthreads();   // every slot of the sub-chunk is taken
        // placement: tile f's records go to [base_f, base_f + n_f) in slot order,
        // n_f = cursor now - cursor at the start, base_f the exclusive scan of n_f;
        // the offset slot - start_f + base_f = slot + (inclusive scan_f - cursor now)
        for (int i = threadIdx.x; i < C2; i += kBlock) s_adj[i] = s_cur[i] - s_adj[i];
        __syncthreads();
        const int32_t n_sub = block_scan_incl(s_adj, C2);
        for (int i = threadIdx.x; i < C2; i += kBlock) s_adj[i] -= s_cur[i];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kSubPer; ++j) {
            if (slot[j] >= 0) {
                const int32_t e = slot[j] + s_adj[tile[j]];
                s_slot[e] = slot[j];
                s_pos[e] = pos[j];
                s_v[2 * e] = vr[j];
                s_v[2 * e + 1] = vi[j];
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < n_sub; e += kBlock) {
            const int32_t sl = s_slot[e];
            rec_pos[sl] = s_pos[e];
            store2(rec_vis + 2 * (int64_t)sl, s_v[2 * e], s_v[2 * e + 1]);
        }
        __syncthreads();   // the staging arrays and placement offsets are reused
    }
    if constexpr (VMAX)
        for (int i = threadIdx.x; i < C2; i += kBlock) vmax2[(int64_t)chunk * C2 + i] = s_m[i];
}

// ---- scan of per-bin record counts in bin order ----
// gridding work items of a bin: none for an empty bin (its tile is not written)
__device__ __forceinline__ int32_t chunks_of(int32_t count, int32_t CH) {
    return (count + CH - 1) / CH;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_partials(const int32_t *__restrict__ counts, int32_t n,
                                                              int32_t CH, int32_t *__restrict__ bsum) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanPer;
    int32_t a = 0, b = 0;
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) {
            const int32_t c = counts[base + k];
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
    for (int32_t s0 = 0; s0 < nblk; s0 += kScanBlock) {
        const int32_t i = s0 + threadIdx.x;
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
                                                           BinScan *__restrict__ scan, int32_t *__restrict__ item_bin,
                                                           int32_t *__restrict__ heavy_bins, Stats *__restrict__ st) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanPer;
    int32_t c[kScanPer], a = 0, b = 0;
    for (int k = 0; k < kScanPer; ++k) {
        c[k] = base + k < n ? counts[base + k] : 0;
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

}  // namespace

__global__ void k_stamp(uint64_t *slot) {
    if (threadIdx.x == 0) *slot = wall_clock64();
}

hipError_t launch_stamp(uint64_t *slot, hipStream_t s) {
    hipLaunchKernelGGL(k_stamp, dim3(1), dim3(64), 0, s, slot);
    return hipGetLastError();
}

hipError_t launch_zero_stats(Stats *st, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_stats, dim3(1), dim3(64), 0, s, st);
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

// level-1 partition of nvis visibilities over at most kL1Blocks blocks
static L1Part l1_part(int64_t nvis) {
    int64_t nb = (nvis + kL1Block - 1) / kL1Block;
    if (nb < 1) nb = 1;
    if (nb > kL1Blocks) nb = kL1Blocks;
    int64_t per = (nvis + nb - 1) / nb;
    per = (per + kL1Block - 1) / kL1Block * kL1Block;
    if (per < kL1Block) per = kL1Block;
    nb = (nvis + per - 1) / per;
    if (nb < 1) nb = 1;
    return L1Part{(int32_t)nb, (int32_t)per};
}

namespace {
void *g_scratch_ptr[kMaxDevices];
hipError_t g_scratch_err[kMaxDevices];
std::once_flag g_scratch_once[kMaxDevices];
}  // namespace

hipError_t static_scratch_setup() {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::call_once(g_scratch_once[dev], [dev] {
        void *ptr = nullptr;
        const hipError_t r = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        g_scratch_err[dev] = r;
        g_scratch_ptr[dev] = r == hipSuccess ? ptr : nullptr;
    });
    return g_scratch_err[dev];
}

hipError_t static_scratch(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    e = static_scratch_setup();
    if (e != hipSuccess) return e;
    *out = g_scratch_ptr[device];
    return *out ? hipSuccess : hipErrorInvalidSymbol;
}

int64_t flat_scan_partials(int64_t n) { return (n + 1 + kScanTile - 1) / kScanTile; }

hipError_t launch_flat_scan(int32_t *a, int64_t n, int32_t *bsum, hipStream_t s) {
    const int32_t nblk = (int32_t)flat_scan_partials(n);
    hipLaunchKernelGGL(k_flat_partials, dim3(nblk), dim3(kScanBlock), 0, s, a, n, bsum);
    hipLaunchKernelGGL(k_flat_top, dim3(1), dim3(kScanBlock), 0, s, bsum, nblk);
    hipLaunchKernelGGL(k_flat_apply, dim3(nblk), dim3(kScanBlock), 0, s, a, n, bsum);
    return hipGetLastError();
}

int32_t bin_max_chunks(const Geom &g, int64_t max_records) {
    return (int32_t)(g.n1 + (max_records + g.CHK - 1) / g.CHK);
}

template <typename real>
hipError_t launch_bin_level1(const Geom &g, const BinBufs &bb, const double *uvw, const double *scales_dev,
                             const real *vis, const float *weight, int64_t nrow, int32_t nchan, Stats *st, int phase,
                             hipStream_t s) {
    const int64_t nvis = nrow * nchan;
    const L1Part part = l1_part(nvis);
    const size_t lds = size_t(g.n1) * sizeof(int32_t);
    const bool cpt = g.cpt1 && sizeof(real) == 4;
    real *vis1 = reinterpret_cast<real *>(static_cast<unsigned char *>(bb.rec1) + l1_vis_offset(nvis, cpt));
    if (phase == 0) {
        hipLaunchKernelGGL(k_l1_count, dim3(part.nb1), dim3(kL1Block), lds, s, g, uvw, scales_dev, weight, nvis,
                           nchan, part, bb.cnt1);
    } else if (phase == 1) {
        const int64_t n = (int64_t)g.n1 * part.nb1;
        const int32_t nblk = (int32_t)((n + 1 + kScanTile - 1) / kScanTile);
        hipLaunchKernelGGL(k_flat_partials, dim3(nblk), dim3(kScanBlock), 0, s, bb.cnt1, n, bb.bsum);
        hipLaunchKernelGGL(k_flat_top, dim3(1), dim3(kScanBlock), 0, s, bb.bsum, nblk);
        hipLaunchKernelGGL(k_flat_apply, dim3(nblk), dim3(kScanBlock), 0, s, bb.cnt1, n, bb.bsum);
        hipLaunchKernelGGL(k_l2_chunks, dim3(1), dim3(kScanBlock), 0, s, g, bb.cnt1, part.nb1, bb.key_chunk0,
                           bb.chunk_key, st);
    } else if (cpt) {
        hipLaunchKernelGGL((k_l1_scatter<real, true>), dim3(part.nb1), dim3(kL1Block), lds, s, g, uvw, scales_dev,
                           vis, weight, nvis, nchan, part, bb.cnt1, (P1<true> *)bb.rec1, vis1, st);
    } else {
        hipLaunchKernelGGL((k_l1_scatter<real, false>), dim3(part.nb1), dim3(kL1Block), lds, s, g, uvw, scales_dev,
                           vis, weight, nvis, nchan, part, bb.cnt1, (P1<false> *)bb.rec1, vis1, st);
    }
    return hipGetLastError();
}

template <typename real>
hipError_t launch_bin_level2(const Geom &g, const BinBufs &bb, int64_t nrow, int32_t nchan, Stats *st, int phase,
                             hipStream_t s) {
    const int64_t nvis = nrow * nchan;
    const L1Part part = l1_part(nvis);
    // chunks of this call: at most one per coarse bin plus one per CHK level-1 records (one per visibility)
    const int32_t nchunk = bin_max_chunks(g, nvis);
    const size_t lds = size_t(g.C) * g.C * sizeof(int32_t);
    const int32_t nbb = (g.nbins + kBlock - 1) / kBlock;
    const bool cpt = g.cpt1 && sizeof(real) == 4;
    const real *vis1 =
        reinterpret_cast<const real *>(static_cast<const unsigned char *>(bb.rec1) + l1_vis_offset(nvis, cpt));
    if (phase == 0) {
        if (cpt)
            hipLaunchKernelGGL((k_l2_count<real, true>), dim3(nchunk), dim3(kBlock), lds, s, g, bb.cnt1, part.nb1,
                               bb.key_chunk0, bb.chunk_key, st, (const P1<true> *)bb.rec1, vis1, bb.cnt2);
        else
            hipLaunchKernelGGL((k_l2_count<real, false>), dim3(nchunk), dim3(kBlock), lds, s, g, bb.cnt1, part.nb1,
                               bb.key_chunk0, bb.chunk_key, st, (const P1<false> *)bb.rec1, vis1, bb.cnt2);
    } else if (phase == 1) {
        hipLaunchKernelGGL(k_l2_totals, dim3(nbb), dim3(kBlock), 0, s, g, bb.key_chunk0, bb.cnt2, bb.counts);
        const int32_t n = g.nbins;
        const int32_t nblk = (n + 1 + kScanTile - 1) / kScanTile;
        hipLaunchKernelGGL(k_scan_partials, dim3(nblk), dim3(kScanBlock), 0, s, bb.counts, n, g.CH, bb.bsum);
        hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, s, bb.bsum, nblk);
        hipLaunchKernelGGL(k_scan_apply, dim3(nblk), dim3(kScanBlock), 0, s, bb.counts, n, g.CH, bb.bsum, bb.scan,
                           bb.item_bin, bb.heavy_bins, st);
        hipLaunchKernelGGL(k_l2_bases, dim3(nbb), dim3(kBlock), 0, s, g, bb.key_chunk0, bb.scan, bb.cnt2);
    } else {
        // cursors, placement offsets and (float32 records) the per-tile maxima
        const size_t lds2 = (sizeof(real) == 4 ? 3 : 2) * lds;
        if (cpt)
            hipLaunchKernelGGL((k_l2_scatter<real, true>), dim3(nchunk), dim3(kBlock), lds2, s, g, bb.cnt1, part.nb1,
                               bb.key_chunk0, bb.chunk_key, st, (const P1<true> *)bb.rec1, vis1, bb.cnt2, bb.rec_pos,
                               (real *)bb.rec_vis, bb.vmax2);
        else
            hipLaunchKernelGGL((k_l2_scatter<real, false>), dim3(nchunk), dim3(kBlock), lds2, s, g, bb.cnt1,
                               part.nb1, bb.key_chunk0, bb.chunk_key, st, (const P1<false> *)bb.rec1, vis1, bb.cnt2,
                               bb.rec_pos, (real *)bb.rec_vis, bb.vmax2);
        if (sizeof(real) == 4)
            hipLaunchKernelGGL(k_bin_vmax, dim3(nbb), dim3(kBlock), 0, s, g, bb.key_chunk0, bb.vmax2, bb.bin_vmax);
    }
    return hipGetLastError();
}

template hipError_t launch_bin_level1<float>(const Geom &, const BinBufs &, const double *, const double *,
                                             const float *, const float *, int64_t, int32_t, Stats *, int,
                                             hipStream_t);
template hipError_t launch_bin_level1<double>(const Geom &, const BinBufs &, const double *, const double *,
                                              const double *, const float *, int64_t, int32_t, Stats *, int,
                                              hipStream_t);
template hipError_t launch_bin_level2<float>(const Geom &, const BinBufs &, int64_t, int32_t, Stats *, int,
                                             hipStream_t);
template hipError_t launch_bin_level2<double>(const Geom &, const BinBufs &, int64_t, int32_t, Stats *, int,
                                              hipStream_t);

}  // namespace rick
