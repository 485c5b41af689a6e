// Batched, centred 2-D inverse FFT of every w-plane (the FFT step of
// Sec. 2.1), in place in HBM, in two passes:
//   fft_rows         one block per row (several rows for small N),
//   fft_cols         one block per strip of V adjacent columns of one plane,
//   fft_cols_screen  the column pass fused with the w-correction and the sum
//                    over planes: one block per strip, looping over planes.
//
// Each transform is a Stockham autosort FFT held in registers: a thread owns
// 16 elements per stage (one radix-16 butterfly, or 16/R butterflies of the
// first stage's radix R in {2, 4, 8} when log2 N is not a multiple of 4).
// Stage of radix R over L-point sub-transforms (butterfly b, k = b mod L):
//   a_j = x[b + j N/R] w_{L R}^{j k},  A = DFT_R(a),  y[(b / L) L R + k + q L] = A_q,
// with w_M = exp(+2 pi i / M).  The first stage reads its inputs straight
// from HBM and the last stage writes straight to HBM (both coalesced); only
// the exchanges between stages go through LDS (two for N = 4096).
//
// Twiddles come from a table of exp(+2 pi i m / N) computed in float64 on the
// host and rounded.  A radix-16 butterfly reads w^j for j in {1, 2, 3, 4, 8,
// 12} and forms each other power as one product of two table entries.
//
// Centring: for N divisible by 4,
//   sum_i x_i exp(+2 pi i (i - N/2)(p - N/2) / N) = (-1)^p sum_i (-1)^i x_i exp(+2 pi i i p / N),
// so each pass flips signs on load and on store.
//
// LDS element e is stored at e + e / 16, which keeps the stride-16 writes of
// the first exchange on distinct banks.
//
// Tile occupancy: the gridder writes only the tiles that received records,
// so the row passes read a row segment only where its tile is set and take
// zeros elsewhere; rows of an empty tile row are written as zeros (in place)
// or not at all (fused path, whose column pass then takes them as zeros).
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

// inverse DFTs (positive exponent), natural order in and out
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
    const real r = (real)0.70710678118654752440;              // 1/sqrt(2)
    const C t1 = C{(o1.x - o1.y) * r, (o1.x + o1.y) * r};     // * exp(+i pi/4)
    const C t2 = mul_pi(o2);                                  // * i
    const C t3 = C{(-o3.x - o3.y) * r, (o3.x - o3.y) * r};    // * exp(+3i pi/4)
    a[0] = cadd(e0, o0);
    a[4] = csub(e0, o0);
    a[1] = cadd(e1, t1);
    a[5] = csub(e1, t1);
    a[2] = cadd(e2, t2);
    a[6] = csub(e2, t2);
    a[3] = cadd(e3, t3);
    a[7] = csub(e3, t3);
}
// 16 = 4 x 4: DFT4 over n1 for each n2, twiddle exp(+2 pi i n2 k1 / 16), DFT4 over n2
template <typename C>
__device__ __forceinline__ void dft16(C *a) {
    using real = decltype(a[0].x);
    const real c1 = (real)0.92387953251128675613;   // cos(pi/8)
    const real s1 = (real)0.38268343236508977173;   // sin(pi/8)
    const real h = (real)0.70710678118654752440;    // cos(pi/4)
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) dft4(a[n2], a[n2 + 4], a[n2 + 8], a[n2 + 12]);
    // a[n2 + 4 k1] now holds the inner DFT of index n2 at frequency k1
    a[5] = cmul(a[5], C{c1, s1});      // n2=1, k1=1: w16^1
    a[9] = cmul(a[9], C{h, h});        // n2=1, k1=2: w16^2
    a[13] = cmul(a[13], C{s1, c1});    // n2=1, k1=3: w16^3
    a[6] = cmul(a[6], C{h, h});        // n2=2, k1=1: w16^2
    a[10] = mul_pi(a[10]);             // n2=2, k1=2: w16^4
    a[14] = cmul(a[14], C{-h, h});     // n2=2, k1=3: w16^6
    a[7] = cmul(a[7], C{s1, c1});      // n2=3, k1=1: w16^3
    a[11] = cmul(a[11], C{-h, h});     // n2=3, k1=2: w16^6
    a[15] = cmul(a[15], C{-c1, -s1});  // n2=3, k1=3: w16^9
    C o[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        C b0 = a[4 * k1], b1 = a[4 * k1 + 1], b2 = a[4 * k1 + 2], b3 = a[4 * k1 + 3];
        dft4(b0, b1, b2, b3);
        o[k1] = b0;
        o[k1 + 4] = b1;
        o[k1 + 8] = b2;
        o[k1 + 12] = b3;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) a[i] = o[i];
}

template <int R, typename C>
__device__ __forceinline__ void dftR(C *a) {
    if constexpr (R == 2) dft2(a[0], a[1]);
    else if constexpr (R == 4) dft4(a[0], a[1], a[2], a[3]);
    else if constexpr (R == 8) dft8(a);
    else dft16(a);
}

constexpr int ilog2c(int n) { return n <= 1 ? 0 : 1 + ilog2c(n / 2); }

__device__ __forceinline__ int padi(int e) { return e + (e >> 4); }

template <int N>
struct Shape {
    static constexpr int LG = ilog2c(N);
    static constexpr int R0 = (LG % 4) == 0 ? 16 : (1 << (LG % 4));   // first-stage radix
    static constexpr int S = 1 + (LG - ilog2c(R0)) / 4;               // number of stages (>= 2 for N >= 64)
    static constexpr int NT = N / 16;                                 // threads per transform
    static constexpr int PADN = N + N / 16;                           // padded LDS elements
};

// Multiplies x[1..15] of a radix-16 butterfly by w^j, w = exp(+2 pi i k / (16 L)).
template <int N, typename C>
__device__ __forceinline__ void twiddle16(C *x, int k, int L, const C *__restrict__ tw) {
    const int st = k * (N / (16 * L));
    const C w1 = tw[st], w2 = tw[2 * st], w3 = tw[3 * st], w4 = tw[4 * st], w8 = tw[8 * st], w12 = tw[12 * st];
    x[1] = cmul(x[1], w1);
    x[2] = cmul(x[2], w2);
    x[3] = cmul(x[3], w3);
    x[4] = cmul(x[4], w4);
    x[5] = cmul(x[5], cmul(w4, w1));
    x[6] = cmul(x[6], cmul(w4, w2));
    x[7] = cmul(x[7], cmul(w4, w3));
    x[8] = cmul(x[8], w8);
    x[9] = cmul(x[9], cmul(w8, w1));
    x[10] = cmul(x[10], cmul(w8, w2));
    x[11] = cmul(x[11], cmul(w8, w3));
    x[12] = cmul(x[12], w12);
    x[13] = cmul(x[13], cmul(w12, w1));
    x[14] = cmul(x[14], cmul(w12, w2));
    x[15] = cmul(x[15], cmul(w12, w3));
}

// One N-point transform per vector lane, VC vector lanes per thread.  `x`
// arrives in the first stage's input layout,
//   x[i R0 + j][v] = element (tb + i NT) + j N/R0 of vector lane v0 + v,
// and leaves in the last stage's output layout, x[q][v] = element tb + q NT.
// buf: LDS with V vector lanes per element, element e at padi(e) * V.
template <int N, int V, int VC, typename C>
__device__ __forceinline__ void fft_regs(C (&x)[16][VC], C *buf, int tb, int v0, const C *__restrict__ tw) {
    using SH = Shape<N>;
    constexpr int NT = SH::NT, R0 = SH::R0, S = SH::S;
    static_assert(S >= 2, "N >= 64");
    // stage 0 (L = 1, no twiddles)
#pragma unroll
    for (int v = 0; v < VC; ++v) {
        C tmp[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) tmp[i] = x[i][v];
#pragma unroll
        for (int i = 0; i < 16 / R0; ++i) dftR<R0>(tmp + i * R0);
#pragma unroll
        for (int i = 0; i < 16; ++i) x[i][v] = tmp[i];
    }
    int L = R0;
#pragma unroll
    for (int s = 1; s < S; ++s) {
        // previous stage's outputs y[(b / Lp) Lp Rp + b mod Lp + q Lp] -> LDS
        if (s > 1) __syncthreads();   // every thread has read the previous exchange
        if (s == 1) {
#pragma unroll
            for (int i = 0; i < 16 / R0; ++i) {
                const int b = tb + i * NT;   // Lp = 1, Rp = R0
#pragma unroll
                for (int q = 0; q < R0; ++q)
#pragma unroll
                    for (int v = 0; v < VC; ++v) buf[padi(b * R0 + q) * V + v0 + v] = x[i * R0 + q][v];
            }
        } else {
            const int Lp = L / 16;
            const int b = tb, k = b % Lp;
            const int base = (b / Lp) * Lp * 16 + k;
#pragma unroll
            for (int q = 0; q < 16; ++q)
#pragma unroll
                for (int v = 0; v < VC; ++v) buf[padi(base + q * Lp) * V + v0 + v] = x[q][v];
        }
        __syncthreads();
        // this stage's inputs: x[j] = element tb + j NT
#pragma unroll
        for (int j = 0; j < 16; ++j)
#pragma unroll
            for (int v = 0; v < VC; ++v) x[j][v] = buf[padi(tb + j * NT) * V + v0 + v];
        const int k = tb % L;
#pragma unroll
        for (int v = 0; v < VC; ++v) {
            C tmp[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) tmp[i] = x[i][v];
            twiddle16<N>(tmp, k, L, tw);
            dft16(tmp);
#pragma unroll
            for (int i = 0; i < 16; ++i) x[i][v] = tmp[i];
        }
        L *= 16;
    }
}

// first-stage input element of slot i (< 16) for thread tb
template <int N>
__device__ __forceinline__ int in_elem(int tb, int i) {
    using SH = Shape<N>;
    return (tb + (i / SH::R0) * SH::NT) + (i % SH::R0) * (N / SH::R0);
}
// Occupancy word of slot i.  Slot i of thread tb is element tb + c NT (c
// fixed by i, tb < NT), and NT = N / 16 <= 64 T, so the element's tile index
// divided by 64 -- its word in a tile-row or row bitmap -- is the same for
// every thread: the word is a uniform load.
template <int N>
__device__ __forceinline__ int occ_word(int i, int log2T) {
    return in_elem<N>(0, i) >> (log2T + 6);
}
__device__ __forceinline__ bool bit_of(uint64_t word, int idx) { return (word >> (idx & 63)) & 1ull; }
// A bitmap word at a wave-uniform index, read through the scalar cache (the
// bitmaps are not written while the FFT kernels run).
typedef __attribute__((address_space(4))) const uint64_t const_u64;
__device__ __forceinline__ uint64_t uniform_word(const uint64_t *bits, int64_t i) {
    return ((const_u64 *)bits)[i];
}

// last-stage output element of slot q for thread tb
template <int N>
__device__ __forceinline__ int out_elem(int tb, int q) {
    return tb + q * Shape<N>::NT;
}

// ---- the same transform with 8 elements per thread ----
// Radix-8 stages after a first stage of radix R0 in {2, 4, 8}: twice the
// threads per transform and half the registers per thread of the radix-16
// form, for the sizes where a transform's block is the only one its CU holds.
template <int N>
struct Shape8 {
    static constexpr int LG = ilog2c(N);
    static constexpr int R0 = (LG % 3) == 0 ? 8 : (1 << (LG % 3));   // first-stage radix
    static constexpr int S = 1 + (LG - ilog2c(R0)) / 3;               // number of stages
    static constexpr int NT = N / 8;                                  // threads per transform
};

// Multiplies x[1..7] of a radix-8 butterfly by w^j, w = exp(+2 pi i k / (8 L)):
// three table reads and four products.
template <int TN, typename C>
__device__ __forceinline__ void twiddle8(C *x, int k, int L, const C *__restrict__ tw) {
    const int st = k * (TN / (8 * L));
    const C w1 = tw[st], w2 = tw[2 * st], w4 = tw[4 * st];
    const C w3 = cmul(w1, w2);
    x[1] = cmul(x[1], w1);
    x[2] = cmul(x[2], w2);
    x[3] = cmul(x[3], w3);
    x[4] = cmul(x[4], w4);
    x[5] = cmul(x[5], cmul(w4, w1));
    x[6] = cmul(x[6], cmul(w4, w2));
    x[7] = cmul(x[7], cmul(w4, w3));
}

// LDS element e of the radix-8 form at e + e / 8 (its first exchange writes
// at a stride of R0 elements).
__device__ __forceinline__ int padi8(int e) { return e + (e >> 3); }
template <int N>
constexpr int padn8() { return N + N / 8; }

// As fft_regs, with slots of 8: x[i R0 + j][v] = element (tb + i NT) + j N/R0
// on entry, x[q][v] = element tb + q NT on exit (NT = N / 8).
template <int N, int V, int VC, int TN = N, typename C>
__device__ __forceinline__ void fft_regs8(C (&x)[8][VC], C *buf, int tb, int v0, const C *__restrict__ tw) {
    using SH = Shape8<N>;
    constexpr int NT = SH::NT, R0 = SH::R0, S = SH::S;
    static_assert(S >= 2, "N >= 16");
#pragma unroll
    for (int v = 0; v < VC; ++v) {
        C tmp[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) tmp[i] = x[i][v];
#pragma unroll
        for (int i = 0; i < 8 / R0; ++i) dftR<R0>(tmp + i * R0);
#pragma unroll
        for (int i = 0; i < 8; ++i) x[i][v] = tmp[i];
    }
    int L = R0;
#pragma unroll
    for (int s = 1; s < S; ++s) {
        if (s > 1) __syncthreads();   // every thread has read the previous exchange
        if (s == 1) {
#pragma unroll
            for (int i = 0; i < 8 / R0; ++i) {
                const int b = tb + i * NT;   // Lp = 1, Rp = R0
#pragma unroll
                for (int q = 0; q < R0; ++q)
#pragma unroll
                    for (int v = 0; v < VC; ++v) buf[padi8(b * R0 + q) * V + v0 + v] = x[i * R0 + q][v];
            }
        } else {
            const int Lp = L / 8;
            const int b = tb, k = b % Lp;
            const int base = (b / Lp) * Lp * 8 + k;
#pragma unroll
            for (int q = 0; q < 8; ++q)
#pragma unroll
                for (int v = 0; v < VC; ++v) buf[padi8(base + q * Lp) * V + v0 + v] = x[q][v];
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 8; ++j)
#pragma unroll
            for (int v = 0; v < VC; ++v) x[j][v] = buf[padi8(tb + j * NT) * V + v0 + v];
        const int k = tb % L;
#pragma unroll
        for (int v = 0; v < VC; ++v) {
            C tmp[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) tmp[i] = x[i][v];
            twiddle8<TN>(tmp, k, L, tw);
            dft8(tmp);
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i][v] = tmp[i];
        }
        L *= 8;
    }
}

// Slot layouts and transform of E (16 or 8) elements per thread.
template <int N, int E>
__device__ __forceinline__ int in_elem_e(int tb, int i) {
    if constexpr (E == 16) return in_elem<N>(tb, i);
    else return (tb + (i / Shape8<N>::R0) * Shape8<N>::NT) + (i % Shape8<N>::R0) * (N / Shape8<N>::R0);
}
template <int N, int E>
__device__ __forceinline__ int out_elem_e(int tb, int q) {
    return tb + q * (N / E);
}
// word of slot i in a tile-row bitmap: uniform while N / E <= 64 T
template <int N, int E>
__device__ __forceinline__ int occ_word_e(int i, int log2T) {
    return in_elem_e<N, E>(0, i) >> (log2T + 6);
}
template <int N, int E, int V, int VC, typename C>
__device__ __forceinline__ void fft_regs_e(C (&x)[E][VC], C *buf, int tb, int v0, const C *__restrict__ tw) {
    if constexpr (E == 16) fft_regs<N, V, VC>(x, buf, tb, v0, tw);
    else fft_regs8<N, V, VC>(x, buf, tb, v0, tw);
}

// XCD-aware order: blocks are dealt to the 8 XCDs round-robin; blocks that
// share an XCD get adjacent strips, so their row segments share L2 lines.
__device__ __forceinline__ int64_t xcd_order(int64_t bid, int64_t nblk) {
    return (nblk & 7) == 0 ? (bid & 7) * (nblk >> 3) + (bid >> 3) : bid;
}

// ---- rows into column panels (for the fused column pass) ----
// The output goes to a separate buffer in column-panel order: panels of PW
// adjacent columns, each panel stored row after row, element (plane k, row q,
// column p) at k N^2 + (p / PW) N PW + q PW + p % PW, so that the column pass
// reads a strip as RB-row runs of whole cache lines.  A block transforms RB
// consecutive rows (PW RB complex values = one 128-byte line per panel),
// stages them in LDS, and writes each panel's RB x PW values as one line;
// blocks are taken in an XCD-aware order.
template <typename real, int N, int RB, int PW>
__global__ __launch_bounds__((N / 16) * RB) void k_fft_rows_panel(Geom g, const real *__restrict__ in,
                                                                  real *__restrict__ out,
                                                                  const real *__restrict__ twr,
                                                                  const uint64_t *__restrict__ tile_bits,
                                                                  const uint64_t *__restrict__ row_bits) {
    using C = typename R2T<real>::t;
    using SH = Shape<N>;
    constexpr int NT = SH::NT;
    constexpr int CE = 16 / (int)sizeof(C);          // complex values per 16-byte chunk
    constexpr int CPP = RB * PW / CE;                // chunks per panel line
    extern __shared__ __align__(16) unsigned char smem[];
    const C *tw = reinterpret_cast<const C *>(twr);
    // Persistent: the block takes groups of RB rows q = blockIdx.x, + gridDim.x, ...
    // (RB divides N, so a group lies in one tile row, RB <= 4 <= T), skipping
    // groups of an empty tile row (not written: the fused column pass reads
    // them as zeros); the next group is loaded while this one is transformed.
    const int64_t ngroup = (int64_t)g.Nw * N / RB;
    auto next = [&](int64_t q) {
        for (; q < ngroup; q += gridDim.x) {
            const int64_t row0 = q * RB;
            if (row_set(row_bits, g, (int32_t)(row0 / N), (int32_t)(row0 % N) >> g.log2T)) break;
        }
        return q;
    };
    // a group's input (zeros where its tile is clear, which is not read)
    auto load = [&](int64_t q, int tb, int rb, C (&v)[16][1]) {
        const int64_t row0 = q * RB;
        const int32_t kp = (int32_t)(row0 / N), ty = (int32_t)(row0 % N) >> g.log2T;
        const C *gi = reinterpret_cast<const C *>(in) + (row0 + rb) * N;
        const uint64_t *tb_row = tile_bits + ((int64_t)kp * g.nt + ty) * g.occw;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = in_elem<N>(tb, i);
            const bool on = bit_of(uniform_word(tb_row, occ_word<N>(i, g.log2T)), e >> g.log2T);
            v[i][0] = on ? cneg_if(gi[e], e & 1) : C{0, 0};
        }
    };
    int64_t q = next(blockIdx.x);
    C pre[16][1];   // the next group's input, loaded while this one is transformed
    if (q < ngroup) load(q, (int)threadIdx.x % NT, (int)threadIdx.x / NT, pre);
    while (q < ngroup) {
        // the lane's index arithmetic and the twiddle loads are redone per
        // group (L1 hits) rather than held in registers across groups, which
        // would not fit beside the transform
        const C *twq = tw;
        int tid = (int)threadIdx.x;
        __asm__ volatile("" : "+s"(twq), "+v"(tid));
        const int rb = tid / NT, tb = tid % NT;
        C *buf = reinterpret_cast<C *>(smem) + rb * SH::PADN;
        const int64_t row0 = q * RB;
        C x[16][1];
#pragma unroll
        for (int i = 0; i < 16; ++i) x[i][0] = pre[i][0];
        const int64_t qn = next(q + gridDim.x);
        if (qn < ngroup) load(qn, tb, rb, pre);
        __syncthreads();   // the previous group's copy-out has read the staging buffer
        fft_regs<N, 1, 1>(x, buf, tb, 0, twq);
        __syncthreads();   // every thread has read the last exchange
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int e = out_elem<N>(tb, j);
            buf[padi(e)] = cneg_if(x[j][0], e & 1);
        }
        __syncthreads();
        const int64_t k = row0 / N, r0 = row0 % N;
        C *go = reinterpret_cast<C *>(out) + k * N * N + r0 * PW;
        const C *stage = reinterpret_cast<const C *>(smem);
        for (int c = tid; c < N / PW * CPP; c += RB * NT) {
            const int pnl = c / CPP, part = c % CPP;
            const int r = (part * CE) / PW, col = pnl * PW + (part * CE) % PW;
            const C *src = stage + r * SH::PADN + padi(col);   // CE values, contiguous (col even when CE = 2)
            C *dst = go + (int64_t)pnl * N * PW + r * PW + (part * CE) % PW;
#pragma unroll
            for (int j = 0; j < CE; ++j) dst[j] = src[j];
        }
        q = qn;
    }
}

// ---- rows: B rows per block, NT threads per row ----
template <typename real, int N, int B>
__global__ __launch_bounds__((N / 16) * B) void k_fft_rows(Geom g, real *__restrict__ mesh,
                                                           const real *__restrict__ twr,
                                                           const uint64_t *__restrict__ tile_bits,
                                                           const uint64_t *__restrict__ row_bits) {
    using C = typename R2T<real>::t;
    using SH = Shape<N>;
    extern __shared__ __align__(16) unsigned char smem[];
    const C *tw = reinterpret_cast<const C *>(twr);
    const int rb = threadIdx.x / SH::NT, tb = threadIdx.x % SH::NT;
    const int64_t row = (int64_t)blockIdx.x * B + rb;   // B divides the row count N_w N
    const int32_t kp = (int32_t)(row / N), ty = (int32_t)(row % N) >> g.log2T;
    C *buf = reinterpret_cast<C *>(smem) + rb * SH::PADN;
    C *gm = reinterpret_cast<C *>(mesh) + row * N;
    // clear tiles (and every tile of an empty tile row) are zeros, not read;
    // the transform is written in full
    const bool any = row_set(row_bits, g, kp, ty);
    const uint64_t *tb_row = tile_bits + ((int64_t)kp * g.nt + ty) * g.occw;
    C x[16][1];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int e = in_elem<N>(tb, i);
        x[i][0] = any && bit_of(tb_row[occ_word<N>(i, g.log2T)], e >> g.log2T) ? cneg_if(gm[e], e & 1) : C{0, 0};
    }
    fft_regs<N, 1, 1>(x, buf, tb, 0, tw);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = out_elem<N>(tb, q);
        gm[e] = cneg_if(x[q][0], e & 1);
    }
}

// ---- columns: one block per (plane, strip of V columns) ----
// thread tid: vector group vg = tid % (V / VC) (fastest: adjacent columns),
// butterfly lane tb = tid / (V / VC).  PW = 0: rows of N elements; PW > 0:
// column-panel order (row e of column c at (c / PW) N PW + e PW + c % PW, the
// strip inside one panel), so that a strip's row segments fill whole lines.
template <typename real, int N, int V, int VC, int PW>
__global__ __launch_bounds__((N / 16) * (V / VC)) void k_fft_cols(real *__restrict__ mesh,
                                                                  const real *__restrict__ twr, int32_t nw) {
    using C = typename R2T<real>::t;
    constexpr int NSTRIP = N / V;
    constexpr int64_t RS = PW > 0 ? PW : N;   // element stride between rows of a column
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);
    const C *tw = reinterpret_cast<const C *>(twr);
    const int64_t logical = xcd_order(blockIdx.x, (int64_t)nw * NSTRIP);
    const int64_t plane = logical / NSTRIP;
    const int c0 = (int)(logical % NSTRIP) * V;
    const int vg = threadIdx.x % (V / VC), tb = threadIdx.x / (V / VC), v0 = vg * VC;
    const int64_t col_off = PW > 0 ? (int64_t)(c0 / PW) * N * PW + c0 % PW : c0;
    C *g = reinterpret_cast<C *>(mesh) + plane * (int64_t)N * N + col_off + v0;
    C x[16][VC];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int e = in_elem<N>(tb, i);
#pragma unroll
        for (int v = 0; v < VC; ++v) x[i][v] = cneg_if(g[(int64_t)e * RS + v], e & 1);
    }
    fft_regs<N, V, VC>(x, buf, tb, v0, tw);
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const int e = out_elem<N>(tb, q);
#pragma unroll
        for (int v = 0; v < VC; ++v) g[(int64_t)e * RS + v] = cneg_if(x[q][v], e & 1);
    }
}

// Re(exp(+i pi t2) f) (-1)^flip for a phase t2 in float64 half turns.
// t2 = q + g with q the nearest integer, so exp(+i pi t2) = (-1)^q exp(+i pi g),
// |g| <= 1/2.  float32: sincospi_half (rick_internal.h).  float64: sincospi
// of the float64 remainder.
__device__ __forceinline__ float screen_term(double t2, float2 f, int flip) {
    const double qd = rint(t2);
    float sn, pc;
    sincospi_half((float)(t2 - qd), sn, pc);
    const float t = fmaf(pc, f.x, -sn * f.y);
    return (((int)qd ^ flip) & 1) ? -t : t;
}
__device__ __forceinline__ double screen_term(double t2, double2 f, int flip) {
    const double qd = rint(t2);
    double sn, cs;
    sincospi(t2 - qd, &sn, &cs);
    const double t = cs * f.x - sn * f.y;
    return (((int)qd ^ flip) & 1) ? -t : t;
}

// ---- columns fused with the w-correction and the plane sum ----
// One block per strip of V columns loops over the planes: the strip of plane
// k (already transformed along rows) is transformed along columns in
// registers, and each thread adds Re(exp(+2 pi i w_k (n - 1)) F_k) for the E
// x VC pixels it owns (E = 16 elements per thread; 8 in the radix-8 form
// used where a strip's block is the only one its CU holds); the next plane
// is fetched into registers meanwhile.
// The transformed planes are never written back, and the image is written
// once.  n - 1 of the strip's pixels is kept in LDS in float64; the phase
// 2 w_k (n - 1) is formed in float64 half turns.  Planes without a set tile
// are skipped (their F_k is zero).  Pass 0 takes the planes stored as they
// are and writes the image; pass 1 takes the planes stored transposed, whose
// strip of columns is a strip of image rows (n - 1 and the taper are
// symmetric in l and m, so the same values serve), and adds its sums to the
// image there, unless no plane was taken.
template <typename real, int N, int V, int VC, int PW, bool KAHAN, int E>
__device__ __forceinline__ void cols_screen_strip(const Geom &g, const real *__restrict__ mesh,
                                                  const real *__restrict__ twr, const double *__restrict__ corr,
                                                  const Stats *__restrict__ st, const uint64_t *__restrict__ row_bits,
                                                  const int32_t *__restrict__ plane_tr, int pass,
                                                  real *__restrict__ image, int strip) {
    using C = typename R2T<real>::t;
    using SH = Shape<N>;
    extern __shared__ __align__(16) unsigned char smem[];
    C *buf = reinterpret_cast<C *>(smem);
    constexpr int PADN = E == 8 ? padn8<N>() : SH::PADN;   // LDS elements of the exchange
    double *s_nm1 = reinterpret_cast<double *>(buf + PADN * V);
    const C *tw = reinterpret_cast<const C *>(twr);
    const int c0 = strip * V;
    const int vg = threadIdx.x % (V / VC), tb = threadIdx.x / (V / VC), v0 = vg * VC;
    // the row transforms in column-panel order: row e of column c at
    // (c / PW) N PW + e PW + c % PW (the strip lies inside one panel)
    const C *gbase = reinterpret_cast<const C *>(mesh) + (int64_t)(c0 / PW) * N * PW + c0 % PW + v0;
    const int64_t plane_stride = (int64_t)N * N;
    const double dl = g.fov / N;
    // owned pixels: rows out_elem(tb, q), columns c0 + v0 + v
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int e = out_elem_e<N, E>(tb, q);
#pragma unroll
        for (int v = 0; v < VC; ++v) {
            const double l = (double)(c0 + v0 + v - N / 2) * dl, m = (double)(e - N / 2) * dl;
            const double r2 = l * l + m * m;
            s_nm1[e * V + v0 + v] = r2 < 1.0 ? -r2 / (1.0 + sqrt(1.0 - r2)) : 0.0;
        }
    }
    // the planes of this pass holding a set tile, in order (uniform loads)
    typedef __attribute__((address_space(4))) const int32_t const_i32;
    auto taken = [&](int32_t k) {
        if (plane_tr != nullptr && (((const_i32 *)plane_tr)[k] != 0) != (pass != 0)) return false;
        uint64_t any = 0;
        for (int32_t w = 0; w < g.occw; ++w) any |= uniform_word(row_bits, (int64_t)k * g.occw + w);
        return any != 0;
    };
    auto next_plane = [&](int32_t k) {
        while (k < g.Nw && !taken(k)) ++k;
        return k;
    };
    // rows of an empty tile row were not written by the row pass: zeros
    real acc[E][VC], comp[E][VC];
    C pre[E][VC];
    int32_t k = next_plane(0);
    const bool any_plane = k < g.Nw;
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int e = in_elem_e<N, E>(tb, i);
        const bool on = k < g.Nw &&
                        bit_of(uniform_word(row_bits, (int64_t)k * g.occw + occ_word_e<N, E>(i, g.log2T)), e >> g.log2T);
        const C *gk = gbase + (int64_t)k * plane_stride;
#pragma unroll
        for (int v = 0; v < VC; ++v) {
            acc[i][v] = 0;
            comp[i][v] = 0;
            pre[i][v] = on ? gk[(int64_t)e * PW + v] : C{0, 0};
        }
    }
    while (k < g.Nw) {
        // at N >= 8192, and at every N with the compensated sum, the lane
        // indices and the twiddle pointer are laundered per plane, so that
        // the compiler recomputes addresses and reloads twiddles (L1 hits)
        // instead of keeping every stage's values live across the plane
        // loop: kept live they spill (36 registers at 8192 with the
        // compensated sum: 47.6 ms instead of 42.7 for 128 planes of 8192^2;
        // 70 at 4096: 4.73 ms instead of 3.02 for 64 planes of 4096^2);
        // without the compensated sum at N <= 4096 they fit and keeping them
        // is faster (2.50 ms against 2.88 for 64 planes of 4096^2)
        const C *twk = tw;
        int tid = (int)threadIdx.x;
        if (N >= 8192 || KAHAN) __asm__ volatile("" : "+s"(twk), "+v"(tid));
        const int vg = tid % (V / VC), tb = tid / (V / VC), v0 = vg * VC;
        C x[E][VC];
#pragma unroll
        for (int i = 0; i < E; ++i) {
            const int e = in_elem_e<N, E>(tb, i);
#pragma unroll
            for (int v = 0; v < VC; ++v) x[i][v] = cneg_if(pre[i][v], e & 1);
        }
        const int32_t kn = next_plane(k + 1);
        if (kn < g.Nw) {
            const C *gk = gbase + (int64_t)kn * plane_stride;
#pragma unroll
            for (int i = 0; i < E; ++i) {
                const int e = in_elem_e<N, E>(tb, i);
                const bool on =
                    bit_of(uniform_word(row_bits, (int64_t)kn * g.occw + occ_word_e<N, E>(i, g.log2T)), e >> g.log2T);
#pragma unroll
                for (int v = 0; v < VC; ++v) pre[i][v] = on ? gk[(int64_t)e * PW + v] : C{0, 0};
            }
        }
        // the LDS strip is reused plane after plane: every thread must have
        // read the previous plane's last exchange before this plane's first
        __syncthreads();
        fft_regs_e<N, E, V, VC>(x, buf, tb, v0, twk);
        const double w2 = 2.0 * plane_centre(g, k);
#pragma unroll
        for (int q = 0; q < E; ++q) {
            const int e = out_elem_e<N, E>(tb, q);
#pragma unroll
            for (int v = 0; v < VC; ++v) {
                const real term = screen_term(w2 * s_nm1[e * V + v0 + v], x[q][v], e & 1);
                if (KAHAN) {
                    const real y = term - comp[q][v];
                    const real t = acc[q][v] + y;
                    comp[q][v] = (t - acc[q][v]) - y;
                    acc[q][v] = t;
                } else {
                    acc[q][v] += term;
                }
            }
        }
        k = kn;
    }
    if (pass != 0 && !any_plane) return;   // (uniform) nothing to add
    const double sw = st->sum_w;
#pragma unroll
    for (int q = 0; q < E; ++q) {
        const int e = out_elem_e<N, E>(tb, q);
#pragma unroll
        for (int v = 0; v < VC; ++v) {
            const int p = c0 + v0 + v;
            const double l = (double)(p - N / 2) * dl, m = (double)(e - N / 2) * dl;
            const bool in_sky = l * l + m * m < 1.0;
            const double nm1 = s_nm1[e * V + v0 + v];
            // pass 1: the strip's column p is image row p, its row e image column e
            const int64_t row = pass ? p : e, col = pass ? e : p;
            const double val =
                (sw > 0.0 && in_sky) ? (1.0 + nm1) * (double)acc[q][v] / (taper_at(g, corr, row, col) * sw) : 0.0;
            if (pass) image[row * N + col] += (real)val;
            else image[row * N + col] = (real)val;
        }
    }
}

template <typename real, int N, int V, int VC, int PW, bool KAHAN, int E>
__global__ __launch_bounds__((N / E) * (V / VC)) void k_fft_cols_screen(Geom g, const real *__restrict__ mesh,
                                                                         const real *__restrict__ twr,
                                                                         const double *__restrict__ corr,
                                                                         const Stats *__restrict__ st,
                                                                         const uint64_t *__restrict__ row_bits,
                                                                         const int32_t *__restrict__ plane_tr,
                                                                         int pass, real *__restrict__ image) {
    cols_screen_strip<real, N, V, VC, PW, KAHAN, E>(g, mesh, twr, corr, st, row_bits, plane_tr, pass, image,
                                                    (int)xcd_order(blockIdx.x, N / V));
}

// The fused column pass of several plans of one grid size in one launch,
// one block per (job, strip), with that job's operands read from its device
// slot (uniform: scalar loads).  The per-strip work is the single-plan
// kernel's.  Blocks go to the 8 XCDs round-robin; each XCD takes the same
// eighth of every job's strips (adjacent strips, sharing L2 lines), job
// after job, so that jobs of unequal work keep every XCD busy.
typedef __attribute__((address_space(4))) const uint32_t const_u32_cols;
__device__ __forceinline__ ColJob load_col_job(const ColJob *p) {
    static_assert(sizeof(ColJob) % 4 == 0, "whole words");
    ColJob v;
    uint32_t *dst = reinterpret_cast<uint32_t *>(&v);
    const const_u32_cols *src = (const const_u32_cols *)p;
#pragma unroll
    for (int i = 0; i < (int)(sizeof(ColJob) / 4); ++i) dst[i] = src[i];
    return v;
}
template <typename real, int N, int V, int VC, int PW, bool KAHAN, int E>
__global__ __launch_bounds__((N / E) * (V / VC)) void k_fft_cols_screen_jobs(ColJobList list, int pass) {
    constexpr int NSTRIP = N / V;
    int32_t j, strip;
    if constexpr (NSTRIP % 8 == 0) {
        constexpr int PER = NSTRIP / 8;   // strips of one job per XCD
        const int32_t x = (int32_t)(blockIdx.x & 7), r = (int32_t)(blockIdx.x >> 3);
        j = r / PER;
        strip = x * PER + (r - j * PER);
    } else {
        j = (int32_t)(blockIdx.x / NSTRIP);
        strip = (int32_t)(blockIdx.x - j * NSTRIP);
    }
    j = __builtin_amdgcn_readfirstlane(j);
    const ColJob J = load_col_job(list.job[j]);
    cols_screen_strip<real, N, V, VC, PW, KAHAN, E>(J.g, (const real *)J.mesh, (const real *)J.tw, J.corr, J.st,
                                                    J.row_bits, J.plane_tr, pass, (real *)J.image, strip);
}

// strip width V (columns per block) and columns per thread VC
template <typename real, int N>
struct ColShape {
    using C = typename R2T<real>::t;
    // the strip fills about 70 KB of LDS (16 columns for small N)
    static constexpr int VRAW = (8192 * 8 / (int)sizeof(C)) / N;
    static constexpr int V = VRAW < 1 ? 1 : (VRAW > 16 ? 16 : VRAW);
    static constexpr int NT = N / 16;
    static constexpr int VC0 = (NT * V > 512) ? (NT * V) / 512 : 1;   // at most 512 threads
    static constexpr int VC = VC0 < V ? VC0 : V;                       // (N = 16384: 1024 threads, V = VC = 1)
    static constexpr int THREADS = NT * (V / VC);
};

template <typename real, int N>
hipError_t rows_n(const Geom &g, real *mesh, const real *tw, const uint64_t *tile_bits, const uint64_t *row_bits,
                  hipStream_t s) {
    using C = typename R2T<real>::t;
    constexpr int NT = Shape<N>::NT;
    constexpr int B = NT >= 256 ? 1 : 256 / NT;
    const int64_t nrows = (int64_t)g.Nw * N;
    const size_t lds = size_t(B) * Shape<N>::PADN * sizeof(C);
    static std::once_flag attr_once[kMaxDevices];
    once_per_device(attr_once, [&] {
        (void)hipFuncSetAttribute((const void *)k_fft_rows<real, N, B>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds);
    });
    hipLaunchKernelGGL((k_fft_rows<real, N, B>), dim3((unsigned)(nrows / B)), dim3(NT * B), lds, s, g, mesh, tw,
                       tile_bits, row_bits);
    return hipGetLastError();
}

template <typename real, int N, int PW>
hipError_t cols_n(const Geom &g, real *mesh, const real *tw, hipStream_t s) {
    using CS = ColShape<real, N>;
    const size_t lds = size_t(Shape<N>::PADN) * CS::V * sizeof(typename CS::C);
    static std::once_flag attr_once[kMaxDevices];
    once_per_device(attr_once, [&] {
        (void)hipFuncSetAttribute((const void *)k_fft_cols<real, N, CS::V, CS::VC, PW>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    });
    const int64_t nblk = (int64_t)g.Nw * (N / CS::V);
    hipLaunchKernelGGL((k_fft_cols<real, N, CS::V, CS::VC, PW>), dim3((unsigned)nblk), dim3(CS::THREADS), lds, s,
                       mesh, tw, g.Nw);
    return hipGetLastError();
}

// Column panels of the fused path: PW columns by RB rows make one 128-byte
// line (RB <= 4 and at most 1024 threads per row block); PW >= V.
template <typename real, int N>
struct PanelShape {
    static constexpr int L = 128 / (2 * (int)sizeof(real));   // complex values per 128-byte line
    static constexpr int NT = N / 16;
    static constexpr int RBT = 1024 / NT < 4 ? (1024 / NT < 1 ? 1 : 1024 / NT) : 4;          // threads
    static constexpr int RBL = (160 * 1024) / (Shape<N>::PADN * 2 * (int)sizeof(real));      // LDS
    static constexpr int RBMAX = RBT < RBL ? RBT : (RBL < 1 ? 1 : RBL);
    static constexpr int PW0 = L / RBMAX > 0 ? L / RBMAX : 1;
    static constexpr int PW = PW0 > ColShape<real, N>::V ? PW0 : ColShape<real, N>::V;
    static constexpr int RB = L / PW > 0 ? (L / PW < RBMAX ? L / PW : RBMAX) : 1;
};

template <typename real, int N>
hipError_t rows_panel_n(const Geom &g, const real *in, real *out, const real *tw, const uint64_t *tile_bits,
                        const uint64_t *row_bits, hipStream_t s) {
    using C = typename R2T<real>::t;
    using PS = PanelShape<real, N>;
    const int64_t nrows = (int64_t)g.Nw * N;
    const size_t lds = size_t(PS::RB) * Shape<N>::PADN * sizeof(C);
    static std::once_flag attr_once[kMaxDevices];
    once_per_device(attr_once, [&] {
        (void)hipFuncSetAttribute((const void *)k_fft_rows_panel<real, N, PS::RB, PS::PW>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    });
    // persistent blocks: as many as fit on the device at once
    const int cus = device_cus();
    int per_cu = int((160 * 1024) / lds);
    const int by_threads = 2048 / (PS::NT * PS::RB);
    per_cu = per_cu < by_threads ? per_cu : by_threads;
    per_cu = per_cu < 1 ? 1 : per_cu;
    const int64_t ngroup = nrows / PS::RB;
    const int64_t nblk = (int64_t)cus * per_cu < ngroup ? (int64_t)cus * per_cu : ngroup;
    hipLaunchKernelGGL((k_fft_rows_panel<real, N, PS::RB, PS::PW>), dim3((unsigned)nblk), dim3(PS::NT * PS::RB), lds,
                       s, g, in, out, tw, tile_bits, row_bits);
    return hipGetLastError();
}

template <typename real, int N>
hipError_t cols_screen_n(const Geom &g, const real *mesh, const real *tw, const double *corr, const Stats *st,
                         const uint64_t *row_bits, const int32_t *plane_tr, int pass, real *image, int kahan,
                         hipStream_t s) {
    using CS = ColShape<real, N>;
    constexpr int PW = PanelShape<real, N>::PW;
    // elements per thread: 8 (radix-8 stages, 1024 threads) for the float32
    // strip of 8192, whose block is alone on its CU; 16 otherwise
    constexpr int E = (N == 8192 && sizeof(real) == 4) ? 8 : 16;
    constexpr int THREADS = (N / E) * (CS::V / CS::VC);
    static_assert(THREADS <= 1024, "one block of at most 1024 threads");
    const size_t lds = size_t(E == 8 ? padn8<N>() : Shape<N>::PADN) * CS::V * sizeof(typename CS::C) +
                       size_t(N) * CS::V * sizeof(double);
    static std::once_flag attr_once[kMaxDevices];
    once_per_device(attr_once, [&] {
        (void)hipFuncSetAttribute((const void *)k_fft_cols_screen<real, N, CS::V, CS::VC, PW, false, E>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipFuncSetAttribute((const void *)k_fft_cols_screen<real, N, CS::V, CS::VC, PW, true, E>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    });
    if (kahan)
        hipLaunchKernelGGL((k_fft_cols_screen<real, N, CS::V, CS::VC, PW, true, E>), dim3(N / CS::V), dim3(THREADS),
                           lds, s, g, mesh, tw, corr, st, row_bits, plane_tr, pass, image);
    else
        hipLaunchKernelGGL((k_fft_cols_screen<real, N, CS::V, CS::VC, PW, false, E>), dim3(N / CS::V), dim3(THREADS),
                           lds, s, g, mesh, tw, corr, st, row_bits, plane_tr, pass, image);
    return hipGetLastError();
}

template <typename real, int N>
hipError_t cols_screen_jobs_n(const ColJobList &list, int pass, int kahan, hipStream_t s) {
    using CS = ColShape<real, N>;
    constexpr int PW = PanelShape<real, N>::PW;
    constexpr int E = (N == 8192 && sizeof(real) == 4) ? 8 : 16;   // as the single-plan launch
    constexpr int THREADS = (N / E) * (CS::V / CS::VC);
    const size_t lds = size_t(E == 8 ? padn8<N>() : Shape<N>::PADN) * CS::V * sizeof(typename CS::C) +
                       size_t(N) * CS::V * sizeof(double);
    static std::once_flag attr_once[kMaxDevices];
    once_per_device(attr_once, [&] {
        (void)hipFuncSetAttribute((const void *)k_fft_cols_screen_jobs<real, N, CS::V, CS::VC, PW, false, E>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        (void)hipFuncSetAttribute((const void *)k_fft_cols_screen_jobs<real, N, CS::V, CS::VC, PW, true, E>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    });
    const dim3 grid((unsigned)(list.n * (N / CS::V)));
    if (kahan)
        hipLaunchKernelGGL((k_fft_cols_screen_jobs<real, N, CS::V, CS::VC, PW, true, E>), grid, dim3(THREADS), lds, s,
                           list, pass);
    else
        hipLaunchKernelGGL((k_fft_cols_screen_jobs<real, N, CS::V, CS::VC, PW, false, E>), grid, dim3(THREADS), lds,
                           s, list, pass);
    return hipGetLastError();
}

__global__ void k_put_col_job(ColJob *__restrict__ dst, ColJob v) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *dst = v;
}

}  // namespace

hipError_t launch_put_col_job(ColJob *dst, const ColJob &v, hipStream_t s) {
    hipLaunchKernelGGL(k_put_col_job, dim3(1), dim3(64), 0, s, dst, v);
    return hipGetLastError();
}

template <typename real>
hipError_t launch_fft_cols_screen_jobs(const ColJobList &list, int N, int pass, int kahan, hipStream_t s) {
    if (list.n < 1 || list.n > kMaxGridJobs) return hipErrorInvalidValue;
    switch (N) {
#define CASE(n) \
    case n: return cols_screen_jobs_n<real, n>(list, pass, kahan, s);
        CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096) CASE(8192)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

bool fft_supported(int N, size_t real_bytes) {
    return (N & (N - 1)) == 0 && N >= 64 && (N <= 8192 || (N == 16384 && real_bytes == 4));
}

size_t fused_screen_lds_bytes(int N, size_t real_bytes) {
    const int cbytes = (int)(2 * real_bytes);
    int v = (8192 * 8 / cbytes) / N;
    v = v < 1 ? 1 : (v > 16 ? 16 : v);
    // (the float32 strip of 8192 runs the radix-8 form, padded every 8 elements)
    const int padn = (N == 8192 && real_bytes == 4) ? N + N / 8 : N + N / 16;
    return size_t(padn) * v * cbytes + size_t(N) * v * sizeof(double);
}

template <typename real>
hipError_t launch_fft_rows(const Geom &g, real *mesh, const real *tw, const uint64_t *tile_bits,
                           const uint64_t *row_bits, hipStream_t s) {
    switch (g.N) {
#define CASE(n) \
    case n: return rows_n<real, n>(g, mesh, tw, tile_bits, row_bits, s);
        CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096) CASE(8192)
#undef CASE
        case 16384:   // float32 only: a float64 row does not fit in LDS
            if constexpr (sizeof(real) == 4) return rows_n<real, 16384>(g, mesh, tw, tile_bits, row_bits, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

int fused_panel_width(int N, size_t real_bytes) {
    switch (N) {
#define CASE(n) \
    case n: return real_bytes == 8 ? PanelShape<double, n>::PW : PanelShape<float, n>::PW;
        CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096) CASE(8192)
#undef CASE
        default: return 0;
    }
}

template <typename real>
hipError_t launch_fft_rows_panel(const Geom &g, const real *in, real *out, const real *tw,
                                 const uint64_t *tile_bits, const uint64_t *row_bits, hipStream_t s) {
    switch (g.N) {
#define CASE(n) \
    case n: return rows_panel_n<real, n>(g, in, out, tw, tile_bits, row_bits, s);
        CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096) CASE(8192)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename real>
hipError_t launch_fft_cols(const Geom &g, real *mesh, const real *tw, hipStream_t s) {
    switch (g.N) {
#define CASE(n) \
    case n: return cols_n<real, n, 0>(g, mesh, tw, s);
        CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096) CASE(8192)
#undef CASE
        case 16384:
            if constexpr (sizeof(real) == 4) return cols_n<real, 16384, 0>(g, mesh, tw, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <typename real>
hipError_t launch_fft_cols_panel(const Geom &g, real *row_mesh, const real *tw, hipStream_t s) {
    switch (g.N) {
#define CASE(n) \
    case n: return cols_n<real, n, PanelShape<real, n>::PW>(g, row_mesh, tw, s);
        CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096) CASE(8192)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

template <typename real>
hipError_t launch_fft_cols_screen(const Geom &g, const real *mesh, const real *tw, const double *corr,
                                  const Stats *st, const uint64_t *row_bits, const int32_t *plane_tr, int pass,
                                  real *image, int kahan, hipStream_t s) {
    switch (g.N) {
#define CASE(n) \
    case n: return cols_screen_n<real, n>(g, mesh, tw, corr, st, row_bits, plane_tr, pass, image, kahan, s);
        CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096) CASE(8192)
#undef CASE
        default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_fft_rows<float>(const Geom &, float *, const float *, const uint64_t *, const uint64_t *,
                                           hipStream_t);
template hipError_t launch_fft_rows<double>(const Geom &, double *, const double *, const uint64_t *,
                                            const uint64_t *, hipStream_t);
template hipError_t launch_fft_rows_panel<float>(const Geom &, const float *, float *, const float *,
                                                 const uint64_t *, const uint64_t *, hipStream_t);
template hipError_t launch_fft_rows_panel<double>(const Geom &, const double *, double *, const double *,
                                                  const uint64_t *, const uint64_t *, hipStream_t);
template hipError_t launch_fft_cols<float>(const Geom &, float *, const float *, hipStream_t);
template hipError_t launch_fft_cols<double>(const Geom &, double *, const double *, hipStream_t);
template hipError_t launch_fft_cols_panel<float>(const Geom &, float *, const float *, hipStream_t);
template hipError_t launch_fft_cols_panel<double>(const Geom &, double *, const double *, hipStream_t);
template hipError_t launch_fft_cols_screen<float>(const Geom &, const float *, const float *, const double *,
                                                  const Stats *, const uint64_t *, const int32_t *, int, float *,
                                                  int, hipStream_t);
template hipError_t launch_fft_cols_screen<double>(const Geom &, const double *, const double *, const double *,
                                                   const Stats *, const uint64_t *, const int32_t *, int, double *,
                                                   int, hipStream_t);
template hipError_t launch_fft_cols_screen_jobs<float>(const ColJobList &, int, int, int, hipStream_t);
template hipError_t launch_fft_cols_screen_jobs<double>(const ColJobList &, int, int, int, hipStream_t);

}  // namespace rick
