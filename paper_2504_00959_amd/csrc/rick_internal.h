// Internal declarations shared by the host plan and the HIP kernels of the
// w-stacking imager.  Not part of the public ABI (see include/rick.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <utility>

#include "../../include/rick.h"

namespace rick {

constexpr double kC0 = 299792458.0;      // speed of light, m/s
constexpr int kMaxInlineChan = 32;       // channel scale factors per kernel-argument upload
constexpr int kMaxChan = 1 << 16;        // capacity of the plan's channel scale buffer
constexpr int kMaxTimers = 16;
constexpr int kL1Blocks = 512;           // blocks of the level-1 binning passes (at most)
constexpr int kMaxCoarse = 8192;         // coarse bins of level-1 binning (LDS counters per block)
constexpr int kMaxPlanes = 8192;         // w-planes per plan
constexpr int kTimerRing = 64;         // launches per kernel whose times are kept between reads

constexpr int kMaxDevices = 64;          // device ordinals with their own once-per-device set-up

// Runs f once per device for one call site (the site keeps one flag per
// device ordinal): kernel attributes are per device, so a plan on a second
// GPU sets them there too.  Concurrent first callers on one device wait until
// the first has finished.
template <class F>
inline void once_per_device(std::once_flag (&flags)[kMaxDevices], F &&f) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        f();
        return;
    }
    std::call_once(flags[dev], std::forward<F>(f));
}

// A batch of channel scale factors nu_c / c0, passed by value.
struct ChanScales {
    double s[kMaxInlineChan];
};

// Geometry of one plan, passed by value to kernels.
struct Geom {
    int32_t N;          // grid edge
    int32_t Nw;         // number of w-planes
    int32_t W;          // kernel support
    int32_t h;          // (W - 1) / 2
    int32_t OS;         // oversampling
    int32_t log2OS;
    int32_t T;          // tile edge
    int32_t log2T;
    int32_t nt;         // tiles per axis, N / T
    int32_t nbins;      // Nw * nt * nt
    int32_t CH;         // records per gridding chunk
    int32_t pitch;      // LDS row pitch (floats) of the gridding tile
    int32_t C;          // tiles per coarse-tile edge (level-1 binning)
    int32_t log2C;
    int32_t nct;        // coarse tiles per axis, nt / C
    int32_t n1;         // coarse bins, Nw * nct * nct
    int32_t CHK;        // level-1 records per level-2 chunk
    int32_t occw;       // 64-bit words of tile occupancy per tile row, ceil(nt / 64)
    float gmax2;        // square of the largest tap of the tap table (as the device holds it)
    int32_t cpt1;       // level-1 records in the compact 12-byte format (float32 mode, when it fits)
    int32_t nwf;        // w-fraction bins of a non-separable tap table (1 otherwise)
    int32_t lut3;       // 1: the taps come from a non-separable table T[nwf][OS][OS][W][W]
    double fov;
    double half;        // N * OS / 2
    double w_min;
    double dw;
};

// Device-side counters of one plan (zeroed by rick_reset).
struct Stats {
    unsigned long long n_gridded;
    unsigned long long n_dropped;
    unsigned long long n_records;   // records written by the last rick_grid
    unsigned long long n_heavy;     // bins of the last rick_grid split over several chunks
    double sum_w;
    unsigned long long n_chunks;    // level-2 binning chunks of the last rick_grid
    unsigned long long grid_next;   // gridding work items handed out (zeroed before each gridding launch)
    unsigned long long n_dead;      // level-1 records of the last rick_grid without a finite W V
};

// Binning bookkeeping written by the scan: per bin, exclusive prefix sums of
// the record count (x) and of the number of gridding chunks (y).
struct BinScan {
    int32_t rec;
    int32_t item;
};

// Tile occupancy.  Tile (plane k, tile row ty, tile column tx) holds gridded
// values since the last reset iff bit tx % 64 of tile_bits[(k nt + ty) occw +
// tx / 64] is set; the mesh contents of a clear tile are never read and stand
// for zeros (the gridder writes only tiles that receive records).  Bit ty % 64
// of row_bits[k occw + ty / 64] is set iff any tile of tile row (k, ty) is.
__device__ __forceinline__ bool tile_set(const uint64_t *__restrict__ tile_bits, const Geom &g, int32_t k,
                                         int32_t ty, int32_t tx) {
    return (tile_bits[((int64_t)k * g.nt + ty) * g.occw + (tx >> 6)] >> (tx & 63)) & 1ull;
}
__device__ __forceinline__ bool row_set(const uint64_t *__restrict__ row_bits, const Geom &g, int32_t k,
                                        int32_t ty) {
    return (row_bits[(int64_t)k * g.occw + (ty >> 6)] >> (ty & 63)) & 1ull;
}

// Plane orientation.  A plan with RICK_FLAG_PLANE_ORIENT may store plane k
// transposed -- cell (y, x) of G_k at row x, column y of the stored plane --
// iff plane_tr[k] != 0 (plane_tr NULL: no plane is).  The tile bits, the row
// bits and the row transforms then follow the stored orientation.
__device__ __forceinline__ bool plane_transposed(const int32_t *__restrict__ plane_tr, int32_t k) {
    return plane_tr != nullptr && plane_tr[k] != 0;
}

// sin(pi g) and cos(pi g) for |g| <= 1/2 in float32: sin(pi g) = g P(g^2),
// cos(pi g) = Q(g^2), minimax polynomials fitted on [-1/2, 1/2] (Horner form,
// float32 fma; absolute error below 2.5e-7).
__device__ __forceinline__ void sincospi_half(float g, float &sn, float &cs) {
    const float g2 = g * g;
    float ps = fmaf(g2, 0.07805382838216549f, -0.5985074114168937f);
    ps = fmaf(g2, ps, 2.5501159030870695f);
    ps = fmaf(g2, ps, -5.167712346356822f);
    ps = fmaf(g2, ps, 3.141592653446274f);
    sn = g * ps;
    float pc = fmaf(g2, -0.02468992584886284f, 0.23511454480404714f);
    pc = fmaf(g2, pc, -1.3352479005812146f);
    pc = fmaf(g2, pc, 4.05871189644457f);
    pc = fmaf(g2, pc, -4.934802200064621f);
    cs = fmaf(g2, pc, 1.0f);
}

// Image-plane taper of pixel (q, p): C(l'_p) C(m'_q) for a separable
// kernel (corr holds the 1-D taper), or the 2-D taper corr[q][p] of a
// non-separable table.
__device__ __forceinline__ double taper_at(const Geom &g, const double *__restrict__ corr, int64_t q, int64_t p) {
    return g.lut3 ? corr[q * g.N + p] : corr[p] * corr[q];
}

// Centre of plane k: w_k = w_min + (k + 1/2) dw, in float64, multiply then
// add, each rounded (no contraction), as on the host.
__device__ __forceinline__ double plane_centre(const Geom &g, int32_t k) {
    return __dadd_rn(g.w_min, __dmul_rn((double)k + 0.5, g.dw));
}

// ---- kernel launchers (each returns hipGetLastError() of its launches) ----
hipError_t launch_zero_stats(Stats *st, hipStream_t s);
template <typename real>
hipError_t launch_zero_mesh(real *mesh, int64_t n_real, hipStream_t s);

// Channel scale factors nu_c / c0 into the plan's device buffer (kernel arguments, no copies).
hipError_t launch_set_scales(double *dst, const double *host_scales, int32_t nchan, hipStream_t s);

// Device buffers of the two-level bin-and-sort.
struct BinBufs {
    int32_t *cnt1;        // [n1 * kL1Blocks + 1] per (coarse bin, block) counts, scanned in place
    int32_t *bsum;        // partial sums of the scans
    void *rec1;           // level-1 records: positions, then W V at l1_vis_offset (binsort.hip)
    int32_t *key_chunk0;  // [n1 + 1] first level-2 chunk of each coarse bin
    int32_t *chunk_key;   // [max chunks] coarse bin of each level-2 chunk
    int32_t *cnt2;        // [max chunks][C^2] per (chunk, tile) counts, then record offsets
    uint32_t *vmax2;      // [max chunks][C^2] per (chunk, tile) largest |W V| (float bits; float32 records)
    int32_t *counts;      // [nbins] records per bin
    uint32_t *bin_vmax;   // [nbins] largest |W V| of the bin's records (float bits; float32 records)
    BinScan *scan;        // [nbins + 1]
    int32_t *item_bin;    // gridding work items
    int32_t *heavy_bins;  // bins split over several gridding chunks
    uint32_t *rec_pos;    // records: packed position in the tile
    void *rec_vis;        // records: W V (2 reals)
};
// Upper bound of level-2 chunks for max_records level-1 records.
int32_t bin_max_chunks(const Geom &g, int64_t max_records);
// Exclusive scan of a[0..n) in place, a[n] receiving the total (a holds n + 1
// entries, every partial sum below 2^31); bsum holds flat_scan_partials(n) ints.
int64_t flat_scan_partials(int64_t n);
hipError_t launch_flat_scan(int32_t *a, int64_t n, int32_t *bsum, hipStream_t s);
// Level 1 of bin-and-sort.  phase 0: coarse counts, drop test, weight sum;
// 1: scan of the count table and level-2 chunk list; 2: level-1 records.
template <typename real>
hipError_t launch_bin_level1(const Geom &g, const BinBufs &bb, const double *uvw, const double *scales_dev,
                             const real *vis, const float *weight, int64_t nrow, int32_t nchan, Stats *st, int phase,
                             hipStream_t s);
// Level 2.  phase 0: per (chunk, tile) counts; 1: per-bin totals, scan in
// bin order (gridding items, heavy bins), per (chunk, tile) offsets; 2: records.
template <typename real>
hipError_t launch_bin_level2(const Geom &g, const BinBufs &bb, int64_t nrow, int32_t nchan, Stats *st, int phase,
                             hipStream_t s);
// Gridding: zero the heavy tiles that hold nothing yet (and the margin
// buffers of heavy bins, and the work-item counter), then persistent blocks
// that take (bin, chunk) items from the counter; tiles set in
// tile_bits are added to, others stored; each bin's margins go to its margin
// buffer (grid_margin_len complex values per bin).
// With tapmax non-NULL, lut is a non-separable table T[N_f][OS][OS][W][W]
// in device memory and *tapmax its largest |entry|.
template <typename real>
hipError_t launch_grid(const Geom &g, const BinScan *scan, const int32_t *item_bin, const uint32_t *rec_pos,
                       const real *rec_vis, const real *lut, real *mesh, const uint64_t *tile_bits, real *margin,
                       const uint32_t *bin_vmax, const float *tapmax, Stats *st, const int32_t *plane_tr,
                       int32_t max_items, hipStream_t s);
// One plan's gridding operands as the multi-job gridder reads them (a
// device copy per plan, written by launch_put_grid_job before the launch).
struct GridJob {
    Geom g;
    const BinScan *scan;
    const int32_t *item_bin;
    const uint32_t *rec_pos;
    const void *rec_vis;
    const void *lut;   // separable tap table (real[OS][W])
    void *mesh;
    const uint64_t *tile_bits;
    void *margin;
    const uint32_t *bin_vmax;
    const int32_t *plane_tr;
};
constexpr int kMaxGridJobs = 64;   // jobs of one multi-job gridding launch
struct GridJobList {
    int32_t n;
    const GridJob *job[kMaxGridJobs];
};
hipError_t launch_put_grid_job(GridJob *dst, const GridJob &v, hipStream_t s);
// Gridding of list.n binned jobs in one persistent launch (every job of
// support W, tile edge T, separable table); next is the shared work-item
// counter (zero at launch), lds the largest of the jobs' grid_lds_bytes,
// max_items the sum of the jobs' bounds on work items.
template <typename real>
hipError_t launch_grid_jobs(const GridJobList &list, int W, int T, size_t lds, int64_t max_items,
                            unsigned long long *next, hipStream_t s);
// One fused plan's operands as the multi-job column pass reads them (a
// device copy per plan, written by launch_put_col_job before the launch).
struct ColJob {
    Geom g;
    const void *mesh;   // row transforms, column-panel order
    const void *tw;
    const double *corr;   // the taper the screen divides by
    const Stats *st;
    const uint64_t *row_bits;
    const int32_t *plane_tr;
    void *image;
};
struct ColJobList {
    int32_t n;
    const ColJob *job[kMaxGridJobs];
};
hipError_t launch_put_col_job(ColJob *dst, const ColJob &v, hipStream_t s);
// The fused column pass (pass 0 or 1, as launch_fft_cols_screen) of list.n
// fused plans of grid size N in one launch.
template <typename real>
hipError_t launch_fft_cols_screen_jobs(const ColJobList &list, int N, int pass, int kahan, hipStream_t s);
// Orientation of every plane that holds no set tile yet: transposed iff this
// call's records (with the margins they spill right and down) occupy fewer
// tile columns than tile rows.  Planes already holding tiles keep theirs.
hipError_t launch_orient(const Geom &g, const BinScan *scan, const uint64_t *row_bits, int32_t *plane_tr,
                         hipStream_t s);
// LDS bytes of one gridding block (64-bit accumulators + tap table)
size_t grid_lds_bytes(const Geom &g, size_t real_bytes);
int64_t grid_margin_len(const Geom &g);
template <typename real>
hipError_t launch_zero_heavy(const Geom &g, const int32_t *heavy_bins, Stats *st, const uint64_t *tile_bits,
                             const int32_t *plane_tr, real *mesh, real *margin, hipStream_t s);
// After gridding: add the margins to the neighbouring tiles, set the tile
// bits (records or margins received) and rebuild the row bits.
template <typename real>
hipError_t launch_merge_margins(const Geom &g, const BinScan *scan, const real *margin, uint64_t *tile_bits,
                                uint64_t *row_bits, const int32_t *plane_tr, real *mesh, hipStream_t s);
// The library's static device scratch (rick_grid_static): kStaticScratchBytes
// per device, in a file-scope __device__ array.  static_scratch_setup takes
// its address on the current device, once per device (plan creation calls
// it); static_scratch returns that address for `device`, or an error when
// the setup failed or never ran there.
constexpr size_t kStaticScratchBytes = size_t(256) << 20;
hipError_t static_scratch_setup();
hipError_t static_scratch(int device, void **out);
// Device clock value (constant rate) into *slot once the stream's preceding work is done.
hipError_t launch_stamp(uint64_t *slot, hipStream_t s);
// Clear both occupancy bitmaps (a fill kernel; no memset node in captured work).
hipError_t launch_clear_bits(const Geom &g, uint64_t *tile_bits, uint64_t *row_bits, hipStream_t s);
// Batched centred 2-D inverse FFT, in place, all planes.  Rows of an empty
// tile row are written as zeros; clear tiles are read as zeros.
template <typename real>
hipError_t launch_fft_rows(const Geom &g, real *mesh, const real *twiddle, const uint64_t *tile_bits,
                           const uint64_t *row_bits, hipStream_t s);
template <typename real>
hipError_t launch_fft_cols(const Geom &g, real *mesh, const real *twiddle, hipStream_t s);
// Column pass in place on column-panel order (the row pass's panel output).
template <typename real>
hipError_t launch_fft_cols_panel(const Geom &g, real *row_mesh, const real *tw, hipStream_t s);
// Row pass of the fused path: from the mesh into `out` in column-panel order
// (panels of fused_panel_width(N) columns, each stored row after row).  Rows
// of an empty tile row are not written (the fused column pass reads them as zeros).
template <typename real>
hipError_t launch_fft_rows_panel(const Geom &g, const real *in, real *out, const real *twiddle,
                                 const uint64_t *tile_bits, const uint64_t *row_bits, hipStream_t s);
int fused_panel_width(int N, size_t real_bytes);
// CUs of the current device (queried once per device)
int device_cus();
bool fft_supported(int N, size_t real_bytes);   // N = 16384 in float32 modes only
// Column transform fused with the w-correction, plane sum and normalisation.
size_t fused_screen_lds_bytes(int N, size_t real_bytes);
// pass 0: the planes stored as they are (all planes without plane_tr), the
// image written; pass 1: the planes stored transposed, added to the image
// transposed.  Planes without a set tile are skipped.
template <typename real>
hipError_t launch_fft_cols_screen(const Geom &g, const real *mesh, const real *tw, const double *corr,
                                  const Stats *st, const uint64_t *row_bits, const int32_t *plane_tr, int pass,
                                  real *image, int kahan, hipStream_t s);
// Phase screen + plane sum + normalisation.
template <typename real>
hipError_t launch_wscreen(const Geom &g, const real *mesh, const double *corr,
                          const Stats *st, real *image, int kahan, hipStream_t s);

// ---- learned gridding kernel (learned.hip) ----
// Scratch of the 2-D taper of a non-separable table: A [M][M] (the table
// averaged over w-fraction bins, M = OS W offsets per axis), Ec/Es [M][N]
// (cos/sin of 2 pi d l'), Uc/Us [M][N] (row-pass results).
struct TaperBufs {
    double *A, *Ec, *Es, *Uc, *Us;
};
int mlp_param_count();
template <typename real>
hipError_t launch_table_install(const float *src, real *dst, int64_t n, float *tapmax, hipStream_t s);
template <typename real>
hipError_t launch_taper2d(const Geom &g, const real *T, const TaperBufs &tb, double *C, hipStream_t s);
template <typename real>
hipError_t launch_taper2d_adjoint(const Geom &g, const double *dC, const TaperBufs &tb, double *dT, hipStream_t s);
template <typename real>
hipError_t launch_image_loss(const Geom &g, const real *I, const double *D, const double *taper, double *dA,
                             double *dC, double *sums, hipStream_t s);
template <typename real>
hipError_t launch_grad_screen(const Geom &g, const double *dA, const Stats *st, real *mesh, hipStream_t s);
template <typename real>
hipError_t launch_table_grad(const Geom &g, const double *uvw, const double *scales, const real *vis,
                             const float *weight, int64_t nrow, int32_t nchan, const real *mesh, double *dT,
                             int64_t n_table, hipStream_t s);
hipError_t launch_mlp_table(const float *theta, int W, int OS, int nwf, float *T, float *rowsum, hipStream_t s);
hipError_t launch_mlp_backward(const float *theta, int W, int OS, int nwf, const float *T, const double *dT,
                               float *dtheta, hipStream_t s);
hipError_t launch_adam(float *theta, const float *grad, float *m, float *v, int n, int step, float lr, float b1,
                       float b2, float eps, hipStream_t s);
template <typename real>
hipError_t launch_dft(const Geom &g, const double *uvw, const double *scales, const real *vis, const float *weight,
                      int64_t nrow, int32_t nchan, int q0, int p0, int nq, int np, double *out, double *wsum,
                      hipStream_t s);
template <typename real>
hipError_t launch_separable_table(const real *g, int nwf, int OS, int W, float *out, hipStream_t s);
hipError_t launch_table_residual(const float *T, const float *R, int64_t n, double *dT, double *sums, hipStream_t s);
// Every tile bit and row bit of every plane set (degrid.hip).
hipError_t launch_fill_bits(const Geom &g, uint64_t *tile_bits, uint64_t *row_bits, hipStream_t s);

// Prediction: conj(P_k) of the model image into every plane of the mesh, and
// every tile bit and row bit set (the FFT then reads whole planes).
template <typename real>
hipError_t launch_predict_screen(const Geom &g, const real *model, const double *corr, real *mesh,
                                 uint64_t *tile_bits, uint64_t *row_bits, hipStream_t s);

// Prediction at fixed positions: sort keys and values of every visibility,
// their stable LSD radix sort on bits [begin_bit, end_bit) (temp == nullptr
// queries temp_bytes; keys_in and vals_in are overwritten, being the other
// half of the ping-pong; n < 2^31), and interpolation in sorted order.
template <typename real>
hipError_t launch_order_keys(const Geom &g, const double *uvw, const double *scales, int64_t nrow, int32_t nchan,
                             int32_t panel, uint64_t *keys, uint64_t *vals, hipStream_t s);
hipError_t sort_order(void *temp, size_t &temp_bytes, uint64_t *keys_in, uint64_t *keys_out, uint64_t *vals_in,
                      uint64_t *vals_out, int64_t n, int begin_bit, int end_bit, hipStream_t s);
template <typename real>
hipError_t launch_degrid_sorted(const Geom &g, const uint64_t *keys, const uint64_t *vals, int64_t nvis,
                                const real *lut, const real *mesh, int32_t panel, real *out, hipStream_t s);

// Prediction: interpolate visibilities from planes holding conj(H_k).
// panel = 0: planes in row order (the mesh); panel = PW: column-panel order
// (the fused plan's row_mesh), element (k, j, i) at k N^2 + (i / PW) N PW + j PW + i % PW.
template <typename real>
hipError_t launch_degrid(const Geom &g, const double *uvw, const double *scales, int64_t nrow, int32_t nchan,
                         const real *lut, const real *mesh, int32_t panel, real *out, hipStream_t s);

}  // namespace rick
