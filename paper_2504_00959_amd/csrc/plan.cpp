// Host side of the w-stacking imager: argument validation, float64 tables,
// one-time device allocation, and the C ABI entry points of include/rick.h.
//
// Everything the device needs is allocated in rick_plan; the per-image
// calls only queue kernels on the caller's stream (the paper's GPU gridder
// lost most of its time to per-sector hipMalloc/hipFree, Sec. 4.2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "rick_internal.h"

using namespace rick;

namespace {

constexpr uint32_t kMagic = 0x5249434bu;  // "RICK"
constexpr uint32_t kDead = 0xdeadbeefu;

thread_local char g_err[512] = "";

rick_status fail(rick_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

rick_status hip_fail(hipError_t e, const char *what) {
    return fail(RICK_E_HIP, "%s: %s", what, hipGetErrorString(e));
}

bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int ilog2(int64_t x) {
    int r = 0;
    while ((int64_t(1) << r) < x) ++r;
    return r;
}

// Modified Bessel function I0 from its power series sum ((x/2)^k / k!)^2.
double bessel_i0(double x) {
    const double q = 0.25 * x * x;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / (double(k) * double(k));
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

// Continuous kernel g(d), zero for |d| >= W/2 (Sec. 2.1: Gaussian or Kaiser-Bessel).
double kernel_at(double d, int W, int kind, double param) {
    const double half = 0.5 * W;
    if (!(std::fabs(d) < half)) return 0.0;
    if (kind == RICK_KERNEL_GAUSSIAN) {
        return std::exp(-d * d / (2.0 * param * param));
    }
    const double a = 1.0 - (2.0 * d / W) * (2.0 * d / W);
    return bessel_i0(param * std::sqrt(a > 0.0 ? a : 0.0)) / bessel_i0(param);
}

double default_param(int W, int kind) {
    if (kind == RICK_KERNEL_GAUSSIAN) return (0.5 * W) / std::sqrt(2.0 * std::log(1000.0));
    // Beatty, Nishimura & Pauly (2005), oversampling ratio 2
    const double alpha = 2.0;
    const double x = (W / alpha) * (W / alpha) * (alpha - 0.5) * (alpha - 0.5) - 0.8;
    return x > 0.0 ? M_PI * std::sqrt(x) : 0.0;
}

}  // namespace

struct rick_plan_s {
    uint32_t magic;
    rick_plan_desc d;
    Geom g;
    bool fp64;
    int state;               // 0 empty, 1 gridded, 2 transformed, 3 predicted planes (conj(H_k))
    double du, dl;
    int64_t max_items;       // gridding launch bound per visibility (items <= nbins + 4 nvis / CH)
    size_t real_bytes;
    // device buffers
    void *mesh = nullptr;
    size_t mesh_bytes = 0;
    void *row_mesh = nullptr;   // fused: row transforms in column-panel order
    uint64_t *tile_bits = nullptr;   // tiles written since the reset, [N_w][nt][occw] words
    uint64_t *row_bits = nullptr;    // tile rows with a written tile, [N_w][occw] words
    int32_t *plane_tr = nullptr;     // RICK_FLAG_PLANE_ORIENT: per plane, 1 if stored transposed
    void *margin = nullptr;          // per bin: the accumulator margins right of and below the tile
    int32_t panel = 0;
    void *lut = nullptr;
    void *twiddle = nullptr;
    double *corr = nullptr;
    double *scales = nullptr;
    Stats *stats = nullptr;
    GridJob *job_dev = nullptr;   // this plan's operands for the multi-job gridder
    ColJob *coljob_dev = nullptr;   // ... and for the multi-job column pass
    int32_t *counts = nullptr;
    BinScan *scan = nullptr;
    int32_t *block_sums = nullptr;
    int32_t *cnt1 = nullptr;
    void *rec1 = nullptr;
    int32_t *key_chunk0 = nullptr;
    int32_t *chunk_key = nullptr;
    int32_t *cnt2 = nullptr;
    uint32_t *vmax2 = nullptr;
    uint32_t *bin_vmax = nullptr;
    int32_t max_chunks = 0;
    int32_t *item_bin = nullptr;
    int32_t *heavy_bins = nullptr;
    uint32_t *rec_pos = nullptr;
    void *rec_vis = nullptr;
    int64_t rec_cap = 0;
    // non-separable table (RICK_KERNEL_USER_LUT): lut holds T[N_f][OS][OS][W][W],
    // corr2 its 2-D taper [N][N], tapmax its largest |entry|
    bool lut3 = false;
    bool lut_ready = false;
    size_t lut_bytes = 0;
    float *tapmax = nullptr;
    double *corr2 = nullptr;
    TaperBufs taper_bufs{};
    double *dft_wsum = nullptr;   // weight sum of the last rick_dft_image
    std::vector<double> w_k_host;
    // host copies of tables (for tests and info)
    std::vector<double> lut_host, corr_host;
    // timing: per kernel slot a ring of (start, stop) event pairs
    hipEvent_t ev[kMaxTimers][2 * kTimerRing] = {};
    const char *ev_name[kMaxTimers] = {};
    int64_t ev_calls[kMaxTimers] = {};
    bool timing = false;
    bool fused = false;      // column transform fused into rick_wstack_image
};

namespace {

bool plan_ok(const rick_plan_t *p) { return p != nullptr && p->magic == kMagic; }

// The image-plane taper the screens divide by: the 1-D taper of the
// separable kernel, or the 2-D taper [N][N] of a user table.
const double *taper_of(const rick_plan_t *p) { return p->lut3 ? p->corr2 : p->corr; }

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

void free_all(rick_plan_t *p) {
    void *bufs[] = {p->mesh,      p->row_mesh,  p->tile_bits,  p->row_bits,  p->plane_tr, p->margin, p->lut, p->twiddle,
                    p->corr,
                    p->scales,
                    p->stats,     p->counts,     p->scan,      p->block_sums, p->cnt1,  p->rec1,
                    p->key_chunk0, p->chunk_key, p->cnt2,   p->vmax2,    p->bin_vmax, p->item_bin, p->heavy_bins,
                    p->rec_pos,   p->rec_vis,   p->dft_wsum,  p->tapmax,    p->corr2,     p->taper_bufs.A,
                    p->job_dev,   p->coljob_dev};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    for (int i = 0; i < kMaxTimers; ++i)
        for (int j = 0; j < 2 * kTimerRing; ++j)
            if (p->ev[i][j]) (void)hipEventDestroy(p->ev[i][j]);
}

rick_status validate(const rick_plan_desc *d) {
    if (!d) return fail(RICK_E_INVALID_ARG, "desc is NULL");
    if (!is_pow2(d->grid_n) || d->grid_n < 64 || d->grid_n > 16384)
        return fail(RICK_E_INVALID_ARG, "grid_n=%d: must be a power of two in [64, 16384]", d->grid_n);
    if (d->n_wplanes < 1 || d->n_wplanes > kMaxPlanes)
        return fail(RICK_E_INVALID_ARG, "n_wplanes=%d: must be in [1, %d]", d->n_wplanes, kMaxPlanes);
    if (d->support < 1 || d->support > 15 || (d->support & 1) == 0)
        return fail(RICK_E_INVALID_ARG, "support=%d: must be odd in [1, 15]", d->support);
    if (!is_pow2(d->oversample) || d->oversample > 256)
        return fail(RICK_E_INVALID_ARG, "oversample=%d: must be a power of two in [1, 256]", d->oversample);
    if (d->kernel != RICK_KERNEL_GAUSSIAN && d->kernel != RICK_KERNEL_KAISER_BESSEL &&
        d->kernel != RICK_KERNEL_USER_LUT)
        return fail(RICK_E_INVALID_ARG, "kernel=%d: unknown", d->kernel);
    if (d->kernel == RICK_KERNEL_USER_LUT && (!is_pow2(d->lut_wbins) || d->lut_wbins > 8))
        return fail(RICK_E_INVALID_ARG, "lut_wbins=%d: must be 1, 2, 4 or 8 with RICK_KERNEL_USER_LUT", d->lut_wbins);
    if (d->precision < RICK_PREC_FP32 || d->precision > RICK_PREC_FP64)
        return fail(RICK_E_INVALID_ARG, "precision=%d: unknown", d->precision);
    if (!std::isfinite(d->kernel_param))
        return fail(RICK_E_INVALID_ARG, "kernel_param is not finite");
    if (!(d->fov_rad > 0.0) || !(d->fov_rad * d->fov_rad / 2.0 < 1.0))
        return fail(RICK_E_INVALID_ARG, "fov_rad=%g: need 0 < fov and fov^2/2 < 1", d->fov_rad);
    if (!std::isfinite(d->w_min) || !std::isfinite(d->w_max) || !(d->w_max > d->w_min))
        return fail(RICK_E_INVALID_ARG, "w range [%g, %g]: need finite w_min < w_max", d->w_min, d->w_max);
    if (d->max_vis < 0 || d->max_vis >= (int64_t(1) << 29))
        return fail(RICK_E_INVALID_ARG, "max_vis=%lld: must be in [0, 2^29)", (long long)d->max_vis);
    if (d->device < 0) return fail(RICK_E_INVALID_ARG, "device=%d", d->device);
    if (d->flags & ~int32_t(RICK_FLAG_TIMING | RICK_FLAG_FUSED_SCREEN | RICK_FLAG_PLANE_ORIENT))
        return fail(RICK_E_INVALID_ARG, "flags=%d: unknown bits", d->flags);
    if ((d->flags & RICK_FLAG_PLANE_ORIENT) && !(d->flags & RICK_FLAG_FUSED_SCREEN))
        return fail(RICK_E_INVALID_ARG, "RICK_FLAG_PLANE_ORIENT needs RICK_FLAG_FUSED_SCREEN");
    if (d->tile != 0) {
        if (!is_pow2(d->tile) || d->tile < 16 || d->tile > 64 || d->tile < d->support || d->tile > d->grid_n)
            return fail(RICK_E_INVALID_ARG, "tile=%d: power of two in [16, 64], >= support, <= grid_n", d->tile);
    }
    if (d->chunk < 0 || d->chunk > (1 << 24)) return fail(RICK_E_INVALID_ARG, "chunk=%d", d->chunk);
    return RICK_OK;
}

// Timer slots: per kernel a ring of (start, stop) event pairs, so that the
// mean over every launch since the last rick_plan_info can be reported.
void timer_begin(rick_plan_t *p, int slot, const char *name, hipStream_t s) {
    if (!p->timing) return;
    p->ev_name[slot] = name;
    const int r = int(p->ev_calls[slot] % kTimerRing);
    (void)hipEventRecord(p->ev[slot][2 * r], s);
}
void timer_end(rick_plan_t *p, int slot, hipStream_t s) {
    if (!p->timing) return;
    const int r = int(p->ev_calls[slot] % kTimerRing);
    (void)hipEventRecord(p->ev[slot][2 * r + 1], s);
    ++p->ev_calls[slot];
}

enum TimerSlot {
    T_COUNT = 0, T_SCAN, T_SCATTER, T_ZERO_HEAVY, T_GRID, T_FFT_ROWS, T_FFT_COLS, T_SCREEN, T_RESET,
    T_FINE_COUNT, T_FINE_SCAN, T_FINE_SCATTER, T_MARK, T_PRED_SCREEN, T_PRED_FFT, T_DEGRID
};

}  // namespace

extern "C" {

const char *rick_status_str(rick_status s) {
    switch (s) {
        case RICK_OK: return "success";
        case RICK_E_INVALID_ARG: return "invalid argument";
        case RICK_E_NO_DEVICE: return "no usable HIP device";
        case RICK_E_OOM: return "not enough device memory for the plan";
        case RICK_E_HIP: return "HIP runtime error";
        case RICK_E_CAPACITY: return "more visibilities than the plan's max_vis";
        case RICK_E_BAD_PLAN: return "invalid plan handle";
        case RICK_E_STATE: return "call out of order for the plan's state";
        case RICK_E_UNSUPPORTED: return "unsupported configuration";
        default: return "unknown status";
    }
}

const char *rick_last_error(void) { return g_err; }

rick_status rick_plan(const rick_plan_desc *d, rick_plan_t **out) {
    if (!out) return fail(RICK_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    rick_status st = validate(d);
    if (st != RICK_OK) return st;
    if (!fft_supported(d->grid_n, d->precision == RICK_PREC_FP64 ? 8 : 4))
        return fail(RICK_E_UNSUPPORTED, "no FFT kernel for N=%d in this precision", d->grid_n);
    if ((d->flags & RICK_FLAG_FUSED_SCREEN) &&
        fused_screen_lds_bytes(d->grid_n, d->precision == RICK_PREC_FP64 ? 8 : 4) > size_t(160) * 1024)
        return fail(RICK_E_UNSUPPORTED, "fused screen: a column strip of N=%d does not fit in LDS", d->grid_n);
    if ((d->flags & RICK_FLAG_PLANE_ORIENT) && d->kernel == RICK_KERNEL_USER_LUT)
        return fail(RICK_E_UNSUPPORTED, "transposed planes with a user table are not built");

    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0)
        return fail(RICK_E_NO_DEVICE, "no HIP device available");
    if (d->device >= ndev) return fail(RICK_E_NO_DEVICE, "device %d of %d", d->device, ndev);

    rick_plan_t *p = new (std::nothrow) rick_plan_t();
    if (!p) return fail(RICK_E_OOM, "host allocation");
    p->magic = kMagic;
    p->d = *d;
    p->fp64 = d->precision == RICK_PREC_FP64;
    p->real_bytes = p->fp64 ? 8 : 4;
    p->timing = (d->flags & RICK_FLAG_TIMING) != 0;
    p->fused = (d->flags & RICK_FLAG_FUSED_SCREEN) != 0;

    Geom &g = p->g;
    g.N = d->grid_n;
    g.Nw = d->n_wplanes;
    g.W = d->support;
    g.h = (d->support - 1) / 2;
    g.OS = d->oversample;
    g.log2OS = ilog2(d->oversample);
    g.T = d->tile ? d->tile : (g.N >= 64 ? 64 : g.N);
    if (g.T < g.W) g.T = 16 >= g.W ? 16 : 32;
    g.log2T = ilog2(g.T);
    g.nt = g.N / g.T;
    g.occw = (g.nt + 63) / 64;
    const int64_t nbins64 = int64_t(g.Nw) * g.nt * g.nt;
    if (nbins64 >= (int64_t(1) << 26)) {
        delete p;
        return fail(RICK_E_INVALID_ARG, "too many (plane, tile) bins: %lld", (long long)nbins64);
    }
    g.nbins = int32_t(nbins64);
    // records per gridding work item by default (of 4096 ... 32768, 16384 was
    // fastest for 4096^2 x 64 planes and within 1 % of the best for 8192^2 x 128)
    g.CH = d->chunk ? d->chunk : 16384;
    {
        // level-1 binning: coarse tiles of C x C tiles, the smallest C (a
        // power of two) that leaves at most kMaxCoarse coarse bins
        int C = 1;
        while (C < g.nt && int64_t(g.Nw) * (g.nt / C) * (g.nt / C) > kMaxCoarse) C *= 2;
        g.C = C;
        g.log2C = ilog2(C);
        g.nct = g.nt / C;
        g.n1 = g.Nw * g.nct * g.nct;
        g.CHK = 16 * C * C > 16384 ? 16 * C * C : 16384;
        // (a level-2 block keeps three C^2 tables in LDS)
        if (g.n1 > kMaxCoarse || int64_t(C) * C > 4096) {
            delete p;
            return fail(RICK_E_INVALID_ARG, "no coarse binning fits %d planes of %d x %d tiles", g.Nw, g.nt, g.nt);
        }
    }
    {
        // LDS row pitch: at least the tile plus its W - 1 margin, congruent to W
        // mod 32, so a W x W footprint spreads over distinct banks (one tap per
        // lane, see grid.hip)
        int pitch = g.T + g.W - 1;
        while ((pitch - g.W) % 32 != 0) ++pitch;
        g.pitch = pitch;
    }
    {
        // the gridding block keeps its (T + W - 1) x pitch 64-bit accumulators and the tap table in LDS
        const size_t lds = grid_lds_bytes(g, p->fp64 ? 8 : 4);
        if (lds > size_t(160) * 1024 - 64) {   // (64 bytes stay for the kernel's static LDS)
            delete p;
            return fail(RICK_E_INVALID_ARG, "tile=%d with support %d, oversample %d needs %zu B of LDS (> 160 KB)",
                        g.T, g.W, g.OS, lds);
        }
    }
    // a non-separable table: the w-fraction bin rides in spare bits of the
    // full-format level-1 records and of the gridding records
    p->lut3 = d->kernel == RICK_KERNEL_USER_LUT;
    g.lut3 = p->lut3 ? 1 : 0;
    g.nwf = p->lut3 ? d->lut_wbins : 1;
    // compact level-1 records: origin in the coarse tile and sub-cell in one word
    g.cpt1 = (!p->fp64 && !p->lut3 && 2 * (g.log2C + g.log2T + g.log2OS) <= 32) ? 1 : 0;
    g.fov = d->fov_rad;
    g.half = double(int64_t(g.N) * g.OS) / 2.0;
    g.w_min = d->w_min;
    g.dw = (d->w_max - d->w_min) / double(g.Nw);
    p->du = 1.0 / d->fov_rad;
    p->dl = d->fov_rad / g.N;
    p->rec_cap = d->max_vis;   // one record per visibility (the tile of its footprint origin)
    p->max_items = g.nbins + (p->rec_cap + g.CH - 1) / g.CH;

    // ---- float64 tables on the host ----
    // (a plan with a user table keeps a Gaussian separable table here, which
    // no kernel of that plan reads: its taps and taper come with the table)
    const int kind = p->lut3 ? RICK_KERNEL_GAUSSIAN : d->kernel;
    const double param = (d->kernel_param > 0 && !p->lut3) ? d->kernel_param : default_param(g.W, kind);
    if (!(param > 0.0) && kind == RICK_KERNEL_GAUSSIAN) {
        delete p;
        return fail(RICK_E_INVALID_ARG, "Gaussian width must be positive");
    }
    p->lut_host.assign(size_t(g.OS) * g.W, 0.0);
    for (int r = 0; r < g.OS; ++r) {
        const int s = r - g.OS / 2;
        double sum = 0.0;
        for (int t = 0; t < g.W; ++t) {
            const double dist = double(t - g.h) - double(s) / g.OS;
            p->lut_host[size_t(r) * g.W + t] = kernel_at(dist, g.W, kind, param);
            sum += p->lut_host[size_t(r) * g.W + t];
        }
        for (int t = 0; t < g.W; ++t) p->lut_host[size_t(r) * g.W + t] /= sum;
    }
    {
        // largest tap as the device holds it; its square bounds |g_y g_x|
        double gm = 0.0;
        for (double v : p->lut_host) gm = std::max(gm, p->fp64 ? v : double(float(v)));
        g.gmax2 = float(gm * gm * (1.0 + 1e-6));
    }
    // taper C(l') = (1/OS) sum_s sum_t g_s[t] cos(2 pi (t - h - s/OS) l'), l' = (p - N/2)/N
    p->corr_host.assign(g.N, 0.0);
    for (int px = 0; px < g.N; ++px) {
        const double lp = double(px - g.N / 2) / g.N;
        double c = 0.0;
        for (int r = 0; r < g.OS; ++r) {
            const int s = r - g.OS / 2;
            for (int t = 0; t < g.W; ++t) {
                const double dist = double(t - g.h) - double(s) / g.OS;
                c += p->lut_host[size_t(r) * g.W + t] * std::cos(2.0 * M_PI * dist * lp);
            }
        }
        p->corr_host[px] = c / g.OS;
    }

    // ---- device allocation, once ----
    DeviceGuard guard(d->device);
    // address of the library's static scratch on this device, taken once per
    // device; a failure is kept and reported by rick_grid_static, the only
    // call that uses the scratch
    (void)static_scratch_setup();
    const size_t rb = p->real_bytes;
    p->mesh_bytes = size_t(g.Nw) * g.N * g.N * 2 * rb;
    const size_t sz_lut = p->lut3 ? size_t(g.nwf) * g.OS * g.OS * g.W * g.W * rb : size_t(g.OS) * g.W * rb;
    const size_t taper_m = size_t(g.OS) * g.W;
    const size_t sz_taper = p->lut3 ? (taper_m * taper_m + 4 * taper_m * g.N) * sizeof(double) : 0;
    const size_t sz_corr2 = p->lut3 ? size_t(g.N) * g.N * sizeof(double) : 0;
    p->lut_bytes = sz_lut;
    const size_t sz_tw = size_t(g.N) * 2 * rb;
    const size_t sz_counts = size_t(g.nbins + 1) * sizeof(int32_t);
    const size_t sz_items = size_t(p->max_items + 1) * sizeof(int32_t);
    const size_t sz_heavy = size_t(p->rec_cap / (g.CH + 1) + 2) * sizeof(int32_t);
    const size_t sz_scan = size_t(g.nbins + 1) * sizeof(BinScan);
    const size_t n_cnt1 = size_t(g.n1) * kL1Blocks + 1;
    const size_t n_scanned = n_cnt1 > size_t(g.nbins) + 1 ? n_cnt1 : size_t(g.nbins) + 1;
    const size_t sz_bsum = (n_scanned + 2047) / 2048 * 2 * sizeof(int32_t) + 64;
    const size_t sz_cnt1 = n_cnt1 * sizeof(int32_t);
    // level-1 records: a footprint touches at most four coarse bins
    const size_t sz_rec1 = size_t(p->rec_cap) * (8 + 2 * rb) + 256;   // positions, then W V (256-byte aligned)
    p->max_chunks = bin_max_chunks(g, p->rec_cap);
    const size_t sz_kc0 = size_t(g.n1 + 1) * sizeof(int32_t);
    const size_t sz_ckey = size_t(p->max_chunks) * sizeof(int32_t);
    const size_t sz_cnt2 = size_t(p->max_chunks) * g.C * g.C * sizeof(int32_t);
    const size_t sz_pos = size_t(p->rec_cap) * sizeof(uint32_t);
    const size_t sz_rvis = size_t(p->rec_cap) * 2 * rb;
    const size_t sz_rbits = size_t(g.Nw) * g.occw * sizeof(uint64_t);
    const size_t sz_tbits = sz_rbits * g.nt;
    const size_t sz_margin = size_t(g.nbins) * size_t(grid_margin_len(g)) * 2 * rb + 64;
    const size_t total = p->mesh_bytes * (p->fused ? 2 : 1) + sz_lut + sz_taper + sz_corr2 + sz_tw + size_t(g.N) * 8 + size_t(g.Nw) * 8 +
                         size_t(kMaxChan) * 8 + sizeof(Stats) + sz_counts + sz_scan + sz_bsum + sz_cnt1 + sz_rec1 + sz_kc0 + sz_ckey + 2 * sz_cnt2 + sz_counts + sz_items + sz_heavy + sz_pos + sz_rvis + sz_tbits + sz_rbits + sz_margin;
    size_t free_b = 0, total_b = 0;
    hipError_t e = hipMemGetInfo(&free_b, &total_b);
    if (e != hipSuccess) {
        delete p;
        return hip_fail(e, "hipMemGetInfo");
    }
    if (total + (size_t(256) << 20) > free_b) {
        delete p;
        return fail(RICK_E_OOM, "plan needs %.3f GB, device has %.3f GB free", total / 1e9, free_b / 1e9);
    }
#define ALLOC(ptr, bytes)                                        \
    do {                                                         \
        e = hipMalloc((void **)&(ptr), (bytes) > 256 ? (bytes) : 256); \
        if (e != hipSuccess) {                                   \
            free_all(p);                                         \
            delete p;                                            \
            return e == hipErrorOutOfMemory ? fail(RICK_E_OOM, "hipMalloc %zu bytes", size_t(bytes)) \
                                            : hip_fail(e, "hipMalloc");                               \
        }                                                        \
    } while (0)
    ALLOC(p->mesh, p->mesh_bytes);
    if (p->fused) {
        p->panel = fused_panel_width(g.N, rb);
        ALLOC(p->row_mesh, p->mesh_bytes);
    }
    ALLOC(p->tile_bits, sz_tbits);
    ALLOC(p->row_bits, sz_rbits);
    if (d->flags & RICK_FLAG_PLANE_ORIENT) ALLOC(p->plane_tr, size_t(g.Nw) * sizeof(int32_t));
    ALLOC(p->margin, sz_margin);
    ALLOC(p->lut, sz_lut);
    ALLOC(p->twiddle, sz_tw);
    ALLOC(p->corr, size_t(g.N) * 8);
    ALLOC(p->scales, size_t(kMaxChan) * 8);
    ALLOC(p->stats, sizeof(Stats));
    ALLOC(p->job_dev, sizeof(GridJob));
    ALLOC(p->coljob_dev, sizeof(ColJob));
    ALLOC(p->counts, sz_counts);
    ALLOC(p->scan, sz_scan);
    ALLOC(p->block_sums, sz_bsum);
    ALLOC(p->cnt1, sz_cnt1);
    ALLOC(p->rec1, sz_rec1);
    ALLOC(p->key_chunk0, sz_kc0);
    ALLOC(p->chunk_key, sz_ckey);
    ALLOC(p->cnt2, sz_cnt2);
    ALLOC(p->vmax2, sz_cnt2);
    ALLOC(p->bin_vmax, sz_counts);
    ALLOC(p->item_bin, sz_items);
    ALLOC(p->heavy_bins, sz_heavy);
    ALLOC(p->rec_pos, sz_pos);
    ALLOC(p->rec_vis, sz_rvis);
    ALLOC(p->dft_wsum, sizeof(double));
    if (p->lut3) {
        ALLOC(p->tapmax, sizeof(float));
        ALLOC(p->corr2, sz_corr2);
        double *tb = nullptr;
        ALLOC(tb, sz_taper);
        p->taper_bufs.A = tb;
        p->taper_bufs.Ec = tb + taper_m * taper_m;
        p->taper_bufs.Es = p->taper_bufs.Ec + taper_m * g.N;
        p->taper_bufs.Uc = p->taper_bufs.Es + taper_m * g.N;
        p->taper_bufs.Us = p->taper_bufs.Uc + taper_m * g.N;
    }
#undef ALLOC

    // tables: tap LUT and twiddles rounded to the plan's real type
    std::vector<double> tw(size_t(g.N) * 2);
    for (int i = 0; i < g.N; ++i) {
        // exp(+2 pi i i / N), evaluated in long double and rounded
        const long double a = 2.0L * M_PI * (long double)i / (long double)g.N;
        tw[2 * i] = (double)std::cos(a);
        tw[2 * i + 1] = (double)std::sin(a);
    }
    const size_t sz_lut_sep = size_t(g.OS) * g.W * rb;   // the separable table's bytes
    std::vector<char> lut_dev(sz_lut_sep), tw_dev(sz_tw);
    if (p->fp64) {
        std::memcpy(lut_dev.data(), p->lut_host.data(), sz_lut_sep);
        std::memcpy(tw_dev.data(), tw.data(), sz_tw);
    } else {
        float *lf = reinterpret_cast<float *>(lut_dev.data());
        for (size_t i = 0; i < p->lut_host.size(); ++i) lf[i] = float(p->lut_host[i]);
        float *tf = reinterpret_cast<float *>(tw_dev.data());
        for (size_t i = 0; i < tw.size(); ++i) tf[i] = float(tw[i]);
    }
    struct Cp { void *dst; const void *src; size_t n; } cps[] = {
        {p->twiddle, tw_dev.data(), sz_tw},
        {p->corr, p->corr_host.data(), size_t(g.N) * 8},
        {p->lut, lut_dev.data(), sz_lut_sep},   // (a user table arrives with rick_plan_set_lut)
    };
    for (auto &c : cps) {
        if (c.dst == p->lut && p->lut3) continue;
        e = hipMemcpy(c.dst, c.src, c.n, hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            free_all(p);
            delete p;
            return hip_fail(e, "hipMemcpy tables");
        }
    }
    e = hipMemset(p->stats, 0, sizeof(Stats));
    if (e == hipSuccess) e = hipMemset(p->mesh, 0, p->mesh_bytes);
    if (e == hipSuccess) e = hipMemset(p->tile_bits, 0, sz_tbits);
    if (e == hipSuccess) e = hipMemset(p->row_bits, 0, sz_rbits);
    if (e == hipSuccess && p->plane_tr) e = hipMemset(p->plane_tr, 0, size_t(g.Nw) * sizeof(int32_t));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_all(p);
        delete p;
        return hip_fail(e, "plan initialisation");
    }
    if (p->timing) {
        for (int i = 0; i < kMaxTimers; ++i) {
            for (int j = 0; j < 2 * kTimerRing; ++j) {
                e = hipEventCreate(&p->ev[i][j]);
                if (e != hipSuccess) {
                    free_all(p);
                    delete p;
                    return hip_fail(e, "hipEventCreate");
                }
            }
        }
    }
    p->state = 0;
    *out = p;
    return RICK_OK;
}

rick_status rick_plan_destroy(rick_plan_t *p) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    DeviceGuard guard(p->d.device);
    free_all(p);
    p->magic = kDead;
    delete p;
    return RICK_OK;
}

rick_status rick_reset(rick_plan_t *p, void *stream) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    DeviceGuard guard(p->d.device);
    hipStream_t s = (hipStream_t)stream;
    timer_begin(p, T_RESET, "reset", s);
    hipError_t e = launch_zero_stats(p->stats, s);
    if (e == hipSuccess) e = launch_clear_bits(p->g, p->tile_bits, p->row_bits, s);
    timer_end(p, T_RESET, s);
    if (e != hipSuccess) return hip_fail(e, "reset");
    p->state = 0;
    return RICK_OK;
}

}  // extern "C"

namespace {

// Checks of a call's visibility arguments (before any device work).
rick_status check_vis_args(rick_plan_t *p, const double *uvw, const double *freq_hz, const void *vis,
                           const float *weight, int64_t nrow, int32_t nchan) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    if (nrow < 0) return fail(RICK_E_INVALID_ARG, "nrow=%lld", (long long)nrow);
    if (nchan < 1) return fail(RICK_E_INVALID_ARG, "nchan=%d", nchan);
    if (!freq_hz && nchan != 1) return fail(RICK_E_INVALID_ARG, "nchan=%d without freq_hz", nchan);
    if (nchan > kMaxChan) return fail(RICK_E_INVALID_ARG, "nchan=%d > %d", nchan, kMaxChan);
    if (nrow > 0 && (!uvw || !vis)) return fail(RICK_E_INVALID_ARG, "uvw or vis is NULL");
    if (((uintptr_t)uvw & 7) || ((uintptr_t)vis & (p->fp64 ? 15 : 7)) || ((uintptr_t)weight & 3))
        return fail(RICK_E_INVALID_ARG, "misaligned input pointer");
    if (nrow > (int64_t(1) << 40) / nchan) return fail(RICK_E_CAPACITY, "nrow*nchan too large");
    if (freq_hz) {
        for (int c = 0; c < nchan; ++c)
            if (!std::isfinite(freq_hz[c]) || !(freq_hz[c] > 0.0))
                return fail(RICK_E_INVALID_ARG, "freq_hz[%d]=%g", c, freq_hz[c]);
    }
    return RICK_OK;
}

// Argument checks shared by rick_grid and rick_grid_static (before any device work).
rick_status check_grid_args(rick_plan_t *p, const double *uvw, const double *freq_hz, const void *vis,
                            const float *weight, int64_t nrow, int32_t nchan) {
    const rick_status st = check_vis_args(p, uvw, freq_hz, vis, weight, nrow, nchan);
    if (st != RICK_OK) return st;
    if (p->state == 2) return fail(RICK_E_STATE, "planes already transformed; call rick_reset first");
    if (p->state == 3) return fail(RICK_E_STATE, "mesh holds predicted planes; call rick_reset first");
    if (p->lut3 && !p->lut_ready) return fail(RICK_E_STATE, "no table installed; call rick_plan_set_lut first");
    return RICK_OK;
}

// Channel scales nu_c / c0 into the plan's device buffer, in batches of
// kMaxInlineChan passed as kernel arguments (no host or device allocation).
hipError_t upload_scales(rick_plan_t *p, const double *freq_hz, int32_t nchan, hipStream_t s) {
    double sc[kMaxInlineChan];
    for (int32_t c0 = 0; c0 < nchan; c0 += kMaxInlineChan) {
        const int32_t n = nchan - c0 < kMaxInlineChan ? nchan - c0 : kMaxInlineChan;
        for (int32_t j = 0; j < n; ++j) sc[j] = freq_hz ? freq_hz[c0 + j] / kC0 : 1.0;
        const hipError_t e = launch_set_scales(p->scales + c0, sc, n, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Bound on the gridding work items of a call of nvis visibilities: one per
// chunk of a non-empty bin (one record per visibility).
int32_t grid_items_bound(const Geom &g, int64_t nvis) {
    return int32_t((nvis < g.nbins ? nvis : g.nbins) + (nvis + g.CH - 1) / g.CH + 1);
}

// Bin-and-sort of one call (sort buffers in bb), the orientation of new
// planes and the zeroing of split bins' tiles: everything before gridding.
rick_status bin_impl(rick_plan_t *p, const BinBufs &bb, const double *uvw, const double *freq_hz, const void *vis,
                     const float *weight, int64_t nrow, int32_t nchan, hipStream_t s) {
    hipError_t e = upload_scales(p, freq_hz, nchan, s);
    if (e != hipSuccess) return hip_fail(e, "channel scales upload");
    const Geom &g = p->g;
    struct Pass {
        int slot;
        const char *name;
        int level, phase;
    } passes[] = {
        {T_COUNT, "bin_count", 1, 0},       {T_SCAN, "bin_scan", 1, 1},        {T_SCATTER, "bin_scatter", 1, 2},
        {T_FINE_COUNT, "fine_count", 2, 0}, {T_FINE_SCAN, "fine_scan", 2, 1}, {T_FINE_SCATTER, "fine_scatter", 2, 2},
    };
    for (const Pass &ps : passes) {
        timer_begin(p, ps.slot, ps.name, s);
        if (ps.level == 1)
            e = p->fp64 ? launch_bin_level1<double>(g, bb, uvw, p->scales, (const double *)vis, weight, nrow, nchan,
                                                    p->stats, ps.phase, s)
                        : launch_bin_level1<float>(g, bb, uvw, p->scales, (const float *)vis, weight, nrow, nchan,
                                                   p->stats, ps.phase, s);
        else
            e = p->fp64 ? launch_bin_level2<double>(g, bb, nrow, nchan, p->stats, ps.phase, s)
                        : launch_bin_level2<float>(g, bb, nrow, nchan, p->stats, ps.phase, s);
        timer_end(p, ps.slot, s);
        if (e != hipSuccess) return hip_fail(e, ps.name);
    }
    if (p->plane_tr) {
        // orientation of the planes this call is the first to grid onto
        e = launch_orient(g, bb.scan, p->row_bits, p->plane_tr, s);
        if (e != hipSuccess) return hip_fail(e, "orient");
    }
    timer_begin(p, T_ZERO_HEAVY, "zero_heavy", s);
    if (p->fp64)
        e = launch_zero_heavy<double>(g, bb.heavy_bins, p->stats, p->tile_bits, p->plane_tr, (double *)p->mesh,
                                      (double *)p->margin, s);
    else
        e = launch_zero_heavy<float>(g, bb.heavy_bins, p->stats, p->tile_bits, p->plane_tr, (float *)p->mesh,
                                     (float *)p->margin, s);
    timer_end(p, T_ZERO_HEAVY, s);
    if (e != hipSuccess) return hip_fail(e, "zero_heavy");
    return RICK_OK;
}

// Margins of the gridded tiles added to their neighbours, tile and row bits.
rick_status merge_impl(rick_plan_t *p, const BinBufs &bb, hipStream_t s) {
    const Geom &g = p->g;
    timer_begin(p, T_MARK, "merge_margins", s);
    const hipError_t e =
        p->fp64 ? launch_merge_margins<double>(g, bb.scan, (const double *)p->margin, p->tile_bits, p->row_bits,
                                               p->plane_tr, (double *)p->mesh, s)
                : launch_merge_margins<float>(g, bb.scan, (const float *)p->margin, p->tile_bits, p->row_bits,
                                              p->plane_tr, (float *)p->mesh, s);
    timer_end(p, T_MARK, s);
    if (e != hipSuccess) return hip_fail(e, "merge_margins");
    p->state = 1;
    return RICK_OK;
}

// Bin-and-sort, gridding and margin merge of one call, with the sort buffers in bb.
rick_status grid_impl(rick_plan_t *p, const BinBufs &bb, const double *uvw, const double *freq_hz, const void *vis,
                      const float *weight, int64_t nrow, int32_t nchan, hipStream_t s) {
    rick_status r = bin_impl(p, bb, uvw, freq_hz, vis, weight, nrow, nchan, s);
    if (r != RICK_OK) return r;
    const Geom &g = p->g;
    const int32_t max_items = grid_items_bound(g, nrow * nchan);
    timer_begin(p, T_GRID, "grid", s);
    hipError_t e;
    if (p->fp64)
        e = launch_grid<double>(g, bb.scan, bb.item_bin, bb.rec_pos, (const double *)bb.rec_vis,
                                (const double *)p->lut, (double *)p->mesh, p->tile_bits, (double *)p->margin,
                                bb.bin_vmax, p->lut3 ? p->tapmax : nullptr, p->stats, p->plane_tr, max_items, s);
    else
        e = launch_grid<float>(g, bb.scan, bb.item_bin, bb.rec_pos, (const float *)bb.rec_vis, (const float *)p->lut,
                               (float *)p->mesh, p->tile_bits, (float *)p->margin, bb.bin_vmax,
                               p->lut3 ? p->tapmax : nullptr, p->stats, p->plane_tr, max_items, s);
    timer_end(p, T_GRID, s);
    if (e != hipSuccess) return hip_fail(e, "grid");
    return merge_impl(p, bb, s);
}

// The plan's own sort buffers (those of rick_grid).
BinBufs plan_bufs(rick_plan_t *p) {
    return BinBufs{p->cnt1,   p->block_sums, p->rec1, p->key_chunk0, p->chunk_key,  p->cnt2,    p->vmax2,
                   p->counts, p->bin_vmax,   p->scan, p->item_bin,   p->heavy_bins, p->rec_pos, p->rec_vis};
}

// Byte offsets, in the static scratch, of the per-visibility sort buffers of
// one rick_grid_static call of nvis visibilities (each 256-byte aligned).
struct StaticLayout {
    size_t rec1, chunk_key, cnt2, vmax2, item_bin, heavy, rec_pos, rec_vis, total;
};
StaticLayout static_layout(const Geom &g, size_t rb, int64_t nvis) {
    auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
    const size_t chunks = size_t(bin_max_chunks(g, nvis));
    const size_t items = size_t((nvis < g.nbins ? nvis : g.nbins) + (nvis + g.CH - 1) / g.CH + 2);
    StaticLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += up(bytes > 0 ? bytes : 1);
        return at;
    };
    L.rec1 = take(size_t(nvis) * (8 + 2 * rb) + 256);
    L.chunk_key = take(chunks * sizeof(int32_t));
    L.cnt2 = take(chunks * g.C * g.C * sizeof(int32_t));
    L.vmax2 = take(chunks * g.C * g.C * sizeof(uint32_t));
    L.item_bin = take(items * sizeof(int32_t));
    L.heavy = take((size_t(nvis) / (g.CH + 1) + 2) * sizeof(int32_t));
    L.rec_pos = take(size_t(nvis) * sizeof(uint32_t));
    L.rec_vis = take(size_t(nvis) * 2 * rb);
    L.total = off;
    return L;
}

}  // namespace

extern "C" {

rick_status rick_grid(rick_plan_t *p, const double *uvw, const double *freq_hz, const void *vis,
                      const float *weight, int64_t nrow, int32_t nchan, void *stream) {
    const rick_status st = check_grid_args(p, uvw, freq_hz, vis, weight, nrow, nchan);
    if (st != RICK_OK) return st;
    if (nrow * int64_t(nchan) > p->d.max_vis)
        return fail(RICK_E_CAPACITY, "nrow*nchan=%lld > max_vis=%lld", (long long)(nrow * nchan),
                    (long long)p->d.max_vis);
    DeviceGuard guard(p->d.device);
    return grid_impl(p, plan_bufs(p), uvw, freq_hz, vis, weight, nrow, nchan, (hipStream_t)stream);
}

static_assert(RICK_MAX_GRID_JOBS == kMaxGridJobs, "one job limit for the header and the kernel");

rick_status rick_grid_jobs(const rick_grid_job *jobs, int32_t n, void *stream) {
    if (!jobs) return fail(RICK_E_INVALID_ARG, "jobs is NULL");
    if (n < 1 || n > kMaxGridJobs) return fail(RICK_E_INVALID_ARG, "n=%d (1 ... %d jobs)", n, kMaxGridJobs);
    for (int32_t i = 0; i < n; ++i) {
        const rick_grid_job &J = jobs[i];
        rick_plan_t *p = J.plan;
        if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "job %d: invalid plan", i);
        if (p->lut3) return fail(RICK_E_UNSUPPORTED, "job %d: a user table (the joint gridder takes separable kernels)", i);
        const rick_status st = check_grid_args(p, J.uvw, J.freq_hz, J.vis, J.weight, J.nrow, J.nchan);
        if (st != RICK_OK) return st;
        if (J.reserved != 0) return fail(RICK_E_INVALID_ARG, "job %d: reserved=%d (must be 0)", i, J.reserved);
        if (J.nrow * int64_t(J.nchan) > p->d.max_vis)
            return fail(RICK_E_CAPACITY, "job %d: nrow*nchan=%lld > max_vis=%lld", i,
                        (long long)(J.nrow * J.nchan), (long long)p->d.max_vis);
        if (p->fp64 != jobs[0].plan->fp64) return fail(RICK_E_INVALID_ARG, "job %d: precision differs from job 0's", i);
        if (p->d.device != jobs[0].plan->d.device)
            return fail(RICK_E_INVALID_ARG, "job %d: device differs from job 0's", i);
        for (int32_t k = 0; k < i; ++k)
            if (jobs[k].plan == p) return fail(RICK_E_INVALID_ARG, "job %d: same plan as job %d", i, k);
    }
    DeviceGuard guard(jobs[0].plan->d.device);
    hipStream_t s = (hipStream_t)stream;
    const bool fp64 = jobs[0].plan->fp64;
    for (int32_t i = 0; i < n; ++i) {
        const rick_grid_job &J = jobs[i];
        const rick_status r = bin_impl(J.plan, plan_bufs(J.plan), J.uvw, J.freq_hz, J.vis, J.weight, J.nrow, J.nchan, s);
        if (r != RICK_OK) return r;
    }
    // one persistent launch per (support, tile edge); the shared work-item
    // counter is the first job's (zeroed by its binning)
    bool done[kMaxGridJobs] = {};
    for (int32_t i = 0; i < n; ++i) {
        if (done[i]) continue;
        const Geom &gi = jobs[i].plan->g;
        GridJobList list{};
        size_t lds = 0;
        int64_t max_items = 0;
        for (int32_t j = i; j < n; ++j) {
            rick_plan_t *p = jobs[j].plan;
            if (done[j] || p->g.W != gi.W || p->g.T != gi.T) continue;
            done[j] = true;
            const GridJob d{p->g,     p->scan,      p->item_bin, p->rec_pos, p->rec_vis,   p->lut,
                            p->mesh,  p->tile_bits, p->margin,   p->bin_vmax, p->plane_tr};
            hipError_t e = launch_put_grid_job(p->job_dev, d, s);
            if (e != hipSuccess) return hip_fail(e, "grid job table");
            list.job[list.n++] = p->job_dev;
            const size_t b = grid_lds_bytes(p->g, p->real_bytes);
            lds = b > lds ? b : lds;
            max_items += grid_items_bound(p->g, jobs[j].nrow * jobs[j].nchan);
        }
        unsigned long long *next = &jobs[i].plan->stats->grid_next;
        const hipError_t e = fp64 ? launch_grid_jobs<double>(list, gi.W, gi.T, lds, max_items, next, s)
                                  : launch_grid_jobs<float>(list, gi.W, gi.T, lds, max_items, next, s);
        if (e != hipSuccess) return hip_fail(e, "grid_jobs");
    }
    for (int32_t i = 0; i < n; ++i) {
        const rick_status r = merge_impl(jobs[i].plan, plan_bufs(jobs[i].plan), s);
        if (r != RICK_OK) return r;
    }
    return RICK_OK;
}

rick_status rick_grid_static(rick_plan_t *p, const double *uvw, const double *freq_hz, const void *vis,
                             const float *weight, int64_t nrow, int32_t nchan, void *stream) {
    const rick_status st = check_grid_args(p, uvw, freq_hz, vis, weight, nrow, nchan);
    if (st != RICK_OK) return st;
    const int64_t nvis = nrow * int64_t(nchan);
    const StaticLayout L = static_layout(p->g, p->real_bytes, nvis);
    if (L.total > kStaticScratchBytes)
        return fail(RICK_E_CAPACITY,
                    "nrow*nchan=%lld needs %zu B of sort scratch; the static scratch holds %zu B "
                    "(use rick_grid with a plan's max_vis for larger calls)",
                    (long long)nvis, L.total, kStaticScratchBytes);
    DeviceGuard guard(p->d.device);
    void *base = nullptr;
    const hipError_t e = static_scratch(p->d.device, &base);
    if (e != hipSuccess) return hip_fail(e, "static scratch address");
    unsigned char *b = static_cast<unsigned char *>(base);
    // per-bin tables stay the plan's (sized by the mesh shape at rick_plan);
    // the buffers that grow with the number of visibilities come from the scratch
    const BinBufs bb{p->cnt1,
                     p->block_sums,
                     b + L.rec1,
                     p->key_chunk0,
                     reinterpret_cast<int32_t *>(b + L.chunk_key),
                     reinterpret_cast<int32_t *>(b + L.cnt2),
                     reinterpret_cast<uint32_t *>(b + L.vmax2),
                     p->counts,
                     p->bin_vmax,
                     p->scan,
                     reinterpret_cast<int32_t *>(b + L.item_bin),
                     reinterpret_cast<int32_t *>(b + L.heavy),
                     reinterpret_cast<uint32_t *>(b + L.rec_pos),
                     b + L.rec_vis};
    return grid_impl(p, bb, uvw, freq_hz, vis, weight, nrow, nchan, (hipStream_t)stream);
}

rick_status rick_fft_planes(rick_plan_t *p, void *stream) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    if (p->state == 2) return fail(RICK_E_STATE, "planes already transformed");
    if (p->state == 3) return fail(RICK_E_STATE, "mesh holds predicted planes; call rick_reset first");
    DeviceGuard guard(p->d.device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    // tiles nothing was gridded onto since the reset are read as zeros
    timer_begin(p, T_FFT_ROWS, "fft_rows", s);
    if (p->fused)
        e = p->fp64 ? launch_fft_rows_panel<double>(p->g, (const double *)p->mesh, (double *)p->row_mesh,
                                                    (const double *)p->twiddle, p->tile_bits, p->row_bits, s)
                    : launch_fft_rows_panel<float>(p->g, (const float *)p->mesh, (float *)p->row_mesh,
                                                   (const float *)p->twiddle, p->tile_bits, p->row_bits, s);
    else if (p->fp64)
        e = launch_fft_rows<double>(p->g, (double *)p->mesh, (const double *)p->twiddle, p->tile_bits, p->row_bits,
                                    s);
    else
        e = launch_fft_rows<float>(p->g, (float *)p->mesh, (const float *)p->twiddle, p->tile_bits, p->row_bits, s);
    timer_end(p, T_FFT_ROWS, s);
    if (e != hipSuccess) return hip_fail(e, "fft_rows");
    if (!p->fused) {
        timer_begin(p, T_FFT_COLS, "fft_cols", s);
        if (p->fp64) e = launch_fft_cols<double>(p->g, (double *)p->mesh, (const double *)p->twiddle, s);
        else e = launch_fft_cols<float>(p->g, (float *)p->mesh, (const float *)p->twiddle, s);
        timer_end(p, T_FFT_COLS, s);
        if (e != hipSuccess) return hip_fail(e, "fft_cols");
    }
    p->state = 2;
    return RICK_OK;
}

rick_status rick_wstack_image(rick_plan_t *p, void *image, void *stream) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    if (!image) return fail(RICK_E_INVALID_ARG, "image is NULL");
    if (((uintptr_t)image) & (p->fp64 ? 7 : 3)) return fail(RICK_E_INVALID_ARG, "misaligned image");
    if (p->state != 2) return fail(RICK_E_STATE, "planes not transformed; call rick_fft_planes first");
    DeviceGuard guard(p->d.device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    const int kahan = p->d.precision == RICK_PREC_FP32_KAHAN;
    if (p->fused) {
        timer_begin(p, T_SCREEN, "fft_cols_screen", s);
        // pass 0: planes stored as they are (writes the image); pass 1: planes
        // stored transposed (adds to it)
        e = hipSuccess;
        for (int pass = 0; pass < (p->plane_tr ? 2 : 1) && e == hipSuccess; ++pass) {
            if (p->fp64)
                e = launch_fft_cols_screen<double>(p->g, (const double *)p->row_mesh, (const double *)p->twiddle,
                                                   taper_of(p), p->stats, p->row_bits, p->plane_tr, pass,
                                                   (double *)image, 0, s);
            else
                e = launch_fft_cols_screen<float>(p->g, (const float *)p->row_mesh, (const float *)p->twiddle,
                                                  taper_of(p), p->stats, p->row_bits, p->plane_tr, pass,
                                                  (float *)image, kahan, s);
        }
        timer_end(p, T_SCREEN, s);
        if (e != hipSuccess) return hip_fail(e, "fft_cols_screen");
        return RICK_OK;
    }
    timer_begin(p, T_SCREEN, "wscreen", s);
    if (p->fp64)
        e = launch_wscreen<double>(p->g, (const double *)p->mesh, taper_of(p), p->stats, (double *)image, 0, s);
    else
        e = launch_wscreen<float>(p->g, (const float *)p->mesh, taper_of(p), p->stats, (float *)image, kahan, s);
    timer_end(p, T_SCREEN, s);
    if (e != hipSuccess) return hip_fail(e, "wscreen");
    return RICK_OK;
}

rick_status rick_wstack_image_jobs(const rick_image_job *jobs, int32_t n, void *stream) {
    if (!jobs) return fail(RICK_E_INVALID_ARG, "jobs is NULL");
    if (n < 1 || n > kMaxGridJobs) return fail(RICK_E_INVALID_ARG, "n=%d (1 ... %d jobs)", n, kMaxGridJobs);
    for (int32_t i = 0; i < n; ++i) {
        rick_plan_t *p = jobs[i].plan;
        if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "job %d: invalid plan", i);
        if (!p->fused) return fail(RICK_E_INVALID_ARG, "job %d: plan without RICK_FLAG_FUSED_SCREEN", i);
        if (!jobs[i].image) return fail(RICK_E_INVALID_ARG, "job %d: image is NULL", i);
        if (((uintptr_t)jobs[i].image) & (p->fp64 ? 7 : 3)) return fail(RICK_E_INVALID_ARG, "job %d: misaligned image", i);
        if (p->state != 2) return fail(RICK_E_STATE, "job %d: planes not transformed; call rick_fft_planes first", i);
        if (p->fp64 != jobs[0].plan->fp64) return fail(RICK_E_INVALID_ARG, "job %d: precision differs from job 0's", i);
        if (p->d.device != jobs[0].plan->d.device)
            return fail(RICK_E_INVALID_ARG, "job %d: device differs from job 0's", i);
        for (int32_t k = 0; k < i; ++k)
            if (jobs[k].plan == p) return fail(RICK_E_INVALID_ARG, "job %d: same plan as job %d", i, k);
    }
    DeviceGuard guard(jobs[0].plan->d.device);
    hipStream_t s = (hipStream_t)stream;
    const bool fp64 = jobs[0].plan->fp64;
    // one launch per (grid size, compensated sum) and pass: pass 0 over every
    // plan of the group (writes the images), pass 1 over those holding
    // transposed planes (adds to them)
    bool done[kMaxGridJobs] = {};
    for (int32_t i = 0; i < n; ++i) {
        if (done[i]) continue;
        const rick_plan_t *pi = jobs[i].plan;
        const int kahan = pi->d.precision == RICK_PREC_FP32_KAHAN;
        ColJobList all{}, tr{};
        for (int32_t j = i; j < n; ++j) {
            rick_plan_t *p = jobs[j].plan;
            if (done[j] || p->g.N != pi->g.N || (p->d.precision == RICK_PREC_FP32_KAHAN) != (kahan != 0)) continue;
            done[j] = true;
            const ColJob d{p->g, p->row_mesh, p->twiddle, taper_of(p), p->stats, p->row_bits, p->plane_tr,
                           jobs[j].image};
            const hipError_t e = launch_put_col_job(p->coljob_dev, d, s);
            if (e != hipSuccess) return hip_fail(e, "column job table");
            all.job[all.n++] = p->coljob_dev;
            if (p->plane_tr) tr.job[tr.n++] = p->coljob_dev;
        }
        for (int pass = 0; pass < 2; ++pass) {
            const ColJobList &list = pass ? tr : all;
            if (list.n == 0) continue;
            const hipError_t e = fp64 ? launch_fft_cols_screen_jobs<double>(list, pi->g.N, pass, 0, s)
                                      : launch_fft_cols_screen_jobs<float>(list, pi->g.N, pass, kahan, s);
            if (e != hipSuccess) return hip_fail(e, "fft_cols_screen_jobs");
        }
    }
    return RICK_OK;
}

rick_status rick_predict_planes(rick_plan_t *p, const void *model, void *stream) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    if (p->lut3) return fail(RICK_E_UNSUPPORTED, "prediction with a user table is not built");
    if (!model) return fail(RICK_E_INVALID_ARG, "model is NULL");
    if (((uintptr_t)model) & (p->fp64 ? 7 : 3)) return fail(RICK_E_INVALID_ARG, "misaligned model");
    DeviceGuard guard(p->d.device);
    hipStream_t s = (hipStream_t)stream;
    const Geom &g = p->g;
    hipError_t e;
    timer_begin(p, T_PRED_SCREEN, "predict_screen", s);
    if (p->fp64)
        e = launch_predict_screen<double>(g, (const double *)model, p->corr, (double *)p->mesh, p->tile_bits,
                                          p->row_bits, s);
    else
        e = launch_predict_screen<float>(g, (const float *)model, p->corr, (float *)p->mesh, p->tile_bits,
                                         p->row_bits, s);
    timer_end(p, T_PRED_SCREEN, s);
    if (e != hipSuccess) return hip_fail(e, "predict_screen");
    // the inverse transform of conj(P_k) is conj(H_k): rows then columns, in
    // place in the mesh, or (plans with a row_mesh) rows into row_mesh in
    // column-panel order and columns in place there, whose strips then read
    // and write whole lines
    timer_begin(p, T_PRED_FFT, "predict_fft", s);
    if (p->fused) {
        if (p->fp64) {
            e = launch_fft_rows_panel<double>(g, (const double *)p->mesh, (double *)p->row_mesh,
                                              (const double *)p->twiddle, p->tile_bits, p->row_bits, s);
            if (e == hipSuccess)
                e = launch_fft_cols_panel<double>(g, (double *)p->row_mesh, (const double *)p->twiddle, s);
        } else {
            e = launch_fft_rows_panel<float>(g, (const float *)p->mesh, (float *)p->row_mesh,
                                             (const float *)p->twiddle, p->tile_bits, p->row_bits, s);
            if (e == hipSuccess)
                e = launch_fft_cols_panel<float>(g, (float *)p->row_mesh, (const float *)p->twiddle, s);
        }
    } else if (p->fp64) {
        e = launch_fft_rows<double>(g, (double *)p->mesh, (const double *)p->twiddle, p->tile_bits, p->row_bits, s);
        if (e == hipSuccess) e = launch_fft_cols<double>(g, (double *)p->mesh, (const double *)p->twiddle, s);
    } else {
        e = launch_fft_rows<float>(g, (float *)p->mesh, (const float *)p->twiddle, p->tile_bits, p->row_bits, s);
        if (e == hipSuccess) e = launch_fft_cols<float>(g, (float *)p->mesh, (const float *)p->twiddle, s);
    }
    timer_end(p, T_PRED_FFT, s);
    if (e != hipSuccess) return hip_fail(e, "predict_fft");
    p->state = 3;
    return RICK_OK;
}

rick_status rick_degrid(rick_plan_t *p, const double *uvw, const double *freq_hz, void *vis_out, int64_t nrow,
                        int32_t nchan, void *stream) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    if (p->lut3) return fail(RICK_E_UNSUPPORTED, "prediction with a user table is not built");
    if (nrow < 0) return fail(RICK_E_INVALID_ARG, "nrow=%lld", (long long)nrow);
    if (nchan < 1) return fail(RICK_E_INVALID_ARG, "nchan=%d", nchan);
    if (!freq_hz && nchan != 1) return fail(RICK_E_INVALID_ARG, "nchan=%d without freq_hz", nchan);
    if (nchan > kMaxChan) return fail(RICK_E_INVALID_ARG, "nchan=%d > %d", nchan, kMaxChan);
    if (nrow > (int64_t(1) << 40) / nchan) return fail(RICK_E_INVALID_ARG, "nrow*nchan too large");
    if (nrow > 0 && (!uvw || !vis_out)) return fail(RICK_E_INVALID_ARG, "uvw or vis_out is NULL");
    if (((uintptr_t)uvw & 7) || ((uintptr_t)vis_out & (p->fp64 ? 15 : 7)))
        return fail(RICK_E_INVALID_ARG, "misaligned pointer");
    if (p->state != 3) return fail(RICK_E_STATE, "no predicted planes; call rick_predict_planes first");
    std::vector<double> sc(nchan, 1.0);
    if (freq_hz) {
        for (int c = 0; c < nchan; ++c) {
            if (!std::isfinite(freq_hz[c]) || !(freq_hz[c] > 0.0))
                return fail(RICK_E_INVALID_ARG, "freq_hz[%d]=%g", c, freq_hz[c]);
            sc[c] = freq_hz[c] / kC0;
        }
    }
    DeviceGuard guard(p->d.device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_set_scales(p->scales, sc.data(), nchan, s);
    if (e != hipSuccess) return hip_fail(e, "channel scales upload");
    timer_begin(p, T_DEGRID, "degrid", s);
    const void *planes = p->fused ? p->row_mesh : p->mesh;
    const int32_t panel = p->fused ? p->panel : 0;
    if (p->fp64)
        e = launch_degrid<double>(p->g, uvw, p->scales, nrow, nchan, (const double *)p->lut, (const double *)planes,
                                  panel, (double *)vis_out, s);
    else
        e = launch_degrid<float>(p->g, uvw, p->scales, nrow, nchan, (const float *)p->lut, (const float *)planes,
                                 panel, (float *)vis_out, s);
    timer_end(p, T_DEGRID, s);
    if (e != hipSuccess) return hip_fail(e, "degrid");
    return RICK_OK;
}

}  // extern "C"

struct rick_degrid_order_s {
    uint32_t magic;
    int device;
    int64_t nrow, nvis;
    int32_t nchan;
    int32_t panel;   // layout the keys address: 0 row order, else column panels of this width
    uint64_t *keys, *vals;
    Geom g;   // geometry the positions were quantised with
};

namespace {
constexpr uint32_t kOrderMagic = 0x4f524452u, kOrderDead = 0x44454144u;
bool same_geometry(const Geom &a, const Geom &b) {
    return a.N == b.N && a.Nw == b.Nw && a.W == b.W && a.OS == b.OS && a.fov == b.fov && a.half == b.half &&
           a.w_min == b.w_min && a.dw == b.dw;
}
}  // namespace

extern "C" {

rick_status rick_degrid_order_create(rick_plan_t *p, const double *uvw, const double *freq_hz, int64_t nrow,
                                     int32_t nchan, rick_degrid_order_t **out, void *stream) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    if (p->lut3) return fail(RICK_E_UNSUPPORTED, "prediction with a user table is not built");
    if (!out) return fail(RICK_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (nrow < 0) return fail(RICK_E_INVALID_ARG, "nrow=%lld", (long long)nrow);
    if (nchan < 1) return fail(RICK_E_INVALID_ARG, "nchan=%d", nchan);
    if (!freq_hz && nchan != 1) return fail(RICK_E_INVALID_ARG, "nchan=%d without freq_hz", nchan);
    if (nchan > kMaxChan) return fail(RICK_E_INVALID_ARG, "nchan=%d > %d", nchan, kMaxChan);
    if (nrow > ((int64_t(1) << 31) - 1) / nchan) return fail(RICK_E_INVALID_ARG, "nrow*nchan >= 2^31");
    if (nrow > 0 && !uvw) return fail(RICK_E_INVALID_ARG, "uvw is NULL");
    if ((uintptr_t)uvw & 7) return fail(RICK_E_INVALID_ARG, "misaligned uvw");
    std::vector<double> sc(nchan, 1.0);
    if (freq_hz) {
        for (int c = 0; c < nchan; ++c) {
            if (!std::isfinite(freq_hz[c]) || !(freq_hz[c] > 0.0))
                return fail(RICK_E_INVALID_ARG, "freq_hz[%d]=%g", c, freq_hz[c]);
            sc[c] = freq_hz[c] / kC0;
        }
    }
    DeviceGuard guard(p->d.device);
    hipStream_t s = (hipStream_t)stream;
    const Geom &g = p->g;
    const int64_t nvis = nrow * nchan;
    const size_t n = size_t(nvis > 0 ? nvis : 1);
    uint64_t *kin = nullptr, *vin = nullptr, *kout = nullptr, *vout = nullptr;
    void *temp = nullptr;
    auto release = [&]() {
        if (kin) (void)hipFree(kin);
        if (vin) (void)hipFree(vin);
        if (temp) (void)hipFree(temp);
    };
    hipError_t e = hipMalloc(&kin, n * 8);
    if (e == hipSuccess) e = hipMalloc(&vin, n * 8);
    if (e == hipSuccess) e = hipMalloc(&kout, n * 8);
    if (e == hipSuccess) e = hipMalloc(&vout, n * 8);
    if (e != hipSuccess) {
        release();
        if (kout) (void)hipFree(kout);
        if (vout) (void)hipFree(vout);
        return fail(RICK_E_OOM, "sort order buffers for %lld visibilities", (long long)nvis);
    }
    // keys are offsets of the footprint origin in the layout the planes will
    // be held in (row_mesh's column panels for plans that have one): below N_w N^2
    const int32_t panel = p->fused ? p->panel : 0;
    int end_bit = 1;
    while ((uint64_t(1) << end_bit) < uint64_t(g.Nw) * uint64_t(g.N) * uint64_t(g.N)) ++end_bit;
    // the sort ignores the key's lowest bits (the column inside a panel and
    // 3 bits of the row; 3 bits of the column in row order): footprints of one
    // group of PW x 8 cells (8 x 1 in row order) stay together, in visibility order, so
    // that a wave's results land in fewer, longer runs of the output
    int begin_bit = (panel > 0 ? __builtin_ctz((unsigned)panel) : 0) + 3;
    if (begin_bit >= end_bit) begin_bit = 0;
    size_t temp_bytes = 0;
    e = launch_set_scales(p->scales, sc.data(), nchan, s);
    if (e == hipSuccess)
        e = p->fp64 ? launch_order_keys<double>(g, uvw, p->scales, nrow, nchan, panel, kin, vin, s)
                    : launch_order_keys<float>(g, uvw, p->scales, nrow, nchan, panel, kin, vin, s);
    if (e == hipSuccess && nvis > 0)
        e = sort_order(nullptr, temp_bytes, kin, kout, vin, vout, nvis, begin_bit, end_bit, s);
    if (e == hipSuccess && nvis > 0) e = hipMalloc(&temp, temp_bytes > 0 ? temp_bytes : 1);
    if (e == hipSuccess && nvis > 0)
        e = sort_order(temp, temp_bytes, kin, kout, vin, vout, nvis, begin_bit, end_bit, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    release();
    if (e != hipSuccess) {
        (void)hipFree(kout);
        (void)hipFree(vout);
        return hip_fail(e, "degrid order");
    }
    rick_degrid_order_t *o = new rick_degrid_order_t;
    o->magic = kOrderMagic;
    o->device = p->d.device;
    o->nrow = nrow;
    o->nchan = nchan;
    o->nvis = nvis;
    o->panel = panel;
    o->keys = kout;
    o->vals = vout;
    o->g = g;
    *out = o;
    return RICK_OK;
}

rick_status rick_degrid_order_destroy(rick_degrid_order_t *o) {
    if (!o || o->magic != kOrderMagic) return fail(RICK_E_INVALID_ARG, "invalid degrid order");
    DeviceGuard guard(o->device);
    (void)hipFree(o->keys);
    (void)hipFree(o->vals);
    o->magic = kOrderDead;
    delete o;
    return RICK_OK;
}

rick_status rick_degrid_order_info(const rick_degrid_order_t *o, rick_degrid_order_info_t *out) {
    if (!o || o->magic != kOrderMagic) return fail(RICK_E_INVALID_ARG, "invalid degrid order");
    if (!out) return fail(RICK_E_INVALID_ARG, "out is NULL");
    out->keys = o->keys;
    out->vals = o->vals;
    out->n = o->nvis;
    out->panel = o->panel;
    out->pad = 0;
    return RICK_OK;
}

rick_status rick_degrid_sorted(rick_plan_t *p, const rick_degrid_order_t *o, void *vis_out, void *stream) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    if (!o || o->magic != kOrderMagic) return fail(RICK_E_INVALID_ARG, "invalid degrid order");
    if (o->device != p->d.device) return fail(RICK_E_INVALID_ARG, "order and plan on different devices");
    if (!same_geometry(o->g, p->g) || o->panel != (p->fused ? p->panel : 0))
        return fail(RICK_E_INVALID_ARG, "order was made for another grid, field, w range or plane layout");
    if (o->nvis > 0 && !vis_out) return fail(RICK_E_INVALID_ARG, "vis_out is NULL");
    if ((uintptr_t)vis_out & (p->fp64 ? 15 : 7)) return fail(RICK_E_INVALID_ARG, "misaligned vis_out");
    if (p->state != 3) return fail(RICK_E_STATE, "no predicted planes; call rick_predict_planes first");
    DeviceGuard guard(p->d.device);
    hipStream_t s = (hipStream_t)stream;
    timer_begin(p, T_DEGRID, "degrid", s);
    const void *planes = p->fused ? p->row_mesh : p->mesh;
    const int32_t panel = p->fused ? p->panel : 0;
    hipError_t e =
        p->fp64 ? launch_degrid_sorted<double>(p->g, o->keys, o->vals, o->nvis, (const double *)p->lut,
                                               (const double *)planes, panel, (double *)vis_out, s)
                : launch_degrid_sorted<float>(p->g, o->keys, o->vals, o->nvis, (const float *)p->lut,
                                              (const float *)planes, panel, (float *)vis_out, s);
    timer_end(p, T_DEGRID, s);
    if (e != hipSuccess) return hip_fail(e, "degrid_sorted");
    return RICK_OK;
}

rick_status rick_plan_info(rick_plan_t *p, rick_plan_info_t *out) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    if (!out) return fail(RICK_E_INVALID_ARG, "out is NULL");
    DeviceGuard guard(p->d.device);
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "synchronise");
    Stats st;
    e = hipMemcpy(&st, p->stats, sizeof st, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read counters");
    std::memset(out, 0, sizeof *out);
    out->n_gridded = (int64_t)st.n_gridded;
    out->n_dropped = (int64_t)st.n_dropped;
    out->n_records = (int64_t)st.n_records;
    out->sum_weights = st.sum_w;
    out->du = p->du;
    out->dl = p->dl;
    out->dw = p->g.dw;
    out->mesh = p->mesh;
    out->row_mesh = p->row_mesh;
    out->tile_bits = p->tile_bits;
    out->occ_words = p->g.occw;
    {
        const Geom &g = p->g;
        std::vector<uint64_t> bits(size_t(g.Nw) * g.nt * g.occw);
        e = hipMemcpy(bits.data(), p->tile_bits, bits.size() * sizeof(uint64_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "read tile bitmap");
        int64_t tiles = 0, rows = 0;
        for (size_t r = 0; r < size_t(g.Nw) * g.nt; ++r) {
            int64_t c = 0;
            for (int j = 0; j < g.occw; ++j) c += __builtin_popcountll(bits[r * g.occw + j]);
            tiles += c;
            rows += c > 0;
        }
        out->tiles_set = tiles;
        out->tile_rows_set = rows;
        out->rec1_bytes = p->g.cpt1 ? 12 : int32_t(8 + 2 * p->real_bytes);
    }
    out->panel = p->panel;
    out->mesh_bytes = (int64_t)p->mesh_bytes;
    if (p->w_k_host.size() != size_t(p->g.Nw)) {
        p->w_k_host.resize(p->g.Nw);
        for (int k = 0; k < p->g.Nw; ++k) p->w_k_host[k] = p->g.w_min + (double(k) + 0.5) * p->g.dw;
    }
    out->w_k = p->w_k_host.data();
    out->taper = taper_of(p);
    out->lut_wbins = p->lut3 ? p->g.nwf : 0;
    out->plane_transposed = p->plane_tr;
    out->tile = p->g.T;
    out->chunk = p->g.CH;
    out->state = p->state;
    out->n_timers = 0;
    if (p->timing) {
        int nt = 0;
        for (int i = 0; i < kMaxTimers && nt < 16; ++i) {
            if (!p->ev_name[i] || p->ev_calls[i] == 0) continue;
            const int64_t n = p->ev_calls[i] < kTimerRing ? p->ev_calls[i] : kTimerRing;
            double sum = 0.0;
            int64_t ok = 0;
            for (int64_t j = 0; j < n; ++j) {
                float ms = 0.0f;
                if (hipEventElapsedTime(&ms, p->ev[i][2 * j], p->ev[i][2 * j + 1]) == hipSuccess) {
                    sum += ms;
                    ++ok;
                }
            }
            out->kernel_ms[nt] = ok ? float(sum / ok) : -1.0f;
            out->kernel_calls[nt] = (int32_t)ok;
            out->kernel_names[nt] = p->ev_name[i];
            ++nt;
            p->ev_calls[i] = 0;
        }
        out->n_timers = nt;
        (void)hipGetLastError();
    }
    return RICK_OK;
}

rick_status rick_plan_bin_counts(rick_plan_t *p, int32_t *counts, int64_t n) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    if (!counts) return fail(RICK_E_INVALID_ARG, "counts is NULL");
    if (n != p->g.nbins) return fail(RICK_E_INVALID_ARG, "n=%lld, plan has %d bins", (long long)n, p->g.nbins);
    DeviceGuard guard(p->d.device);
    hipError_t e = hipDeviceSynchronize();
    std::vector<BinScan> sc(size_t(n) + 1);
    if (e == hipSuccess) e = hipMemcpy(sc.data(), p->scan, (size_t(n) + 1) * sizeof(BinScan), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read bin counts");
    for (int64_t i = 0; i < n; ++i) counts[i] = sc[i + 1].rec - sc[i].rec;
    return RICK_OK;
}

rick_status rick_plan_retarget(rick_plan_t *p, double fov_rad, double w_min, double w_max) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    rick_plan_desc d = p->d;
    d.fov_rad = fov_rad;
    d.w_min = w_min;
    d.w_max = w_max;
    const rick_status st = validate(&d);
    if (st != RICK_OK) return st;
    p->d = d;
    p->g.fov = fov_rad;
    p->g.w_min = w_min;
    p->g.dw = (w_max - w_min) / double(p->g.Nw);
    p->du = 1.0 / fov_rad;
    p->dl = fov_rad / p->g.N;
    return RICK_OK;
}

// ---- batches: graph recording, timestamps, autotuning ----

struct rick_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct rick_stamps_s {
    uint64_t *dev = nullptr;   // device clock values, one per slot
    int32_t n = 0;
    double khz = 0.0;          // device clock rate
};

rick_status rick_capture_begin(void *stream) {
    hipError_t e = hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal);
    return e == hipSuccess ? RICK_OK : hip_fail(e, "hipStreamBeginCapture");
}

rick_status rick_capture_end(void *stream, rick_graph_t **out) {
    if (!out) return fail(RICK_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    rick_graph_t *g = new (std::nothrow) rick_graph_t;
    if (!g) return fail(RICK_E_OOM, "graph handle");
    hipError_t e = hipStreamEndCapture((hipStream_t)stream, &g->graph);
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (g->graph) (void)hipGraphDestroy(g->graph);
        delete g;
        return hip_fail(e, "graph capture");
    }
    *out = g;
    return RICK_OK;
}

rick_status rick_graph_launch(rick_graph_t *g, void *stream) {
    if (!g || !g->exec) return fail(RICK_E_INVALID_ARG, "graph is NULL");
    hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    return e == hipSuccess ? RICK_OK : hip_fail(e, "hipGraphLaunch");
}

rick_status rick_graph_destroy(rick_graph_t *g) {
    if (!g) return fail(RICK_E_INVALID_ARG, "graph is NULL");
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return RICK_OK;
}

rick_status rick_stamps_create(int32_t n, rick_stamps_t **out) {
    if (!out || n < 1) return fail(RICK_E_INVALID_ARG, "n=%d", n);
    *out = nullptr;
    rick_stamps_t *t = new (std::nothrow) rick_stamps_t;
    if (!t) return fail(RICK_E_OOM, "stamps handle");
    int dev = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e == hipSuccess && khz <= 0) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = hipMalloc((void **)&t->dev, size_t(n) * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMemset(t->dev, 0, size_t(n) * sizeof(uint64_t));
    // the memset is ordered on the null stream only, not against non-blocking
    // streams: it must be done before a stamp on such a stream can land
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        if (t->dev) (void)hipFree(t->dev);
        delete t;
        return hip_fail(e, "stamps");
    }
    t->n = n;
    t->khz = double(khz);
    *out = t;
    return RICK_OK;
}

rick_status rick_stamp(rick_stamps_t *t, int32_t i, void *stream) {
    if (!t || i < 0 || i >= t->n) return fail(RICK_E_INVALID_ARG, "stamp %d", i);
    hipError_t e = launch_stamp(t->dev + i, (hipStream_t)stream);
    return e == hipSuccess ? RICK_OK : hip_fail(e, "stamp");
}

rick_status rick_stamps_elapsed(rick_stamps_t *t, int32_t i, int32_t j, float *ms) {
    if (!t || !ms || i < 0 || j < 0 || i >= t->n || j >= t->n) return fail(RICK_E_INVALID_ARG, "stamps %d, %d", i, j);
    uint64_t a = 0, b = 0;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(&a, t->dev + i, sizeof a, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&b, t->dev + j, sizeof b, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "read stamps");
    *ms = float(double(int64_t(b - a)) / t->khz);
    return RICK_OK;
}

rick_status rick_stamps_destroy(rick_stamps_t *t) {
    if (!t) return fail(RICK_E_INVALID_ARG, "stamps is NULL");
    if (t->dev) (void)hipFree(t->dev);
    delete t;
    return RICK_OK;
}

rick_status rick_autotune(const rick_plan_desc *d, const double *uvw, const double *freq_hz, const void *vis,
                          const float *weight, int64_t nrow, int32_t nchan, void *stream, int32_t *tile,
                          int32_t *chunk, float *ms) {
    if (!d || !tile || !chunk || !ms) return fail(RICK_E_INVALID_ARG, "NULL argument");
    rick_status st = validate(d);
    if (st != RICK_OK) return st;
    DeviceGuard guard(d->device);
    hipStream_t s = (hipStream_t)stream;
    const size_t real_bytes = d->precision == RICK_PREC_FP64 ? 8 : 4;
    void *image = nullptr;
    hipError_t e = hipMalloc(&image, size_t(d->grid_n) * d->grid_n * real_bytes);
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(RICK_E_OOM, "autotune image") : hip_fail(e, "hipMalloc");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float best = -1.0f;
    int32_t best_t = 0, best_c = 0;
    rick_status result = RICK_OK;
    const int32_t tiles[] = {16, 32, 64}, chunks[] = {2048, 8192, 32768};
    for (int32_t T : tiles) {
        if (e != hipSuccess || result != RICK_OK) break;
        if (T < d->support || T > d->grid_n) continue;
        for (int32_t CH : chunks) {
            rick_plan_desc dd = *d;
            dd.tile = T;
            dd.chunk = CH;
            dd.flags &= ~RICK_FLAG_TIMING;
            rick_plan_t *p = nullptr;
            st = rick_plan(&dd, &p);
            if (st == RICK_E_INVALID_ARG) continue;   // tile does not fit this support / LDS
            if (st != RICK_OK) {
                result = st;
                break;
            }
            float t_ms = 0.0f;
            for (int it = 0; it < 3 && st == RICK_OK; ++it) {
                if (it == 1) e = hipEventRecord(e0, s);
                st = rick_reset(p, stream);
                if (st == RICK_OK) st = rick_grid(p, uvw, freq_hz, vis, weight, nrow, nchan, stream);
                if (st == RICK_OK) st = rick_fft_planes(p, stream);
                if (st == RICK_OK) st = rick_wstack_image(p, image, stream);
            }
            if (st == RICK_OK) {
                e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                if (e == hipSuccess) e = hipEventElapsedTime(&t_ms, e0, e1);
                t_ms *= 0.5f;
            }
            (void)rick_plan_destroy(p);
            if (st != RICK_OK) {
                result = st;
                break;
            }
            if (e != hipSuccess) break;
            if (best < 0.0f || t_ms < best) {
                best = t_ms;
                best_t = T;
                best_c = CH;
            }
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(image);
    if (result != RICK_OK) return result;
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    if (best < 0.0f) return fail(RICK_E_INVALID_ARG, "no tile fits support %d", d->support);
    *tile = best_t;
    *chunk = best_c;
    *ms = best;
    return RICK_OK;
}


rick_status rick_plan_set_lut(rick_plan_t *p, const float *table, int32_t on_device, void *stream) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    if (!p->lut3) return fail(RICK_E_STATE, "the plan's kernel is not RICK_KERNEL_USER_LUT");
    if (!table) return fail(RICK_E_INVALID_ARG, "table is NULL");
    if (on_device && ((uintptr_t)table & 3)) return fail(RICK_E_INVALID_ARG, "misaligned table");
    DeviceGuard guard(p->d.device);
    hipStream_t s = (hipStream_t)stream;
    const Geom &g = p->g;
    const int64_t n = int64_t(g.nwf) * g.OS * g.OS * g.W * g.W;
    hipError_t e = hipSuccess;
    if (on_device) {
        e = p->fp64 ? launch_table_install<double>(table, (double *)p->lut, n, p->tapmax, s)
                    : launch_table_install<float>(table, (float *)p->lut, n, p->tapmax, s);
    } else {
        // a host table: converted and its largest |entry| found here, copied
        // synchronously (the caller's buffer may go away after the call)
        float mx = 0.0f;
        for (int64_t i = 0; i < n; ++i) {
            if (!std::isfinite(table[i])) return fail(RICK_E_INVALID_ARG, "table[%lld] is not finite", (long long)i);
            mx = std::max(mx, std::fabs(table[i]));
        }
        if (p->fp64) {
            std::vector<double> t(table, table + n);
            e = hipMemcpy(p->lut, t.data(), size_t(n) * sizeof(double), hipMemcpyHostToDevice);
        } else {
            e = hipMemcpy(p->lut, table, size_t(n) * sizeof(float), hipMemcpyHostToDevice);
        }
        if (e == hipSuccess) e = hipMemcpy(p->tapmax, &mx, sizeof mx, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess)
        e = p->fp64 ? launch_taper2d<double>(g, (const double *)p->lut, p->taper_bufs, p->corr2, s)
                    : launch_taper2d<float>(g, (const float *)p->lut, p->taper_bufs, p->corr2, s);
    if (e != hipSuccess) return hip_fail(e, "install table");
    p->lut_ready = true;
    return RICK_OK;
}

static rick_status check_table_shape(int32_t support, int32_t oversample, int32_t n_wbins) {
    if (support < 1 || support > 15 || (support & 1) == 0)
        return fail(RICK_E_INVALID_ARG, "support=%d: must be odd in [1, 15]", support);
    if (!is_pow2(oversample) || oversample > 256)
        return fail(RICK_E_INVALID_ARG, "oversample=%d: must be a power of two in [1, 256]", oversample);
    if (!is_pow2(n_wbins) || n_wbins > 8) return fail(RICK_E_INVALID_ARG, "n_wbins=%d: must be 1, 2, 4 or 8", n_wbins);
    return RICK_OK;
}

rick_status rick_mlp_tabulate(const float *theta, int32_t support, int32_t oversample, int32_t n_wbins,
                              float *table, void *stream) {
    const rick_status st = check_table_shape(support, oversample, n_wbins);
    if (st != RICK_OK) return st;
    if (!theta || !table) return fail(RICK_E_INVALID_ARG, "theta or table is NULL");
    if (((uintptr_t)theta & 3) || ((uintptr_t)table & 3)) return fail(RICK_E_INVALID_ARG, "misaligned pointer");
    const hipError_t e = launch_mlp_table(theta, support, oversample, n_wbins, table, nullptr, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mlp tabulate");
    return RICK_OK;
}

rick_status rick_mlp_backward(const float *theta, int32_t support, int32_t oversample, int32_t n_wbins,
                              const float *table, const double *dtable, float *dtheta, void *stream) {
    const rick_status st = check_table_shape(support, oversample, n_wbins);
    if (st != RICK_OK) return st;
    if (!theta || !table || !dtable || !dtheta) return fail(RICK_E_INVALID_ARG, "NULL pointer");
    if (((uintptr_t)theta & 3) || ((uintptr_t)table & 3) || ((uintptr_t)dtable & 7) || ((uintptr_t)dtheta & 3))
        return fail(RICK_E_INVALID_ARG, "misaligned pointer");
    const hipError_t e = launch_mlp_backward(theta, support, oversample, n_wbins, table, dtable, dtheta,
                                             (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "mlp backward");
    return RICK_OK;
}

rick_status rick_adam_step(float *theta, const float *grad, float *m, float *v, int32_t n, int32_t step, float lr,
                           float beta1, float beta2, float eps, void *stream) {
    if (!theta || !grad || !m || !v) return fail(RICK_E_INVALID_ARG, "NULL pointer");
    if (n < 1 || step < 1) return fail(RICK_E_INVALID_ARG, "n=%d, step=%d", n, step);
    if (!(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return fail(RICK_E_INVALID_ARG, "Adam hyper-parameters");
    const hipError_t e = launch_adam(theta, grad, m, v, n, step, lr, beta1, beta2, eps, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "adam");
    return RICK_OK;
}

rick_status rick_image_loss(rick_plan_t *p, const void *image, const double *target, double *dimage,
                            double *dtaper, double *sums, void *stream) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    if (!image || !target || !dimage || !dtaper || !sums) return fail(RICK_E_INVALID_ARG, "NULL pointer");
    if (((uintptr_t)image & (p->fp64 ? 7 : 3)) || ((uintptr_t)target & 7) || ((uintptr_t)dimage & 7) ||
        ((uintptr_t)dtaper & 7) || ((uintptr_t)sums & 7))
        return fail(RICK_E_INVALID_ARG, "misaligned pointer");
    DeviceGuard guard(p->d.device);
    hipStream_t s = (hipStream_t)stream;
    const hipError_t e =
        p->fp64 ? launch_image_loss<double>(p->g, (const double *)image, target, taper_of(p), dimage, dtaper, sums, s)
                : launch_image_loss<float>(p->g, (const float *)image, target, taper_of(p), dimage, dtaper, sums, s);
    if (e != hipSuccess) return hip_fail(e, "image loss");
    return RICK_OK;
}

rick_status rick_table_gradient(rick_plan_t *p, const double *dimage, const double *dtaper, const double *uvw,
                                const double *freq_hz, const void *vis, const float *weight, int64_t nrow,
                                int32_t nchan, double *dtable, void *stream) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    if (!p->lut3) return fail(RICK_E_STATE, "the plan's kernel is not RICK_KERNEL_USER_LUT");
    if (p->state != 2) return fail(RICK_E_STATE, "the planes of the imaged visibilities are not transformed");
    if (!dimage || !dtaper || !dtable) return fail(RICK_E_INVALID_ARG, "NULL pointer");
    if (((uintptr_t)dimage & 7) || ((uintptr_t)dtaper & 7) || ((uintptr_t)dtable & 7))
        return fail(RICK_E_INVALID_ARG, "misaligned pointer");
    const rick_status st = check_vis_args(p, uvw, freq_hz, vis, weight, nrow, nchan);
    if (st != RICK_OK) return st;
    DeviceGuard guard(p->d.device);
    hipStream_t s = (hipStream_t)stream;
    const Geom &g = p->g;
    const int64_t n_table = int64_t(g.nwf) * g.OS * g.OS * g.W * g.W;
    hipError_t e = upload_scales(p, freq_hz, nchan, s);
    // dL/dG_k of every plane (conjugated, then inverse-transformed in place:
    // the mesh then holds the conjugate of the forward transform)
    if (e == hipSuccess)
        e = p->fp64 ? launch_grad_screen<double>(g, dimage, p->stats, (double *)p->mesh, s)
                    : launch_grad_screen<float>(g, dimage, p->stats, (float *)p->mesh, s);
    if (e == hipSuccess) e = launch_fill_bits(g, p->tile_bits, p->row_bits, s);
    if (e == hipSuccess)
        e = p->fp64 ? launch_fft_rows<double>(g, (double *)p->mesh, (const double *)p->twiddle, p->tile_bits,
                                              p->row_bits, s)
                    : launch_fft_rows<float>(g, (float *)p->mesh, (const float *)p->twiddle, p->tile_bits,
                                             p->row_bits, s);
    if (e == hipSuccess)
        e = p->fp64 ? launch_fft_cols<double>(g, (double *)p->mesh, (const double *)p->twiddle, s)
                    : launch_fft_cols<float>(g, (float *)p->mesh, (const float *)p->twiddle, s);
    if (e == hipSuccess)
        e = p->fp64 ? launch_table_grad<double>(g, uvw, p->scales, (const double *)vis, weight, nrow, nchan,
                                                (const double *)p->mesh, dtable, n_table, s)
                    : launch_table_grad<float>(g, uvw, p->scales, (const float *)vis, weight, nrow, nchan,
                                               (const float *)p->mesh, dtable, n_table, s);
    if (e == hipSuccess)
        e = p->fp64 ? launch_taper2d_adjoint<double>(g, dtaper, p->taper_bufs, dtable, s)
                    : launch_taper2d_adjoint<float>(g, dtaper, p->taper_bufs, dtable, s);
    if (e != hipSuccess) return hip_fail(e, "table gradient");
    p->state = 3;   // the mesh holds gradient planes: a reset comes next
    return RICK_OK;
}

rick_status rick_dft_image(rick_plan_t *p, const double *uvw, const double *freq_hz, const void *vis,
                           const float *weight, int64_t nrow, int32_t nchan, int32_t q0, int32_t p0, int32_t nq,
                           int32_t np, double *out, void *stream) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    if (!out || ((uintptr_t)out & 7)) return fail(RICK_E_INVALID_ARG, "out is NULL or misaligned");
    const int32_t N = p->g.N;
    if (nq < 1 || np < 1 || q0 < 0 || p0 < 0 || q0 > N - nq || p0 > N - np)
        return fail(RICK_E_INVALID_ARG, "pixel rectangle (%d, %d) + (%d, %d) outside the %d^2 image", q0, p0, nq, np,
                    N);
    const rick_status st = check_vis_args(p, uvw, freq_hz, vis, weight, nrow, nchan);
    if (st != RICK_OK) return st;
    if (nrow * int64_t(nchan) > int64_t(65535) * 16384)
        return fail(RICK_E_CAPACITY, "nrow*nchan=%lld: at most %lld visibilities per call",
                    (long long)(nrow * nchan), (long long)(int64_t(65535) * 16384));
    DeviceGuard guard(p->d.device);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = upload_scales(p, freq_hz, nchan, s);
    if (e == hipSuccess)
        e = p->fp64 ? launch_dft<double>(p->g, uvw, p->scales, (const double *)vis, weight, nrow, nchan, q0, p0, nq,
                                         np, out, p->dft_wsum, s)
                    : launch_dft<float>(p->g, uvw, p->scales, (const float *)vis, weight, nrow, nchan, q0, p0, nq, np,
                                        out, p->dft_wsum, s);
    if (e != hipSuccess) return hip_fail(e, "direct sum");
    return RICK_OK;
}


rick_status rick_separable_table(rick_plan_t *p, int32_t n_wbins, float *table, void *stream) {
    if (!plan_ok(p)) return fail(RICK_E_BAD_PLAN, "invalid plan");
    if (p->lut3) return fail(RICK_E_STATE, "the plan's kernel is a user table, not a separable one");
    if (!is_pow2(n_wbins) || n_wbins > 8) return fail(RICK_E_INVALID_ARG, "n_wbins=%d: must be 1, 2, 4 or 8", n_wbins);
    if (!table || ((uintptr_t)table & 3)) return fail(RICK_E_INVALID_ARG, "table is NULL or misaligned");
    DeviceGuard guard(p->d.device);
    const hipError_t e =
        p->fp64 ? launch_separable_table<double>((const double *)p->lut, n_wbins, p->g.OS, p->g.W, table,
                                                 (hipStream_t)stream)
                : launch_separable_table<float>((const float *)p->lut, n_wbins, p->g.OS, p->g.W, table,
                                                (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "separable table");
    return RICK_OK;
}

rick_status rick_table_residual(const float *table, const float *target, int64_t n, double *dtable, double *sums,
                                void *stream) {
    if (!table || !target || !dtable || !sums || n < 1) return fail(RICK_E_INVALID_ARG, "NULL pointer or n < 1");
    if (((uintptr_t)table & 3) || ((uintptr_t)target & 3) || ((uintptr_t)dtable & 7) || ((uintptr_t)sums & 7))
        return fail(RICK_E_INVALID_ARG, "misaligned pointer");
    const hipError_t e = launch_table_residual(table, target, n, dtable, sums, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "table residual");
    return RICK_OK;
}

}  // extern "C"
