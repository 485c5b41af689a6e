/*
 * rick.h -- C ABI of the MI355X (gfx950) w-stacking imager.
 *
 * The library computes a dirty image from interferometric visibilities by
 * w-stacking (Sec. 2.1 of "Green computing toward SKA era with RICK",
 * arXiv:2504.00959): every visibility is mapped to the closest w-plane and
 * convolved onto that plane's (u, v) mesh with a finite Gaussian or
 * Kaiser-Bessel kernel (Eq. 3), every plane is inverse-FFT'd, plane k is
 * multiplied by the w phase screen exp(+2 pi i w_k (n - 1)) and the planes
 * are summed into the image (Eq. 1, whose visibility model is Eq. 2).
 *
 * Four calls make one image, each asynchronous on the caller's stream:
 *   rick_grid          bin-and-sort by (w-plane, uv tile), then LDS-tiled gridding
 *   rick_fft_planes    batched, centred 2-D inverse FFT of every plane
 *   rick_wstack_image  phase screen + sum over planes + normalisation
 *   rick_reset         start a new image (clears the weight sum and counters)
 *   rick_predict_planes, rick_degrid
 *                      prediction: model image -> visibilities (Eq. 2), the
 *                      adjoint of the imaging steps
 *   rick_degrid_order_create, rick_degrid_sorted, rick_degrid_order_destroy
 *                      prediction at fixed positions: quantise and sort once,
 *                      interpolate in sorted order every time
 *   rick_plan_retarget, rick_grid_jobs, rick_wstack_image_jobs,
 *   rick_capture_begin/_end,
 *   rick_graph_launch/_destroy, rick_stamps_create/_stamp/_elapsed/_destroy,
 *   rick_autotune
 *                      many jobs: one plan per shape retargeted per job, the
 *                      gridding of many jobs in one persistent launch and
 *                      their column passes in one launch per grid size, work
 *                      recorded into a graph and replayed, device timestamps,
 *                      tile and chunk chosen by measurement
 *
 * Conventions shared by every call:
 *   - All entry points return a rick_status; no exception, abort or exit
 *     crosses the ABI.  Arguments are validated on the host before any
 *     device work is queued.  A launch failure returns RICK_E_HIP; a fault
 *     inside a kernel surfaces at the caller's next synchronisation.
 *   - Device pointers are HIP device (or managed) addresses on the plan's
 *     device.  Host pointers are ordinary process memory.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - A plan is used by one host thread and one stream at a time; distinct
 *     plans are independent.
 *   - The plan owns every device buffer it allocates; rick_plan allocates
 *     them all once, and the calls on a plan allocate nothing.  The calls
 *     that create other objects (rick_degrid_order_create, rick_capture_end,
 *     rick_stamps_create) and rick_autotune (trial plans) allocate, and say
 *     so.
 *
 * Coordinates (the paper leaves them implicit; these are this library's):
 *   cell i of the N-cell axis sits at u_i = (i - N/2) du, du = 1 / FoV;
 *   pixel p sits at l_p = (p - N/2) dl, dl = FoV / N; the mesh and the
 *   image are row-major with rows along v (resp. m) and columns along u
 *   (resp. l); the image is Re of the plane sum times n = sqrt(1 - l^2 - m^2)
 *   divided by the sum of gridded weights and by the kernel taper
 *   C(l') C(m'); pixels with l^2 + m^2 >= 1 are 0.
 */
#ifndef RICK_H
#define RICK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rick_status;

enum {
    RICK_OK = 0,
    RICK_E_INVALID_ARG = 1,   /* bad pointer, size, alignment or plan parameter */
    RICK_E_NO_DEVICE = 2,     /* no HIP device, or the requested ordinal does not exist */
    RICK_E_OOM = 3,           /* the plan's buffers do not fit the device's free memory */
    RICK_E_HIP = 4,           /* a HIP runtime call or kernel launch failed */
    RICK_E_CAPACITY = 5,      /* nrow * nchan exceeds the plan's max_vis */
    RICK_E_BAD_PLAN = 6,      /* NULL or destroyed plan handle */
    RICK_E_STATE = 7,         /* call out of order (e.g. rick_wstack_image before rick_fft_planes) */
    RICK_E_UNSUPPORTED = 8    /* valid but not built (e.g. a grid size without an FFT kernel) */
};

enum {
    RICK_KERNEL_GAUSSIAN = 0,
    RICK_KERNEL_KAISER_BESSEL = 1,
    RICK_KERNEL_USER_LUT = 2   /* a non-separable table T[lut_wbins][OS][OS][W][W] installed with rick_plan_set_lut */
};

enum {
    RICK_PREC_FP32 = 0,        /* float mesh, FFT and plane sum; float64 phase argument and normalisation;
                                  gridding sums each cell as integers (terms rounded at 2^-21 of the
                                  largest possible term of their bin) */
    RICK_PREC_FP32_KAHAN = 1,  /* as FP32, compensated (Kahan) summation over w-planes */
    RICK_PREC_FP64 = 2         /* every step in float64 (complex128 mesh) */
};

enum {
    RICK_FLAG_TIMING = 1,       /* record per-kernel HIP events; read them with rick_plan_info */
    RICK_FLAG_FUSED_SCREEN = 2, /* rick_fft_planes transforms rows only, into a second buffer (row_mesh,
                                   in column-panel order); rick_wstack_image transforms the columns plane by
                                   plane and screens and sums them in the same pass, so F_k is never
                                   written to HBM.  The mesh keeps G_k.  Needs a second mesh-sized buffer. */
    RICK_FLAG_PLANE_ORIENT = 4  /* with RICK_FLAG_FUSED_SCREEN (not with RICK_KERNEL_USER_LUT): the first
                                   rick_grid after a reset stores a plane transposed (cell (y, x) of G_k at
                                   row x, column y) when its visibilities reach fewer tile columns than tile
                                   rows, so that the row pass of rick_fft_planes transforms the fewer lines;
                                   rick_wstack_image then takes such planes in a second column pass whose
                                   strips are image rows.  tile_bits, the row transforms and the mesh
                                   follow the stored orientation (rick_plan_info_t.plane_transposed).
                                   The image is the same up to float rounding. */
};

/* Plan parameters (Sec. 2.1: mesh N_u x N_v x N_w, kernel type and support). */
typedef struct rick_plan_desc {
    int32_t grid_n;        /* N = N_u = N_v: power of two, 64..16384 (16384: without RICK_FLAG_FUSED_SCREEN) */
    int32_t n_wplanes;     /* N_w >= 1 */
    int32_t support;       /* kernel support W in cells: odd, 1..15 */
    int32_t oversample;    /* OS sub-cell positions per cell: power of two, 1..256 */
    int32_t kernel;        /* RICK_KERNEL_* */
    int32_t precision;     /* RICK_PREC_* */
    double kernel_param;   /* Gaussian sigma in cells, or Kaiser-Bessel beta; <= 0 selects the default
                              (sigma with g(W/2) = 1e-3; beta of Beatty et al. 2005 at alpha = 2) */
    double fov_rad;        /* field of view FoV: 0 < FoV and FoV^2 / 2 < 1 (image corners inside the sky) */
    double w_min, w_max;   /* w range in wavelengths covered by the planes; w_max > w_min.  Plane k
                              spans [w_min + k dw, w_min + (k+1) dw), dw = (w_max - w_min) / N_w, with
                              centre w_k; w outside the range goes to the nearest end plane. */
    int64_t max_vis;       /* largest nrow * nchan one rick_grid call accepts; 0..2^29.  0: the plan
                              allocates no per-visibility sort buffers and grids only through
                              rick_grid_static */
    int32_t device;        /* HIP device ordinal */
    int32_t flags;         /* RICK_FLAG_* */
    int32_t tile;          /* uv tile edge T in cells for binning and gridding: 0 = default (64), else a
                              power of two 16..64 with T >= W */
    int32_t chunk;         /* largest number of binned records one gridding block takes: 0 = default */
    int32_t lut_wbins;     /* RICK_KERNEL_USER_LUT: w-fraction bins N_f of the table, 1, 2, 4 or 8 (ignored
                              otherwise) */
} rick_plan_desc;

typedef struct rick_plan_s rick_plan_t;   /* opaque plan handle */

/* Counters and layout of a plan (read back synchronously). */
typedef struct rick_plan_info_t {
    int64_t n_gridded;       /* visibilities gridded since the last reset */
    int64_t n_dropped;       /* visibilities dropped since the last reset (non-finite input, weight <= 0,
                                kernel footprint leaving the mesh) */
    int64_t n_records;       /* binned records written by the last rick_grid: one per gridded visibility,
                                in the tile holding the top-left cell of its footprint */
    double sum_weights;      /* sum of the weights of gridded visibilities since the last reset */
    double du, dl, dw;       /* cell size [wavelengths], pixel size [rad], plane width [wavelengths] */
    void *mesh;              /* device pointer to the planes, [N_w][N][N] complex64 (complex128 in FP64
                                mode), interleaved (re, im): G_k after rick_grid, F_k after rick_fft_planes
                                (with RICK_FLAG_FUSED_SCREEN it keeps G_k).  G_k is held only in the tiles
                                set in tile_bits; every other tile holds stale values and stands for zeros
                                (F_k is complete) */
    int64_t mesh_bytes;
    void *row_mesh;          /* with RICK_FLAG_FUSED_SCREEN (else NULL): the row transforms H_k written by
                                rick_fft_planes, mesh_bytes long, in column-panel order: element (plane k,
                                row q, column p) at k N^2 + (p / panel) N panel + q panel + p % panel.
                                Rows of a tile row with no set tile are not written and stand for zeros */
    int32_t panel;           /* columns per panel of row_mesh (0 without RICK_FLAG_FUSED_SCREEN) */
    int32_t occ_words;       /* 64-bit words of tile_bits per tile row: ceil(N / tile / 64) */
    const uint64_t *tile_bits; /* device bitmap of the tiles gridded onto since the last reset: tile (plane
                                k, tile row ty, tile column tx) is set iff bit tx % 64 of word
                                (k N / tile + ty) occ_words + tx / 64 is */
    int64_t tiles_set;       /* tiles set in tile_bits */
    int64_t tile_rows_set;   /* tile rows (plane, ty) with at least one set tile */
    int32_t rec1_bytes;      /* bytes of a first-level binning record (12, 16 or 24) */
    int32_t pad1;
    int32_t tile, chunk;     /* effective tile edge and chunk size */
    int32_t state;           /* 0 = empty, 1 = gridded, 2 = transformed, 3 = predicted planes */
    int32_t n_timers;        /* number of valid entries in kernel_ms / kernel_calls / kernel_names */
    float kernel_ms[16];     /* with RICK_FLAG_TIMING: mean device time per launch of each kernel over the
                                launches since the previous rick_plan_info (the last 64 at most) */
    int32_t kernel_calls[16];/* launches the mean covers */
    const char *kernel_names[16];
    const double *w_k;       /* HOST [N_w]: plane centres w_k = w_min + (k + 1/2) dw, owned by the plan */
    const double *taper;     /* device: the taper the image is divided by, C(l') [N] for a separable kernel
                                (pixel (q, p) divided by C[p] C[q]), or [N][N] for a user table */
    int32_t lut_wbins;       /* w-fraction bins of the installed user table (0 for a separable kernel) */
    int32_t pad2;
    const int32_t *plane_transposed; /* device [N_w] with RICK_FLAG_PLANE_ORIENT (else NULL): 1 if plane k
                                is stored transposed (tile_bits, mesh and row_mesh then hold G_k^T and its
                                row transforms), 0 if not */
} rick_plan_info_t;

/*
 * rick_plan -- validate `d`, build the kernel tap table, the taper C(l'),
 * the plane centres w_k and the FFT twiddles in float64 on the host, and
 * allocate every device buffer the plan needs (mesh, binning scratch,
 * tables) once.  Device memory is checked against hipMemGetInfo first.
 * On success *out receives the plan; on failure *out is NULL.
 * Errors: RICK_E_INVALID_ARG, RICK_E_NO_DEVICE, RICK_E_OOM, RICK_E_HIP,
 * RICK_E_UNSUPPORTED.
 */
rick_status rick_plan(const rick_plan_desc *d, rick_plan_t **out);

/*
 * rick_grid -- map visibilities to the closest w-plane and convolve them onto
 * the mesh (Sec. 2.1, Eq. 3), accumulating onto what earlier rick_grid calls
 * since the last reset gridded (frequency or time chunks, Sec. 2.2).
 *   uvw      device, float64 [nrow][3]: metres if freq_hz != NULL, else wavelengths
 *   freq_hz  HOST, float64 [nchan] channel frequencies, or NULL (then nchan must be 1)
 *   vis      device, complex64 [nrow][nchan] interleaved (re, im) (complex128 in FP64 mode)
 *   weight   device, float32 [nrow][nchan], or NULL for unit weights
 * u [wavelengths] = uvw[r][0] * freq_hz[c] / c0, c0 = 299792458 m/s, and
 * likewise v, w.  Position quantised to 1/OS cell, nearest cell, plane by
 * floor((w - w_min) / dw) clamped; a visibility is dropped (counted, not an
 * error) if any input is non-finite, its weight is <= 0 or its W x W
 * footprint leaves the mesh.  uvw and vis must be 8-byte (16-byte in FP64
 * mode) aligned.  Inputs must stay alive until `stream` reaches this work.
 * Errors: RICK_E_BAD_PLAN, RICK_E_INVALID_ARG (NULL pointer, nrow < 0,
 * nchan < 1, nchan > 1 without freq_hz, misalignment, non-finite or
 * non-positive frequency), RICK_E_CAPACITY, RICK_E_STATE (after
 * rick_fft_planes without a reset), RICK_E_HIP.
 */
rick_status rick_grid(rick_plan_t *p, const double *uvw, const double *freq_hz, const void *vis,
                      const float *weight, int64_t nrow, int32_t nchan, void *stream);

/*
 * rick_grid_static -- rick_grid for callers that cannot allocate device
 * memory (work recorded into a graph, tight serving loops, hosts that forbid
 * hipMalloc).  Same arguments, result and errors as rick_grid, but the
 * buffers of bin-and-sort that grow with the number of visibilities (level-1
 * and gridding records, chunk tables, work items) live in the library's
 * static device scratch of RICK_STATIC_SCRATCH_BYTES (256 MiB) per device,
 * allocated when the library's device code is loaded and held until the
 * process ends, instead of in the plan; the plan's max_vis does not apply
 * (a plan made with max_vis = 0 holds no such buffers).  This call allocates
 * nothing, host or device.
 *   - nrow * nchan is limited by the scratch: about 9.5 M visibilities in
 *     FP32 modes and 6 M in FP64 (28 and 44 bytes per visibility plus
 *     per-chunk tables); a larger call returns RICK_E_CAPACITY before any
 *     device work.
 *   - Every call on one device shares that device's scratch, and the scratch
 *     keeps the last call's contents (nothing in it needs to start at zero).
 *     Calls whose device work overlaps on one device -- on different streams,
 *     from different threads, or on different plans -- race on the scratch
 *     and give wrong results: order them on one stream or synchronise between
 *     them.  rick_grid is unaffected (its buffers are the plan's).
 * Errors: as rick_grid, and RICK_E_HIP if the scratch's address could not be
 * taken on this device.
 */
#define RICK_STATIC_SCRATCH_BYTES (256ull << 20)
rick_status rick_grid_static(rick_plan_t *p, const double *uvw, const double *freq_hz, const void *vis,
                             const float *weight, int64_t nrow, int32_t nchan, void *stream);

/*
 * rick_grid_jobs -- rick_grid for several independent imaging jobs at once,
 * each on its own plan: the gridding of Sec. 2.1 (Eq. 3) for a batch of
 * jobs of uneven grid size and visibility count.  The result on every plan
 * is that of rick_grid with the job's arguments (planes equal up to the
 * order of float additions where a bin spans several gridding chunks).  Each
 * job is binned on its own plan's buffers; then the gridding work items of
 * all jobs form one device-side queue taken by ONE persistent launch per
 * (kernel support, uv tile edge) among the jobs: a block claims items from a
 * shared counter and grids each with its job's plan, so small jobs do not
 * leave the device idle between launches.  Everything runs on `stream`, in
 * job order for the binning; nothing is allocated (may be recorded into a
 * graph).
 *   jobs   HOST array of n job descriptors (plan and the arguments of
 *          rick_grid, same meaning, layout and lifetime rules); the array
 *          itself may be freed when the call returns
 *   n      1 ... RICK_MAX_GRID_JOBS
 * Every plan must be a different one, on one device, all in float32 modes
 * or all in FP64 mode, with a separable kernel (not RICK_KERNEL_USER_LUT).
 * All arguments are checked before any device work.
 * Errors: RICK_E_INVALID_ARG (NULL jobs, n out of range, a plan given twice,
 * plans on different devices or of different precisions, a job's arguments
 * as for rick_grid), RICK_E_BAD_PLAN, RICK_E_UNSUPPORTED (a user table),
 * RICK_E_CAPACITY, RICK_E_STATE (as for rick_grid), RICK_E_HIP.
 */
#define RICK_MAX_GRID_JOBS 64
typedef struct rick_grid_job {
    rick_plan_t *plan;
    const double *uvw;
    const double *freq_hz;
    const void *vis;
    const float *weight;
    int64_t nrow;
    int32_t nchan;
    int32_t reserved; /* set to 0 */
} rick_grid_job;
rick_status rick_grid_jobs(const rick_grid_job *jobs, int32_t n, void *stream);

/*
 * rick_fft_planes -- in place, every plane becomes its centred inverse DFT
 * (the FFT step of Sec. 2.1):
 *   F_k[q][p] = sum_{j,i} G_k[j][i] exp(+2 pi i ((i - N/2)(p - N/2) + (j - N/2)(q - N/2)) / N)
 * (unnormalised).  With RICK_FLAG_FUSED_SCREEN only the sum over i (the row
 * transform) is done here, into row_mesh (see rick_plan_info_t; the mesh
 * keeps G_k), and the sum over j happens in rick_wstack_image.  Tiles that
 * nothing was gridded onto since the reset are taken as zeros without being
 * read (a plan with nothing gridded transforms to zeros).
 * Errors: RICK_E_BAD_PLAN, RICK_E_STATE, RICK_E_HIP.
 */
rick_status rick_fft_planes(rick_plan_t *p, void *stream);

/*
 * rick_wstack_image -- w-correction and plane reduction (Sec. 2.1, Eq. 1):
 *   I[q][p] = n_pq sum_k Re(exp(+2 pi i w_k (n_pq - 1)) F_k[q][p]) / (C(l'_p) C(l'_q) sum W)
 * with n - 1 formed as -r^2 / (1 + sqrt(1 - r^2)) in float64, the phase
 * w_k (n - 1) formed and range-reduced in float64, and the sum over planes
 * in the plan's precision.  `image` is device float32 [N][N] (float64 in FP64
 * mode), owned by the caller.  May be called again on the same planes.
 * Errors: RICK_E_BAD_PLAN, RICK_E_INVALID_ARG (NULL image), RICK_E_STATE
 * (planes not transformed), RICK_E_HIP.
 */
rick_status rick_wstack_image(rick_plan_t *p, void *image, void *stream);

/*
 * rick_wstack_image_jobs -- rick_wstack_image for several plans made with
 * RICK_FLAG_FUSED_SCREEN at once (the w-correction and plane sum of
 * Sec. 2.1, Eq. 1-2, of a batch of jobs): every image is the one
 * rick_wstack_image would write for its plan, bit for bit.  The fused
 * column pass of all plans of one grid size (and one precision mode) is
 * ONE launch over their column strips together, so that small grids, whose
 * own pass has few strips, fill the device.  Runs on `stream`; allocates
 * nothing (may be recorded into a graph).
 *   jobs   HOST array of n {plan, image} pairs (image: device, as for
 *          rick_wstack_image); the array may be freed when the call returns
 *   n      1 ... RICK_MAX_GRID_JOBS
 * Every plan must be a different one, fused, after rick_fft_planes, on one
 * device, all in float32 modes or all in FP64 mode.  All arguments are
 * checked before any device work.
 * Errors: RICK_E_INVALID_ARG (NULL jobs or image, n out of range, a plan
 * given twice, a plan without the fused screen, misalignment, mixed devices
 * or precisions), RICK_E_BAD_PLAN, RICK_E_STATE (planes not transformed),
 * RICK_E_HIP.
 */
typedef struct rick_image_job {
    rick_plan_t *plan;
    void *image;
} rick_image_job;
rick_status rick_wstack_image_jobs(const rick_image_job *jobs, int32_t n, void *stream);

/*
 * rick_predict_planes -- the first half of prediction (degridding): the
 * visibility model of Eq. 2 discretised by w-stacking, Sec. 2.1 run the other
 * way.  For every plane k of the plan's w range, the mesh receives the
 * centred forward DFT H_k of the plane image
 *   P_k[q][p] = M[q][p] exp(-2 pi i w_k (n_pq - 1)) / (n_pq C(l'_p) C(l'_q))
 *   H_k[j][i] = sum_{q,p} P_k[q][p] exp(-2 pi i ((i - N/2)(p - N/2) + (j - N/2)(q - N/2)) / N)
 * (zero outside the unit circle; phase and n - 1 in float64 as in
 * rick_wstack_image).  The forward DFT runs as the inverse DFT of the
 * conjugate, so conj(H_k) is what is held afterwards: in the mesh, or with
 * RICK_FLAG_FUSED_SCREEN in row_mesh in column-panel order (the mesh then
 * holds conj(P_k)); every tile is marked set.
 *   model  device float32 [N][N] (float64 in FP64 mode), indexed [q = m][p = l],
 *          the sky brightness per pixel; read only, owned by the caller
 * Overwrites what was gridded; call rick_reset before gridding again.
 * Errors: RICK_E_BAD_PLAN, RICK_E_INVALID_ARG (NULL or misaligned model), RICK_E_HIP.
 */
rick_status rick_predict_planes(rick_plan_t *p, const void *model, void *stream);

/*
 * rick_degrid -- the second half of prediction: every visibility is
 * interpolated from its closest plane with the gridding kernel's tap table
 * (Eq. 3 read backwards),
 *   V = sum_{t_y, t_x} g_{s_y}[t_y] g_{s_x}[t_x] H_k[c_y + t_y - h][c_x + t_x - h],
 * with cell, sub-cell offset, plane and drop decision exactly those of
 * rick_grid (a visibility rick_grid would drop for its position is predicted
 * as 0), so that prediction is the adjoint of the imaging steps.
 *   uvw      device, float64 [nrow][3]: metres if freq_hz != NULL, else wavelengths
 *   freq_hz  HOST, float64 [nchan] channel frequencies, or NULL (then nchan must be 1)
 *   vis_out  device complex [nrow][nchan] (interleaved float32 re, im; float64 in
 *            FP64 mode), written completely; owned by the caller
 * May be called any number of times on the same predicted planes.  Not
 * limited by max_vis.
 * Errors: RICK_E_BAD_PLAN, RICK_E_INVALID_ARG, RICK_E_STATE (no
 * rick_predict_planes since the last reset or gridding), RICK_E_HIP.
 */
rick_status rick_degrid(rick_plan_t *p, const double *uvw, const double *freq_hz, void *vis_out, int64_t nrow,
                        int32_t nchan, void *stream);

/*
 * Prediction at fixed positions (the same observation predicted again and
 * again, e.g. every cycle of a deconvolution): the positions are quantised
 * and sorted once by the offset of their footprint origin in the layout the
 * plan holds predicted planes in (plane, then row and column: row order, or
 * column panels with RICK_FLAG_FUSED_SCREEN), down to groups of PW x 8 cells
 * (a panel's width by 8 rows; 8 x 1 in row order) whose visibilities keep
 * their own order, so that neighbouring threads of rick_degrid_sorted read
 * neighbouring footprints and write neighbouring results where they can.
 *
 * rick_degrid_order_create -- quantise (exactly as rick_grid and rick_degrid
 * do, for the plan's current grid, field and w range) and sort (the
 * library's stable LSD radix sort, one pass per 8 bits of the key width).
 * uvw and freq_hz as for rick_degrid; nrow * nchan < 2^31.  Allocates device
 * memory (16 B per visibility kept, 32 B per visibility plus the sort's
 * scratch, about 0.5 B per visibility, during the call) and synchronises
 * `stream`.  *out receives the handle.
 * Errors: RICK_E_BAD_PLAN, RICK_E_INVALID_ARG, RICK_E_OOM, RICK_E_HIP.
 */
typedef struct rick_degrid_order_s rick_degrid_order_t;
rick_status rick_degrid_order_create(rick_plan_t *p, const double *uvw, const double *freq_hz, int64_t nrow,
                                     int32_t nchan, rick_degrid_order_t **out, void *stream);

/*
 * rick_degrid_sorted -- rick_degrid over the order's visibilities, walked in
 * sorted order; vis_out [nrow][nchan] as for rick_degrid (each visibility
 * written at its own index).  The plan must hold predicted planes and have
 * the grid, field, w range and plane layout the order was made with.
 * Errors: RICK_E_BAD_PLAN, RICK_E_INVALID_ARG (bad order, other geometry,
 * NULL or misaligned vis_out), RICK_E_STATE, RICK_E_HIP.
 */
rick_status rick_degrid_sorted(rick_plan_t *p, const rick_degrid_order_t *o, void *vis_out, void *stream);

/* rick_degrid_order_destroy -- free the order.  Errors: RICK_E_INVALID_ARG. */
rick_status rick_degrid_order_destroy(rick_degrid_order_t *o);

/*
 * rick_degrid_order_info -- the order's sorted arrays, device memory owned by
 * the order (valid until rick_degrid_order_destroy), n = nrow * nchan
 * entries each, ascending by key:
 *   keys[j]  the footprint origin (c_x - h, c_y - h) of the visibility as an
 *            offset in the planes' layout, plane k times N^2 plus j N + i in
 *            row order (panel == 0) or (i / panel) N panel + j panel + i % panel
 *            in column panels; all ones for a dropped visibility;
 *   vals[j]  its index r * nchan + c in bits 0-31, s_x + OS/2 in bits 32-39,
 *            s_y + OS/2 in bits 40-47.
 * These are the decisions of Sec. 2.1's discretisation that rick_grid takes
 * for the same positions (quant.h): cell, sub-cell offset, plane and drop.
 * Errors: RICK_E_INVALID_ARG (bad order, NULL out).
 */
typedef struct rick_degrid_order_info_t {
    const uint64_t *keys;
    const uint64_t *vals;
    int64_t n;
    int32_t panel;
    int32_t pad;
} rick_degrid_order_info_t;
rick_status rick_degrid_order_info(const rick_degrid_order_t *o, rick_degrid_order_info_t *out);

/*
 * rick_reset -- begin a new image: zero the weight sum and the counters and
 * clear the tile bitmap, so the next rick_grid stores its tiles instead of
 * adding to them and every other tile reads as zero.
 * Errors: RICK_E_BAD_PLAN, RICK_E_HIP.
 */
rick_status rick_reset(rick_plan_t *p, void *stream);

/*
 * rick_plan_retarget -- give the plan another field of view and w range
 * (fov_rad, w_min, w_max as in rick_plan_desc) for the work issued after this
 * call: the cell size, pixel size and plane centres follow; the grid size,
 * planes, kernel, precision and buffers stay.  Host-side only (no device work),
 * so it may be called while recording a graph: each recorded job keeps the
 * field it was recorded with.  Call rick_reset before gridding a new field.
 * Errors: RICK_E_BAD_PLAN, RICK_E_INVALID_ARG (as for rick_plan).
 */
rick_status rick_plan_retarget(rick_plan_t *p, double fov_rad, double w_min, double w_max);

/*
 * rick_plan_info -- fill *out.  Synchronises the plan's device (it copies
 * counters back), so call it outside timed regions.
 * Errors: RICK_E_BAD_PLAN, RICK_E_INVALID_ARG (NULL out), RICK_E_HIP.
 */
rick_status rick_plan_info(rick_plan_t *p, rick_plan_info_t *out);

/*
 * rick_plan_destroy -- free every buffer of the plan.  The caller must have
 * synchronised the streams that used it.  Destroying NULL returns
 * RICK_E_BAD_PLAN; the handle is invalid afterwards.
 */
rick_status rick_plan_destroy(rick_plan_t *p);

/*
 * rick_plan_bin_counts -- copy the per-bin record counts of the last
 * rick_grid to HOST memory `counts` [n], n = N_w * (N/T)^2, bin index
 * (k * (N/T) + tile_row) * (N/T) + tile_col.  A gridded visibility adds
 * one record, to the tile holding the top-left cell of its W x W footprint.
 * Synchronises the device.
 * Errors: RICK_E_BAD_PLAN, RICK_E_INVALID_ARG (NULL counts, wrong n), RICK_E_HIP.
 */
rick_status rick_plan_bin_counts(rick_plan_t *p, int32_t *counts, int64_t n);

/*
 * Batches of imaging jobs (Sec. 2.2 processes the data in independent
 * chunks; here many independent jobs are recorded once and replayed).
 *
 * rick_capture_begin -- start recording the work the library (and anything
 * else) issues on `stream` into a graph instead of running it: rick_reset,
 * rick_grid, rick_fft_planes, rick_wstack_image, rick_predict_planes,
 * rick_degrid, rick_degrid_sorted and rick_stamp on any plans, each with the
 * same stream.  None of them allocates or synchronises, so a whole sequence
 * of jobs can be recorded.  rick_plan_info, rick_plan_bin_counts,
 * rick_autotune, rick_degrid_order_create and plan creation synchronise and
 * must not be called while recording.
 * rick_capture_end -- stop recording and instantiate the graph; *out
 * receives it (NULL on failure).
 * rick_graph_launch -- run the recorded work once on `stream` (asynchronous;
 * may be launched again: every launch redoes the recorded work with the
 * buffers as they are then).  The plans, inputs and outputs used while
 * recording must stay alive while the graph is used.
 * rick_graph_destroy -- free the graph (after its launches completed).
 * Errors: RICK_E_INVALID_ARG (NULL stream handle pointer or graph), RICK_E_HIP.
 */
typedef struct rick_graph_s rick_graph_t;
rick_status rick_capture_begin(void *stream);
rick_status rick_capture_end(void *stream, rick_graph_t **out);
rick_status rick_graph_launch(rick_graph_t *g, void *stream);
rick_status rick_graph_destroy(rick_graph_t *g);

/*
 * Device timestamps for per-job latencies inside a graph.
 * rick_stamps_create -- n timestamp slots (allocates 8 n bytes of device
 * memory, zeroed; synchronises the device); rick_stamp -- a one-thread kernel
 * on `stream` writes the device's constant-rate clock into slot i when the
 * preceding work on the stream has finished (may be recorded into a graph);
 * rick_stamps_elapsed -- synchronise the device and give, in *ms, the time
 * from slot i to slot j of their last writes; rick_stamps_destroy.
 * Errors: RICK_E_INVALID_ARG (n < 1, index out of range, NULL pointer), RICK_E_HIP.
 */
typedef struct rick_stamps_s rick_stamps_t;
rick_status rick_stamps_create(int32_t n, rick_stamps_t **out);
rick_status rick_stamp(rick_stamps_t *t, int32_t i, void *stream);
rick_status rick_stamps_elapsed(rick_stamps_t *t, int32_t i, int32_t j, float *ms);
rick_status rick_stamps_destroy(rick_stamps_t *t);

/*
 * rick_autotune -- pick the uv tile edge and gridding chunk for plan
 * parameters `d` and one job's inputs (same meaning as rick_grid): each
 * candidate (tile 16, 32 or 64 where it holds the footprint and fits LDS;
 * chunk 2048, 8192 or 32768 records) gets a plan of its own, one untimed and
 * two timed runs of reset + grid + fft + image on `stream`, and is freed;
 * *tile, *chunk receive the fastest and *ms its time per run.  Synchronises;
 * needs memory for one plan of `d` at a time.  d->tile and d->chunk are
 * ignored.
 * Errors: as rick_plan and rick_grid; RICK_E_INVALID_ARG (NULL outputs).
 */
rick_status rick_autotune(const rick_plan_desc *d, const double *uvw, const double *freq_hz, const void *vis,
                          const float *weight, int64_t nrow, int32_t nchan, void *stream, int32_t *tile,
                          int32_t *chunk, float *ms);

/* Static message for a status code (never NULL). */
/*
 * Learned gridding kernel.  The paper convolves with a Gaussian or
 * Kaiser-Bessel kernel (Sec. 2.1, Eq. 3); these calls let a kernel be learned
 * instead and used through a plan with kernel = RICK_KERNEL_USER_LUT:
 *   - the kernel is a table T[iw][s_y + OS/2][s_x + OS/2][t_y][t_x] (float32,
 *     row-major) of the tap at cell offset (t_x - h - s_x / OS, t_y - h - s_y / OS)
 *     for a visibility whose w-fraction bin is iw: with r = (w - w_min) / dw and
 *     plane k = clamp(floor(r), 0, N_w - 1), iw = clamp(floor((r - k) N_f), 0, N_f - 1);
 *   - the image is divided by the table's 2-D taper C(l', m') = (1 / (N_f OS^2))
 *     sum over every entry of T cos(2 pi (dx l' + dy m')), computed on the device
 *     when the table is installed.
 * A 3 -> 32 -> 32 -> 1 MLP (tanh after both hidden layers, linear output)
 * tabulates such a table, K = exp(mlp(dx / (W/2), dy / (W/2), f_iw)) inside
 * |dx|, |dy| < W/2 (0 outside), f_iw = (iw + 1/2) / N_f - 1/2, each
 * (iw, s_y, s_x) row normalised to sum 1.  Its RICK_MLP_PARAMS float32
 * parameters are packed W1 [32][3], b1 [32], W2 [32][32], b2 [32], w3 [32], b3.
 * Training against the direct Fourier sum (Eq. 1) chains rick_image_loss,
 * rick_table_gradient (the adjoint of the imaging steps: a degridding of the
 * loss gradient) and rick_mlp_backward, then rick_adam_step.
 */
#define RICK_MLP_PARAMS 1217

/* rick_plan_set_lut -- install the table (host or device float32, N_f OS^2 W^2
 * values, every entry finite) into a RICK_KERNEL_USER_LUT plan and compute its
 * taper; a host table is copied before the call returns, a device table is
 * read on `stream`.  The plan grids with it from then on.
 * Errors: RICK_E_BAD_PLAN, RICK_E_STATE (not a user-table plan),
 * RICK_E_INVALID_ARG (NULL, misaligned, non-finite host entry), RICK_E_HIP. */
rick_status rick_plan_set_lut(rick_plan_t *p, const float *table, int32_t on_device, void *stream);

/* rick_mlp_tabulate -- table [n_wbins][OS][OS][W][W] (device float32) of the MLP
 * with parameters theta (device float32 [RICK_MLP_PARAMS]), on the current
 * device.  Errors: RICK_E_INVALID_ARG (shape as in rick_plan_desc, NULL,
 * misaligned), RICK_E_HIP. */
rick_status rick_mlp_tabulate(const float *theta, int32_t support, int32_t oversample, int32_t n_wbins,
                              float *table, void *stream);

/* rick_mlp_backward -- dtheta (device float32 [RICK_MLP_PARAMS], overwritten) =
 * gradient of sum(dtable T) with respect to theta, T the table rick_mlp_tabulate
 * made from theta (device, same shape) and dtable device float64 of that shape
 * (through the row normalisation, exp and the MLP).  Errors as rick_mlp_tabulate. */
rick_status rick_mlp_backward(const float *theta, int32_t support, int32_t oversample, int32_t n_wbins,
                              const float *table, const double *dtable, float *dtheta, void *stream);

/* rick_adam_step -- one Adam update (Kingma & Ba 2015, Algorithm 1: bias-corrected
 * moments, theta -= lr m_hat / (sqrt(v_hat) + eps)) of theta [n] with gradient
 * grad and moment buffers m, v (device float32, m and v zero before step 1);
 * step counts from 1.  Errors: RICK_E_INVALID_ARG, RICK_E_HIP. */
rick_status rick_adam_step(float *theta, const float *grad, float *m, float *v, int32_t n, int32_t step, float lr,
                           float beta1, float beta2, float eps, void *stream);

/* rick_image_loss -- for the plan's image I (device [N][N], plan's real type) and
 * a target D (device float64 [N][N], the direct sum): sums[0] = sum_Omega (I - D)^2,
 * sums[1] = sum_Omega D^2 over Omega = {|q - N/2| < N/4, |p - N/2| < N/4} (the loss
 * is sums[0] / sums[1]); dimage = dL/dA for the apparent image A = I C and
 * dtaper = dL/dC (device float64 [N][N], zero outside Omega), C the plan's taper.
 * Errors: RICK_E_BAD_PLAN, RICK_E_INVALID_ARG, RICK_E_HIP. */
rick_status rick_image_loss(rick_plan_t *p, const void *image, const double *target, double *dimage,
                            double *dtaper, double *sums, void *stream);

/* rick_table_gradient -- dtable (device float64, N_f OS^2 W^2, overwritten) =
 * dL/dT for a RICK_KERNEL_USER_LUT plan that has just gridded (rick_grid) and
 * transformed (rick_fft_planes) exactly these visibilities, given dimage and
 * dtaper from rick_image_loss: the planes dA n exp(-2 pi i w_k (n - 1)) / sum W
 * go through the centred forward transform (the adjoint of imaging, as in
 * prediction), each visibility adds Re(dL/dG_k[cell] conj(W V)) to the entries
 * its taps read, and the taper's dependence on T is added.  The mesh is used
 * as scratch: the plan needs rick_reset afterwards.
 * Errors: RICK_E_BAD_PLAN, RICK_E_STATE (not a user-table plan, or its planes
 * not transformed), RICK_E_INVALID_ARG, RICK_E_HIP. */
rick_status rick_table_gradient(rick_plan_t *p, const double *dimage, const double *dtaper, const double *uvw,
                                const double *freq_hz, const void *vis, const float *weight, int64_t nrow,
                                int32_t nchan, double *dtable, void *stream);

/* rick_dft_image -- the direct Fourier sum (Eq. 1 over the measured samples)
 * at the pixels q0 <= q < q0 + nq, p0 <= p < p0 + np of the plan's image:
 *   out[q - q0][p - p0] = n Re(sum W V exp(+2 pi i (u l_p + v m_q + w (n - 1)))) / sum W
 * over the visibilities the plan keeps (its drop rule; inputs as rick_grid),
 * exact (unquantised) u, v, w; phase and sums in float64, sin and cos of the
 * phase reduced to half a turn in float32 (about 2.5e-7 per term).  out:
 * device float64 [nq][np]; at most 65535 * 16384 visibilities per call.  The
 * plan's state is unchanged.  Errors: RICK_E_BAD_PLAN, RICK_E_INVALID_ARG,
 * RICK_E_CAPACITY, RICK_E_HIP. */
rick_status rick_dft_image(rick_plan_t *p, const double *uvw, const double *freq_hz, const void *vis,
                           const float *weight, int64_t nrow, int32_t nchan, int32_t q0, int32_t p0, int32_t nq,
                           int32_t np, double *out, void *stream);

/* rick_separable_table -- the plan's separable tap table (Gaussian or
 * Kaiser-Bessel) in the user-table layout: table[iw][s_y][s_x][t_y][t_x] =
 * g[s_y][t_y] g[s_x][t_x] for every iw < n_wbins (device float32).  For
 * comparing kernels at equal support and as a starting point for learning.
 * Errors: RICK_E_BAD_PLAN, RICK_E_STATE (a user-table plan), RICK_E_INVALID_ARG, RICK_E_HIP. */
rick_status rick_separable_table(rick_plan_t *p, int32_t n_wbins, float *table, void *stream);

/* rick_table_residual -- least-squares fit of a table to a target (device
 * float32, n entries each): dtable = 2 (table - target) / n (device float64) and
 * sums[0] = sum (table - target)^2 / n (device float64).  With
 * rick_mlp_backward it fits the MLP to a given table.
 * Errors: RICK_E_INVALID_ARG, RICK_E_HIP. */
rick_status rick_table_residual(const float *table, const float *target, int64_t n, double *dtable, double *sums,
                                void *stream);

const char *rick_status_str(rick_status s);

/* Detail of the last failing call on this host thread (static storage, never NULL). */
const char *rick_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RICK_H */
