"""GPU path (through the C ABI) against the float64 oracle, element by element.

Stage by stage on the tiny workload: integer binning (bit-exact), the gridded
planes G_k, the FFT of the GPU's own planes, the screen of the GPU's own
F_k, and the end-to-end image; then precision modes, kernels, supports,
oversampling, tile sizes, heavy-bin splitting, accumulation, edge cases.
Tolerances are relative RMS errors (||a - b|| / ||b||): per-stage FP32 1e-6;
end-to-end FP32 image 1e-5 on the apparent image (before the division by the
kernel taper, which both sides apply as the same float64 per-pixel scale) and
on the corrected image where the taper product C(l')C(m') >= 0.1; FP64 mode
1e-10 on the whole corrected image.  (Behind the split: the taper division
amplifies any float32 rounding by up to 1/C^2 at the image edge -- 6.4e3 for
the default Gaussian, unbounded for wide ones -- and a float32 numpy/scipy
pipeline shows the same whole-image errors.)
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import wstack as ow
from paper_2504_00959_amd import rick
from tests.helpers import image_errors, oracle_bin_counts, rel_rms, to_device

pytestmark = pytest.mark.gpu

FP32_IMG = 1e-5
FP32_STAGE = 1e-6
# gridded planes of the float32 modes: re and im are summed as 32-bit
# fixed-point halves of one word, each term rounded at 2^-21 of its bin's
# largest possible term
FP32_GRID = 5e-6
FP64_IMG = 1e-10


def run_gpu(ds, precision="fp32", **kw):
    """Grid, transform and image through the C ABI; with fused=True rick_fft_planes
    writes the row transforms only, into the column-panel buffer (returned as F)."""
    import torch
    uvw, vis, wt = to_device(ds, precision)
    p = rick.Plan.for_dataset(ds, precision=precision, **kw)
    p.reset()
    p.grid(uvw, vis, wt, ds.freq)
    torch.cuda.synchronize()
    G = p.mesh().cpu().numpy()
    info = p.info()
    nt = ds.grid_n // info["tile"]
    counts = p.bin_counts(ds.n_wplanes * nt * nt)
    p.fft()
    torch.cuda.synchronize()
    if p.fused:
        # the mesh keeps G_k; the row transforms went to the column-panel buffer
        assert np.array_equal(p.mesh().cpu().numpy(), G)
        F = p.row_mesh().cpu().numpy()
    else:
        F = p.mesh().cpu().numpy()
    img = p.image().double().cpu().numpy()
    torch.cuda.synchronize()
    p.close()
    return dict(G=G, F=F, img=img, info=info, counts=counts, precision=precision)


def oracle_of(ds, **over):
    return oracle.wstack.wstack_dataset(ds, **over)


def check_stages(ds, gpu, ref, stage_tol=FP32_STAGE, img_tol=FP32_IMG, fused=False):
    info = gpu["info"]
    b = ref.binned
    # integer decisions: exact
    assert info["n_gridded"] == int(b.keep.sum())
    assert info["n_dropped"] == int((~b.keep).sum())
    oc = oracle_bin_counts(b, ds.grid_n, ds.n_wplanes, ds.support, info["tile"])
    assert np.array_equal(gpu["counts"].astype(np.int64), oc)
    assert info["n_records"] == int(oc.sum())
    assert abs(info["sum_weights"] - ref.sum_w) <= 1e-12 * max(1.0, ref.sum_w)
    # gridded planes
    grid_tol = max(stage_tol, FP32_GRID) if gpu["precision"] in ("fp32", "fp32_kahan") else stage_tol
    assert rel_rms(gpu["G"], ref.planes) <= grid_tol
    G = gpu["G"].astype(np.complex128)
    if fused:
        # rows transformed only: H_k[j][p] = sum_i G_k[j][i] exp(+2 pi i (i - N/2)(p - N/2) / N)
        N = ds.grid_n
        H = np.fft.fftshift(np.fft.ifft(np.fft.ifftshift(G, axes=-1), axis=-1), axes=-1) * N
        assert rel_rms(gpu["F"], H) <= stage_tol
        F_own = ow.ifft_planes(G)
    else:
        # FFT of the GPU's own planes
        assert rel_rms(gpu["F"], ow.ifft_planes(G)) <= stage_tol
        F_own = gpu["F"].astype(np.complex128)
    # screen + normalisation of the GPU's own transformed planes
    S = ow.screen_sum(F_own, ref.w_k, ds.fov)
    mine = ow.normalise(S, ref.corr, ref.sum_w, ds.fov)
    assert rel_rms(gpu["img"] * np.outer(ref.corr, ref.corr), mine * np.outer(ref.corr, ref.corr)) <= stage_tol
    # end to end
    err = image_errors(gpu["img"], ref.image, ref.corr)
    assert err["apparent"] <= img_tol, err
    assert err["central"] <= img_tol, err
    return err


def test_tiny_stagewise_fp32():
    ds = synth.tiny()
    check_stages(ds, run_gpu(ds), oracle_of(ds))


@pytest.mark.parametrize("precision", ["fp32", "fp32_kahan"])
def test_tiny_fused_screen(precision):
    """Column transform fused with the screen: same image, F_k never written."""
    ds = synth.tiny()
    check_stages(ds, run_gpu(ds, precision=precision, fused=True), oracle_of(ds), fused=True)


@pytest.mark.parametrize("N", [64, 256, 1024, 4096, 8192])
def test_fused_screen_grid_sizes(N):
    ds = synth.tiny(nrow=5000, seed=16, grid_n=N, n_wplanes=3, uv_radius=120.0 * N / 256)
    check_stages(ds, run_gpu(ds, fused=True), oracle_of(ds), fused=True)


def test_fused_screen_fp64():
    ds = synth.tiny()
    gpu = run_gpu(ds, precision="fp64", fused=True)
    assert rel_rms(gpu["img"], oracle_of(ds).image) <= FP64_IMG


@pytest.mark.parametrize("N,fused", [(1024, False), (8192, False), (4096, True)])
def test_fp64_grid_sizes(N, fused):
    """All-float64 path at large meshes (the precision form's comparison run)."""
    ds = synth.tiny(nrow=5000, seed=17, grid_n=N, n_wplanes=2, uv_radius=120.0 * N / 256)
    if N == 8192:
        # a float64 column strip of 8192 does not fit in LDS beside its screen table
        with pytest.raises(rick.RickError, match="UNSUPPORTED"):
            rick.Plan.for_dataset(ds, precision="fp64", fused=True)
    gpu = run_gpu(ds, precision="fp64", fused=fused)
    ref = oracle_of(ds)
    assert rel_rms(gpu["G"], ref.planes) <= 1e-12
    assert rel_rms(gpu["img"], ref.image) <= FP64_IMG


def test_tiny_fp64_mode():
    ds = synth.tiny()
    gpu = run_gpu(ds, precision="fp64")
    ref = oracle_of(ds)
    assert rel_rms(gpu["G"], ref.planes) <= 1e-12
    assert rel_rms(gpu["img"], ref.image) <= FP64_IMG


def test_tiny_kahan():
    ds = synth.tiny()
    gpu = run_gpu(ds, precision="fp32_kahan")
    ref = oracle_of(ds)
    err = image_errors(gpu["img"], ref.image, ref.corr)
    assert err["apparent"] <= FP32_IMG and err["central"] <= FP32_IMG, err


def test_heavy_bins_split_over_chunks():
    """Small chunks force the dense central bins through the multi-chunk path."""
    ds = synth.tiny()
    gpu = run_gpu(ds, chunk=64)
    check_stages(ds, gpu, oracle_of(ds))


@pytest.mark.parametrize("grid_n,tile,n_wplanes", [(1024, 16, 8), (512, 16, 40)])
def test_binning_with_coarse_tiles(grid_n, tile, n_wplanes):
    """More (plane, tile) bins than one level of LDS counters holds: coarse
    tiles of several tiles (1024/16: 2 x 2; 512/16 with 40 planes: 4 x 4),
    with many footprints straddling coarse-tile edges."""
    ds = synth.tiny(nrow=40000, seed=21, grid_n=grid_n, n_wplanes=n_wplanes, uv_radius=120.0 * grid_n / 256)
    check_stages(ds, run_gpu(ds, tile=tile), oracle_of(ds))


@pytest.mark.parametrize("tile,chunk", [(16, 512), (32, 2048)])
def test_split_bins_at_other_tiles_and_chunks(tile, chunk):
    """bins split over several chunks at smaller tiles: partial tiles merged onto the mesh"""
    ds = synth.tiny()
    gpu = run_gpu(ds, tile=tile, chunk=chunk)
    assert gpu["counts"].max() > chunk              # split bins occur
    check_stages(ds, gpu, oracle_of(ds))


@pytest.mark.parametrize("kernel", ["gaussian", "kaiser_bessel"])
@pytest.mark.parametrize("W,OS,tile", [(1, 1, 16), (3, 4, 32), (5, 256, 64), (7, 64, 64), (9, 8, 16),
                                       (15, 2, 32)])
def test_kernels_supports_oversampling_tiles(kernel, W, OS, tile):
    ds = synth.tiny(nrow=20000, seed=4, support=W, oversample=OS, kernel=kernel)
    check_stages(ds, run_gpu(ds, tile=tile), oracle_of(ds))


def test_multichannel_metres_and_weights():
    ds = synth.ska_low_small()
    rng = np.random.default_rng(5)
    ds.weight = rng.uniform(0.2, 2.0, (ds.nrow, ds.nchan)).astype(np.float32)
    check_stages(ds, run_gpu(ds), oracle_of(ds))


def test_many_channels_beyond_one_scale_upload():
    ds = synth.ska_low_small(n_chan=40, n_times=4, n_src=3)
    check_stages(ds, run_gpu(ds), oracle_of(ds))


@pytest.mark.parametrize("N", [64, 128, 512, 1024, 2048, 4096, 8192])
def test_grid_sizes(N):
    ds = synth.tiny(nrow=5000, seed=6, grid_n=N, n_wplanes=2, uv_radius=120.0 * N / 256)
    check_stages(ds, run_gpu(ds), oracle_of(ds))


def test_dropped_inputs_match_oracle():
    ds = synth.tiny(nrow=6000, seed=9, weights=True)
    uvw = ds.uvw.copy()
    vis = np.asarray(ds.vis).copy()
    wt = ds.weight.copy()
    uvw[0, 0] = np.nan
    uvw[1, 2] = np.inf
    vis[2, 0] = np.nan
    wt[3, 0] = 0.0
    wt[4, 0] = -1.0
    wt[5, 0] = np.nan
    uvw[6, 0] = 5000.0      # far outside the grid
    uvw[7, 1] = -633.0      # footprint leaves the low edge
    uvw[8, 2] = 1e6         # beyond w_max: last plane
    ds.uvw, ds.vis, ds.weight = uvw, vis, wt
    ref = oracle_of(ds)
    assert (~ref.binned.keep).sum() >= 8
    check_stages(ds, run_gpu(ds), ref)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_many_nonfinite_visibilities(precision):
    """Visibilities whose position passes every test but whose V is not
    finite: the binning's counting pass does not read V, so they take level-1
    slots and are skipped at level 2; counts, sums and image stay the
    oracle's (every seventh visibility NaN or infinite, small tiles and chunks)"""
    ds = synth.tiny(nrow=20000, seed=12)
    vis = np.asarray(ds.vis).copy()
    vis[::7, 0] = np.nan
    vis[3::14, 0] = np.complex64(complex(np.inf, 0.0))
    vis[5::21, 0] = np.complex64(complex(0.0, -np.inf))
    ds.vis = vis
    ref = oracle_of(ds)
    assert (~ref.binned.keep).sum() > 2800
    gpu = run_gpu(ds, precision=precision, tile=16, chunk=64)
    if precision == "fp64":
        assert rel_rms(gpu["G"], ref.planes) <= 1e-12 and rel_rms(gpu["img"], ref.image) <= FP64_IMG
        assert gpu["info"]["n_gridded"] == int(ref.binned.keep.sum())
    else:
        check_stages(ds, gpu, ref)


@pytest.mark.parametrize("tile,chunk", [(0, 0), (16, 512), (16, 64)])
def test_accumulating_two_grid_calls_equals_one(tile, chunk):
    """also with bins split over several chunks (16, 512) and (16, 64)"""
    import torch
    ds = synth.tiny(nrow=30000, seed=10)
    uvw, vis, _ = to_device(ds)
    with rick.Plan.for_dataset(ds, tile=tile, chunk=chunk) as p:
        p.reset()
        p.grid(uvw[:12345], vis[:12345])
        p.grid(uvw[12345:], vis[12345:])
        p.fft()
        img2 = p.image().double().cpu().numpy()
        n2 = p.info()["n_gridded"]
        # reuse after reset
        p.reset()
        p.grid(uvw, vis)
        p.fft()
        img1 = p.image().double().cpu().numpy()
        torch.cuda.synchronize()
    ref = oracle_of(ds)
    assert n2 == ds.nvis
    for img in (img1, img2):
        err = image_errors(img, ref.image, ref.corr)
        assert err["apparent"] <= FP32_IMG and err["central"] <= FP32_IMG, err


@pytest.mark.parametrize("fused", [False, True])
def test_tile_bitmap_across_calls_and_resets(fused):
    """Tiles are written only where records land and a bitmap says which:
    a second rick_grid over other tiles stores those and adds to shared ones,
    and after a reset the first image's tiles must not leak into the next."""
    import torch
    ds = synth.tiny(nrow=20000, seed=18)
    uvw, vis, _ = to_device(ds)
    east = np.nonzero(ds.uvw[:, 0] > 20.0)[0]      # first call: one half-plane of u
    west = np.nonzero(ds.uvw[:, 0] <= 20.0)[0]
    e_t = torch.as_tensor(east, device=uvw.device)
    w_t = torch.as_tensor(west, device=uvw.device)
    with rick.Plan.for_dataset(ds, fused=fused) as p:
        p.reset()
        p.grid(uvw[e_t].contiguous(), vis[e_t].contiguous())
        nt = ds.grid_n // p.info()["tile"]
        t_east = p.tile_mask()
        p.grid(uvw[w_t].contiguous(), vis[w_t].contiguous())
        t_all = p.tile_mask()
        assert t_east.sum() > 0 and t_all.sum() > t_east.sum() and np.all(t_all[t_east])
        p.fft()
        img_two = p.image().double().cpu().numpy()
        # a new image of the west half only: the east tiles still sit in the
        # mesh and must read as zeros
        p.reset()
        assert p.tile_mask().sum() == 0
        p.grid(uvw[w_t].contiguous(), vis[w_t].contiguous())
        p.fft()
        img_west = p.image().double().cpu().numpy()
        # nothing gridded since the reset: a zero image
        p.reset()
        p.fft()
        img_none = p.image().double().cpu().numpy()
        torch.cuda.synchronize()
    assert t_all.shape == (ds.n_wplanes, nt, nt)
    ref = oracle_of(ds)
    err = image_errors(img_two, ref.image, ref.corr)
    assert err["apparent"] <= FP32_IMG and err["central"] <= FP32_IMG, err
    dsw = synth.tiny(nrow=20000, seed=18)
    dsw.uvw = ds.uvw[west]
    dsw.vis = np.asarray(ds.vis)[west]
    refw = oracle_of(dsw)
    err = image_errors(img_west, refw.image, refw.corr)
    assert err["apparent"] <= FP32_IMG and err["central"] <= FP32_IMG, err
    assert float(np.abs(img_none).max()) == 0.0


def test_fixed_point_scale_follows_each_bin():
    """Float32-mode gridding sums in fixed point scaled per bin by the bin's
    largest |W V|: tiles of faint visibilities keep their relative precision
    next to tiles 1e10 times brighter (both float32 modes)."""
    ds = synth.tiny(nrow=20000, seed=19)
    u = ds.uvw[:, 0]
    keep = np.abs(u) > 25.0          # faint (u < -25) and bright (u > 25) never share a tile
    ds.uvw = ds.uvw[keep]
    vis = np.asarray(ds.vis)[keep].copy()
    vis[ds.uvw[:, 0] > 0] *= np.float32(1e10)
    ds.vis = vis
    ref = oracle_of(ds)
    N = ds.grid_n
    faint = (slice(None), slice(None), slice(0, N // 2))              # cells x < 128: faint tiles only
    bright = (slice(None), slice(None), slice(N // 2 + 8, None))
    for precision, tol in (("fp32", FP32_GRID), ("fp32_kahan", FP32_GRID)):
        gpu = run_gpu(ds, precision=precision)
        assert rel_rms(gpu["G"][faint], ref.planes[faint]) <= tol, precision
        assert rel_rms(gpu["G"][bright], ref.planes[bright]) <= tol, precision
    assert np.abs(ref.planes[faint]).max() > 0 and np.abs(ref.planes[bright]).max() > 1e8 * np.abs(ref.planes[faint]).max()


def test_empty_and_all_dropped_give_zero_image():
    import torch
    ds = synth.tiny(nrow=100, seed=11)
    uvw, vis, _ = to_device(ds)
    with rick.Plan.for_dataset(ds) as p:
        p.reset()
        p.grid(uvw[:0], vis[:0])
        p.fft()
        img = p.image()
        torch.cuda.synchronize()
        assert float(img.abs().max()) == 0.0
        p.reset()
        p.grid(uvw * 1000.0, vis)           # every footprint leaves the grid
        p.fft()
        img = p.image()
        inf = p.info()
        assert inf["n_gridded"] == 0 and inf["n_dropped"] == 100
        assert float(img.abs().max()) == 0.0


def test_call_order_and_capacity_errors():
    ds = synth.tiny(nrow=1000, seed=12)
    uvw, vis, _ = to_device(ds)
    with rick.Plan.for_dataset(ds, max_vis=1000) as p:
        with pytest.raises(rick.RickError) as e:
            p.image()
        assert e.value.status == 7
        p.reset()
        with pytest.raises(rick.RickError) as e:
            import torch
            p.grid(torch.cat([uvw, uvw]), torch.cat([vis, vis]))
        assert e.value.status == 5
        p.grid(uvw, vis)
        p.fft()
        with pytest.raises(rick.RickError) as e:
            p.grid(uvw, vis)
        assert e.value.status == 7


def test_gpu_error_vs_dft_equals_oracle_error_vs_dft():
    """The GPU image's distance to the direct DFT equals the oracle's within 1 %."""
    ds = synth.tiny()
    ref = oracle_of(ds)
    gpu = run_gpu(ds)
    rows = cols = slice(96, 160)
    D = oracle.dft.dft_of_binned(ref.binned, ds.fov, ds.grid_n, rows=rows, cols=cols)
    e_or = rel_rms(ref.image[rows, cols], D)
    e_gpu = rel_rms(gpu["img"][rows, cols], D)
    assert abs(e_gpu - e_or) <= 0.01 * e_or, (e_gpu, e_or)


def test_phase_centre_source_unit_peak():
    ds = synth.tiny(nrow=20000, seed=13)
    ds.vis = np.full((ds.nrow, 1), 1.5, np.complex64)
    gpu = run_gpu(ds)
    assert abs(gpu["img"][128, 128] - 1.5) < 1e-5


@pytest.mark.parametrize("fused", [False, True])
def test_per_visibility_decisions_match_oracle(fused):
    """The discretisation of Sec. 2.1 visibility by visibility: footprint
    origin cell, sub-cell offsets, plane and drop decision of every
    visibility, read back through a prediction order (the same quantisation
    code as gridding, rick_degrid_order_info), equal the oracle's bit for bit.
    The order is a permutation of the visibilities sorted by its keys (the
    library's radix sort).  Multichannel positions in metres, with positions
    that are dropped (non-finite, beyond the grid, footprint leaving it) and
    w beyond the planes' range."""
    import torch
    ds = synth.ska_low_small()
    uvw = ds.uvw.copy()
    uvw[0, 0] = np.nan
    uvw[1, 2] = np.inf
    uvw[2, 0] = 1e7
    uvw[3, 1] = -uvw[3, 1] * 50.0
    uvw[4, 2] = 1e9
    uvw[5, 2] = -1e9
    ds.uvw = uvw
    N, OS, h = ds.grid_n, ds.oversample, (ds.support - 1) // 2
    zeros = np.zeros((ds.nrow, ds.nchan), dtype=np.complex64)
    b = ow.bin_visibilities(ds.uvw, ds.freq, zeros, None, grid_n=N, n_wplanes=ds.n_wplanes, support=ds.support,
                            oversample=OS, fov=ds.fov, w_min=ds.w_min, w_max=ds.w_max)
    assert (~b.keep).sum() >= 4 * ds.nchan
    with rick.Plan.for_dataset(ds, fused=fused) as p:
        plan_panel = p.info()["panel"]
        with p.degrid_order(torch.as_tensor(ds.uvw).to("cuda:0"), ds.freq) as o:
            keys, vals, panel = o.arrays()
    assert panel == plan_panel and (panel > 0) == fused
    n = ds.nvis
    # sorted on the key's bits above the group bits (the column inside a
    # panel and 3 row bits; 3 column bits in row order), equal groups in
    # visibility order
    lo = np.uint64((int(panel).bit_length() - 1 if panel else 0) + 3)
    hi = keys >> lo
    idx = (vals & np.uint64(0xffffffff)).astype(np.int64)
    assert keys.shape == (n,) and np.all(hi[1:] >= hi[:-1])
    same = hi[1:] == hi[:-1]
    assert np.all(idx[1:][same] > idx[:-1][same])
    assert np.array_equal(np.sort(idx), np.arange(n))
    dropped = keys == np.uint64(0xffffffffffffffff)
    assert np.array_equal(~dropped, b.keep[idx])
    kk = keys[~dropped].astype(np.uint64)
    ii = idx[~dropped]
    k = (kk // np.uint64(N * N)).astype(np.int64)
    off = (kk % np.uint64(N * N)).astype(np.int64)
    if panel:
        y0, x0 = (off // panel) % N, (off // (N * panel)) * panel + off % panel
    else:
        y0, x0 = off // N, off % N
    sx = ((vals[~dropped] >> np.uint64(32)) & np.uint64(0xff)).astype(np.int64) - OS // 2
    sy = ((vals[~dropped] >> np.uint64(40)) & np.uint64(0xff)).astype(np.int64) - OS // 2
    assert np.array_equal(k, b.k[ii])
    assert np.array_equal(x0, b.cx[ii] - h) and np.array_equal(y0, b.cy[ii] - h)
    assert np.array_equal(sx, b.sx[ii]) and np.array_equal(sy, b.sy[ii])
