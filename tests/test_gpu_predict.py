"""Prediction (degridding) through the C ABI against the float64 prediction
oracle: the model image's plane transforms and the interpolated visibilities,
element by element on small grids (several tiles, ragged channel counts,
dropped visibilities), the adjoint identity with the GPU imaging path, the
call-order rules shared with imaging, and sampled visibilities at the full
4096^2 x 64-plane size.

Tolerances: float32 mode carries float32 plane values through a float32 FFT
of log2(N^2) radix passes and a W^2-term interpolation.  The planes hold the
model divided by the taper C(l'_p) C(l'_q) (up to 1/min(C)^2 = 6.4e3 at the
corners for the support-7 Gaussian), and the interpolation takes the taper
back out, so the float32 rounding of the planes reaches V magnified by
A = ||M / (C C)|| / ||M||: the relative RMS error is gated at
max(1e-5, 1e-7 A) (measured 2.7e-8 A for a white-noise model, A = 384).
Float64 mode is gated at 1e-11.  Dropped visibilities are exactly 0 on both
sides.
"""
import numpy as np
import pytest

import synth
from oracle import predict as op
from oracle import wstack as ow
from paper_2504_00959_amd import rick
from tests.helpers import rel_rms

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-11}


def _tol(precision, M, ds):
    if precision == "fp64":
        return TOL["fp64"]
    C = ow.grid_correction(ow.tap_table(ds.support, ds.oversample, ds.kernel, ds.kernel_param), ds.grid_n)
    A = float(np.linalg.norm(M / np.outer(C, C)) / np.linalg.norm(M))
    return max(TOL["fp32"], 1e-7 * A)


def _model(N, seed, n_src=25, dense=False):
    rng = np.random.default_rng(seed)
    if dense:
        return rng.normal(size=(N, N))
    M = np.zeros((N, N))
    np.add.at(M, (rng.integers(0, N, n_src), rng.integers(0, N, n_src)), rng.uniform(0.05, 3.0, n_src))
    return M


def _predict_gpu(ds, M, precision="fp32", fused=False, freq=None, **plan_kw):
    import torch
    with rick.Plan.for_dataset(ds, precision=precision, fused=fused, **plan_kw) as p:
        m = torch.as_tensor(M, dtype=p.real_dtype).to("cuda:0").contiguous()
        uvw = torch.as_tensor(ds.uvw, dtype=torch.float64).to("cuda:0")
        p.predict_planes(m)
        vis = p.degrid(uvw, freq)
        torch.cuda.synchronize()
        return vis.cpu().numpy().astype(np.complex128).reshape(-1)


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
@pytest.mark.parametrize("dense", [False, True])
def test_tiny_predict_matches_oracle(precision, dense, fused):
    """fused: planes transformed into the plan's row_mesh in column-panel
    order and interpolated from there."""
    ds = synth.tiny(nrow=20000, seed=51)
    M = _model(ds.grid_n, 52, dense=dense)
    got = _predict_gpu(ds, M, precision, fused=fused)
    ref = op.wstack_predict(M, ds.uvw, None, **ds.plan_kwargs(), keep_planes=False)
    kept = ref.binned.keep
    assert np.all(got[~kept] == 0)
    assert rel_rms(got[kept], ref.vis[kept]) <= _tol(precision, M, ds)


@pytest.mark.parametrize("fused", [False, True])
def test_multichannel_metres_matches_oracle(fused):
    ds = synth.ska_low_small()
    M = _model(ds.grid_n, 53, n_src=40)
    got = _predict_gpu(ds, M, "fp32", fused=fused, freq=ds.freq)
    ref = op.wstack_predict(M, ds.uvw, ds.freq, **ds.plan_kwargs(), keep_planes=False)
    kept = ref.binned.keep
    assert kept.sum() > 0.5 * kept.size
    assert np.all(got[~kept] == 0)
    assert rel_rms(got[kept], ref.vis[kept]) <= _tol("fp32", M, ds)


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("kernel,W,OS,N", [("kaiser_bessel", 5, 16, 512), ("gaussian", 9, 128, 128),
                                           ("gaussian", 1, 1, 64)])
def test_kernels_supports_and_sizes(kernel, W, OS, N, fused):
    ds = synth.tiny(nrow=6000, seed=54, grid_n=N)
    kw = {**ds.plan_kwargs(), "kernel": kernel, "support": W, "oversample": OS}
    ds.kernel, ds.support, ds.oversample = kernel, W, OS
    M = _model(N, 55, dense=True)
    got = _predict_gpu(ds, M, "fp64", fused=fused)
    ref = op.wstack_predict(M, ds.uvw, None, **kw, keep_planes=False)
    kept = ref.binned.keep
    assert np.all(got[~kept] == 0)
    assert rel_rms(got[kept], ref.vis[kept]) <= TOL["fp64"]


def test_dropped_positions_and_empty_inputs():
    import torch
    ds = synth.tiny(nrow=3000, seed=56)
    uvw = ds.uvw.copy()
    uvw[:10, 0] = 1e9          # footprint off the grid
    uvw[10:20, 1] = np.nan     # non-finite
    ds.uvw = uvw
    M = _model(ds.grid_n, 57)
    got = _predict_gpu(ds, M, "fp32")
    assert np.all(got[:20] == 0)
    ref = op.wstack_predict(M, uvw, None, **ds.plan_kwargs(), keep_planes=False)
    kept = ref.binned.keep
    assert not kept[:20].any() and np.all(got[~kept] == 0)
    assert rel_rms(got[kept], ref.vis[kept]) <= _tol("fp32", M, ds)
    with rick.Plan.for_dataset(ds) as p:
        p.predict_planes(torch.zeros((ds.grid_n, ds.grid_n), dtype=torch.float32, device="cuda:0"))
        v0 = p.degrid(torch.as_tensor(uvw[:500]).to("cuda:0"))
        empty = p.degrid(torch.zeros((0, 3), dtype=torch.float64, device="cuda:0"))
        torch.cuda.synchronize()
        assert torch.all(v0 == 0) and empty.numel() == 0


def test_adjoint_of_gpu_imaging_fp64():
    """sum_pq M I / n^2 * sum W = Re <V, predict(M)> with both sides on the
    GPU in float64 (the imaging path and the prediction path are adjoint)."""
    import torch
    ds = synth.tiny(nrow=8000, seed=58)
    rng = np.random.default_rng(59)
    V = (rng.normal(size=(ds.nrow, 1)) + 1j * rng.normal(size=(ds.nrow, 1)))
    N = ds.grid_n
    M = rng.normal(size=(N, N))
    with rick.Plan.for_dataset(ds, precision="fp64") as p:
        uvw = torch.as_tensor(ds.uvw).to("cuda:0")
        p.reset()
        p.grid(uvw, torch.as_tensor(V).to("cuda:0").contiguous())
        p.fft()
        img = p.image().cpu().numpy()
        sum_w = p.info()["sum_weights"]
        p.predict_planes(torch.as_tensor(M).to("cuda:0").contiguous())
        pred = p.degrid(uvw).cpu().numpy().reshape(-1)
    l = ow.pixel_lm(N, ds.fov)
    nm1 = ow.nm1_of(l[None, :], l[:, None])
    n2 = np.where(np.isfinite(nm1), (1.0 + np.nan_to_num(nm1)) ** 2, 1.0)
    lhs = float((M * img / n2).sum() * sum_w)
    rhs = float(np.real(np.vdot(pred, V.reshape(-1))))
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs), (lhs, rhs)


def test_call_order_with_imaging():
    """Prediction overwrites the mesh: gridding or transforming after it needs
    a reset, degridding needs predicted planes, and imaging after a reset is
    unaffected by the prediction that came before."""
    import torch
    ds = synth.tiny(nrow=5000, seed=60)
    uvw = torch.as_tensor(ds.uvw).to("cuda:0")
    vis = torch.as_tensor(ds.vis).to("cuda:0").contiguous()
    M = torch.as_tensor(_model(ds.grid_n, 61), dtype=torch.float32).to("cuda:0")
    with rick.Plan.for_dataset(ds, fused=True) as p:
        with pytest.raises(rick.RickError):
            p.degrid(uvw)                                   # nothing predicted
        p.reset()
        p.grid(uvw, vis)
        p.fft()
        first = p.image().double().cpu().numpy()
        p.predict_planes(M)
        with pytest.raises(rick.RickError):
            p.grid(uvw, vis)
        with pytest.raises(rick.RickError):
            p.fft()
        with pytest.raises(rick.RickError):
            p.image()
        a = p.degrid(uvw).cpu().numpy()
        b = p.degrid(uvw).cpu().numpy()                     # repeatable on the same planes
        assert np.array_equal(a, b)
        p.reset()
        p.grid(uvw, vis)
        p.fft()
        second = p.image().double().cpu().numpy()
        torch.cuda.synchronize()
    assert np.array_equal(first, second)


@pytest.mark.parametrize("fused", [False, True])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_sorted_order_equals_direct_order(precision, fused):
    """Prediction through a sort order (quantised and sorted once) gives each
    visibility the same value as the direct walk, at its own index; dropped
    visibilities are 0; channels in metres."""
    import torch
    ds = synth.ska_low_small()
    uvw_h = ds.uvw.copy()
    uvw_h[:5, 0] = 1e9
    M = _model(ds.grid_n, 63, n_src=40)
    with rick.Plan.for_dataset(ds, precision=precision, fused=fused) as p:
        uvw = torch.as_tensor(uvw_h).to("cuda:0")
        p.predict_planes(torch.as_tensor(M, dtype=p.real_dtype).to("cuda:0"))
        direct = p.degrid(uvw, ds.freq).cpu().numpy()
        with p.degrid_order(uvw, ds.freq) as order:
            out = torch.full((ds.nrow, len(ds.freq)), 7.0, dtype=p.complex_dtype, device="cuda:0")
            srt = p.degrid_sorted(order, out).cpu().numpy()
            again = p.degrid_sorted(order).cpu().numpy()
        torch.cuda.synchronize()
    assert np.all(srt[:5] == 0)
    assert np.max(np.abs(srt - direct)) <= 1e-6 * np.max(np.abs(direct))
    assert np.array_equal(srt, again)
    ref = op.wstack_predict(M, uvw_h, ds.freq, **ds.plan_kwargs(), keep_planes=False)
    kept = ref.binned.keep
    assert rel_rms(srt.reshape(-1)[kept], ref.vis[kept]) <= _tol(precision, M, ds)


def test_sorted_order_checks_geometry_and_empty():
    import torch
    ds = synth.tiny(nrow=4000, seed=64)
    uvw = torch.as_tensor(ds.uvw).to("cuda:0")
    M = torch.as_tensor(_model(ds.grid_n, 65), dtype=torch.float32).to("cuda:0")
    with rick.Plan.for_dataset(ds) as p:
        order = p.degrid_order(uvw)
        with pytest.raises(rick.RickError):
            p.degrid_sorted(order)                 # nothing predicted yet
        p.retarget(ds.fov * 1.1, ds.w_min, ds.w_max)
        p.predict_planes(M)
        with pytest.raises(rick.RickError):
            p.degrid_sorted(order)                 # order made for another field
        p.retarget(ds.fov, ds.w_min, ds.w_max)
        p.predict_planes(M)
        a = p.degrid_sorted(order)
        b = p.degrid(uvw)
        with p.degrid_order(torch.zeros((0, 3), dtype=torch.float64, device="cuda:0")) as empty:
            assert p.degrid_sorted(empty).numel() == 0
        torch.cuda.synchronize()
        order.close()
    assert torch.equal(a, b) or float((a - b).abs().max()) <= 1e-6 * float(b.abs().max())


@pytest.fixture(scope="module")
def share_predict():
    import torch
    print("[predict fullsize] generating ska_low_share positions on cuda:0", flush=True)
    ds = synth.ska_low_share(device="cuda:0", with_vis=False)
    N = ds.grid_n
    dl = ds.fov / N
    pp = np.rint(ds.sources["l"] / dl).astype(np.int64) + N // 2
    qq = np.rint(ds.sources["m"] / dl).astype(np.int64) + N // 2
    fl = np.asarray(ds.sources["flux"], dtype=np.float64)
    M = torch.zeros((N, N), dtype=torch.float32, device="cuda:0")
    M.index_put_((torch.as_tensor(qq).cuda(), torch.as_tensor(pp).cuda()),
                 torch.as_tensor(fl, dtype=torch.float32).cuda(), accumulate=True)
    uvw = torch.as_tensor(ds.uvw, dtype=torch.float64).to("cuda:0")
    with rick.Plan.for_dataset(ds, fused=True) as p:
        p.predict_planes(M)
        vis = p.degrid(uvw, ds.freq)
        with p.degrid_order(uvw, ds.freq) as order:
            vis_sorted = p.degrid_sorted(order)
        torch.cuda.synchronize()
        sorted_diff = float((vis_sorted - vis).abs().max() / vis.abs().max())
        del vis_sorted
        rng = np.random.default_rng(62)
        rows = np.sort(rng.choice(ds.nrow, 40, replace=False))
        got = vis[torch.as_tensor(rows).cuda()].cpu().numpy().astype(np.complex128).reshape(-1)
        finite = bool(torch.isfinite(torch.view_as_real(vis)).all())
    print("[predict fullsize] GPU done; oracle at sampled rows", flush=True)
    uvw_h = uvw[torch.as_tensor(rows).cuda()].cpu().numpy()
    ref = op.wstack_predict_sparse(pp, qq, fl, uvw_h, ds.freq, **ds.plan_kwargs())
    Mh = np.zeros((N, N))
    np.add.at(Mh, (qq, pp), fl)
    return dict(got=got, ref=ref, finite=finite, tol=_tol("fp32", Mh, ds), sorted_diff=sorted_diff)


def test_fullsize_sampled_visibilities(share_predict):
    """4096^2 x 64 planes, 209.3M visibility positions, the 1000-source model
    on pixels: 40 rows x 16 channels against the oracle's sparse-model form."""
    got, ref = share_predict["got"], share_predict["ref"]
    assert share_predict["finite"]
    assert rel_rms(got, ref) <= share_predict["tol"]
    assert share_predict["sorted_diff"] <= 1e-6


def test_recorded_prediction_replays_like_eager():
    """rick_predict_planes, rick_degrid and rick_degrid_sorted recorded into a
    graph and replayed three times, with an eager imaging run on the same
    plan and synchronisations between the replays: every replay equals the
    eager prediction."""
    import torch
    ds = synth.tiny(nrow=6000, seed=66)
    uvw = torch.as_tensor(ds.uvw).to("cuda:0")
    vis = torch.as_tensor(ds.vis).to("cuda:0").contiguous()
    M = torch.as_tensor(_model(ds.grid_n, 67), dtype=torch.float32).to("cuda:0")
    stream = torch.cuda.Stream()
    with rick.Plan.for_dataset(ds, fused=True) as p, torch.cuda.stream(stream):
        p.predict_planes(M, stream)
        eager = p.degrid(uvw, None, None, stream).clone()
        order = p.degrid_order(uvw, None, stream)
        eager_sorted = p.degrid_sorted(order, None, stream).clone()
        stream.synchronize()
        out1 = torch.empty_like(eager)
        out2 = torch.empty_like(eager)
        with rick.Graph.record(stream) as graph:
            p.predict_planes(M, stream)
            p.degrid(uvw, None, out1, stream)
            p.degrid_sorted(order, out2, stream)
        for rep in range(3):
            out1.fill_(-1.0)
            out2.fill_(-1.0)
            p.reset(stream)
            p.grid(uvw, vis, None, None, stream)
            p.fft(stream)
            p.image(None, stream)
            torch.cuda.synchronize()
            graph.launch(stream)
            stream.synchronize()
            assert torch.equal(out1, eager), rep
            assert torch.equal(out2, eager_sorted), rep
        graph.close()
        order.close()
