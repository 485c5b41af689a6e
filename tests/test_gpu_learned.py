"""GPU path of the learned gridding kernel (user tables), the direct Fourier
sum kernel, and the 16384^2 grid, through the C ABI, against the float64
oracle (``oracle.learned``, ``oracle.dft``, ``oracle.pixels``).

Tolerances: float32 stages 1e-6 relative RMS (planes 5e-6: packed 32-bit
fixed-point sums; taper exact to 1e-12 as it is float64 on both sides), end-to-end float32 image 1e-5 on the
apparent image and the central region (as in the other parity tests), the
float32 MLP 2e-6 absolute on table entries (each row sums to 1) and 1e-4
relative on parameter gradients, the direct sum 2e-6 relative (float32
sin/cos of the reduced phase, about 2.5e-7 per term).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import dft as od
from oracle import learned as ol
from oracle import wstack as ow
from paper_2504_00959_amd import rick
from tests.helpers import image_errors, rel_rms, to_device

pytestmark = pytest.mark.gpu


def _scene(seed=61, nrow=3000, N=128, Nw=6, W=7, OS=16, fov=0.5, wmax=60.0, nsrc=6):
    rng = np.random.default_rng(seed)
    r = 0.4 * N / fov * np.sqrt(rng.uniform(0, 1, nrow))
    ph = rng.uniform(0, 2 * np.pi, nrow)
    uvw = np.stack([r * np.cos(ph), r * np.sin(ph), rng.uniform(-wmax, wmax, nrow)], 1)
    l = rng.uniform(-0.3, 0.3, nsrc) * fov
    m = rng.uniform(-0.3, 0.3, nsrc) * fov
    S = rng.uniform(0.5, 1.5, nsrc)
    vis = synth.point_source_vis_np(uvw[:, 0], uvw[:, 1], uvw[:, 2], l, m, S).astype(np.complex64).reshape(-1, 1)
    wt = rng.uniform(0.5, 2.0, (nrow, 1)).astype(np.float32)
    geo = dict(grid_n=N, n_wplanes=Nw, support=W, oversample=OS, fov=fov, w_min=-wmax, w_max=wmax)
    return uvw, vis, wt, geo


def _dev(uvw, vis, wt, precision="fp32"):
    import torch
    cd = torch.complex128 if precision == "fp64" else torch.complex64
    return (torch.as_tensor(uvw, dtype=torch.float64).cuda(), torch.as_tensor(vis).to(cd).cuda().contiguous(),
            torch.as_tensor(wt, dtype=torch.float32).cuda().contiguous())


def _image(plan, uvw_d, vis_d, wt_d):
    import torch
    plan.reset()
    plan.grid(uvw_d, vis_d, wt_d, None)
    torch.cuda.synchronize()
    G = plan.mesh().cpu().numpy()
    plan.fft()
    img = plan.image().double().cpu().numpy()
    torch.cuda.synchronize()
    return G, img


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_separable_table_matches_gaussian_plan(precision):
    """The Gaussian tap table laid out as a user table (4 identical w-fraction
    bins) images exactly like the separable Gaussian plan, and its 2-D taper
    is C(l') C(m')."""
    uvw, vis, wt, geo = _scene()
    g = ow.tap_table(geo["support"], geo["oversample"])
    T = ol.separable_table(g, g, 4).astype(np.float32)
    dev = _dev(uvw, vis, wt, precision)
    with rick.Plan(**geo, precision=precision, max_vis=len(uvw)) as pg, \
            rick.Plan(**geo, precision=precision, max_vis=len(uvw), kernel="user_lut", lut_wbins=4) as pu:
        pu.set_lut(T)
        Gg, ig = _image(pg, *dev)
        Gu, iu = _image(pu, *dev)
        C2 = pu.taper().cpu().numpy()
        c1 = pg.taper().cpu().numpy()
    # the float32 table entries are the float32 rounding of g_y g_x, not the
    # product of the rounded rows: agreement to float32 rounding, and in the
    # float32 mode to the packed sums' rounding of each term (2^-21 of the
    # bin's largest), which a one-ulp difference in a tap can move by one step
    tol = 5e-6 if precision == "fp32" else 1e-7
    assert rel_rms(Gu, Gg) <= tol
    assert np.max(np.abs(C2 - np.outer(c1, c1))) < 1e-7
    assert image_errors(iu, ig, c1)["apparent"] <= tol


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp64", 1e-10)])
def test_learned_table_image_parity(precision, tol):
    """A table tabulated from an MLP (different in every w-fraction bin)
    installed from the host: planes, taper and image against the oracle with
    the same (float32) table."""
    uvw, vis, wt, geo = _scene(seed=62)
    th = ol.init_params(21, scale=0.4)
    T = ol.tabulate(th, geo["support"], geo["oversample"], 4).astype(np.float32)
    ref = ol.image_with_table(uvw, None, vis, wt, T.astype(np.float64), **geo)
    assert len(np.unique(ref.iw[ref.binned.keep])) == 4
    dev = _dev(uvw, vis, wt, precision)
    with rick.Plan(**geo, precision=precision, max_vis=len(uvw), kernel="user_lut", lut_wbins=4) as pu:
        pu.set_lut(T)
        G, img = _image(pu, *dev)
        C2 = pu.taper().cpu().numpy()
        info = pu.info()
    assert info["n_gridded"] == int(ref.binned.keep.sum())
    assert np.max(np.abs(C2 - ref.corr2)) < 1e-12
    # float32: packed 32-bit fixed-point sums (terms rounded at 2^-21 of the bin's largest)
    assert rel_rms(G, ref.planes) <= (5e-6 if precision == "fp32" else 1e-12)
    err = image_errors(img, ref.image, np.ones(geo["grid_n"]))   # compare with the 2-D taper below
    app = rel_rms(img * ref.corr2, ref.apparent)
    print(f"[learned] {precision}: planes {rel_rms(G, ref.planes):.2e}, apparent {app:.2e}, image {err['full']:.2e}")
    assert app <= tol


def test_table_from_device_and_fused_plan():
    """A table installed from device memory into a plan with the fused
    column transform gives the host-installed, unfused result."""
    import torch
    uvw, vis, wt, geo = _scene(seed=63)
    T = ol.tabulate(ol.init_params(22, scale=0.4), geo["support"], geo["oversample"], 2).astype(np.float32)
    dev = _dev(uvw, vis, wt)
    with rick.Plan(**geo, max_vis=len(uvw), kernel="user_lut", lut_wbins=2) as pa, \
            rick.Plan(**geo, max_vis=len(uvw), kernel="user_lut", lut_wbins=2, fused=True) as pb:
        pa.set_lut(T)
        pb.set_lut(torch.as_tensor(T).cuda())
        _, ia = _image(pa, *dev)
        _, ib = _image(pb, *dev)
        C2 = pa.taper().cpu().numpy()
    assert rel_rms(ia * C2, ib * C2) <= 1e-6


def test_user_lut_plan_refuses_grid_before_table_and_prediction():
    uvw, vis, wt, geo = _scene(seed=64, nrow=100)
    dev = _dev(uvw, vis, wt)
    with rick.Plan(**geo, max_vis=100, kernel="user_lut", lut_wbins=1) as pu:
        with pytest.raises(rick.RickError, match="RICK_E_STATE"):
            pu.grid(*dev[:2], dev[2], None)
        pu.set_lut(np.full((1, geo["oversample"], geo["oversample"], geo["support"], geo["support"]),
                           1.0 / geo["support"] ** 2, np.float32))
        import torch
        with pytest.raises(rick.RickError, match="RICK_E_UNSUPPORTED"):
            pu.predict_planes(torch.zeros((geo["grid_n"], geo["grid_n"]), dtype=torch.float32, device="cuda:0"))


def test_mlp_tabulate_and_backward_parity():
    import torch
    W, OS, nf = 7, 16, 4
    th = ol.init_params(23, scale=0.5)
    v32 = ol.flatten(th).astype(np.float32)
    th32 = ol.unflatten(v32.astype(np.float64))
    theta = torch.as_tensor(v32).cuda()
    T = rick.mlp_tabulate(theta, W, OS, nf)
    Tref = ol.tabulate(th32, W, OS, nf)
    assert np.max(np.abs(T.cpu().numpy() - Tref)) < 2e-6
    rng = np.random.default_rng(24)
    dT = rng.normal(size=Tref.shape)
    g = rick.mlp_backward(theta, T, torch.as_tensor(dT).cuda()).cpu().numpy()
    gref = ol.flatten(ol.tabulate_backward(th32, W, OS, nf, dT))
    print(f"[learned] mlp backward rel-RMS {rel_rms(g, gref):.2e}")
    assert rel_rms(g, gref) <= 1e-4


def test_adam_step_matches_definition():
    import torch
    rng = np.random.default_rng(25)
    n = 1217
    th, gr = rng.normal(size=n).astype(np.float32), rng.normal(size=n).astype(np.float32)
    m, v = np.zeros(n, np.float32), np.zeros(n, np.float32)
    td, gd = torch.as_tensor(th).cuda(), torch.as_tensor(gr).cuda()
    md, vd = torch.as_tensor(m).cuda(), torch.as_tensor(v).cuda()
    lr, b1, b2, eps = 1e-3, 0.9, 0.999, 1e-8
    want, mm, vv = th.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in (1, 2, 3):
        rick.adam_step(td, gd, md, vd, step, lr, b1, b2, eps)
        mm = b1 * mm + (1 - b1) * gr
        vv = b2 * vv + (1 - b2) * gr.astype(np.float64) ** 2
        mh, vh = mm / (1 - b1 ** step), vv / (1 - b2 ** step)
        want = want - lr * mh / (np.sqrt(vh) + eps)
    assert np.max(np.abs(td.cpu().numpy() - want)) < 1e-6


@pytest.mark.parametrize("channels", [False, True])
def test_dft_image_parity(channels):
    """The direct-sum kernel against the oracle's float64 direct sum, with
    dropped visibilities (off-grid, zero weight) left out of both."""
    rng = np.random.default_rng(26)
    N, fov = 128, 0.6
    if channels:
        nrow, nchan = 800, 3
        uvw = np.stack([rng.normal(0, 800, nrow), rng.normal(0, 800, nrow), rng.normal(0, 200, nrow)], 1)
        freq = np.array([140e6, 150e6, 160e6])
    else:
        nrow, nchan = 4000, 1
        uvw = np.stack([rng.normal(0, 30, nrow), rng.normal(0, 30, nrow), rng.normal(0, 20, nrow)], 1)
        uvw[:10, 0] = 1e6          # off the grid: dropped
        freq = None
    vis = (rng.normal(size=(nrow, nchan)) + 1j * rng.normal(size=(nrow, nchan))).astype(np.complex64)
    wt = rng.uniform(0.5, 2.0, (nrow, nchan)).astype(np.float32)
    wt[10:20] = 0.0                 # dropped
    geo = dict(grid_n=N, n_wplanes=4, support=7, oversample=16, fov=fov, w_min=-800.0, w_max=800.0)
    b = ow.bin_visibilities(uvw, freq, vis, wt, **geo)
    ref = od.dft_of_binned(b, fov, N, rows=slice(40, 72), cols=slice(10, 58))
    import torch
    with rick.Plan(**geo, max_vis=nrow * nchan) as p:
        out = p.dft_image(torch.as_tensor(uvw).cuda(), torch.as_tensor(vis).cuda(), torch.as_tensor(wt).cuda(),
                          freq, q0=40, p0=10, nq=32, np_=48).cpu().numpy()
    print(f"[dft] rel-RMS {rel_rms(out, ref):.2e}")
    assert rel_rms(out, ref) <= 2e-6


def test_loss_and_table_gradient_parity():
    """Loss against the direct sum and dL/dT (gridding part through the
    adjoint transform, and the taper part) against the oracle's exact
    gradient, with the same float32 table."""
    import torch
    uvw, vis, wt, geo = _scene(seed=65, nrow=2500, N=64, Nw=4, W=5, OS=8, fov=0.5, wmax=40.0)
    th = ol.init_params(27, scale=0.3)
    T = ol.tabulate(th, geo["support"], geo["oversample"], 2).astype(np.float32)
    b = ow.bin_visibilities(uvw, None, vis, wt, **geo)
    D = od.dft_of_binned(b, geo["fov"], geo["grid_n"])
    L, dT, r = ol.loss_and_table_grad(uvw, None, vis, wt, T.astype(np.float64), D, **geo)
    N = geo["grid_n"]
    uvw_d, vis_d, wt_d = _dev(uvw, vis, wt)
    with rick.Plan(**geo, max_vis=len(uvw), kernel="user_lut", lut_wbins=2) as pu:
        pu.set_lut(T)
        pu.reset()
        pu.grid(uvw_d, vis_d, wt_d, None)
        pu.fft()
        img = pu.image()
        Dd = torch.as_tensor(D).cuda()
        dA = torch.empty((N, N), dtype=torch.float64, device="cuda:0")
        dC = torch.empty_like(dA)
        sums = torch.zeros(2, dtype=torch.float64, device="cuda:0")
        pu.image_loss(img, Dd, dA, dC, sums)
        dTd = torch.empty(T.shape, dtype=torch.float64, device="cuda:0")
        pu.table_gradient(dA, dC, uvw_d, vis_d, wt_d, None, dTd)
        torch.cuda.synchronize()
        s = sums.cpu().numpy()
        g = dTd.cpu().numpy()
    Lg = s[0] / s[1]
    print(f"[learned] loss {Lg:.6e} (oracle {L:.6e}), gradient rel-RMS {rel_rms(g, dT):.2e}")
    assert abs(Lg - L) <= 1e-4 * L
    assert rel_rms(g, dT) <= 1e-4


def test_grid_16384():
    """A 16384^2 plan (unfused, float32): a few hundred visibilities imaged,
    the image at sampled pixels against the oracle's per-pixel regrouping."""
    import torch
    rng = np.random.default_rng(28)
    N, fov, nrow = 16384, 0.5, 600
    uvw = np.stack([rng.normal(0, 2000, nrow), rng.normal(0, 2000, nrow), rng.uniform(-30, 30, nrow)], 1)
    vis = (rng.normal(size=(nrow, 1)) + 1j * rng.normal(size=(nrow, 1))).astype(np.complex64)
    geo = dict(grid_n=N, n_wplanes=2, support=7, oversample=32, fov=fov, w_min=-30.0, w_max=30.0)
    pp = np.r_[N // 2, rng.integers(N // 4, 3 * N // 4, 7)]
    qq = np.r_[N // 2, rng.integers(N // 4, 3 * N // 4, 7)]
    ref, _, kept, _ = oracle.pixels.wstack_pixels(uvw, None, vis, None, pp, qq, **geo)
    assert kept == nrow
    with rick.Plan(**geo, max_vis=nrow) as p:
        p.reset()
        p.grid(torch.as_tensor(uvw).cuda(), torch.as_tensor(vis).cuda(), None, None)
        p.fft()
        img = p.image()
        got = img[torch.as_tensor(qq).cuda(), torch.as_tensor(pp).cuda()].double().cpu().numpy()
        c = p.taper().cpu().numpy()
    c2 = c[pp] * c[qq]
    print(f"[16384] apparent rel-RMS {rel_rms(got * c2, ref * c2):.2e}")
    assert rel_rms(got * c2, ref * c2) <= 1e-5
    with pytest.raises(rick.RickError, match="RICK_E_UNSUPPORTED"):
        rick.Plan(**geo, max_vis=nrow, precision="fp64")


def test_training_steps_reduce_the_loss():
    """The training driver (library calls only): fitting the MLP to the
    Gaussian table reproduces the Gaussian image's loss, and steps on one
    scene lower its loss against the direct sum."""
    import torch
    import synth
    from paper_2504_00959_amd.learned import LearnedKernel
    kw = dict(nvis=30000, grid_n=64, n_wplanes=4, support=5, oversample=8)
    s0 = synth.learned_scene(0, **kw)
    lk = LearnedKernel(grid_n=64, n_wplanes=4, support=5, oversample=8, fov=s0.fov, w_min=s0.w_min, w_max=s0.w_max,
                       max_vis=s0.nvis, n_wbins=2, seed=1)
    try:
        ds = synth.learned_scene(3, device="cuda:0", **kw)
        uvw = torch.as_tensor(ds.uvw, dtype=torch.float64, device="cuda:0")
        D = lk.target(uvw, ds.vis)
        sums = torch.zeros((3, 2), dtype=torch.float64, device="cuda:0")
        lk.loss(lk.gauss, uvw, ds.vis, D, sums[0])
        mse = lk.fit_table(lk.gaussian_table(), steps=800, lr=3e-3)
        lk.install()
        lk.loss(lk.plan, uvw, ds.vis, D, sums[1])
        for _ in range(40):
            lk.step(uvw, ds.vis, D, sums[2], 1e-3)
        lk.install()
        lk.loss(lk.plan, uvw, ds.vis, D, sums[2])
        s = sums.cpu().numpy()
        L = s[:, 0] / s[:, 1]
        print(f"[learned] fit mse {mse:.2e}; loss gaussian {L[0]:.4e}, fitted {L[1]:.4e}, after 40 steps {L[2]:.4e}")
        assert mse < 1e-5
        assert abs(L[1] - L[0]) < 0.1 * L[0]
        assert L[2] < L[1]
    finally:
        lk.close()
