"""Full-size parity: the SKA-LOW-like one-GPU share (209,305,600 visibilities,
4096^2 x 64 planes, W = 7, OS = 64), in the launch configuration the benchmark
times (fused column transform + screen) and in the unfused one, checked where
the float64 oracle can follow at this size:
  - binning: kept count, per-(plane, tile) record counts (bit-exact), sum W;
  - gridding: every plane's cell sum equals its sum of W V (rows of taps sum to 1);
  - F_k and the image at sampled pixels (bright sources, centre, random) against
    the oracle's per-pixel regrouping, which is linear in the visibilities.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2504_00959_amd import rick
from tests.helpers import rel_rms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def share():
    import torch
    print("[fullsize] generating ska_low_share on cuda:0", flush=True)
    ds = synth.ska_low_share(device="cuda:0")
    uvw = torch.as_tensor(ds.uvw, dtype=torch.float64).to("cuda:0")
    vis = ds.vis
    p = rick.Plan.for_dataset(ds)
    p.reset()
    p.grid(uvw, vis, None, ds.freq)
    torch.cuda.synchronize()
    info = p.info()
    nt = ds.grid_n // info["tile"]
    counts = p.bin_counts(ds.n_wplanes * nt * nt)
    G = p.mesh()
    plane_sums = G.to(torch.complex128).sum(dim=(1, 2)).cpu().numpy()
    del G
    p.fft()
    F = p.mesh()
    img = p.image()
    torch.cuda.synchronize()
    p.close()
    # the benchmark's configuration: column transform fused with the screen
    pf = rick.Plan.for_dataset(ds, fused=True)
    pf.reset()
    pf.grid(uvw, vis, None, ds.freq)
    pf.fft()
    img_fused = pf.image()
    torch.cuda.synchronize()
    pf.close()
    vis_host = vis.cpu().numpy()
    # sampled pixels: source positions (bright), the centre, random
    lm = ds.fov / ds.grid_n
    order = np.argsort(-ds.sources["flux"])[:6]
    ps = np.rint(ds.sources["l"][order] / lm).astype(int) + ds.grid_n // 2
    qs = np.rint(ds.sources["m"][order] / lm).astype(int) + ds.grid_n // 2
    rng = np.random.default_rng(7)
    pp = np.r_[ps, ds.grid_n // 2, rng.integers(0, ds.grid_n, 5)]
    qq = np.r_[qs, ds.grid_n // 2, rng.integers(0, ds.grid_n, 5)]
    Fs = F[:, qq, pp].cpu().numpy().T.astype(np.complex128)       # [npix][N_w]
    img_s = img.double().cpu().numpy()[qq, pp]
    img_fused_s = img_fused.double().cpu().numpy()[qq, pp]
    img_rms = float(img.double().pow(2).mean().sqrt())
    del F
    print("[fullsize] GPU path done; running oracle passes", flush=True)
    return dict(ds=ds, vis_host=vis_host, info=info, counts=counts, plane_sums=plane_sums, pp=pp, qq=qq, Fs=Fs,
                img_s=img_s, img_fused_s=img_fused_s, img_rms=img_rms)


def test_fullsize_binning_and_plane_sums(share):
    ds, info = share["ds"], share["info"]
    counts, psum, kept, sw = oracle.pixels.bin_stats(ds.uvw, ds.freq, share["vis_host"], None, tile=info["tile"],
                                                     **ds.plan_kwargs())
    assert info["n_gridded"] == kept
    assert info["n_gridded"] + info["n_dropped"] == ds.nvis
    assert np.array_equal(share["counts"].astype(np.int64), counts)
    assert abs(info["sum_weights"] - sw) <= 1e-12 * sw
    assert rel_rms(share["plane_sums"], psum) <= 1e-6


def test_fullsize_sampled_pixels(share):
    ds = share["ds"]
    ref, Fref, kept, sw = oracle.pixels.wstack_pixels(ds.uvw, ds.freq, share["vis_host"], None, share["pp"],
                                                      share["qq"], **ds.plan_kwargs())
    # compared before the division by the kernel taper (the same float64
    # per-pixel scale on both sides), as in the small-size parity tests
    corr = oracle.wstack.grid_correction(oracle.wstack.tap_table(ds.support, ds.oversample), ds.grid_n)
    c2 = corr[share["pp"]] * corr[share["qq"]]
    e_f = rel_rms(share["Fs"], Fref)
    e_img = rel_rms(share["img_s"] * c2, ref * c2)
    e_fused = rel_rms(share["img_fused_s"] * c2, ref * c2)
    print(f"[fullsize] F rel-RMS {e_f:.2e}, apparent image rel-RMS {e_img:.2e} (fused {e_fused:.2e})", flush=True)
    assert e_f <= 1e-5
    assert e_img <= 1e-5
    assert e_fused <= 1e-5
    # every sampled pixel within 1e-5 of the image RMS
    assert np.max(np.abs(share["img_s"] - ref) * c2) <= 1e-5 * max(share["img_rms"], np.max(np.abs(ref)))
