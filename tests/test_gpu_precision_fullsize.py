"""Full-size parity of the precision form: the 418,611,200-visibility
SKA-LOW-like workload (32 channels, 8192^2 x 128 planes, W = 7, OS = 64) in
the launch configuration the benchmark times (float32 with the compensated
plane sum, column transform fused with the screen), checked where the
float64 oracle can follow at this size:
  - binning: kept count, sum W and every per-(plane, tile) record count
    (bit-exact) against the oracle's C pass;
  - the image at sampled pixels (a patch at the phase centre and the
    brightest sources) against the oracle's per-pixel regrouping, before the
    taper division (the same float64 per-pixel scale on both sides).
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2504_00959_amd import rick
from tests.helpers import rel_rms

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def precision_run():
    import torch
    print("[precision-fullsize] generating ska_low_precision on cuda:0", flush=True)
    ds = synth.ska_low_precision(device="cuda:0")
    uvw = torch.as_tensor(ds.uvw, dtype=torch.float64).to("cuda:0")
    p = rick.Plan.for_dataset(ds, precision="fp32_kahan", fused=True)
    p.reset()
    p.grid(uvw, ds.vis, None, ds.freq)
    p.fft()
    img = p.image()
    torch.cuda.synchronize()
    info = p.info()
    nt = ds.grid_n // info["tile"]
    counts = p.bin_counts(ds.n_wplanes * nt * nt)
    p.close()
    N = ds.grid_n
    half = 2
    qq, pp = np.meshgrid(np.arange(N // 2 - half, N // 2 + half), np.arange(N // 2 - half, N // 2 + half),
                         indexing="ij")
    order = np.argsort(-ds.sources["flux"])[:4]
    dl = ds.fov / N
    pp = np.r_[pp.ravel(), np.rint(ds.sources["l"][order] / dl).astype(int) + N // 2]
    qq = np.r_[qq.ravel(), np.rint(ds.sources["m"][order] / dl).astype(int) + N // 2]
    img_s = img.double().cpu().numpy()[qq, pp]
    del img, uvw
    torch.cuda.empty_cache()
    vis_host = ds.vis.cpu().numpy()
    print("[precision-fullsize] GPU path done; running oracle passes", flush=True)
    return dict(ds=ds, vis_host=vis_host, info=info, counts=counts, pp=pp, qq=qq, img_s=img_s)


def test_precision_fullsize_binning(precision_run):
    ds, info = precision_run["ds"], precision_run["info"]
    counts, _, kept, sw = oracle.pixels.bin_stats(ds.uvw, ds.freq, precision_run["vis_host"], None,
                                                  tile=info["tile"], **ds.plan_kwargs())
    assert info["n_gridded"] == kept == ds.nvis
    assert abs(info["sum_weights"] - sw) <= 1e-12 * sw
    assert np.array_equal(precision_run["counts"].astype(np.int64), counts)


def test_precision_fullsize_sampled_pixels(precision_run):
    ds = precision_run["ds"]
    pp, qq = precision_run["pp"], precision_run["qq"]
    ref, _, kept, _ = oracle.pixels.wstack_pixels(ds.uvw, ds.freq, precision_run["vis_host"], None, pp, qq,
                                                  **ds.plan_kwargs())
    corr = oracle.wstack.grid_correction(oracle.wstack.tap_table(ds.support, ds.oversample), ds.grid_n)
    c2 = corr[pp] * corr[qq]
    e = rel_rms(precision_run["img_s"] * c2, ref * c2)
    print(f"[precision-fullsize] apparent image rel-RMS at {len(pp)} pixels: {e:.2e}", flush=True)
    assert kept == ds.nvis
    assert e <= 1e-5
