"""rick_grid_static (sort buffers in the library's static device scratch,
nothing allocated) against rick_grid (sort buffers in the plan), through the
C ABI, on two calls in a row on one plan, the second with a smaller input:
the same kept and dropped counts, weight sum and per-bin record counts
(exact), the same gridded planes and image (float32 rounding of split bins
aside), and the image against the float64 oracle; plus the capacity error
for a call larger than the scratch.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from paper_2504_00959_amd import rick
from tests.helpers import image_errors, rel_rms, to_device

pytestmark = pytest.mark.gpu


def _grid_image(p, ds, uvw, vis, wt, static):
    import torch
    p.reset()
    p.grid(uvw, vis, wt, ds.freq, static_scratch=static)
    torch.cuda.synchronize()
    info = p.info()
    nt = ds.grid_n // info["tile"]
    counts = p.bin_counts(ds.n_wplanes * nt * nt)
    G = p.mesh().cpu().numpy()
    p.fft()
    img = p.image().double().cpu().numpy()
    torch.cuda.synchronize()
    return info, counts, G, img


def _subset(ds, nrow):
    sub = synth.Dataset(**{**ds.__dict__})
    sub.uvw = ds.uvw[:nrow]
    sub.vis = ds.vis[:nrow]
    sub.weight = None if ds.weight is None else ds.weight[:nrow]
    return sub


@pytest.mark.parametrize("precision,g_tol,i_tol", [("fp32", 1e-6, 1e-5), ("fp64", 1e-12, 1e-10)])
def test_grid_static_matches_grid_on_two_calls(precision, g_tol, i_tol):
    import torch
    big = synth.ska_low_small()
    small = _subset(big, big.nrow // 3)
    ref_plan = rick.Plan.for_dataset(big, precision=precision)
    st_plan = rick.Plan.for_dataset(big, precision=precision, max_vis=0)   # no sort buffers of its own
    try:
        for ds in (big, small):
            uvw, vis, wt = to_device(ds, precision)
            ri, rc, rG, rimg = _grid_image(ref_plan, ds, uvw, vis, wt, static=False)
            si, sc, sG, simg = _grid_image(st_plan, ds, uvw, vis, wt, static=True)
            ref = oracle.wstack.wstack_dataset(ds)
            # image against image: before the taper division in float32 (the
            # division magnifies rounding at the edge), whole image in float64
            pair = image_errors(simg, rimg, ref.corr)
            print(f"[no-alloc] {precision} nvis={ds.nvis}: gridded {si['n_gridded']}, "
                  f"G rel-RMS {rel_rms(sG, rG):.2e}, image {pair}", flush=True)
            assert si["n_gridded"] == ri["n_gridded"] > 0
            assert si["n_dropped"] == ri["n_dropped"]
            assert si["n_gridded"] + si["n_dropped"] == ds.nvis
            assert si["sum_weights"] == ri["sum_weights"]
            assert np.array_equal(sc, rc)
            assert rel_rms(sG, rG) <= g_tol
            assert pair["apparent"] <= g_tol and pair["central"] <= g_tol
            if precision == "fp64":
                assert pair["full"] <= g_tol
            errs = image_errors(simg, ref.image, ref.corr)
            gated = [errs["apparent"], errs["central"]] + ([errs["full"]] if precision == "fp64" else [])
            assert max(gated) <= i_tol, errs
            del uvw, vis, wt
            torch.cuda.empty_cache()
    finally:
        ref_plan.close()
        st_plan.close()


def test_grid_static_capacity_and_plain_grid_refused_without_buffers():
    import torch
    ds = synth.tiny(nrow=4096)
    uvw, vis, wt = to_device(ds, "fp32")
    p = rick.Plan.for_dataset(ds, max_vis=0)
    try:
        L = rick.lib()
        # larger than the static scratch: refused on the host, before any device work
        st = L.rick_grid_static(p._h, uvw.data_ptr(), None, vis.data_ptr(), None, 1 << 28, 1, None)
        assert st == 5   # RICK_E_CAPACITY
        assert b"static scratch" in L.rick_last_error()
        # a plan without sort buffers refuses rick_grid of any visibility
        st = L.rick_grid(p._h, uvw.data_ptr(), None, vis.data_ptr(), None, 16, 1, None)
        assert st == 5
        # and grids through the static scratch
        p.reset()
        p.grid(uvw, vis, wt, ds.freq, static_scratch=True)
        torch.cuda.synchronize()
        assert p.info()["n_gridded"] > 0
    finally:
        p.close()
