"""w-stacking image at chosen pixels, from raw inputs -- TEST INFRASTRUCTURE ONLY.

Same result as ``oracle.wstack.wstack_image`` at the requested pixels (the
per-plane sums are regrouped per pixel, see ``csrc/pixels.c``), at a cost
linear in the number of visibilities, so that full-size workloads can be
checked at sampled pixels.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import dft as _dft
from .wstack import tap_table, grid_correction, plane_centres, pixel_lm, nm1_of, scales_of

_sig_done = False


def _lib():
    global _sig_done
    L = _dft.lib()
    if not _sig_done:
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        ip = ctypes.POINTER(ctypes.c_int32)
        L.oracle_wstack_pixels.argtypes = [
            ctypes.c_int64, ctypes.c_int32, dp, dp, fp, fp,
            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
            ctypes.c_double, ctypes.c_double, dp,
            ctypes.c_int64, ip, ip, dp, dp]
        L.oracle_wstack_pixels.restype = ctypes.c_int64
        _sig_done = True
    return L


def wstack_pixels(uvw, freq, vis, weight, pix_p, pix_q, *, grid_n, n_wplanes, support, oversample,
                  fov, w_min, w_max, kernel="gaussian", kernel_param=0.0):
    """Returns (image values at (q, p) pairs, per-plane F_k at those pixels [npix][N_w], kept count, sum W)."""
    uvw = np.ascontiguousarray(uvw, dtype=np.float64)
    nrow = uvw.shape[0]
    sc = scales_of(freq)
    nchan = 1 if sc is None else len(sc)
    vis = np.ascontiguousarray(np.asarray(vis).reshape(nrow, nchan), dtype=np.complex64)
    visf = vis.view(np.float32)
    wt = None if weight is None else np.ascontiguousarray(weight, dtype=np.float32).reshape(nrow, nchan)
    table = np.ascontiguousarray(tap_table(support, oversample, kernel, kernel_param))
    pix_p = np.ascontiguousarray(pix_p, dtype=np.int32)
    pix_q = np.ascontiguousarray(pix_q, dtype=np.int32)
    npix = pix_p.shape[0]
    acc = np.zeros((npix, n_wplanes, 2))
    sum_w = ctypes.c_double(0.0)
    dw = (w_max - w_min) / n_wplanes
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    ip = ctypes.POINTER(ctypes.c_int32)
    sc_arr = None if sc is None else np.ascontiguousarray(sc)
    kept = _lib().oracle_wstack_pixels(
        nrow, nchan, uvw.ctypes.data_as(dp), None if sc_arr is None else sc_arr.ctypes.data_as(dp),
        visf.ctypes.data_as(fp), None if wt is None else wt.ctypes.data_as(fp),
        grid_n, n_wplanes, support, oversample, fov, w_min, dw, table.ctypes.data_as(dp),
        npix, pix_p.ctypes.data_as(ip), pix_q.ctypes.data_as(ip), acc.ctypes.data_as(dp),
        ctypes.byref(sum_w))
    F = acc[..., 0] + 1j * acc[..., 1]          # [npix][N_w]
    lm = pixel_lm(grid_n, fov)
    nm1 = nm1_of(lm[pix_p], lm[pix_q])
    inside = np.isfinite(nm1)
    nm1z = np.where(inside, nm1, 0.0)
    w_k = plane_centres(w_min, w_max, n_wplanes)
    tau = nm1z[:, None] * w_k[None, :]
    tr = tau - np.rint(tau)
    S = (np.cos(2 * np.pi * tr) * F.real - np.sin(2 * np.pi * tr) * F.imag).sum(axis=1)
    corr = grid_correction(table, grid_n)
    if not sum_w.value > 0.0:
        return np.zeros(npix), F, int(kept), 0.0
    img = (1.0 + nm1z) * S / (corr[pix_p] * corr[pix_q] * sum_w.value)
    return np.where(inside, img, 0.0), F, int(kept), float(sum_w.value)


def wstack_pixels_dataset(ds, pix_p, pix_q, vis=None):
    v = ds.vis if vis is None else vis
    if hasattr(v, "detach"):
        v = v.detach().cpu().numpy()
    return wstack_pixels(ds.uvw, ds.freq, v, ds.weight, pix_p, pix_q, **ds.plan_kwargs())


def bin_stats(uvw, freq, vis, weight, *, tile, grid_n, n_wplanes, support, oversample, fov, w_min, w_max,
              **_ignored):
    """Whole-input binning statistics (see ``csrc/binstats.c``): per-(plane, tile)
    record counts [N_w * (N/T)^2] (int64), per-plane sums of W V (complex), kept count, sum W."""
    L = _lib()
    if not getattr(L, "_binstats_sig", False):
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        lp = ctypes.POINTER(ctypes.c_int64)
        L.oracle_bin_stats.argtypes = [ctypes.c_int64, ctypes.c_int32, dp, dp, fp, fp, ctypes.c_int32,
                                       ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_int32, lp, dp, dp]
        L.oracle_bin_stats.restype = ctypes.c_int64
        L._binstats_sig = True
    uvw = np.ascontiguousarray(uvw, dtype=np.float64)
    nrow = uvw.shape[0]
    sc = scales_of(freq)
    nchan = 1 if sc is None else len(sc)
    vis = np.ascontiguousarray(np.asarray(vis).reshape(nrow, nchan), dtype=np.complex64)
    wt = None if weight is None else np.ascontiguousarray(weight, dtype=np.float32).reshape(nrow, nchan)
    nt = grid_n // tile
    counts = np.zeros(n_wplanes * nt * nt, dtype=np.int64)
    psum = np.zeros((n_wplanes, 2))
    sum_w = ctypes.c_double(0.0)
    dp = ctypes.POINTER(ctypes.c_double)
    fp = ctypes.POINTER(ctypes.c_float)
    sc_arr = None if sc is None else np.ascontiguousarray(sc)
    kept = L.oracle_bin_stats(
        nrow, nchan, uvw.ctypes.data_as(dp), None if sc_arr is None else sc_arr.ctypes.data_as(dp),
        vis.view(np.float32).ctypes.data_as(fp), None if wt is None else wt.ctypes.data_as(fp), grid_n, n_wplanes,
        support, oversample, fov, w_min, (w_max - w_min) / n_wplanes, tile,
        counts.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), psum.ctypes.data_as(dp), ctypes.byref(sum_w))
    return counts, psum[:, 0] + 1j * psum[:, 1], int(kept), float(sum_w.value)
