"""Direct DFT dirty image -- TEST INFRASTRUCTURE ONLY.

I_DFT[q][p] = n_pq * sum_j W_j Re(V_j exp(+2 pi i (u_j l_p + v_j m_q + w_j (n_pq - 1)))) / sum_j W_j

over the visibilities that the imager keeps, with exact (unquantised) u, v, w
in wavelengths.  This is Eq. 1 with the (u, v, w) integral replaced by the
weighted sum over measured samples (natural weighting), and the left-hand
1/n moved to the right.  The brute-force sum lives in ``csrc/dft.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names another build of the same C sources (a sanitized one)
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "_liboracle.so")
_SOURCES = [os.path.join(_HERE, "csrc", f) for f in ("dft.c", "pixels.c", "binstats.c")]
_lib = None


def build(force: bool = False) -> str:
    """Compile the C part of the oracle with gcc (OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
               "-I", os.path.join(_HERE, "csrc"), "-o", tmp] + [s for s in _SOURCES if os.path.exists(s)] + ["-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.oracle_dft.argtypes = [ctypes.c_int64, dp, dp, dp, dp, dp, ctypes.c_int64, dp, dp, dp,
                                 ctypes.c_int, dp, dp]
        L.oracle_dft.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def dft_sum(u, v, w, a, l, m, nm1, reverse: bool = False) -> np.ndarray:
    """Complex D at each direction: sum_j a_j exp(+2 pi i (u_j l + v_j m + w_j nm1))."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    a = np.asarray(a, dtype=np.complex128)
    are = np.ascontiguousarray(a.real)
    aim = np.ascontiguousarray(a.imag)
    l = np.ascontiguousarray(l, dtype=np.float64).reshape(-1)
    m = np.ascontiguousarray(m, dtype=np.float64).reshape(-1)
    nm1 = np.ascontiguousarray(nm1, dtype=np.float64).reshape(-1)
    out_re = np.empty(l.shape[0])
    out_im = np.empty(l.shape[0])
    lib().oracle_dft(u.shape[0], _p(u), _p(v), _p(w), _p(are), _p(aim), l.shape[0],
                     _p(l), _p(m), _p(nm1), int(reverse), _p(out_re), _p(out_im))
    return out_re + 1j * out_im


def dft_image(u, v, w, wv, wt_sum: float, fov: float, grid_n: int,
              rows: Optional[slice] = None, cols: Optional[slice] = None,
              complex_out: bool = False, reverse: bool = False) -> np.ndarray:
    """Dirty image (or a rectangular patch of it) by the direct sum.

    ``wv`` = W V of the kept visibilities, ``wt_sum`` = sum of their W.
    Pixels with l^2 + m^2 >= 1 are 0."""
    from .wstack import pixel_lm, nm1_of
    lm = pixel_lm(grid_n, fov)
    rows = rows if rows is not None else slice(0, grid_n)
    cols = cols if cols is not None else slice(0, grid_n)
    ls = lm[cols]
    ms = lm[rows]
    L, M = np.meshgrid(ls, ms)              # [q][p]
    nm1 = nm1_of(L, M)
    inside = np.isfinite(nm1)
    nm1z = np.where(inside, nm1, 0.0)
    D = dft_sum(u, v, w, wv, L, M, nm1z, reverse=reverse).reshape(L.shape)
    n = 1.0 + nm1z
    out = n * D / wt_sum
    if not complex_out:
        out = out.real
    return np.where(inside, out, 0.0)


def dft_of_binned(b, fov: float, grid_n: int, **kw) -> np.ndarray:
    """Direct-DFT image over the visibilities that binning kept."""
    idx = np.nonzero(b.keep)[0]
    return dft_image(b.u[idx], b.v[idx], b.w[idx], b.wv[idx], float(b.wt[idx].sum()), fov, grid_n, **kw)


def dft_pixels_rows(uvw_m, freq_hz, vis, weight, pix_p, pix_q, *, grid_n: int, fov: float,
                    sum_w: float) -> np.ndarray:
    """Dirty-image values by the direct sum at chosen pixels (p, q), for
    visibilities laid out [row][channel] with equally spaced channels and uvw
    in metres (``csrc/dft.c``, ``oracle_dft_rows``: the channel phases of a
    row advance as a geometric progression).  ``sum_w`` is the weight sum of
    the visibilities summed; every visibility given is summed, so the caller
    passes only workloads where the imager keeps them all.  Returns
    n Re(D) / sum_w per pixel; pixels with l^2 + m^2 >= 1 give 0."""
    from .wstack import pixel_lm, nm1_of, C0
    uvw = np.ascontiguousarray(uvw_m, dtype=np.float64)
    nrow = uvw.shape[0]
    s = np.asarray(freq_hz, dtype=np.float64) / C0
    nchan = s.shape[0]
    s0 = float(s[0])
    ds = float(s[1] - s[0]) if nchan > 1 else 0.0
    if nchan > 2 and np.max(np.abs(s - (s0 + np.arange(nchan) * ds))) > 1e-12 * np.max(np.abs(s)):
        raise ValueError("channels are not equally spaced")
    visf = np.ascontiguousarray(np.asarray(vis).reshape(nrow, nchan), dtype=np.complex64).view(np.float32)
    wt = None if weight is None else np.ascontiguousarray(weight, dtype=np.float32).reshape(nrow, nchan)
    lm = pixel_lm(grid_n, fov)
    L = np.ascontiguousarray(lm[np.asarray(pix_p)], dtype=np.float64)
    M = np.ascontiguousarray(lm[np.asarray(pix_q)], dtype=np.float64)
    nm1 = nm1_of(L, M)
    inside = np.isfinite(nm1)
    nm1z = np.ascontiguousarray(np.where(inside, nm1, 0.0))
    out_re = np.empty(L.shape[0])
    out_im = np.empty(L.shape[0])
    fp = ctypes.POINTER(ctypes.c_float)
    L_ = lib()
    L_.oracle_dft_rows.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                   ctypes.c_double, ctypes.c_double, fp, fp, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]
    L_.oracle_dft_rows.restype = None
    L_.oracle_dft_rows(nrow, nchan, _p(uvw), s0, ds, visf.ctypes.data_as(fp),
                       None if wt is None else wt.ctypes.data_as(fp), L.shape[0], _p(L), _p(M), _p(nm1z),
                       _p(out_re), _p(out_im))
    return np.where(inside, (1.0 + nm1z) * out_re / sum_w, 0.0)
