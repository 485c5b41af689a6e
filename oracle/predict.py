"""Float64 w-stacking prediction (degridding) -- TEST INFRASTRUCTURE ONLY.

Evaluates the visibility model of Eq. 2 from a model sky image with the same
discretisation the imaging steps of Sec. 2.1 use, run the other way:

 1. plane images
      P_k[q][p] = M[q][p] exp(-2 pi i w_k (n_pq - 1)) / (n_pq C(l'_p) C(l'_q)),
    zero outside the unit circle;
 2. centred forward DFT of every plane
      H_k[j][i] = sum_{q,p} P_k[q][p] exp(-2 pi i ((i-N/2)(p-N/2) + (j-N/2)(q-N/2)) / N);
 3. interpolation with the gridding kernel's tap table (Eq. 3 read backwards)
    at the visibility's quantised position on its closest plane:
      V = sum_{t_y, t_x} g_{s_y}[t_y] g_{s_x}[t_x] H_k[c_y + t_y - h][c_x + t_x - h].

Readings (the paper describes imaging only; prediction is Eq. 2 discretised so
that it is the adjoint of the imaging steps, before their real part and
weight normalisation):

* quantisation, plane choice and drop rule are imaging's
  (``wstack.bin_visibilities``); a visibility imaging would drop (a non-finite
  coordinate, or a footprint leaving the grid) is predicted as 0; weights and
  visibility values play no part;
* M is the brightness per pixel: a point source of flux S at pixel (p0, q0)
  predicts S / n_0 exp(-2 pi i (u l_0 + v m_0 + w (n_0 - 1))) (Eq. 2);
* the phase w_k (n - 1) is taken in turns and reduced to tau - rint(tau)
  before the trigonometric evaluation, as in imaging.

Array conventions as in ``wstack``: planes [N_w][N][N] indexed [k][v][u],
images [N][N] indexed [q = m][p = l], visibilities flattened row * n_chan +
chan.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

from . import wstack as ow


def plane_images(M: np.ndarray, w_k: np.ndarray, corr: np.ndarray, fov: float) -> np.ndarray:
    """Step 1: P_k = M exp(-2 pi i w_k (n - 1)) / (n C_p C_q), zero where r >= 1."""
    N = M.shape[-1]
    l = ow.pixel_lm(N, fov)
    nm1 = ow.nm1_of(l[None, :], l[:, None])          # [q][p]
    inside = np.isfinite(nm1)
    nm1z = np.where(inside, nm1, 0.0)
    base = np.where(inside, M / ((1.0 + nm1z) * corr[None, :] * corr[:, None]), 0.0)
    P = np.empty((len(w_k), N, N), dtype=np.complex128)
    for k, wk in enumerate(w_k):
        tau = wk * nm1z
        tr = tau - np.rint(tau)
        P[k] = base * (np.cos(2 * np.pi * tr) - 1j * np.sin(2 * np.pi * tr))
    return P


def fft_planes_forward(P: np.ndarray) -> np.ndarray:
    """Step 2: H_k[j][i] = sum_{q,p} P_k[q][p] exp(-2 pi i ((i-N/2)(p-N/2) + (j-N/2)(q-N/2)) / N)."""
    ax = (-2, -1)
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(P, axes=ax), axes=ax), axes=ax)


def degrid(H: np.ndarray, b: "ow.Binned", table: np.ndarray) -> np.ndarray:
    """Step 3: V = sum_{t_y,t_x} g_{s_y}[t_y] g_{s_x}[t_x] H_k[c_y + t_y - h][c_x + t_x - h]
    for every kept visibility, 0 for the others; complex128, flattened."""
    OS, support = table.shape
    h = (support - 1) // 2
    V = np.zeros(b.keep.shape[0], dtype=np.complex128)
    idx = np.nonzero(b.keep)[0]
    if idx.size == 0:
        return V
    t = np.arange(support) - h
    gx = table[b.sx[idx] + OS // 2]                       # [n, W]
    gy = table[b.sy[idx] + OS // 2]
    rows = b.cy[idx][:, None] + t[None, :]               # [n, W]
    cols = b.cx[idx][:, None] + t[None, :]
    k = b.k[idx]
    vals = H[k[:, None, None], rows[:, :, None], cols[:, None, :]]        # [n, W, W]
    V[idx] = np.einsum("ny,nx,nyx->n", gy, gx, vals)
    return V


@dataclass
class Predicted:
    vis: np.ndarray        # complex128 [nrow * nchan]
    binned: "ow.Binned"
    planes: Optional[np.ndarray]   # H_k
    table: np.ndarray
    corr: np.ndarray
    w_k: np.ndarray


def _binned_positions(uvw, freq, *, grid_n, n_wplanes, support, oversample, fov, w_min, w_max):
    uvw = np.asarray(uvw, dtype=np.float64)
    nchan = 1 if freq is None else len(freq)
    zeros = np.zeros((uvw.shape[0], nchan), dtype=np.complex64)
    return ow.bin_visibilities(uvw, freq, zeros, None, grid_n=grid_n, n_wplanes=n_wplanes, support=support,
                               oversample=oversample, fov=fov, w_min=w_min, w_max=w_max)


def wstack_predict(model, uvw, freq, *, grid_n, n_wplanes, support, oversample, fov, w_min, w_max,
                   kernel="gaussian", kernel_param=0.0, keep_planes=True) -> Predicted:
    """Visibilities of the model image by w-stacking, float64, steps 1-3 in order."""
    M = np.asarray(model, dtype=np.float64)
    table = ow.tap_table(support, oversample, kernel, kernel_param)
    corr = ow.grid_correction(table, grid_n)
    w_k = ow.plane_centres(w_min, w_max, n_wplanes)
    b = _binned_positions(uvw, freq, grid_n=grid_n, n_wplanes=n_wplanes, support=support,
                          oversample=oversample, fov=fov, w_min=w_min, w_max=w_max)
    H = fft_planes_forward(plane_images(M, w_k, corr, fov))
    V = degrid(H, b, table)
    return Predicted(vis=V, binned=b, planes=H if keep_planes else None, table=table, corr=corr, w_k=w_k)


def wstack_predict_sparse(pix_p, pix_q, flux, uvw, freq, *, grid_n, n_wplanes, support, oversample, fov,
                          w_min, w_max, kernel="gaussian", kernel_param=0.0) -> np.ndarray:
    """The same three steps for a model that is zero except at the listed
    pixels, with H_k evaluated only at the cells each visibility reads, by the
    sum of step 2 over the listed pixels (no FFT).  For checking a few
    visibilities of a large grid.  Returns complex128 [nrow * nchan]."""
    N = grid_n
    table = ow.tap_table(support, oversample, kernel, kernel_param)
    corr = ow.grid_correction(table, N)
    w_k = ow.plane_centres(w_min, w_max, n_wplanes)
    b = _binned_positions(uvw, freq, grid_n=N, n_wplanes=n_wplanes, support=support,
                          oversample=oversample, fov=fov, w_min=w_min, w_max=w_max)
    pp = np.asarray(pix_p, dtype=np.int64)
    qq = np.asarray(pix_q, dtype=np.int64)
    S = np.asarray(flux, dtype=np.float64)
    l = ow.pixel_lm(N, fov)
    nm1 = ow.nm1_of(l[pp], l[qq])
    inside = np.isfinite(nm1)
    nm1z = np.where(inside, nm1, 0.0)
    base = np.where(inside, S / ((1.0 + nm1z) * corr[pp] * corr[qq]), 0.0)
    OS, W = table.shape
    h = (W - 1) // 2
    t = np.arange(W) - h
    V = np.zeros(b.keep.shape[0], dtype=np.complex128)
    for j in np.nonzero(b.keep)[0]:
        tau = w_k[b.k[j]] * nm1z
        tr = tau - np.rint(tau)
        Pk = base * (np.cos(2 * np.pi * tr) - 1j * np.sin(2 * np.pi * tr))           # [n_src]
        ci = b.cx[j] + t                                                              # [W]
        cj = b.cy[j] + t
        ex = np.exp(-2j * np.pi * np.outer(ci - N // 2, pp - N // 2) / N)              # [W, n_src]
        ey = np.exp(-2j * np.pi * np.outer(cj - N // 2, qq - N // 2) / N)
        Hc = (ey[:, None, :] * ex[None, :, :] * Pk[None, None, :]).sum(axis=-1)      # [W_y, W_x]
        gx = table[b.sx[j] + OS // 2]
        gy = table[b.sy[j] + OS // 2]
        V[j] = gy @ Hc @ gx
    return V


def predict_direct(model, uvw, freq, fov, idx=None) -> np.ndarray:
    """Eq. 2 as a sum over the model's pixels, at the exact (unquantised)
    positions: V = sum_{q,p} M[q][p] / n_pq exp(-2 pi i (u l_p + v m_q + w (n_pq - 1))),
    pixels outside the unit circle left out.  ``idx`` selects visibilities
    (flattened indices); returns complex128."""
    M = np.asarray(model, dtype=np.float64)
    N = M.shape[-1]
    uvw = np.asarray(uvw, dtype=np.float64)
    sc = ow.scales_of(freq)
    if sc is None:
        u, v, w = uvw[:, 0:1], uvw[:, 1:2], uvw[:, 2:3]
    else:
        u, v, w = uvw[:, 0:1] * sc, uvw[:, 1:2] * sc, uvw[:, 2:3] * sc
    u, v, w = u.reshape(-1), v.reshape(-1), w.reshape(-1)
    if idx is not None:
        u, v, w = u[idx], v[idx], w[idx]
    l = ow.pixel_lm(N, fov)
    nm1 = ow.nm1_of(l[None, :], l[:, None])
    q, p = np.nonzero(np.isfinite(nm1) & (M != 0))
    lp, mq, n1 = l[p], l[q], nm1[q, p]
    amp = M[q, p] / (1.0 + n1)
    out = np.empty(u.shape[0], dtype=np.complex128)
    for s in range(0, u.shape[0], 256):
        ph = (u[s:s + 256, None] * lp[None, :] + v[s:s + 256, None] * mq[None, :]
              + w[s:s + 256, None] * n1[None, :])
        out[s:s + 256] = (amp[None, :] * np.exp(-2j * np.pi * ph)).sum(axis=1)
    return out
