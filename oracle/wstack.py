"""Float64 w-stacking, one step at a time -- TEST INFRASTRUCTURE ONLY.

The steps follow Sec. 2.1 of the paper in its order: map every visibility to
the closest w-plane and convolve it onto that plane with a finite kernel
(Eq. 3; Gaussian or Kaiser-Bessel), inverse-FFT every plane, multiply plane k
by the w phase screen exp(+2 pi i w_k (n - 1)) of Eq. 1 and sum over planes.

Where the paper is silent these readings are used (each is also recorded in
the design notes of the repository):

* positions are quantised to 1/OS of a cell and the kernel is evaluated at
  the quantised offsets (an oversampled tap table), rows normalised to 1;
* planes are cell-centred, w_k = w_min + (k + 1/2) dw, assignment by floor
  and clamped to [0, N_w - 1];
* the image is Re of the complex sum, multiplied by n (left side of Eq. 1),
  divided by the sum of gridded weights (natural weighting) and by the
  kernel's image-plane taper C(l') C(m');
* pixel p sits at l_p = (p - N/2) FoV/N, cell i at u_i = (i - N/2)/FoV;
* a visibility is dropped (not gridded, not counted in the weight sum) if
  any input is non-finite, its weight is <= 0, or its kernel footprint leaves
  the grid.

Array conventions: planes are [N_w][N][N] indexed [k][row = v][column = u];
the image is [N][N] indexed [q = m][p = l].  Visibilities are flattened as
index = row * n_chan + chan.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

C0 = 299_792_458.0


# ---------------------------------------------------------------------------
# kernels (Sec. 2.1: "either a Gaussian or a Kaiser-Bessel kernel")
# ---------------------------------------------------------------------------
def gaussian_sigma_default(support: int) -> float:
    """Gaussian width (cells) whose value at the support edge W/2 is 1e-3."""
    return (support / 2.0) / math.sqrt(2.0 * math.log(1000.0))


def kb_beta_default(support: int, alpha: float = 2.0) -> float:
    """Kaiser-Bessel shape parameter of Beatty, Nishimura & Pauly (2005) for
    oversampling ratio alpha: beta = pi sqrt((W/alpha)^2 (alpha - 1/2)^2 - 0.8)."""
    x = (support / alpha) ** 2 * (alpha - 0.5) ** 2 - 0.8
    return math.pi * math.sqrt(x) if x > 0.0 else 0.0


def bessel_i0(x: np.ndarray) -> np.ndarray:
    """Modified Bessel function I0 by its power series sum_k ((x/2)^k / k!)^2."""
    x = np.asarray(x, dtype=np.float64)
    q = (x / 2.0) ** 2
    term = np.ones_like(x)
    total = np.ones_like(x)
    for k in range(1, 200):
        term = term * q / (k * k)
        total = total + term
        if np.all(term <= 1e-18 * total):
            break
    return total


def kernel_value(d: np.ndarray, support: int, kernel: str, param: float) -> np.ndarray:
    """Continuous 1-D kernel g(d) at distance d (cells); zero for |d| >= W/2."""
    d = np.asarray(d, dtype=np.float64)
    half = support / 2.0
    inside = np.abs(d) < half
    if kernel == "gaussian":
        sigma = param if param > 0 else gaussian_sigma_default(support)
        g = np.exp(-d * d / (2.0 * sigma * sigma))
    elif kernel in ("kaiser_bessel", "kb"):
        beta = param if param > 0 else kb_beta_default(support)
        arg = 1.0 - (2.0 * d / support) ** 2
        g = bessel_i0(beta * np.sqrt(np.clip(arg, 0.0, None))) / bessel_i0(np.array(beta))
    else:
        raise ValueError(f"unknown kernel {kernel!r}")
    return np.where(inside, g, 0.0)


def tap_table(support: int, oversample: int, kernel: str = "gaussian", param: float = 0.0) -> np.ndarray:
    """Tap weights g_s[t], shape [OS][W]; row index s + OS/2 for the sub-cell
    offset s in [-OS/2, OS/2), column t for the tap at cell offset t - h.

    g_s[t] = g(t - h - s/OS) / sum_t' g(t' - h - s/OS)  (rows sum to 1)."""
    h = (support - 1) // 2
    s = np.arange(-(oversample // 2), oversample - oversample // 2, dtype=np.float64)
    t = np.arange(support, dtype=np.float64) - h
    d = t[None, :] - s[:, None] / oversample
    g = kernel_value(d, support, kernel, param)
    return g / g.sum(axis=1, keepdims=True)


def grid_correction(table: np.ndarray, grid_n: int) -> np.ndarray:
    """Image-plane taper of the tabulated kernel, averaged over sub-cell offsets:
    C(l') = (1/OS) sum_s sum_t g_s[t] cos(2 pi (t - h - s/OS) l'),
    l'_p = (p - N/2)/N for p = 0..N-1."""
    os_, support = table.shape
    h = (support - 1) // 2
    s = np.arange(-(os_ // 2), os_ - os_ // 2, dtype=np.float64)
    d = (np.arange(support, dtype=np.float64) - h)[None, :] - s[:, None] / os_
    lp = (np.arange(grid_n, dtype=np.float64) - grid_n / 2) / grid_n
    # sum over (s, t) of g * cos(2 pi d l')
    ph = 2.0 * np.pi * d.reshape(-1, 1) * lp[None, :]
    return (table.reshape(-1, 1) * np.cos(ph)).sum(axis=0) / os_


# ---------------------------------------------------------------------------
# sky coordinates
# ---------------------------------------------------------------------------
def pixel_lm(grid_n: int, fov: float):
    """Direction cosines of pixel centres: l_p = (p - N/2) FoV/N (same for m)."""
    dl = fov / grid_n
    return (np.arange(grid_n, dtype=np.float64) - grid_n / 2) * dl


def nm1_of(l: np.ndarray, m: np.ndarray) -> np.ndarray:
    """n - 1 = sqrt(1 - l^2 - m^2) - 1, evaluated as -r^2 / (1 + sqrt(1 - r^2));
    NaN where r^2 >= 1."""
    r2 = l * l + m * m
    with np.errstate(invalid="ignore"):
        return np.where(r2 < 1.0, -r2 / (1.0 + np.sqrt(1.0 - r2)), np.nan)


# ---------------------------------------------------------------------------
# step 1: positions, planes, drops
# ---------------------------------------------------------------------------
@dataclass
class Binned:
    X: np.ndarray      # int64 position in 1/OS cells (flattened)
    Y: np.ndarray
    cx: np.ndarray     # int64 nearest cell
    cy: np.ndarray
    sx: np.ndarray     # int64 sub-cell offset in [-OS/2, OS/2)
    sy: np.ndarray
    k: np.ndarray      # int64 w-plane
    keep: np.ndarray   # bool
    u: np.ndarray      # float64 wavelengths (unquantised)
    v: np.ndarray
    w: np.ndarray
    wv: np.ndarray     # complex128 W * V
    wt: np.ndarray     # float64 W


def scales_of(freq: Optional[np.ndarray]) -> Optional[np.ndarray]:
    """Metres -> wavelengths factor nu_c / c0 per channel (None: uvw already in wavelengths)."""
    if freq is None:
        return None
    return np.asarray(freq, dtype=np.float64) / C0


def bin_visibilities(uvw, freq, vis, weight, *, grid_n, n_wplanes, support, oversample,
                     fov, w_min, w_max) -> Binned:
    """Quantise positions to 1/OS cell, choose the closest w-plane, drop.

    For visibility (row r, channel c):
      u = uvw[r,0] * (nu_c/c0)                     (no factor if freq is None)
      X = rint((u * FoV) * OS + N*OS/2)            (round half to even)
      c_x = floor((X + OS/2) / OS),  s_x = X - c_x * OS
      dw = (w_max - w_min) / N_w,  k = clamp(floor((w - w_min) / dw), 0, N_w - 1)
      drop if anything is non-finite, |position| beyond 2^30 sub-cells,
      W <= 0, or c_x - h < 0 or c_x + h > N - 1 (same in y).
    """
    uvw = np.asarray(uvw, dtype=np.float64)
    R = uvw.shape[0]
    sc = scales_of(freq)
    C = 1 if sc is None else len(sc)
    if sc is None:
        u = np.repeat(uvw[:, 0:1], 1, axis=1)
        v = np.repeat(uvw[:, 1:2], 1, axis=1)
        w = np.repeat(uvw[:, 2:3], 1, axis=1)
    else:
        u = uvw[:, 0:1] * sc[None, :]
        v = uvw[:, 1:2] * sc[None, :]
        w = uvw[:, 2:3] * sc[None, :]
    u, v, w = u.reshape(-1), v.reshape(-1), w.reshape(-1)
    vis = np.asarray(vis).reshape(R * C)
    wt = np.ones(R * C) if weight is None else np.asarray(weight, dtype=np.float64).reshape(R * C)
    vr = vis.real.astype(np.float64)
    vi = vis.imag.astype(np.float64)
    OS, N, h = oversample, grid_n, (support - 1) // 2
    finite = (np.isfinite(u) & np.isfinite(v) & np.isfinite(w) & np.isfinite(vr)
              & np.isfinite(vi) & np.isfinite(wt))
    with np.errstate(invalid="ignore", over="ignore"):
        xs = (u * fov) * OS + (N * OS) / 2
        ys = (v * fov) * OS + (N * OS) / 2
        lim = float(2 ** 30)
        inrange = (np.abs(xs) <= lim) & (np.abs(ys) <= lim)
        ok = finite & inrange
        Xf = np.where(ok, np.rint(xs), 0.0)
        Yf = np.where(ok, np.rint(ys), 0.0)
    X = Xf.astype(np.int64)
    Y = Yf.astype(np.int64)
    cx = (X + OS // 2) // OS
    cy = (Y + OS // 2) // OS
    sx = X - cx * OS
    sy = Y - cy * OS
    dw = (w_max - w_min) / n_wplanes
    with np.errstate(invalid="ignore", over="ignore"):
        kf = np.floor((w - w_min) / dw)
        kf = np.where(np.isnan(kf), 0.0, kf)      # w outside the range -> nearest end plane
    k = np.clip(kf, 0, n_wplanes - 1).astype(np.int64)
    keep = (ok & (wt > 0) & (cx - h >= 0) & (cx + h <= N - 1) & (cy - h >= 0) & (cy + h <= N - 1))
    with np.errstate(invalid="ignore"):
        wv = wt * (vr + 1j * vi)
    return Binned(X=X, Y=Y, cx=cx, cy=cy, sx=sx, sy=sy, k=k, keep=keep, u=u, v=v, w=w, wv=wv, wt=wt)


def plane_centres(w_min: float, w_max: float, n_wplanes: int) -> np.ndarray:
    """w_k = w_min + (k + 1/2) dw."""
    dw = (w_max - w_min) / n_wplanes
    return w_min + (np.arange(n_wplanes, dtype=np.float64) + 0.5) * dw


# ---------------------------------------------------------------------------
# step 2: gridding (Eq. 3 with the separable tap table, nearest plane)
# ---------------------------------------------------------------------------
def grid(b: Binned, table: np.ndarray, *, grid_n, n_wplanes) -> np.ndarray:
    """G_k[c_y + t_y - h][c_x + t_x - h] += W V g_{s_y}[t_y] g_{s_x}[t_x]; complex128 [N_w][N][N]."""
    OS, support = table.shape
    h = (support - 1) // 2
    N = grid_n
    G = np.zeros((n_wplanes, N, N), dtype=np.complex128)
    keep = np.nonzero(b.keep)[0]
    for kk in range(n_wplanes):
        grid_plane(G[kk], b, keep[b.k[keep] == kk], table)
    return G


def grid_plane(Gk: np.ndarray, b: Binned, idx: np.ndarray, table: np.ndarray) -> None:
    """Add the visibilities ``idx`` (all of one plane) onto plane ``Gk`` [N][N]:
    Gk[c_y + t_y - h][c_x + t_x - h] += W V g_{s_y}[t_y] g_{s_x}[t_x]."""
    OS, support = table.shape
    h = (support - 1) // 2
    N = Gk.shape[-1]
    if idx.size == 0:
        return
    t = np.arange(support) - h
    gx = table[b.sx[idx] + OS // 2]          # [n, W]
    gy = table[b.sy[idx] + OS // 2]
    rows = (b.cy[idx][:, None] + t[None, :]) * N            # [n, W]
    cols = b.cx[idx][:, None] + t[None, :]
    cell = (rows[:, :, None] + cols[:, None, :]).reshape(-1)                 # [n * W * W]
    wgt = (gy[:, :, None] * gx[:, None, :]).reshape(idx.size, -1)           # [n, W * W]
    wv = b.wv[idx][:, None]
    re = np.bincount(cell, weights=(wv.real * wgt).reshape(-1), minlength=N * N)
    im = np.bincount(cell, weights=(wv.imag * wgt).reshape(-1), minlength=N * N)
    Gk += (re + 1j * im).reshape(N, N)


# ---------------------------------------------------------------------------
# step 3: inverse FFT of every plane, centred
# ---------------------------------------------------------------------------
def ifft_planes(G: np.ndarray) -> np.ndarray:
    """F_k[q][p] = sum_{j,i} G_k[j][i] exp(+2 pi i ((i-N/2)(p-N/2) + (j-N/2)(q-N/2)) / N)."""
    N = G.shape[-1]
    ax = (-2, -1)
    return np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(G, axes=ax), axes=ax), axes=ax) * (N * N)


# ---------------------------------------------------------------------------
# step 4: w phase screen, sum over planes, normalise
# ---------------------------------------------------------------------------
def screen_sum(F: np.ndarray, w_k: np.ndarray, fov: float) -> np.ndarray:
    """S[q][p] = sum_k Re(exp(+2 pi i w_k (n_pq - 1)) F_k[q][p]).

    The phase is taken in turns, tau = w_k (n - 1), reduced to
    tau - rint(tau) before the trigonometric evaluation."""
    N = F.shape[-1]
    l = pixel_lm(N, fov)
    nm1 = nm1_of(l[None, :], l[:, None])          # [q][p]
    nm1z = np.where(np.isfinite(nm1), nm1, 0.0)
    S = np.zeros((N, N))
    for k in range(F.shape[0]):
        tau = w_k[k] * nm1z
        tr = tau - np.rint(tau)
        S += np.cos(2 * np.pi * tr) * F[k].real - np.sin(2 * np.pi * tr) * F[k].imag
    return S


def normalise(S: np.ndarray, corr: np.ndarray, sum_w: float, fov: float) -> np.ndarray:
    """I[q][p] = n_pq S[q][p] / (C(l'_p) C(l'_q) sum W); zero outside the unit circle,
    and zero everywhere when no visibility was gridded (sum W = 0)."""
    N = S.shape[-1]
    if not sum_w > 0.0:
        return np.zeros_like(S)
    l = pixel_lm(N, fov)
    nm1 = nm1_of(l[None, :], l[:, None])
    inside = np.isfinite(nm1)
    n = 1.0 + np.where(inside, nm1, 0.0)
    I = n * S / (corr[None, :] * corr[:, None] * sum_w)
    return np.where(inside, I, 0.0)


# ---------------------------------------------------------------------------
# whole pipeline
# ---------------------------------------------------------------------------
@dataclass
class Result:
    image: np.ndarray
    planes: np.ndarray      # G_k
    fplanes: np.ndarray     # F_k
    binned: Binned
    table: np.ndarray
    corr: np.ndarray
    sum_w: float
    w_k: np.ndarray


def wstack_image(uvw, freq, vis, weight, *, grid_n, n_wplanes, support, oversample, fov,
                 w_min, w_max, kernel="gaussian", kernel_param=0.0, keep_planes=True) -> Result:
    """Dirty image by w-stacking, float64, all steps in the paper's order."""
    table = tap_table(support, oversample, kernel, kernel_param)
    b = bin_visibilities(uvw, freq, vis, weight, grid_n=grid_n, n_wplanes=n_wplanes,
                         support=support, oversample=oversample, fov=fov, w_min=w_min, w_max=w_max)
    G = grid(b, table, grid_n=grid_n, n_wplanes=n_wplanes)
    F = ifft_planes(G)
    w_k = plane_centres(w_min, w_max, n_wplanes)
    S = screen_sum(F, w_k, fov)
    corr = grid_correction(table, grid_n)
    sum_w = float(b.wt[b.keep].sum())
    I = normalise(S, corr, sum_w, fov)
    return Result(image=I, planes=G if keep_planes else None, fplanes=F if keep_planes else None,
                  binned=b, table=table, corr=corr, sum_w=sum_w, w_k=w_k)


def wstack_dataset(ds, **over) -> Result:
    kw = ds.plan_kwargs()
    kw.update(over)
    vis = ds.vis
    if hasattr(vis, "detach"):
        vis = vis.detach().cpu().numpy()
    return wstack_image(ds.uvw, ds.freq, vis, ds.weight, **kw)


def bin_keys(b: Binned, *, grid_n: int, tile: int) -> np.ndarray:
    """(plane, tile row, tile column) of every kept visibility's nearest cell,
    as one integer k * (N/T)^2 + (c_y // T) * (N/T) + c_x // T."""
    nt = grid_n // tile
    idx = np.nonzero(b.keep)[0]
    return b.k[idx] * nt * nt + (b.cy[idx] // tile) * nt + (b.cx[idx] // tile)
