"""Learned gridding kernel, float64 -- TEST INFRASTRUCTURE ONLY.

The paper grids with a Gaussian or a Kaiser-Bessel kernel (Sec. 2.1, Eq. 3).
This module is the reference for a kernel learned instead: a small MLP maps
(tap offset in x, tap offset in y, w-fraction) to a tap value; the values are
tabulated into an oversampled, non-separable table indexed by the
visibility's w-fraction bin; the rest of the imaging steps are those of
``wstack`` (closest plane, inverse FFT per plane, w phase screen of Eq. 1,
sum over planes), with the image-plane taper of the non-separable table in
place of the product C(l') C(m').

Readings (none of this is in the paper; each is recorded in the design notes):

* kernel value   K(dx, dy, f) = exp(mlp(dx / (W/2), dy / (W/2), f)) for
  |dx| < W/2 and |dy| < W/2, else 0; the MLP is 3 -> 32 -> 32 -> 1 with tanh
  after both hidden layers and a linear output (exp keeps the kernel
  positive, like the Gaussian and Kaiser-Bessel ones, so the rows can be
  normalised);
* w-fraction     for r = (w - w_min) / dw and the closest plane
  k = clamp(floor(r), 0, N_w - 1): f = r - k, bin iw = clamp(floor(f N_f), 0,
  N_f - 1) of N_f equal bins, tabulated at the bin centre
  f_iw = (iw + 1/2) / N_f - 1/2 (f and f_iw measured from the plane centre);
* table          T[iw][s_y + OS/2][s_x + OS/2][t_y][t_x] =
  K(t_x - h - s_x/OS, t_y - h - s_y/OS, f_iw), each (iw, s_y, s_x) row
  normalised to sum 1 (as the separable tables are);
* gridding       G_k[c_y + t_y - h][c_x + t_x - h] += W V T[iw][s_y][s_x][t_y][t_x];
* taper          C(l', m') = (1 / (N_f OS^2)) sum over every table entry of
  T cos(2 pi (dx l' + dy m')), l' = (p - N/2) / N (the response averaged over
  sub-cell offsets and w-fraction bins; real part);
* image          I = n Re(sum_k exp(+2 pi i w_k (n - 1)) F_k) / (C sum W);
* loss           L = sum_Omega (I - D)^2 / sum_Omega D^2 against the direct
  Fourier sum D, over Omega = the inner half of the field
  (|p - N/2| < N/4 and |q - N/2| < N/4), where the aliasing of a kernel is
  judged;
* gradient       exact, through the adjoint of every step (the taper's
  dependence on the table included).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import wstack as ow
from . import predict as op

HIDDEN = 32


# ---------------------------------------------------------------------------
# the MLP
# ---------------------------------------------------------------------------
def init_params(seed: int = 0, scale: float = 0.5) -> dict:
    """Random parameters: W1 [32][3], b1 [32], W2 [32][32], b2 [32], w3 [32], b3 (scalar)."""
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.normal(0, scale, (HIDDEN, 3)),
        "b1": rng.normal(0, scale, HIDDEN),
        "W2": rng.normal(0, scale / np.sqrt(HIDDEN), (HIDDEN, HIDDEN)),
        "b2": rng.normal(0, scale, HIDDEN),
        "w3": rng.normal(0, scale / np.sqrt(HIDDEN), HIDDEN),
        "b3": np.array(0.0),
    }


PARAM_ORDER = ("W1", "b1", "W2", "b2", "w3", "b3")


def flatten(theta: dict) -> np.ndarray:
    """Parameters as one vector in the order W1 (row-major), b1, W2 (row-major), b2, w3, b3."""
    return np.concatenate([np.asarray(theta[k], dtype=np.float64).reshape(-1) for k in PARAM_ORDER])


def unflatten(vec: np.ndarray) -> dict:
    vec = np.asarray(vec, dtype=np.float64)
    shapes = {"W1": (HIDDEN, 3), "b1": (HIDDEN,), "W2": (HIDDEN, HIDDEN), "b2": (HIDDEN,), "w3": (HIDDEN,),
              "b3": ()}
    out, o = {}, 0
    for k in PARAM_ORDER:
        n = int(np.prod(shapes[k])) if shapes[k] else 1
        out[k] = vec[o:o + n].reshape(shapes[k]) if shapes[k] else np.array(vec[o])
        o += n
    assert o == vec.size, (o, vec.size)
    return out


def mlp_forward(theta: dict, x: np.ndarray):
    """y = w3 . tanh(W2 tanh(W1 x + b1) + b2) + b3 for every row of x [n][3];
    returns y [n] and the hidden activations (for the backward pass)."""
    a1 = np.tanh(x @ theta["W1"].T + theta["b1"])
    a2 = np.tanh(a1 @ theta["W2"].T + theta["b2"])
    return a2 @ theta["w3"] + theta["b3"], (x, a1, a2)


def mlp_backward(theta: dict, cache, dy: np.ndarray) -> dict:
    """Gradient of sum(dy * y) with respect to the parameters (chain rule,
    tanh' = 1 - tanh^2)."""
    x, a1, a2 = cache
    g = {"w3": a2.T @ dy, "b3": np.array(dy.sum())}
    d2 = np.outer(dy, theta["w3"]) * (1.0 - a2 * a2)
    g["W2"] = d2.T @ a1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ theta["W2"]) * (1.0 - a1 * a1)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(axis=0)
    return g


# ---------------------------------------------------------------------------
# tabulation
# ---------------------------------------------------------------------------
def table_offsets(support: int, oversample: int):
    """Tap offsets dx[s + OS/2][t] = t - h - s/OS (cells) of every table row."""
    h = (support - 1) // 2
    s = np.arange(-(oversample // 2), oversample - oversample // 2, dtype=np.float64)
    t = np.arange(support, dtype=np.float64) - h
    return t[None, :] - s[:, None] / oversample                       # [OS][W]


def bin_centres(n_fbins: int) -> np.ndarray:
    """w-fraction of bin iw's centre, measured from the plane centre: (iw + 1/2) / N_f - 1/2."""
    return (np.arange(n_fbins, dtype=np.float64) + 0.5) / n_fbins - 0.5


def table_inputs(support: int, oversample: int, n_fbins: int):
    """MLP inputs of every table entry, [N_f][OS][OS][W][W][3] =
    (dx / (W/2), dy / (W/2), f_iw), and the mask |dx| < W/2, |dy| < W/2."""
    d = table_offsets(support, oversample)                            # [OS][W]
    half = support / 2.0
    OS, W = d.shape
    X = np.empty((n_fbins, OS, OS, W, W, 3))
    X[..., 0] = (d / half)[None, None, :, None, :]                    # dx: [s_x][t_x]
    X[..., 1] = (d / half)[None, :, None, :, None]                    # dy: [s_y][t_y]
    X[..., 2] = bin_centres(n_fbins)[:, None, None, None, None]
    inside = np.abs(d) < half
    mask = inside[None, None, :, None, :] & inside[None, :, None, :, None]
    return X, np.broadcast_to(mask, X.shape[:-1])


def tabulate(theta: dict, support: int, oversample: int, n_fbins: int) -> np.ndarray:
    """Table T[N_f][OS][OS][W][W]: exp(mlp) inside the support, 0 outside,
    each (iw, s_y, s_x) row normalised to sum 1."""
    X, mask = table_inputs(support, oversample, n_fbins)
    y, _ = mlp_forward(theta, X.reshape(-1, 3))
    K = np.where(mask, np.exp(y.reshape(mask.shape)), 0.0)
    return K / K.sum(axis=(-2, -1), keepdims=True)


def tabulate_backward(theta: dict, support: int, oversample: int, n_fbins: int, dT: np.ndarray) -> dict:
    """Gradient with respect to the parameters of sum(dT * T)."""
    X, mask = table_inputs(support, oversample, n_fbins)
    y, cache = mlp_forward(theta, X.reshape(-1, 3))
    K = np.where(mask, np.exp(y.reshape(mask.shape)), 0.0)
    S = K.sum(axis=(-2, -1), keepdims=True)
    T = K / S
    # T = K / S: dK = (dT - sum(dT T)) / S; K = exp(y) inside: dy = dK K
    dK = (dT - (dT * T).sum(axis=(-2, -1), keepdims=True)) / S
    dy = np.where(mask, dK * K, 0.0).reshape(-1)
    return mlp_backward(theta, cache, dy)


def separable_table(table_y: np.ndarray, table_x: np.ndarray, n_fbins: int) -> np.ndarray:
    """The non-separable layout of separable taps: T[iw][s_y][s_x][t_y][t_x] = g_y[s_y][t_y] g_x[s_x][t_x]."""
    T = table_y[:, None, :, None] * table_x[None, :, None, :]
    return np.broadcast_to(T, (n_fbins,) + T.shape).copy()


# ---------------------------------------------------------------------------
# imaging with the table
# ---------------------------------------------------------------------------
def wfrac_bins(w: np.ndarray, w_min: float, w_max: float, n_wplanes: int, n_fbins: int) -> np.ndarray:
    """w-fraction bin of every visibility: r = (w - w_min) / dw,
    k = clamp(floor(r), 0, N_w - 1), iw = clamp(floor((r - k) N_f), 0, N_f - 1);
    non-finite w gives bin 0 (such visibilities are dropped anyway)."""
    dw = (w_max - w_min) / n_wplanes
    with np.errstate(invalid="ignore", over="ignore"):
        r = (np.asarray(w, dtype=np.float64) - w_min) / dw
        kf = np.floor(r)
        kf = np.where(np.isnan(kf), 0.0, kf)
        k = np.clip(kf, 0, n_wplanes - 1)
        fb = np.floor((r - k) * n_fbins)
        fb = np.where(np.isfinite(fb), fb, 0.0)
    return np.clip(fb, 0, n_fbins - 1).astype(np.int64)


def grid_table(b: "ow.Binned", iw: np.ndarray, T: np.ndarray, *, grid_n: int, n_wplanes: int) -> np.ndarray:
    """G_k[c_y + t_y - h][c_x + t_x - h] += W V T[iw][s_y][s_x][t_y][t_x]; complex128 [N_w][N][N]."""
    n_f, OS, _, W, _ = T.shape
    h = (W - 1) // 2
    N = grid_n
    G = np.zeros((n_wplanes, N, N), dtype=np.complex128)
    idx = np.nonzero(b.keep)[0]
    if idx.size == 0:
        return G
    t = np.arange(W) - h
    taps = T[iw[idx], b.sy[idx] + OS // 2, b.sx[idx] + OS // 2]                  # [n][W][W]
    rows = (b.cy[idx][:, None] + t[None, :]) * N                                  # [n][W]
    cell = (b.k[idx][:, None, None] * N * N + rows[:, :, None] + (b.cx[idx][:, None] + t[None, :])[:, None, :])
    wv = b.wv[idx][:, None, None]
    re = np.bincount(cell.reshape(-1), weights=(wv.real * taps).reshape(-1), minlength=n_wplanes * N * N)
    im = np.bincount(cell.reshape(-1), weights=(wv.imag * taps).reshape(-1), minlength=n_wplanes * N * N)
    G += (re + 1j * im).reshape(n_wplanes, N, N)
    return G


def fine_average(T: np.ndarray) -> np.ndarray:
    """The table averaged over w-fraction bins, as a matrix over the W OS
    distinct tap offsets of each axis (every (s, t) pair gives its own offset
    t - h - s/OS): A[jy][jx], and the offsets d[j] in cells, ascending."""
    n_f, OS, _, W, _ = T.shape
    d = table_offsets(W, OS)                                   # [OS][W]
    flat = d.reshape(-1)
    order = np.argsort(flat)
    dj = flat[order]
    Tm = T.mean(axis=0)                                        # [s_y][s_x][t_y][t_x]
    A = Tm.transpose(0, 2, 1, 3).reshape(OS * W, OS * W)       # [(s_y, t_y)][(s_x, t_x)]
    return A[np.ix_(order, order)], dj


def taper(T: np.ndarray, grid_n: int) -> np.ndarray:
    """C[q][p] = (1/(N_f OS^2)) sum_{iw, s, t} T cos(2 pi (dx l'_p + dy m'_q)), l' = (p - N/2)/N.

    cos(a + b) = cos a cos b - sin a sin b turns the double sum over the fine
    offsets into two matrix products."""
    n_f, OS, _, W, _ = T.shape
    A, d = fine_average(T)
    lp = (np.arange(grid_n, dtype=np.float64) - grid_n / 2) / grid_n
    ph = 2.0 * np.pi * np.outer(lp, d)                          # [N][W OS]
    Cc, Ss = np.cos(ph), np.sin(ph)
    return (Cc @ A @ Cc.T - Ss @ A @ Ss.T) / (OS * OS)


def taper_backward(dC: np.ndarray, support: int, oversample: int, n_fbins: int) -> np.ndarray:
    """Gradient of sum(dC * taper(T)) with respect to every table entry."""
    N = dC.shape[-1]
    OS, W = oversample, support
    d = table_offsets(W, OS)                                    # [OS][W]
    lp = (np.arange(N, dtype=np.float64) - N / 2) / N
    phx = 2.0 * np.pi * lp[:, None, None] * d[None, :, :]      # [p][s_x][t_x]
    cx, sx = np.cos(phx).reshape(N, -1), np.sin(phx).reshape(N, -1)
    # taper[q][p] = sum_{y,x} A[y][x] (cos_y[q] cos_x[p] - sin_y[q] sin_x[p]) / OS^2, A = mean_iw T
    dA = (cx.T @ dC @ cx - sx.T @ dC @ sx) / (OS * OS)          # [(s_y,t_y)][(s_x,t_x)]
    dA = dA.reshape(OS, W, OS, W).transpose(0, 2, 1, 3)        # [s_y][s_x][t_y][t_x]
    return np.broadcast_to(dA / n_fbins, (n_fbins,) + dA.shape).copy()


@dataclass
class TableResult:
    image: np.ndarray       # I (taper divided)
    apparent: np.ndarray    # n Re(sum_k screen_k F_k) / sum W (before the taper division)
    planes: np.ndarray      # G_k
    binned: "ow.Binned"
    iw: np.ndarray
    corr2: np.ndarray       # taper C[q][p]
    sum_w: float
    w_k: np.ndarray


def image_with_table(uvw, freq, vis, weight, T, *, grid_n, n_wplanes, support, oversample, fov, w_min,
                     w_max, **_ignored) -> TableResult:
    """Dirty image with the non-separable table T, all steps in the paper's order."""
    n_f = T.shape[0]
    assert T.shape[1:] == (oversample, oversample, support, support)
    b = ow.bin_visibilities(uvw, freq, vis, weight, grid_n=grid_n, n_wplanes=n_wplanes, support=support,
                            oversample=oversample, fov=fov, w_min=w_min, w_max=w_max)
    iw = wfrac_bins(b.w, w_min, w_max, n_wplanes, n_f)
    G = grid_table(b, iw, T, grid_n=grid_n, n_wplanes=n_wplanes)
    F = ow.ifft_planes(G)
    w_k = ow.plane_centres(w_min, w_max, n_wplanes)
    S = ow.screen_sum(F, w_k, fov)
    sum_w = float(b.wt[b.keep].sum())
    l = ow.pixel_lm(grid_n, fov)
    nm1 = ow.nm1_of(l[None, :], l[:, None])
    inside = np.isfinite(nm1)
    n = 1.0 + np.where(inside, nm1, 0.0)
    apparent = np.where(inside, n * S / sum_w, 0.0) if sum_w > 0 else np.zeros_like(S)
    C2 = taper(T, grid_n)
    return TableResult(image=apparent / C2, apparent=apparent, planes=G, binned=b, iw=iw, corr2=C2,
                       sum_w=sum_w, w_k=w_k)


def inner_mask(grid_n: int) -> np.ndarray:
    """Omega: |p - N/2| < N/4 and |q - N/2| < N/4."""
    c = np.abs(np.arange(grid_n) - grid_n // 2) < grid_n // 4
    return c[:, None] & c[None, :]


def loss_of(image: np.ndarray, target: np.ndarray) -> float:
    m = inner_mask(image.shape[-1])
    return float(((image - target)[m] ** 2).sum() / (target[m] ** 2).sum())


def loss_and_table_grad(uvw, freq, vis, weight, T, target, *, grid_n, n_wplanes, support, oversample, fov,
                        w_min, w_max, **_ignored):
    """L and dL/dT for the table T against the target image (the direct sum)."""
    r = image_with_table(uvw, freq, vis, weight, T, grid_n=grid_n, n_wplanes=n_wplanes, support=support,
                         oversample=oversample, fov=fov, w_min=w_min, w_max=w_max)
    m = inner_mask(grid_n)
    den = float((target[m] ** 2).sum())
    L = float(((r.image - target)[m] ** 2).sum() / den)
    dI = np.where(m, 2.0 * (r.image - target) / den, 0.0)
    dA = dI / r.corr2                       # I = A / C
    dC = -dI * r.image / r.corr2
    # A = n Re(sum_k e^{+i phi_k} F_k) / sum W: the gradient with respect to
    # G_k (d/dRe + i d/dIm) is the centred forward DFT of dA n e^{-i phi_k} / sum W
    l = ow.pixel_lm(grid_n, fov)
    nm1 = ow.nm1_of(l[None, :], l[:, None])
    inside = np.isfinite(nm1)
    nm1z = np.where(inside, nm1, 0.0)
    base = np.where(inside, dA * (1.0 + nm1z) / r.sum_w, 0.0)
    P = np.empty((n_wplanes, grid_n, grid_n), dtype=np.complex128)
    for k, wk in enumerate(r.w_k):
        tau = wk * nm1z
        tr = tau - np.rint(tau)
        P[k] = base * (np.cos(2 * np.pi * tr) - 1j * np.sin(2 * np.pi * tr))
    dG = op.fft_planes_forward(P)
    # gridding: dL/dT[iw][s_y][s_x][t_y][t_x] = sum_v Re(dG_k[cell] conj(W V))
    b, iw = r.binned, r.iw
    n_f = T.shape[0]
    OS, W = oversample, support
    h = (W - 1) // 2
    dT = np.zeros_like(T)
    idx = np.nonzero(b.keep)[0]
    if idx.size:
        t = np.arange(W) - h
        rows = b.cy[idx][:, None] + t[None, :]
        cols = b.cx[idx][:, None] + t[None, :]
        vals = dG[b.k[idx][:, None, None], rows[:, :, None], cols[:, None, :]]     # [n][W][W]
        contrib = (vals * np.conj(b.wv[idx])[:, None, None]).real
        np.add.at(dT, (iw[idx], b.sy[idx] + OS // 2, b.sx[idx] + OS // 2), contrib)
    dT += taper_backward(dC, W, OS, n_f)
    return L, dT, r
