"""Pins of the learned-kernel oracle (``oracle.learned``) against things other
than itself: the separable oracle it must reduce to, brute-force sums,
closed forms of the MLP and of the table, hand-derived w-fraction bins, and
finite differences for the gradient.  No GPU is used.
"""
import math

import numpy as np
import pytest

import synth
from oracle import dft as od
from oracle import learned as ol
from oracle import wstack as ow


def rel_rms(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _scene(seed=51, nrow=600, N=32, Nw=4, W=5, OS=8, fov=0.8, wmax=40.0, nsrc=3):
    rng = np.random.default_rng(seed)
    r = 0.42 * N / fov * np.sqrt(rng.uniform(0, 1, nrow))
    ph = rng.uniform(0, 2 * np.pi, nrow)
    uvw = np.stack([r * np.cos(ph), r * np.sin(ph), rng.uniform(-wmax, wmax, nrow)], 1)
    l = rng.uniform(-0.15, 0.15, nsrc) * fov
    m = rng.uniform(-0.15, 0.15, nsrc) * fov
    S = rng.uniform(0.5, 1.5, nsrc)
    vis = synth.point_source_vis_np(uvw[:, 0], uvw[:, 1], uvw[:, 2], l, m, S).astype(np.complex64).reshape(-1, 1)
    wt = rng.uniform(0.5, 2.0, (nrow, 1)).astype(np.float32)
    geo = dict(grid_n=N, n_wplanes=Nw, support=W, oversample=OS, fov=fov, w_min=-wmax, w_max=wmax)
    return uvw, vis, wt, geo


# ---------------------------------------------------------------------------
# the MLP and the table
# ---------------------------------------------------------------------------
def test_mlp_closed_forms():
    """Special parameters that reduce the MLP to closed forms: all weights zero
    gives the output bias; a single path x0 -> h1[0] -> h2[0] -> y gives
    a tanh(b tanh(c x0 + d) + e) + f."""
    th = {k: np.zeros_like(v) for k, v in ol.init_params(0).items()}
    th["b3"] = np.array(0.37)
    x = np.random.default_rng(1).uniform(-1, 1, (50, 3))
    y, _ = ol.mlp_forward(th, x)
    assert np.all(y == 0.37)
    a, b, c, d, e, f = 1.3, -0.7, 2.1, 0.2, -0.4, 0.05
    th["W1"][0, 0], th["b1"][0] = c, d
    th["W2"][0, 0], th["b2"][0] = b, e
    th["w3"][0], th["b3"] = a, np.array(f)
    y, _ = ol.mlp_forward(th, x)
    want = a * np.tanh(b * np.tanh(c * x[:, 0] + d) + e) + f + 0.0 * x[:, 1]
    # the other hidden units are tanh(0) = 0 and contribute nothing
    assert np.max(np.abs(y - want)) < 1e-15


def test_mlp_backward_finite_differences():
    """Parameter gradient of sum(dy * y) against central differences."""
    rng = np.random.default_rng(2)
    th = ol.init_params(3)
    x = rng.uniform(-1, 1, (40, 3))
    dy = rng.normal(size=40)
    _, cache = ol.mlp_forward(th, x)
    g = ol.flatten(ol.mlp_backward(th, cache, dy))
    v = ol.flatten(th)
    for i in rng.choice(v.size, 25, replace=False):
        e = np.zeros_like(v)
        e[i] = 1e-6
        fp = float(dy @ ol.mlp_forward(ol.unflatten(v + e), x)[0])
        fm = float(dy @ ol.mlp_forward(ol.unflatten(v - e), x)[0])
        assert abs((fp - fm) / 2e-6 - g[i]) < 1e-7 * max(1.0, abs(g[i])), i


def test_table_constant_mlp_is_uniform_over_support():
    """A constant MLP output gives the same value at every tap inside the
    support, 1 / (taps inside); taps with |d| >= W/2 are zero."""
    th = {k: np.zeros_like(v) for k, v in ol.init_params(0).items()}
    th["b3"] = np.array(-1.7)
    W, OS, nf = 5, 8, 2
    T = ol.tabulate(th, W, OS, nf)
    d = ol.table_offsets(W, OS)
    inside = np.abs(d) < W / 2
    for sy in range(OS):
        for sx in range(OS):
            m = np.outer(inside[sy], inside[sx])
            want = np.where(m, 1.0 / m.sum(), 0.0)
            assert np.allclose(T[1, sy, sx], want, atol=1e-15)
    # the half-cell row s = -OS/2 has its last tap at d = W/2 exactly: zero
    assert np.all(T[:, 0, :, W - 1, :] == 0) and np.all(T[:, :, 0, :, W - 1] == 0)


def test_table_rows_sum_to_one_and_inputs_are_offsets():
    th = ol.init_params(4)
    W, OS, nf = 7, 4, 4
    T = ol.tabulate(th, W, OS, nf)
    assert np.max(np.abs(T.sum(axis=(-2, -1)) - 1.0)) < 1e-14
    X, mask = ol.table_inputs(W, OS, nf)
    # entry (iw, s_y, s_x, t_y, t_x) sits at dx = t_x - h - s_x/OS, dy = t_y - h - s_y/OS
    h = (W - 1) // 2
    iw, sy, sx, ty, tx = 2, 1, 3, 5, 0
    s_y, s_x = sy - OS // 2, sx - OS // 2
    assert X[iw, sy, sx, ty, tx, 0] == (tx - h - s_x / OS) / (W / 2)
    assert X[iw, sy, sx, ty, tx, 1] == (ty - h - s_y / OS) / (W / 2)
    assert X[iw, sy, sx, ty, tx, 2] == (iw + 0.5) / nf - 0.5


def test_tabulate_backward_finite_differences():
    rng = np.random.default_rng(5)
    th = ol.init_params(6)
    W, OS, nf = 5, 4, 2
    dT = rng.normal(size=(nf, OS, OS, W, W))
    g = ol.flatten(ol.tabulate_backward(th, W, OS, nf, dT))
    v = ol.flatten(th)
    for i in rng.choice(v.size, 20, replace=False):
        e = np.zeros_like(v)
        e[i] = 1e-6
        fp = float((dT * ol.tabulate(ol.unflatten(v + e), W, OS, nf)).sum())
        fm = float((dT * ol.tabulate(ol.unflatten(v - e), W, OS, nf)).sum())
        assert abs((fp - fm) / 2e-6 - g[i]) < 1e-7 * max(1.0, abs(g[i])), i


# ---------------------------------------------------------------------------
# w-fraction bins
# ---------------------------------------------------------------------------
def test_wfrac_bins_hand_cases():
    """w_min = -40, w_max = 40, N_w = 4 (dw = 20), N_f = 4 (bins of 5 wavelengths
    inside each plane)."""
    w = np.array([-40.0, -35.0, -35.0001, -20.0, -0.0001, 0.0, 4.9999, 5.0, 19.9999, 39.9999, 40.0, 55.0, -60.0,
                  np.nan])
    want = np.array([0, 1, 0, 0, 3, 0, 0, 1, 3, 3, 3, 3, 0, 0])
    # 40 -> plane 3 (clamped), r - k = 1 -> bin clamp(4) = 3; 55 -> r - k = 1.75 -> 3;
    # -60 -> plane 0, r - k = -1 -> bin 0
    got = ol.wfrac_bins(w, -40.0, 40.0, 4, 4)
    assert np.array_equal(got, want), got


# ---------------------------------------------------------------------------
# imaging with a table
# ---------------------------------------------------------------------------
def test_separable_table_reproduces_separable_oracle():
    """The Gaussian tap table laid out non-separably (same for every w-fraction
    bin) gives the separable oracle's planes and image, and its taper is
    C(l') C(m')."""
    uvw, vis, wt, geo = _scene()
    g = ow.tap_table(geo["support"], geo["oversample"])
    T = ol.separable_table(g, g, 4)
    r = ol.image_with_table(uvw, None, vis, wt, T, **geo)
    ref = ow.wstack_image(uvw, None, vis, wt, **geo)
    assert np.max(np.abs(r.planes - ref.planes)) < 1e-13 * np.max(np.abs(ref.planes))
    assert np.max(np.abs(r.corr2 - np.outer(ref.corr, ref.corr))) < 1e-13
    assert np.max(np.abs(r.image - ref.image)) < 1e-11 * np.max(np.abs(ref.image))


def test_asymmetric_table_against_brute_force_gridding():
    """Different Gaussian widths along x and y (so a transposed table or
    swapped offsets show): planes against gridding written out visibility by
    visibility, tap by tap, from the kernel formula."""
    uvw, vis, wt, geo = _scene(seed=52, nrow=40, N=16, Nw=2, W=5, OS=4, fov=0.5, wmax=20.0)
    W, OS = geo["support"], geo["oversample"]
    gy = ow.tap_table(W, OS, "gaussian", 1.3)
    gx = ow.tap_table(W, OS, "gaussian", 0.7)
    T = ol.separable_table(gy, gx, 2)
    r = ol.image_with_table(uvw, None, vis, wt, T, **geo)
    b = r.binned
    h = (W - 1) // 2
    G = np.zeros_like(r.planes)
    for j in np.nonzero(b.keep)[0]:
        dx = np.arange(W) - h - b.sx[j] / OS
        dy = np.arange(W) - h - b.sy[j] / OS
        kx = np.exp(-dx ** 2 / (2 * 0.7 ** 2)) * (np.abs(dx) < W / 2)
        ky = np.exp(-dy ** 2 / (2 * 1.3 ** 2)) * (np.abs(dy) < W / 2)
        for ty in range(W):
            for tx in range(W):
                G[b.k[j], b.cy[j] + ty - h, b.cx[j] + tx - h] += b.wv[j] * ky[ty] / ky.sum() * kx[tx] / kx.sum()
    assert np.max(np.abs(r.planes - G)) < 1e-13 * np.max(np.abs(G))


def test_wfrac_bins_pick_their_table_slice():
    """A table that differs per w-fraction bin equals the sum over bins of the
    separable oracle run on that bin's visibilities with that bin's taps
    (planes are linear in the visibilities)."""
    uvw, vis, wt, geo = _scene(seed=53)
    W, OS = geo["support"], geo["oversample"]
    sig = [0.6, 0.8, 1.0, 1.2]
    tabs = [ow.tap_table(W, OS, "gaussian", s) for s in sig]
    T = np.stack([ol.separable_table(t, t, 1)[0] for t in tabs])
    r = ol.image_with_table(uvw, None, vis, wt, T, **geo)
    b, iw = r.binned, r.iw
    assert set(np.unique(iw[b.keep])) == {0, 1, 2, 3}
    G = np.zeros_like(r.planes)
    for f in range(4):
        for k in range(geo["n_wplanes"]):
            ow.grid_plane(G[k], b, np.nonzero(b.keep & (iw == f) & (b.k == k))[0], tabs[f])
    assert np.max(np.abs(r.planes - G)) < 1e-13 * np.max(np.abs(G))


def test_taper_against_direct_sum():
    """The taper by two matrix products equals the defining sum over every
    table entry, at a few pixels, for an asymmetric learned table."""
    W, OS, nf, N = 5, 4, 2, 16
    T = ol.tabulate(ol.init_params(7), W, OS, nf)
    C = ol.taper(T, N)
    d = ol.table_offsets(W, OS)
    for (q, p) in [(0, 0), (8, 8), (3, 11), (15, 2)]:
        lp, mq = (p - N / 2) / N, (q - N / 2) / N
        tot = 0.0
        for iw in range(nf):
            for sy in range(OS):
                for sx in range(OS):
                    ph = 2 * np.pi * (d[sx][None, :] * lp + d[sy][:, None] * mq)
                    tot += (T[iw, sy, sx] * np.cos(ph)).sum()
        assert abs(C[q, p] - tot / (nf * OS * OS)) < 1e-14
    assert abs(C[N // 2, N // 2] - 1.0) < 1e-14      # rows sum to one


# ---------------------------------------------------------------------------
# gradient
# ---------------------------------------------------------------------------
def _target(uvw, vis, wt, geo):
    b = ow.bin_visibilities(uvw, None, vis, wt, **{k: geo[k] for k in ("grid_n", "n_wplanes", "support",
                                                                       "oversample", "fov", "w_min", "w_max")})
    return od.dft_of_binned(b, geo["fov"], geo["grid_n"])


def test_table_gradient_finite_differences():
    """dL/dT of the loss against the direct sum, including the taper's
    dependence on T, against central differences at table entries that many
    visibilities use."""
    uvw, vis, wt, geo = _scene(seed=54, nrow=300, N=32, Nw=3, W=5, OS=4)
    D = _target(uvw, vis, wt, geo)
    T = ol.tabulate(ol.init_params(8, scale=0.3), geo["support"], geo["oversample"], 2)
    L, dT, r = ol.loss_and_table_grad(uvw, None, vis, wt, T, D, **geo)
    assert L > 0
    rng = np.random.default_rng(9)
    cnt = np.zeros(T.shape[:3])
    np.add.at(cnt, (r.iw[r.binned.keep], r.binned.sy[r.binned.keep] + 2, r.binned.sx[r.binned.keep] + 2), 1)
    rows = np.argwhere(cnt > 0)
    for i in rng.choice(len(rows), 12, replace=False):
        f, sy, sx = rows[i]
        ty, tx = rng.integers(0, geo["support"], 2)
        e = np.zeros_like(T)
        e[f, sy, sx, ty, tx] = 1e-6
        Lp = ol.loss_of(ol.image_with_table(uvw, None, vis, wt, T + e, **geo).image, D)
        Lm = ol.loss_of(ol.image_with_table(uvw, None, vis, wt, T - e, **geo).image, D)
        fd = (Lp - Lm) / 2e-6
        assert abs(fd - dT[f, sy, sx, ty, tx]) < 1e-6 * max(abs(fd), 1e-3 * np.abs(dT).max()), (fd, dT[f, sy, sx, ty, tx])


def test_parameter_gradient_finite_differences():
    """dL/dtheta through the table, the normalisation and the MLP."""
    uvw, vis, wt, geo = _scene(seed=55, nrow=250, N=32, Nw=3, W=5, OS=4)
    D = _target(uvw, vis, wt, geo)
    th = ol.init_params(10, scale=0.3)
    W, OS, nf = geo["support"], geo["oversample"], 2
    T = ol.tabulate(th, W, OS, nf)
    L, dT, _ = ol.loss_and_table_grad(uvw, None, vis, wt, T, D, **geo)
    g = ol.flatten(ol.tabulate_backward(th, W, OS, nf, dT))
    v = ol.flatten(th)
    rng = np.random.default_rng(11)
    for i in rng.choice(v.size, 10, replace=False):
        e = np.zeros_like(v)
        e[i] = 1e-5
        Lp = ol.loss_of(ol.image_with_table(uvw, None, vis, wt, ol.tabulate(ol.unflatten(v + e), W, OS, nf),
                                            **geo).image, D)
        Lm = ol.loss_of(ol.image_with_table(uvw, None, vis, wt, ol.tabulate(ol.unflatten(v - e), W, OS, nf),
                                            **geo).image, D)
        fd = (Lp - Lm) / 2e-5
        assert abs(fd - g[i]) < 1e-5 * max(abs(fd), 1e-3 * np.abs(g).max()), (i, fd, g[i])
