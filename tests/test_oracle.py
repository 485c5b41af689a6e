"""Pins of the float64 oracle against things other than itself.

Each test names the part of the oracle it pins and what pins it: a closed
form, a special case that reduces to a textbook identity, a brute-force sum
written independently, an invariant of the mathematics, or hand-derived
integer decisions.  No GPU is used.
"""
import math
import os

import numpy as np
import pytest
import scipy.special
import scipy.stats

import oracle
import synth
from oracle import wstack as ow
from oracle import dft as od

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel_rms(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


# ---------------------------------------------------------------------------
# P1: direct DFT (Eq. 1 over measured samples)
# ---------------------------------------------------------------------------
def _random_uvw(rng, n, scale=300.0, wscale=80.0):
    return rng.normal(0, scale, n), rng.normal(0, scale, n), rng.normal(0, wscale, n)


def test_dft_point_source_at_pixel_centre_closed_form():
    """A point source of flux S at a pixel centre gives exactly S at that pixel
    (the Eq. 2 phases cancel the Eq. 1 phases, n cancels 1/n), any (u,v,w), any weights."""
    rng = np.random.default_rng(11)
    N, fov = 64, 0.6
    lm = ow.pixel_lm(N, fov)
    p, q = 45, 12
    l0, m0 = lm[p], lm[q]
    nm10 = ow.nm1_of(np.array(l0), np.array(m0))
    S = 2.75
    u, v, w = _random_uvw(rng, 5000, 2000.0, 700.0)
    V = (S / (1 + nm10)) * np.exp(-2j * np.pi * (u * l0 + v * m0 + w * nm10))
    W = rng.uniform(0.2, 3.0, 5000)
    img = od.dft_image(u, v, w, W * V, W.sum(), fov, N, rows=slice(q, q + 1), cols=slice(p, p + 1))
    assert abs(img[0, 0] - S) < 1e-11


def test_dft_cell_centred_flat_sky_equals_library_ifft():
    """With w = 0 and (u, v) on cell centres, the DFT image equals
    n N^2 fftshift(ifft2(ifftshift(A))) / sum W, A = per-cell sum of W V (numpy FFT)."""
    rng = np.random.default_rng(12)
    N, fov = 32, 0.5
    du = 1.0 / fov
    n = 700
    i = rng.integers(0, N, n)
    j = rng.integers(0, N, n)
    u, v, w = (i - N // 2) * du, (j - N // 2) * du, np.zeros(n)
    a = rng.normal(size=n) + 1j * rng.normal(size=n)
    A = np.zeros((N, N), complex)
    np.add.at(A, (j, i), a)
    ref = np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(A))) * N * N
    lm = ow.pixel_lm(N, fov)
    nm1 = ow.nm1_of(lm[None, :], lm[:, None])
    ref = (1 + nm1) * ref / 5.0
    got = od.dft_image(u, v, w, a, 5.0, fov, N, complex_out=True)
    assert np.max(np.abs(got - ref)) < 1e-11 * np.max(np.abs(ref))


def test_dft_linear_hermitian_and_order_independent():
    rng = np.random.default_rng(13)
    N, fov = 24, 0.4
    u, v, w = _random_uvw(rng, 900)
    a1 = rng.normal(size=900) + 1j * rng.normal(size=900)
    a2 = rng.normal(size=900) + 1j * rng.normal(size=900)
    d1 = od.dft_image(u, v, w, a1, 1.0, fov, N, complex_out=True)
    d2 = od.dft_image(u, v, w, a2, 1.0, fov, N, complex_out=True)
    d12 = od.dft_image(u, v, w, 2.0 * a1 - 0.5j * a2, 1.0, fov, N, complex_out=True)
    assert np.max(np.abs(d12 - (2.0 * d1 - 0.5j * d2))) < 1e-11 * np.max(np.abs(d12))
    # Hermitian completion: a real sky -> imaginary part vanishes
    uh, vh, wh = np.r_[u, -u], np.r_[v, -v], np.r_[w, -w]
    ah = np.r_[a1, np.conj(a1)]
    dh = od.dft_image(uh, vh, wh, ah, 1.0, fov, N, complex_out=True)
    assert np.max(np.abs(dh.imag)) < 1e-12 * np.max(np.abs(dh.real))
    # summation order
    dr = od.dft_image(u, v, w, a1, 1.0, fov, N, complex_out=True, reverse=True)
    assert np.max(np.abs(dr - d1)) < 1e-12 * np.max(np.abs(d1))


# ---------------------------------------------------------------------------
# P2: positions, planes, drops (hand-derived integer cases)
# ---------------------------------------------------------------------------
def _load_quantise_cases():
    rows = []
    with open(os.path.join(GOLDEN, "quantise_cases.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            lhs, rhs = line.split("|")
            rows.append((list(map(float, lhs.split())), list(map(int, rhs.split()))))
    return rows


def test_quantisation_hand_cases():
    cases = _load_quantise_cases()
    uvw = np.array([c[0][:3] for c in cases])
    wt = np.array([c[0][3] for c in cases], dtype=np.float32).reshape(-1, 1)
    exp = np.array([c[1] for c in cases])
    vis = np.ones((len(cases), 1), np.complex64)
    b = ow.bin_visibilities(uvw, None, vis, wt, grid_n=16, n_wplanes=4, support=3, oversample=4,
                           fov=0.125, w_min=-8.0, w_max=8.0)
    got = np.stack([b.X, b.Y, b.cx, b.cy, b.sx, b.sy, b.k, b.keep.astype(int)], axis=1)
    assert np.array_equal(got, exp), np.nonzero((got != exp).any(axis=1))


def test_quantisation_drops_non_finite():
    uvw = np.array([[np.nan, 0, 0], [0, np.inf, 0], [0, 0, np.nan], [0, 0, 0], [0, 0, 0], [1e300, 0, 0]])
    vis = np.array([1, 1, 1, np.nan + 0j, 1, 1], np.complex64).reshape(-1, 1)
    wt = np.array([1, 1, 1, 1, np.inf, 1], np.float32).reshape(-1, 1)
    b = ow.bin_visibilities(uvw, None, vis, wt, grid_n=16, n_wplanes=4, support=3, oversample=4,
                           fov=0.125, w_min=-8.0, w_max=8.0)
    assert not b.keep.any()


# ---------------------------------------------------------------------------
# P3: kernel table and grid correction
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kernel", ["gaussian", "kaiser_bessel"])
@pytest.mark.parametrize("W,OS", [(7, 32), (7, 64), (5, 16), (3, 1), (1, 1), (9, 8)])
def test_tap_table_rows_and_symmetry(kernel, W, OS):
    g = ow.tap_table(W, OS, kernel)
    assert g.shape == (OS, W)
    assert np.max(np.abs(g.sum(axis=1) - 1.0)) < 1e-15
    # g_s[t] = g_{-s}[-t] for s != -OS/2 (row s + OS/2, tap t - h)
    for s in range(-(OS // 2) + 1, OS - OS // 2):
        if -s + OS // 2 < OS:
            assert np.allclose(g[s + OS // 2], g[-s + OS // 2][::-1], rtol=0, atol=1e-15)
    if OS > 1 and W > 1:
        assert g[0, W - 1] == 0.0   # d = W/2 exactly: strictly truncated


def test_tap_table_values_vs_scipy():
    """Gaussian taps vs scipy.stats.norm.pdf; Kaiser-Bessel taps vs scipy.special.i0."""
    W, OS = 7, 64
    h = 3
    sigma = ow.gaussian_sigma_default(W)
    assert abs(sigma - 0.9416393) < 1e-6
    beta = ow.kb_beta_default(W)
    assert abs(beta - 16.2522) < 1e-3
    s = np.arange(-OS // 2, OS // 2)
    d = (np.arange(W) - h)[None, :] - s[:, None] / OS
    gg = np.where(np.abs(d) < W / 2, scipy.stats.norm.pdf(d, scale=sigma), 0.0)
    assert np.max(np.abs(ow.tap_table(W, OS, "gaussian") - gg / gg.sum(1, keepdims=True))) < 1e-14
    kb = np.where(np.abs(d) < W / 2,
                  scipy.special.i0(beta * np.sqrt(np.clip(1 - (2 * d / W) ** 2, 0, None))), 0.0)
    assert np.max(np.abs(ow.tap_table(W, OS, "kaiser_bessel") - kb / kb.sum(1, keepdims=True))) < 1e-13
    x = np.linspace(0, 40, 81)
    assert np.max(np.abs(ow.bessel_i0(x) / scipy.special.i0(x) - 1)) < 1e-13


def test_grid_correction_basic():
    g = ow.tap_table(7, 32)
    C = ow.grid_correction(g, 64)
    assert abs(C[32] - 1.0) < 1e-15          # l' = 0
    assert np.max(np.abs(C[1:32] - C[63:32:-1])) < 1e-15   # even in l'
    assert np.all(C > 0) and np.all(np.diff(C[32:]) < 0)


def test_grid_correction_is_offset_averaged_response():
    """C(l') equals the response of gridding + inverse FFT to a unit visibility,
    averaged over all OS sub-cell offsets (1-D cut through the oracle's own grid and FFT)."""
    N, W, OS = 32, 7, 8
    fov = 1.0
    g = ow.tap_table(W, OS)
    # one visibility per sub-cell offset s, at x = s/OS cells from the centre, v = 0, w = 0
    s = np.arange(-OS // 2, OS // 2)
    uvw = np.stack([s / OS, np.zeros(OS), np.zeros(OS)], axis=1)   # wavelengths = cells (fov = 1)
    resp = np.zeros(N)
    for i in range(OS):
        b = ow.bin_visibilities(uvw[i:i + 1], None, np.ones((1, 1), np.complex64), None, grid_n=N,
                               n_wplanes=1, support=W, oversample=OS, fov=fov, w_min=-1, w_max=1)
        F = ow.ifft_planes(ow.grid(b, g, grid_n=N, n_wplanes=1))[0]
        lp = (np.arange(N) - N / 2) / N
        # divide out the true point's phase exp(2 pi i x l')
        resp += (F[N // 2, :] * np.exp(-2j * np.pi * (s[i] / OS) * lp)).real
    resp /= OS
    assert np.max(np.abs(resp - ow.grid_correction(g, N))) < 1e-14


# ---------------------------------------------------------------------------
# P4: gridding
# ---------------------------------------------------------------------------
def test_grid_brute_force_small():
    """N = 16, 5 visibilities: every cell evaluated from the continuous kernel at
    its distance to the quantised position, normalised per visibility and axis."""
    rng = np.random.default_rng(14)
    N, W, OS, Nw, fov = 16, 5, 8, 3, 0.25
    h = 2
    uvw = np.stack([rng.uniform(-20, 20, 5), rng.uniform(-20, 20, 5), rng.uniform(-9, 9, 5)], 1)
    vis = (rng.normal(size=5) + 1j * rng.normal(size=5)).astype(np.complex64).reshape(-1, 1)
    wt = rng.uniform(0.5, 2, 5).astype(np.float32).reshape(-1, 1)
    g = ow.tap_table(W, OS)
    b = ow.bin_visibilities(uvw, None, vis, wt, grid_n=N, n_wplanes=Nw, support=W, oversample=OS,
                           fov=fov, w_min=-9.0, w_max=9.0)
    assert b.keep.all()
    G = ow.grid(b, g, grid_n=N, n_wplanes=Nw)
    ref = np.zeros((Nw, N, N), complex)
    sigma = ow.gaussian_sigma_default(W)
    for n in range(5):
        xq = b.X[n] / OS          # quantised position in cells from the corner
        yq = b.Y[n] / OS
        cells = np.arange(N)
        gx = np.where(np.abs(cells - xq) < W / 2, np.exp(-(cells - xq) ** 2 / (2 * sigma ** 2)), 0)
        gy = np.where(np.abs(cells - yq) < W / 2, np.exp(-(cells - yq) ** 2 / (2 * sigma ** 2)), 0)
        # the footprint is the W cells around the nearest cell
        cx = int(math.floor(xq + 0.5)); cy = int(math.floor(yq + 0.5))
        mx = (cells >= cx - h) & (cells <= cx + h)
        my = (cells >= cy - h) & (cells <= cy + h)
        gx = np.where(mx, gx, 0); gy = np.where(my, gy, 0)
        gx /= gx.sum(); gy /= gy.sum()
        k = int(np.clip(np.floor((uvw[n, 2] + 9.0) / 6.0), 0, Nw - 1))
        ref[k] += float(wt[n, 0]) * complex(vis[n, 0]) * np.outer(gy, gx)
    assert np.max(np.abs(G - ref)) < 1e-14


def test_grid_mass_conservation_and_mirror():
    ds = synth.tiny(nrow=4000, seed=5)
    kw = ds.plan_kwargs()
    g = ow.tap_table(kw["support"], kw["oversample"])
    b = ow.bin_visibilities(ds.uvw, None, ds.vis, None, **{k: kw[k] for k in (
        "grid_n", "n_wplanes", "support", "oversample", "fov", "w_min", "w_max")})
    G = ow.grid(b, g, grid_n=kw["grid_n"], n_wplanes=kw["n_wplanes"])
    for k in range(kw["n_wplanes"]):
        sel = b.keep & (b.k == k)
        assert abs(G[k].sum() - b.wv[sel].sum()) < 1e-11 * max(1.0, abs(b.wv[sel].sum()))
    # mirror: (u,v,w,V) -> (-u,-v,-w,V*) maps cell (j,i) -> (N-j, N-i), plane k -> N_w-1-k
    b2 = ow.bin_visibilities(-ds.uvw, None, np.conj(ds.vis), None, **{k: kw[k] for k in (
        "grid_n", "n_wplanes", "support", "oversample", "fov", "w_min", "w_max")})
    G2 = ow.grid(b2, g, grid_n=kw["grid_n"], n_wplanes=kw["n_wplanes"])
    N = kw["grid_n"]
    mirrored = np.conj(G2[::-1, ::-1, ::-1])            # index N-1-j
    mirrored = np.roll(mirrored, shift=(1, 1), axis=(1, 2))  # -> index N-j
    assert np.max(np.abs(mirrored - G)) < 1e-12


# ---------------------------------------------------------------------------
# P5: inverse FFT
# ---------------------------------------------------------------------------
def test_ifft_planes_brute_force_and_parseval():
    rng = np.random.default_rng(15)
    N = 8
    G = rng.normal(size=(2, N, N)) + 1j * rng.normal(size=(2, N, N))
    F = ow.ifft_planes(G)
    idx = np.arange(N) - N // 2
    ref = np.zeros_like(G)
    for q in range(N):
        for p in range(N):
            ph = np.exp(2j * np.pi * (idx[None, :] * idx[p] + idx[:, None] * idx[q]) / N)
            ref[:, q, p] = (G * ph[None]).sum(axis=(1, 2))
    assert np.max(np.abs(F - ref)) < 1e-12
    assert abs((np.abs(F) ** 2).sum() - N * N * (np.abs(G) ** 2).sum()) < 1e-9 * (np.abs(F) ** 2).sum()


# ---------------------------------------------------------------------------
# P6: screen, plane sum, normalisation
# ---------------------------------------------------------------------------
def test_wstacking_equals_dft_when_exact():
    """W = 1, OS = 1, (u, v) on cell centres, every w on a plane centre: no
    kernel, position or plane error remains, so w-stacking equals the DFT."""
    rng = np.random.default_rng(16)
    N, Nw, fov = 32, 6, 0.9
    w_min, w_max = -30.0, 30.0
    dw = (w_max - w_min) / Nw
    n = 1500
    i = rng.integers(1, N - 1, n)
    j = rng.integers(1, N - 1, n)
    k = rng.integers(0, Nw, n)
    uvw = np.stack([(i - N // 2) / fov, (j - N // 2) / fov, w_min + (k + 0.5) * dw], 1)
    vis = (rng.normal(size=n) + 1j * rng.normal(size=n)).astype(np.complex64).reshape(-1, 1)
    wt = rng.uniform(0.5, 2.0, (n, 1)).astype(np.float32)
    r = ow.wstack_image(uvw, None, vis, wt, grid_n=N, n_wplanes=Nw, support=1, oversample=1, fov=fov,
                        w_min=w_min, w_max=w_max)
    assert np.array_equal(r.binned.k, k) and r.binned.keep.all()
    D = od.dft_of_binned(r.binned, fov, N)
    assert np.max(np.abs(r.image - D)) < 1e-12 * np.max(np.abs(D))


@pytest.mark.parametrize("kernel", ["gaussian", "kaiser_bessel"])
def test_phase_centre_source_gives_flux_at_centre(kernel):
    """V = S for all samples: the centre pixel equals S exactly for any W, OS, N_w
    (n - 1 = 0 there, rows sum to 1, C(0) = 1)."""
    rng = np.random.default_rng(17)
    n = 3000
    uvw = np.stack([rng.normal(0, 60, n), rng.normal(0, 60, n), rng.uniform(-40, 40, n)], 1)
    S = 1.75
    vis = np.full((n, 1), S, np.complex64)
    wt = rng.uniform(0.1, 1.0, (n, 1)).astype(np.float32)
    for W, OS, Nw in [(7, 32, 8), (5, 4, 3), (3, 16, 1)]:
        r = ow.wstack_image(uvw, None, vis, wt, grid_n=128, n_wplanes=Nw, support=W, oversample=OS,
                            fov=0.5, w_min=-40.0, w_max=40.0, kernel=kernel)
        assert abs(r.image[64, 64] - S) < 1e-12


def test_single_plane_zero_w_is_2d_image():
    """N_w = 1 with a symmetric w range: the screen is 1 and the image is the
    2-D gridded image n Re(F_0) / (C C sum W)."""
    ds = synth.tiny(nrow=3000, seed=7)
    uvw = ds.uvw.copy()
    uvw[:, 2] = 0.0
    r = ow.wstack_image(uvw, None, ds.vis, None, **{**ds.plan_kwargs(), "n_wplanes": 1})
    N = ds.grid_n
    l = ow.pixel_lm(N, ds.fov)
    n = 1 + ow.nm1_of(l[None, :], l[:, None])
    ref = n * r.fplanes[0].real / (r.corr[None, :] * r.corr[:, None] * r.sum_w)
    assert np.max(np.abs(r.image - ref)) < 1e-13 * np.max(np.abs(ref))


def test_wstacking_linear_in_visibilities():
    ds = synth.tiny(nrow=3000, seed=8)
    rng = np.random.default_rng(9)
    v2 = (rng.normal(size=ds.vis.shape) + 1j * rng.normal(size=ds.vis.shape)).astype(np.complex64)
    kw = ds.plan_kwargs()
    i1 = ow.wstack_image(ds.uvw, None, ds.vis, None, **kw).image
    i2 = ow.wstack_image(ds.uvw, None, v2, None, **kw).image
    i3 = ow.wstack_image(ds.uvw, None, ds.vis.astype(np.complex128) * 3.0 + v2 * 0.5, None, **kw).image
    assert np.max(np.abs(i3 - (3.0 * i1 + 0.5 * i2))) < 1e-12 * np.max(np.abs(i3))


# ---------------------------------------------------------------------------
# P7: w-stacking vs DFT -- discretisation error behaves as the method says
# ---------------------------------------------------------------------------
def test_wstacking_converges_to_dft_with_more_planes():
    ds = synth.tiny(nrow=16384, seed=1)
    rows = cols = slice(96, 160)
    errs = []
    D = None
    for Nw in (2, 4, 8, 16):
        r = oracle.wstack.wstack_dataset(ds, n_wplanes=Nw)
        if D is None:
            D = od.dft_of_binned(r.binned, ds.fov, ds.grid_n, rows=rows, cols=cols)
        errs.append(rel_rms(r.image[rows, cols], D))
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 2e-3


def test_kernel_only_error_small_without_w():
    """With w = 0 only kernel aliasing and position rounding remain."""
    ds = synth.tiny(nrow=16384, seed=1)
    uvw = ds.uvw.copy()
    uvw[:, 2] = 0.0
    r = ow.wstack_image(uvw, None, ds.vis, None, **ds.plan_kwargs())
    rows = cols = slice(112, 144)
    D = od.dft_of_binned(r.binned, ds.fov, ds.grid_n, rows=rows, cols=cols)
    assert rel_rms(r.image[rows, cols], D) < 1e-3


# ---------------------------------------------------------------------------
# the sampled-pixel regrouping equals the full pipeline
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("maker", ["tiny", "ska_small"])
def test_pixel_oracle_matches_full_pipeline(maker):
    ds = synth.tiny(nrow=8000, weights=True) if maker == "tiny" else synth.ska_low_small()
    r = oracle.wstack.wstack_dataset(ds)
    rng = np.random.default_rng(3)
    N = ds.grid_n
    pp = np.r_[N // 2, rng.integers(0, N, 30)]
    qq = np.r_[N // 2, rng.integers(0, N, 30)]
    img, F, kept, sw = oracle.pixels.wstack_pixels_dataset(ds, pp, qq)
    assert kept == int(r.binned.keep.sum())
    assert abs(sw - r.sum_w) < 1e-9 * r.sum_w
    ref = r.image[qq, pp]
    assert np.max(np.abs(img - ref)) < 1e-12 * np.max(np.abs(r.image))
    assert np.max(np.abs(F - r.fplanes[:, qq, pp].T)) < 1e-12 * np.max(np.abs(r.fplanes))


@pytest.mark.parametrize("maker", ["tiny", "ska_small"])
def test_bin_stats_match_python_oracle(maker):
    """The C whole-input statistics repeat the Python oracle's decisions exactly."""
    from tests.helpers import oracle_bin_counts
    ds = synth.tiny(nrow=20000, weights=True) if maker == "tiny" else synth.ska_low_small()
    uvw = ds.uvw.copy()
    uvw[0, 0] = np.nan
    uvw[1, 0] = 1e6
    ds.uvw = uvw
    r = oracle.wstack.wstack_dataset(ds)
    b = r.binned
    for tile in (16, 64):
        counts, psum, kept, sw = oracle.pixels.bin_stats(ds.uvw, ds.freq, ds.vis, ds.weight, tile=tile,
                                                         **ds.plan_kwargs())
        assert kept == int(b.keep.sum())
        assert np.array_equal(counts, oracle_bin_counts(b, ds.grid_n, ds.n_wplanes, ds.support, tile))
        for k in range(ds.n_wplanes):
            sel = b.keep & (b.k == k)
            assert abs(psum[k] - b.wv[sel].sum()) <= 1e-9 * max(1.0, np.abs(b.wv[sel]).sum())
        assert abs(sw - r.sum_w) <= 1e-9 * r.sum_w


# ---------------------------------------------------------------------------
# n - 1 of Eq. 1-2, pinned without calling the oracle's own formula
# ---------------------------------------------------------------------------
def _nm1_decimal(l: float, m: float) -> float:
    """sqrt(1 - l^2 - m^2) - 1 in 60-digit decimal arithmetic from the exact
    binary values of l and m: no cancellation survives at this precision."""
    import decimal
    with decimal.localcontext() as ctx:
        ctx.prec = 60
        dl, dm = decimal.Decimal(l), decimal.Decimal(m)
        return float((1 - dl * dl - dm * dm).sqrt() - 1)


def test_nm1_closed_forms():
    """Pythagorean direction cosines give n exactly: (0.6, 0) -> n = 0.8,
    (0, 0.8) -> 0.6, (0.36, 0.48) -> 0.8, (0.48, 0.64) -> 0.6,
    (0.6, 0.6) -> sqrt(0.28)."""
    cases = [((0.6, 0.0), -0.2), ((0.0, 0.8), -0.4), ((0.0, 0.6), -0.2),
             ((0.36, 0.48), -0.2), ((0.48, 0.64), -0.4), ((0.6, 0.6), math.sqrt(0.28) - 1.0), ((0.0, 0.0), 0.0)]
    for (l, m), want in cases:
        got = float(ow.nm1_of(np.array(l), np.array(m)))
        assert abs(got - want) <= 4e-16 * max(1.0, abs(want)), (l, m, got, want)
    assert np.isnan(ow.nm1_of(np.array(0.8), np.array(0.6)))      # r^2 = 1: outside the sky
    assert np.isnan(ow.nm1_of(np.array(1.0), np.array(0.5)))


def test_nm1_matches_high_precision_everywhere():
    """n - 1 agrees with a 60-digit evaluation of sqrt(1 - r^2) - 1 to a few
    ulps of relative error from r^2 = 1e-14 up to r^2 = 0.999 (a flipped sign,
    or the small-angle form -r^2/2, is off by up to 100 % there)."""
    rng = np.random.default_rng(41)
    r = np.sqrt(10.0 ** rng.uniform(-14, np.log10(0.999), 400))
    phi = rng.uniform(0, 2 * np.pi, 400)
    l, m = r * np.cos(phi), r * np.sin(phi)
    got = ow.nm1_of(l, m)
    want = np.array([_nm1_decimal(a, b) for a, b in zip(l, m)])
    assert np.all(want < 0)
    assert np.max(np.abs(got - want) / np.abs(want)) < 4e-15


def test_off_centre_large_w_source_recovered_by_dft_and_wstacking():
    """A point source far from the centre (r^2 = 0.46) seen with |w| up to 2000
    wavelengths, its visibilities built with an n - 1 from 60-digit decimal
    arithmetic (not the oracle's formula): the direct sum gives exactly S at its
    pixel, and w-stacking in the exact configuration (W = 1, OS = 1, cell-centred
    (u, v), plane-centred w) gives S there too.  A wrong n - 1 in the oracle
    leaves a phase error of w times the mistake (hundreds of turns) and the
    pixel decorrelates."""
    rng = np.random.default_rng(42)
    N, Nw, fov = 64, 8, 1.2
    w_min, w_max = -2000.0, 2000.0
    dw = (w_max - w_min) / Nw
    lm = ow.pixel_lm(N, fov)
    p, q = 55, 4                                  # l = 0.43125, m = -0.525
    l0, m0 = float(lm[p]), float(lm[q])
    nm10 = _nm1_decimal(l0, m0)
    assert 0.25 < l0 * l0 + m0 * m0 < 0.5
    n = 4000
    i = rng.integers(1, N - 1, n)
    j = rng.integers(1, N - 1, n)
    k = rng.integers(0, Nw, n)
    u, v, w = (i - N // 2) / fov, (j - N // 2) / fov, w_min + (k + 0.5) * dw
    S = 1.5
    V = (S / (1.0 + nm10)) * np.exp(-2j * np.pi * (u * l0 + v * m0 + w * nm10))
    W = rng.uniform(0.5, 2.0, n)
    img = od.dft_image(u, v, w, W * V, W.sum(), fov, N, rows=slice(q, q + 1), cols=slice(p, p + 1))
    assert abs(img[0, 0] - S) < 1e-9
    r = ow.wstack_image(np.stack([u, v, w], 1), None, V.reshape(-1, 1), W.reshape(-1, 1),
                        grid_n=N, n_wplanes=Nw, support=1, oversample=1, fov=fov,
                        w_min=w_min, w_max=w_max)
    assert r.binned.keep.all()
    assert abs(r.image[q, p] - S) < 1e-9


def test_dft_channel_progression_equals_plain_sum():
    """The row-and-channel form of the direct sum (channel phases advanced as a
    geometric progression) equals the plain per-visibility sum of Eq. 1 over
    the same samples, with weights, at pixels all over the field."""
    rng = np.random.default_rng(43)
    nrow, nchan, N, fov = 3000, 24, 128, 0.5
    uvw = np.stack([rng.normal(0, 900, nrow), rng.normal(0, 900, nrow), rng.normal(0, 200, nrow)], 1)
    freq = 140e6 + np.arange(nchan) * 0.625e6
    vis = (rng.normal(size=(nrow, nchan)) + 1j * rng.normal(size=(nrow, nchan))).astype(np.complex64)
    wt = rng.uniform(0.2, 2.0, (nrow, nchan)).astype(np.float32)
    pp = rng.integers(0, N, 40)
    qq = rng.integers(0, N, 40)
    got = od.dft_pixels_rows(uvw, freq, vis, wt, pp, qq, grid_n=N, fov=fov, sum_w=float(wt.sum(dtype=np.float64)))
    sc = freq / ow.C0
    u = (uvw[:, 0:1] * sc[None, :]).ravel()
    v = (uvw[:, 1:2] * sc[None, :]).ravel()
    w = (uvw[:, 2:3] * sc[None, :]).ravel()
    lm = ow.pixel_lm(N, fov)
    L, M = lm[pp], lm[qq]
    nm1 = ow.nm1_of(L, M)
    D = od.dft_sum(u, v, w, (wt.astype(np.float64) * vis.astype(np.complex128)).ravel(), L, M, nm1)
    want = (1 + nm1) * D.real / float(wt.sum(dtype=np.float64))
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))
