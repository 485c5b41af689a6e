"""Pins of the float64 prediction (degridding) oracle against things other
than itself: a special case where the discretisation is exact and the
result must equal Eq. 2 summed over pixels, the adjoint identity with the
(separately pinned) imaging oracle, closed forms, a brute-force DFT, the
w-plane convergence the method promises, and the drop rule.  No GPU.
"""
import numpy as np
import pytest

import synth
from oracle import predict as op
from oracle import wstack as ow


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def test_forward_fft_brute_force():
    """Step 2 against the centred forward DFT written as a double sum."""
    rng = np.random.default_rng(31)
    N = 8
    P = rng.normal(size=(2, N, N)) + 1j * rng.normal(size=(2, N, N))
    H = op.fft_planes_forward(P)
    c = np.arange(N) - N // 2
    E = np.exp(-2j * np.pi * np.outer(c, c) / N)          # [cell][pixel]
    ref = np.einsum("jq,ip,kqp->kji", E, E, P)
    assert np.max(np.abs(H - ref)) < 1e-12 * np.max(np.abs(ref))


def test_exact_case_equals_eq2_sum_over_pixels():
    """W = 1, OS = 1 (no kernel, C = 1), (u, v) on cell centres and every w on
    a plane centre: nothing is approximated, so the w-stacking prediction is
    Eq. 2 summed over the model's pixels."""
    rng = np.random.default_rng(32)
    N, Nw, fov = 32, 6, 0.9
    w_min, w_max = -30.0, 30.0
    dw = (w_max - w_min) / Nw
    n = 600
    i = rng.integers(1, N - 1, n)
    j = rng.integers(1, N - 1, n)
    k = rng.integers(0, Nw, n)
    uvw = np.stack([(i - N // 2) / fov, (j - N // 2) / fov, w_min + (k + 0.5) * dw], 1)
    M = np.zeros((N, N))
    M[rng.integers(0, N, 40), rng.integers(0, N, 40)] = rng.uniform(0.1, 2.0, 40)
    r = op.wstack_predict(M, uvw, None, grid_n=N, n_wplanes=Nw, support=1, oversample=1, fov=fov,
                          w_min=w_min, w_max=w_max)
    assert np.array_equal(r.binned.k, k) and r.binned.keep.all()
    D = op.predict_direct(M, uvw, None, fov)
    assert np.max(np.abs(r.vis - D)) < 1e-11 * np.max(np.abs(D))


@pytest.mark.parametrize("kernel", ["gaussian", "kaiser_bessel"])
def test_adjoint_of_the_imaging_oracle(kernel):
    """<image(V), M / n^2> sum W = Re <V, predict(M)>: prediction is the adjoint
    of the imaging steps (before the real part, with n and sum W undone),
    including visibilities the drop rule removes from both."""
    ds = synth.tiny(nrow=4000, seed=33)
    kw = {**ds.plan_kwargs(), "kernel": kernel, "kernel_param": 0.0}
    uvw = ds.uvw.copy()
    uvw[:7, 0] = 1e9                 # footprints off the grid: dropped by both
    rng = np.random.default_rng(34)
    V = (rng.normal(size=ds.vis.shape) + 1j * rng.normal(size=ds.vis.shape))
    N = ds.grid_n
    M = rng.normal(size=(N, N))
    img = ow.wstack_image(uvw, None, V, None, **kw)
    pred = op.wstack_predict(M, uvw, None, **kw)
    assert not pred.binned.keep[:7].any() and np.array_equal(img.binned.keep, pred.binned.keep)
    assert np.all(pred.vis[:7] == 0)
    l = ow.pixel_lm(N, ds.fov)
    nm1 = ow.nm1_of(l[None, :], l[:, None])
    n2 = np.where(np.isfinite(nm1), (1.0 + np.nan_to_num(nm1)) ** 2, 1.0)
    lhs = float((M * img.image / n2).sum() * img.sum_w)
    rhs = float(np.real(np.vdot(pred.vis, V.reshape(-1))))
    assert abs(lhs - rhs) < 1e-10 * max(abs(lhs), 1.0), (lhs, rhs)


@pytest.mark.parametrize("W,OS,Nw", [(7, 32, 8), (5, 4, 3), (3, 16, 1)])
def test_phase_centre_source_predicts_its_flux(W, OS, Nw):
    """A source at the centre pixel (l = m = 0, n = 1, C(0) = 1) makes every
    H_k constant, so each kept visibility is S exactly (tap rows sum to 1)."""
    rng = np.random.default_rng(35)
    n = 500
    uvw = np.stack([rng.normal(0, 60, n), rng.normal(0, 60, n), rng.uniform(-40, 40, n)], 1)
    N, S = 128, 1.75
    M = np.zeros((N, N))
    M[N // 2, N // 2] = S
    r = op.wstack_predict(M, uvw, None, grid_n=N, n_wplanes=Nw, support=W, oversample=OS, fov=0.5,
                          w_min=-40.0, w_max=40.0)
    kept = r.binned.keep
    assert kept.sum() > 0.9 * n
    assert np.max(np.abs(r.vis[kept] - S)) < 1e-12


def _sources(N, R, seed, n=12):
    rng = np.random.default_rng(seed)
    M = np.zeros((N, N))
    M[rng.integers(N // 2 - R, N // 2 + R, n), rng.integers(N // 2 - R, N // 2 + R, n)] = 1.0
    return M


def test_converges_to_eq2_with_more_planes():
    """Off-centre sources: the error against Eq. 2 is first order in the plane
    width (the screen is exact only at w_k), so it halves with every doubling
    of N_w until the kernel's own error is reached.  OS = 1024 makes the
    position rounding negligible."""
    ds = synth.tiny(nrow=3000, seed=36)
    N = ds.grid_n
    M = _sources(N, 40, 37)
    D = op.predict_direct(M, ds.uvw, None, ds.fov)
    errs = []
    for Nw in (2, 4, 8, 16, 64):
        r = op.wstack_predict(M, ds.uvw, None, **{**ds.plan_kwargs(), "n_wplanes": Nw, "oversample": 1024})
        kept = r.binned.keep
        errs.append(rel(r.vis[kept], D[kept]))
    assert all(b < 0.7 * a for a, b in zip(errs[:4], errs[1:4])), errs
    assert errs[-1] < 2e-3, errs


@pytest.mark.parametrize("OS,bound", [(1024, 1e-3), (32, 1e-2)])
def test_kernel_only_error_small_without_w(OS, bound):
    """w = 0 on one plane centred on 0 (no screen error): only the kernel's
    aliasing and the 1/OS position rounding remain; the rounding moves the
    phase by up to pi (|p - N/2| + |q - N/2|) / (OS N), a few 1e-3 at OS = 32
    for sources 40 pixels out."""
    ds = synth.tiny(nrow=3000, seed=38)
    uvw = ds.uvw.copy()
    uvw[:, 2] = 0.0
    N = ds.grid_n
    M = _sources(N, 40, 37)
    r = op.wstack_predict(M, uvw, None, **{**ds.plan_kwargs(), "n_wplanes": 1, "oversample": OS})
    D = op.predict_direct(M, uvw, None, ds.fov)
    kept = r.binned.keep
    assert rel(r.vis[kept], D[kept]) < bound


def test_sparse_form_equals_full_form():
    """The per-visibility form for sparse models (no FFT) equals steps 1-3 on the whole grid."""
    ds = synth.tiny(nrow=300, seed=39)
    N = ds.grid_n
    rng = np.random.default_rng(40)
    pp = rng.integers(0, N, 9)
    qq = rng.integers(0, N, 9)
    fl = rng.uniform(0.2, 3.0, 9)
    M = np.zeros((N, N))
    np.add.at(M, (qq, pp), fl)
    full = op.wstack_predict(M, ds.uvw, None, **ds.plan_kwargs()).vis
    sparse = op.wstack_predict_sparse(pp, qq, fl, ds.uvw, None, **ds.plan_kwargs())
    assert np.max(np.abs(sparse - full)) < 1e-11 * np.max(np.abs(full))


def test_channels_scale_positions():
    """With channel frequencies, visibility (row, chan) is predicted at uvw * nu / c0."""
    ds = synth.tiny(nrow=200, seed=41)
    N = ds.grid_n
    M = np.zeros((N, N))
    M[N // 2 + 3, N // 2 - 8] = 1.0
    freq = np.array([120e6, 150e6])
    r2 = op.wstack_predict(M, ds.uvw, freq, **ds.plan_kwargs()).vis.reshape(-1, 2)
    for c in range(2):
        r1 = op.wstack_predict(M, ds.uvw * (freq[c] / ow.C0), None, **ds.plan_kwargs()).vis
        assert np.max(np.abs(r2[:, c] - r1)) < 1e-12
