"""Seeded synthetic interferometer data for tests and benchmarks.

This module only *draws inputs*: antenna layouts, earth-rotation (u,v,w)
tracks, channel frequencies, point-source skies and the visibilities those
skies produce through the measurement equation (Eq. 2 of the paper, point
sources: V = sum_s S_s/n_s * exp(-2 pi i (u l_s + v m_s + w (n_s - 1)))).
It contains none of the imaging arithmetic (quantisation, gridding, FFT,
w-correction, normalisation); both the oracle and the GPU path consume what
it returns.

Random draws use numpy's PCG64 ``default_rng(seed)`` in the order written
in each function.  The visibility sum over sources runs in float64 either
with numpy (small cases) or with torch on a chosen device (large cases, so
that the 2e8-visibility workloads can be generated on the GPU in seconds);
the result is rounded to complex64, which is what both sides consume.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

C0 = 299_792_458.0  # speed of light [m/s]
SIDEREAL_DAY_S = 86164.0905


@dataclass
class Dataset:
    """One imaging job: inputs plus the plan parameters that go with them."""
    uvw: np.ndarray                 # float64 [R, 3]; metres if freq is given, else wavelengths
    freq: Optional[np.ndarray]      # float64 [C] in Hz, or None (uvw already in wavelengths)
    vis: object                     # complex64 [R, C]  (numpy array, or torch tensor if generated on a device)
    weight: Optional[np.ndarray]    # float32 [R, C] or None (unit weights)
    grid_n: int
    n_wplanes: int
    support: int
    oversample: int
    fov: float
    w_min: float
    w_max: float
    kernel: str = "gaussian"
    kernel_param: float = 0.0
    sources: dict = field(default_factory=dict)
    name: str = ""

    @property
    def nrow(self) -> int:
        return int(self.uvw.shape[0])

    @property
    def nchan(self) -> int:
        return 1 if self.freq is None else int(len(self.freq))

    @property
    def nvis(self) -> int:
        return self.nrow * self.nchan

    def plan_kwargs(self) -> dict:
        return dict(grid_n=self.grid_n, n_wplanes=self.n_wplanes, support=self.support,
                    oversample=self.oversample, fov=self.fov, w_min=self.w_min,
                    w_max=self.w_max, kernel=self.kernel, kernel_param=self.kernel_param)


def source_nm1(l: np.ndarray, m: np.ndarray) -> np.ndarray:
    """n - 1 for direction cosines (l, m), written without cancellation."""
    r2 = l * l + m * m
    return -r2 / (1.0 + np.sqrt(1.0 - r2))


# --------------------------------------------------------------------------
# measurement equation (point sources), float64
# --------------------------------------------------------------------------
def point_source_vis_np(u: np.ndarray, v: np.ndarray, w: np.ndarray,
                        l: np.ndarray, m: np.ndarray, flux: np.ndarray,
                        chunk: int = 1 << 16) -> np.ndarray:
    """Eq. 2 for point sources, float64 complex, numpy.  u, v, w in wavelengths."""
    nm1 = source_nm1(l, m)
    amp = flux / (1.0 + nm1)
    out = np.empty(u.shape[0], dtype=np.complex128)
    for a in range(0, u.shape[0], chunk):
        b = min(a + chunk, u.shape[0])
        ph = (np.outer(u[a:b], l) + np.outer(v[a:b], m) + np.outer(w[a:b], nm1))
        out[a:b] = np.exp(-2j * np.pi * ph) @ amp
    return out


def point_source_vis_torch(uvw_m, scales, l, m, flux, device, row_chunk: int = 1 << 15):
    """Eq. 2 for point sources on a torch device, float64, per channel.

    ``uvw_m`` float64 [R,3] (metres or wavelengths), ``scales`` float64 [C]
    (nu_c / c0, or 1.0).  Returns complex64 [R, C] on ``device``.
    """
    import torch
    uvw_t = torch.as_tensor(uvw_m, dtype=torch.float64, device=device)
    lt = torch.as_tensor(l, dtype=torch.float64, device=device)
    mt = torch.as_tensor(m, dtype=torch.float64, device=device)
    nm1 = torch.as_tensor(source_nm1(np.asarray(l), np.asarray(m)), dtype=torch.float64, device=device)
    amp = torch.as_tensor(np.asarray(flux) / (1.0 + source_nm1(np.asarray(l), np.asarray(m))),
                          dtype=torch.complex128, device=device)
    R = uvw_t.shape[0]
    C = len(scales)
    out = torch.empty((R, C), dtype=torch.complex64, device=device)
    lmn = torch.stack([lt, mt, nm1], dim=0)  # [3, S]
    for a in range(0, R, row_chunk):
        b = min(a + row_chunk, R)
        base = uvw_t[a:b] @ lmn  # [rows, S] path difference (metres or wavelengths)
        for c, sc in enumerate(scales):
            ph = base * (-2.0 * math.pi * float(sc))
            e = torch.polar(torch.ones_like(ph), ph)
            out[a:b, c] = (e @ amp).to(torch.complex64)
    return out


# --------------------------------------------------------------------------
# tiny workload: 65,536 visibilities, 1 channel, 256^2 x 8 planes
# --------------------------------------------------------------------------
def tiny(seed: int = 1, nrow: int = 65_536, n_src: int = 5, grid_n: int = 256, fov: float = 0.2,
         n_wplanes: int = 8, support: int = 7, oversample: int = 32, uv_radius: float = 120.0,
         w_abs: float = 50.0, kernel: str = "gaussian", kernel_param: float = 0.0,
         weights: bool = False, device: Optional[str] = None) -> Dataset:
    """Uniform-disk (u,v) in wavelengths with uniform w and a few point sources.

    Draw order: source l, m, flux; then radius U, angle U, w U; then (if
    ``weights``) weights U[0.5, 2].
    """
    rng = np.random.default_rng(seed)
    l = rng.uniform(-0.05, 0.05, n_src)
    m = rng.uniform(-0.05, 0.05, n_src)
    flux = rng.uniform(0.1, 1.0, n_src)
    r = uv_radius * np.sqrt(rng.uniform(0.0, 1.0, nrow))
    phi = 2.0 * np.pi * rng.uniform(0.0, 1.0, nrow)
    w = rng.uniform(-w_abs, w_abs, nrow)
    uvw = np.stack([r * np.cos(phi), r * np.sin(phi), w], axis=1)
    wt = rng.uniform(0.5, 2.0, (nrow, 1)).astype(np.float32) if weights else None
    if device is None:
        vis = point_source_vis_np(uvw[:, 0], uvw[:, 1], uvw[:, 2], l, m, flux)
        vis = vis.astype(np.complex64).reshape(nrow, 1)
    else:
        vis = point_source_vis_torch(uvw, [1.0], l, m, flux, device)
    return Dataset(uvw=uvw, freq=None, vis=vis, weight=wt, grid_n=grid_n, n_wplanes=n_wplanes,
                   support=support, oversample=oversample, fov=fov, w_min=-w_abs, w_max=w_abs,
                   kernel=kernel, kernel_param=kernel_param,
                   sources=dict(l=l, m=m, flux=flux), name="tiny")


# --------------------------------------------------------------------------
# SKA-LOW-like array, one GPU's time-slice share
# --------------------------------------------------------------------------
def station_layout(rng, n_stations: int, sigma_m: float) -> np.ndarray:
    """Local (E, N, U) positions: E, N ~ N(0, sigma^2), U = 0."""
    e = rng.normal(0.0, sigma_m, n_stations)
    n = rng.normal(0.0, sigma_m, n_stations)
    return np.stack([e, n, np.zeros(n_stations)], axis=1)


def enu_to_xyz(enu: np.ndarray, lat_rad: float) -> np.ndarray:
    """Local horizon (E, N, U) to equatorial (X, Y, Z) baseline frame
    (Thompson, Moran & Swenson, ch. 4)."""
    e, n, u = enu[:, 0], enu[:, 1], enu[:, 2]
    sl, cl = math.sin(lat_rad), math.cos(lat_rad)
    return np.stack([-sl * n + cl * u, e, cl * n + sl * u], axis=1)


def xyz_to_uvw(bxyz: np.ndarray, ha_rad: np.ndarray, dec_rad: float) -> np.ndarray:
    """Baselines (X, Y, Z) at hour angles H to (u, v, w), time-major rows
    (row = t * n_baselines + b), in metres."""
    sd, cd = math.sin(dec_rad), math.cos(dec_rad)
    sh = np.sin(ha_rad)[:, None]
    ch = np.cos(ha_rad)[:, None]
    X, Y, Z = bxyz[None, :, 0], bxyz[None, :, 1], bxyz[None, :, 2]
    u = sh * X + ch * Y
    v = -sd * ch * X + sd * sh * Y + cd * Z
    w = cd * ch * X - cd * sh * Y + sd * Z
    return np.stack([u, v, w], axis=-1).reshape(-1, 3)


def ska_low(seed: int = 2, n_stations: int = 512, sigma_m: float = 3000.0, n_times: int = 100,
            dump_s: float = 10.0, ha_start_h: float = -2.0, n_chan: int = 16,
            f_centre_hz: float = 150e6, band_hz: float = 20e6, n_src: int = 1000,
            grid_n: int = 4096, n_wplanes: int = 64, support: int = 7, oversample: int = 64,
            lat_deg: float = -26.7, dec_deg: float = -30.0, uv_fill: float = 0.45,
            kernel: str = "gaussian", kernel_param: float = 0.0,
            device: Optional[str] = None, with_vis: bool = True) -> Dataset:
    """Earth-rotation tracks of a Gaussian-distributed station array.

    Stations: E, N ~ N(0, sigma_m^2), U = 0; baselines i < j (no autos).
    Times: hour angle -2 h + t * dump_s (sidereal rate), t = 0..n_times-1.
    Channels: n_chan equally spaced over ``band_hz`` centred on ``f_centre_hz``.
    Field of view: uv_fill * N / u_max, u_max = max(|u|, |v|) in wavelengths
    at the highest channel, so the data fill uv_fill of the half-grid.
    Sources: l, m ~ U(-0.4 FoV, 0.4 FoV); fluxes with N(>S) ~ S^-1.5 on
    [0.01, 10] Jy drawn by the inverse CDF.  Weights: unit (None).
    Draw order: stations E, N; source l, m, flux-U.
    """
    rng = np.random.default_rng(seed)
    enu = station_layout(rng, n_stations, sigma_m)
    xyz = enu_to_xyz(enu, math.radians(lat_deg))
    i, j = np.triu_indices(n_stations, k=1)
    bxyz = xyz[j] - xyz[i]
    ha = (ha_start_h * 3600.0 + dump_s * np.arange(n_times)) * (2.0 * math.pi / SIDEREAL_DAY_S)
    uvw = xyz_to_uvw(bxyz, ha, math.radians(dec_deg))
    dnu = band_hz / n_chan
    freq = f_centre_hz + (np.arange(n_chan) - (n_chan - 1) / 2.0) * dnu
    scales = freq / C0
    umax = float(np.max(np.abs(uvw[:, :2]))) * float(scales.max())
    fov = uv_fill * grid_n / umax
    wl = uvw[:, 2]
    w_lo = min(float(wl.min()) * float(scales.max()), float(wl.min()) * float(scales.min()))
    w_hi = max(float(wl.max()) * float(scales.max()), float(wl.max()) * float(scales.min()))
    l = rng.uniform(-0.4 * fov, 0.4 * fov, n_src)
    m = rng.uniform(-0.4 * fov, 0.4 * fov, n_src)
    a, b = 10.0 ** -1.5, 0.01 ** -1.5
    flux = (a + rng.uniform(0.0, 1.0, n_src) * (b - a)) ** (-1.0 / 1.5)
    vis = None
    if with_vis:
        if device is None:
            cols = [point_source_vis_np(uvw[:, 0] * s, uvw[:, 1] * s, uvw[:, 2] * s, l, m, flux)
                    for s in scales]
            vis = np.stack(cols, axis=1).astype(np.complex64)
        else:
            vis = point_source_vis_torch(uvw, scales, l, m, flux, device)
    return Dataset(uvw=uvw, freq=freq, vis=vis, weight=None, grid_n=grid_n, n_wplanes=n_wplanes,
                   support=support, oversample=oversample, fov=fov, w_min=w_lo, w_max=w_hi,
                   kernel=kernel, kernel_param=kernel_param,
                   sources=dict(l=l, m=m, flux=flux), name="ska_low")


def ska_low_share(device: Optional[str] = None, with_vis: bool = True) -> Dataset:
    """One GPU's time-slice share of the SKA-LOW-like observation:
    512 stations, 100 dumps of 10 s, 16 channels -> 209,305,600 visibilities,
    4096^2 grid, 64 w-planes, support 7, oversample 64."""
    return ska_low(device=device, with_vis=with_vis)


def ska_low_precision(device: Optional[str] = None, with_vis: bool = True) -> Dataset:
    """The precision-form workload: the same array, time slice and sources,
    32 channels over the same 20 MHz band -> 418,611,200 visibilities,
    8192^2 grid, 128 w-planes, support 7, oversample 64."""
    ds = ska_low(n_chan=32, grid_n=8192, n_wplanes=128, device=device, with_vis=with_vis)
    ds.name = "ska_low_precision"
    return ds


def _xyz_to_uvw_torch(bxyz: np.ndarray, ha_rad: np.ndarray, dec_rad: float, device: str):
    """``xyz_to_uvw`` in float64 on a torch device (same formulas and row order)."""
    import torch
    sd, cd = math.sin(dec_rad), math.cos(dec_rad)
    h = torch.as_tensor(ha_rad, dtype=torch.float64, device=device)[:, None]
    sh, ch = torch.sin(h), torch.cos(h)
    b = torch.as_tensor(bxyz, dtype=torch.float64, device=device)
    X, Y, Z = b[None, :, 0], b[None, :, 1], b[None, :, 2]
    u = sh * X + ch * Y
    v = -sd * ch * X + sd * sh * Y + cd * Z
    w = cd * ch * X - cd * sh * Y + sd * Z
    return torch.stack([u, v, w], dim=-1).reshape(-1, 3)


def batched_jobs(seed: int = 4, n_jobs: int = 64, grid_sizes=(512, 1024, 2048, 4096), nvis_range=(1e5, 5e7),
                 n_src: int = 20, n_stations: int = 512, sigma_m: float = 3000.0, dump_s: float = 10.0,
                 n_dumps: int = 1440, ha_start_h: float = -2.0, freq_hz: float = 150e6, support: int = 7,
                 oversample: int = 64, uv_fill: float = 0.45, min_planes: int = 4, max_planes: int = 64,
                 lat_deg: float = -26.7, dec_deg: float = -30.0, device: Optional[str] = None,
                 with_vis: bool = True) -> list:
    """Many independent imaging jobs of uneven size (the batched form).

    The SKA-LOW-like array of ``ska_low`` observed for 4 h at 10 s (1440
    dumps, time-major rows) at one channel.  Job j: grid N_j uniform over
    ``grid_sizes``; visibility count log-uniform over ``nvis_range``; a
    contiguous run of that many rows from a uniform start; FoV = uv_fill N /
    u_max over its rows; w range from its data; planes
    N_w = clamp(2^ceil(log2(4 (w_max - w_min) max|n - 1|)), 4, 64) with
    max|n - 1| at the image corner (a w phase error of at most pi/4 there);
    ``n_src`` point sources as in ``ska_low``.  Draw order: stations E, N;
    then per job N_j, count, start row, source l, m, flux-U.  With a device,
    uvw and visibilities are generated there (uvw then is a device tensor).
    """
    rng = np.random.default_rng(seed)
    enu = station_layout(rng, n_stations, sigma_m)
    xyz = enu_to_xyz(enu, math.radians(lat_deg))
    i, j = np.triu_indices(n_stations, k=1)
    bxyz = xyz[j] - xyz[i]
    nbl = bxyz.shape[0]
    total_rows = n_dumps * nbl
    scale = freq_hz / C0
    jobs = []
    for jj in range(n_jobs):
        N = int(grid_sizes[int(rng.integers(0, len(grid_sizes)))])
        nv = int(round(math.exp(rng.uniform(math.log(nvis_range[0]), math.log(nvis_range[1])))))
        nv = min(nv, total_rows)
        r0 = int(rng.integers(0, total_rows - nv + 1))
        t0, t1 = r0 // nbl, (r0 + nv - 1) // nbl
        ha = (ha_start_h * 3600.0 + dump_s * np.arange(t0, t1 + 1)) * (2.0 * math.pi / SIDEREAL_DAY_S)
        if device is None:
            uvw = xyz_to_uvw(bxyz, ha, math.radians(dec_deg))[r0 - t0 * nbl:r0 - t0 * nbl + nv].copy()
            umax = float(np.max(np.abs(uvw[:, :2]))) * scale
            w_lo, w_hi = float(uvw[:, 2].min()) * scale, float(uvw[:, 2].max()) * scale
        else:
            uvw = _xyz_to_uvw_torch(bxyz, ha, math.radians(dec_deg), device)[r0 - t0 * nbl:r0 - t0 * nbl + nv]
            uvw = uvw.contiguous()
            umax = float(uvw[:, :2].abs().max()) * scale
            w_lo, w_hi = float(uvw[:, 2].min()) * scale, float(uvw[:, 2].max()) * scale
        fov = uv_fill * N / umax
        if not w_hi > w_lo:
            w_hi = w_lo + 1.0
        r2 = 2.0 * (0.5 * fov) ** 2
        nm1_max = r2 / (1.0 + math.sqrt(1.0 - r2))
        x = 4.0 * (w_hi - w_lo) * nm1_max
        nw = 1 << max(0, math.ceil(math.log2(x))) if x > 1.0 else 1
        nw = int(min(max(nw, min_planes), max_planes))
        l = rng.uniform(-0.4 * fov, 0.4 * fov, n_src)
        m = rng.uniform(-0.4 * fov, 0.4 * fov, n_src)
        a, b = 10.0 ** -1.5, 0.01 ** -1.5
        flux = (a + rng.uniform(0.0, 1.0, n_src) * (b - a)) ** (-1.0 / 1.5)
        freq = np.array([freq_hz])
        vis = None
        if with_vis:
            if device is None:
                vis = point_source_vis_np(uvw[:, 0] * scale, uvw[:, 1] * scale, uvw[:, 2] * scale, l, m,
                                          flux)[:, None].astype(np.complex64)
            else:
                vis = point_source_vis_torch(uvw, np.array([scale]), l, m, flux, device)
        jobs.append(Dataset(uvw=uvw, freq=freq, vis=vis, weight=None, grid_n=N, n_wplanes=nw, support=support,
                            oversample=oversample, fov=fov, w_min=w_lo, w_max=w_hi,
                            sources=dict(l=l, m=m, flux=flux), name=f"batch_job{jj}"))
    return jobs


def ska_low_small(seed: int = 3, device: Optional[str] = None, **kw) -> Dataset:
    """Same generator at a size the oracle finishes in seconds."""
    args = dict(seed=seed, n_stations=48, n_times=24, dump_s=60.0, n_chan=4, n_src=20,
                grid_n=256, n_wplanes=12, oversample=32)
    args.update(kw)
    return ska_low(device=device, **args)


# --------------------------------------------------------------------------
# learned-kernel training scenes: tiny-style, 1..20 sources each
# --------------------------------------------------------------------------
def learned_scene(index: int, seed: int = 5, nvis: int = 1_000_000, grid_n: int = 256, n_wplanes: int = 16,
                  fov: float = 0.2, uv_fill: float = 0.45, w_ratio: float = 50.0 / 120.0, max_src: int = 20,
                  support: int = 7, oversample: int = 64, device: Optional[str] = None) -> Dataset:
    """Scene ``index`` of the learned-kernel training set: the tiny workload's
    generator (uniform-disk u, v in wavelengths, uniform w, unit weights) with
    the disk radius u_max = uv_fill N / FoV, |w| <= w_ratio u_max (the tiny
    workload's ratio), and 1..max_src point sources with |l|, |m| < FoV / 4 and
    flux U[0.1, 1].  Each scene has its own generator, seeded (seed, index).
    Draw order: source count, l, m, flux; then radius U, angle U, w U."""
    rng = np.random.default_rng([seed, index])
    n_src = int(rng.integers(1, max_src + 1))
    l = rng.uniform(-0.25 * fov, 0.25 * fov, n_src)
    m = rng.uniform(-0.25 * fov, 0.25 * fov, n_src)
    flux = rng.uniform(0.1, 1.0, n_src)
    umax = uv_fill * grid_n / fov
    wmax = w_ratio * umax
    r = umax * np.sqrt(rng.uniform(0.0, 1.0, nvis))
    phi = 2.0 * np.pi * rng.uniform(0.0, 1.0, nvis)
    w = rng.uniform(-wmax, wmax, nvis)
    uvw = np.stack([r * np.cos(phi), r * np.sin(phi), w], axis=1)
    if device is None:
        vis = point_source_vis_np(uvw[:, 0], uvw[:, 1], uvw[:, 2], l, m, flux).astype(np.complex64).reshape(-1, 1)
    else:
        vis = point_source_vis_torch(uvw, [1.0], l, m, flux, device)
    return Dataset(uvw=uvw, freq=None, vis=vis, weight=None, grid_n=grid_n, n_wplanes=n_wplanes,
                   support=support, oversample=oversample, fov=fov, w_min=-wmax, w_max=wmax,
                   sources=dict(l=l, m=m, flux=flux), name=f"learned_scene{index}")
