"""Shared helpers for the GPU parity tests (inputs, oracle-side bin counts, metrics)."""
import numpy as np


def rel_rms(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / den) if den > 0 else float(np.linalg.norm(a))


def oracle_bin_counts(b, grid_n, n_wplanes, support, tile):
    """Records per (plane, tile) bin implied by the oracle's per-visibility
    decisions: a kept visibility adds one record to the tile holding the
    top-left cell c - h of its footprint."""
    h = (support - 1) // 2
    nt = grid_n // tile
    idx = np.nonzero(b.keep)[0]
    cx, cy, k = b.cx[idx], b.cy[idx], b.k[idx]
    counts = np.zeros(n_wplanes * nt * nt, dtype=np.int64)
    np.add.at(counts, (k * nt + (cy - h) // tile) * nt + (cx - h) // tile, 1)
    return counts


def to_device(ds, precision="fp32", device="cuda:0"):
    import torch
    uvw = torch.as_tensor(ds.uvw, dtype=torch.float64).to(device)
    cd = torch.complex128 if precision == "fp64" else torch.complex64
    vis = ds.vis if isinstance(ds.vis, torch.Tensor) else torch.as_tensor(np.asarray(ds.vis))
    vis = vis.to(device=device, dtype=cd).contiguous()
    wt = None if ds.weight is None else torch.as_tensor(ds.weight, dtype=torch.float32).to(device).contiguous()
    return uvw, vis, wt


def image_errors(img, ref, corr, central=0.1):
    """Errors of an image against the oracle image.

    The last step divides by the kernel's image-plane taper C(l'_p) C(l'_q),
    an exact float64 per-pixel scale applied identically on both sides; it
    amplifies arithmetic noise by up to 1 / min(C)^2 at the image edge
    (6.4e3 for the default support-7 Gaussian, unbounded for wide Gaussians
    whose taper reaches ~0).  So float32 parity is measured
      apparent -- on n S / sum W, i.e. before the taper division, and
      central  -- on the corrected image where C(l'_p) C(l'_q) >= `central`;
    `full` (whole corrected image) is reported, and gated only in float64.
    """
    C2 = np.outer(corr, corr)
    m = C2 >= central
    return dict(apparent=rel_rms(img * C2, ref * C2), central=rel_rms(img[m], ref[m]), full=rel_rms(img, ref))
