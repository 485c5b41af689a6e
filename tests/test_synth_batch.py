"""The batched-form job generator (host only): job shapes follow their rules."""
import math

import numpy as np

import synth


def test_batched_jobs_follow_their_rules():
    jobs = synth.batched_jobs(seed=5, n_jobs=12, grid_sizes=(256, 512, 1024), nvis_range=(1e3, 2e4), n_dumps=100,
                              with_vis=False)
    assert len(jobs) == 12
    scale = 150e6 / synth.C0
    for ds in jobs:
        assert ds.grid_n in (256, 512, 1024)
        assert 1e3 * 0.999 <= ds.nvis <= 2e4 * 1.001 and ds.nchan == 1
        u = ds.uvw[:, :2] * scale
        # field of view by the 0.45 N / u_max rule: the data fill 0.45 of the half grid
        assert math.isclose(np.abs(u).max() * ds.fov, 0.45 * ds.grid_n, rel_tol=1e-12)
        w = ds.uvw[:, 2] * scale
        assert math.isclose(ds.w_min, w.min(), rel_tol=1e-12) and math.isclose(ds.w_max, w.max(), rel_tol=1e-12)
        r2 = 2.0 * (0.5 * ds.fov) ** 2
        x = 4.0 * (ds.w_max - ds.w_min) * r2 / (1.0 + math.sqrt(1.0 - r2))
        want = min(max(2 ** max(0, math.ceil(math.log2(x))) if x > 1 else 1, 4), 64)
        assert ds.n_wplanes == want
        assert len(ds.sources["flux"]) == 20


def test_batched_jobs_are_contiguous_runs_of_the_observation():
    # rows of a job are consecutive rows of the time-major observation
    jobs = synth.batched_jobs(seed=6, n_jobs=2, grid_sizes=(256,), nvis_range=(5e3, 5e3), n_dumps=60,
                              n_stations=32, with_vis=False)
    full = synth.ska_low(seed=6, n_stations=32, n_times=60, n_chan=1, with_vis=False)
    for ds in jobs:
        n = ds.nvis
        hits = [r for r in range(full.uvw.shape[0] - n + 1) if np.array_equal(full.uvw[r], ds.uvw[0])]
        assert any(np.allclose(full.uvw[r:r + n], ds.uvw, rtol=0, atol=1e-9) for r in hits)
