"""Batches of imaging jobs through the C ABI: plan retargeting, work recorded
into a graph and replayed, device timestamps, and the autotuner.

Every replay of a recorded graph is checked against the same jobs run
eagerly, with other eager work and synchronisations between the replays;
retargeted plans are checked against fresh plans and against the oracle.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2504_00959_amd import rick
from tests.helpers import image_errors, rel_rms, to_device

pytestmark = pytest.mark.gpu

FP32_IMG = 1e-5


def _jobs():
    return synth.batched_jobs(seed=21, n_jobs=3, grid_sizes=(256, 512), nvis_range=(2e4, 6e4), n_dumps=200,
                              oversample=32)


def _run_eager(p, ds, uvw, vis, img):
    p.retarget(ds.fov, ds.w_min, ds.w_max)
    p.reset()
    p.grid(uvw, vis, None, ds.freq)
    p.fft()
    p.image(img)


def test_retargeted_plan_matches_a_fresh_plan_and_the_oracle():
    import torch
    a, b = _jobs()[:2]
    b.grid_n = a.grid_n
    b.n_wplanes = a.n_wplanes
    ua, va, _ = to_device(a)
    ub, vb, _ = to_device(b)
    with rick.Plan.for_dataset(a, max_vis=max(a.nvis, b.nvis), fused=True) as p, \
            rick.Plan.for_dataset(b, fused=True) as q:
        img_a = torch.empty((a.grid_n, a.grid_n), dtype=torch.float32, device="cuda:0")
        img_b = torch.empty_like(img_a)
        img_q = torch.empty_like(img_a)
        _run_eager(p, a, ua, va, img_a)
        _run_eager(p, b, ub, vb, img_b)          # same buffers, another field and w range
        _run_eager(q, b, ub, vb, img_q)
        torch.cuda.synchronize()
        got_b, fresh_b = img_b.double().cpu().numpy(), img_q.double().cpu().numpy()
    assert rel_rms(got_b, fresh_b) <= 1e-6
    ref = oracle.wstack.wstack_dataset(b)
    err = image_errors(got_b, ref.image, ref.corr)
    assert err["apparent"] <= FP32_IMG and err["central"] <= FP32_IMG, err


@pytest.mark.parametrize("fused", [True, False])
def test_recorded_jobs_replay_like_eager_runs(fused):
    """Three jobs of two shapes recorded into one graph (two plans, one of them
    retargeted between its jobs), replayed three times with other eager work
    and synchronisations in between; every replay equals the eager images."""
    import torch
    jobs = _jobs()
    dev = [to_device(ds)[:2] for ds in jobs]
    shapes = {}
    for i, ds in enumerate(jobs):
        shapes.setdefault((ds.grid_n, ds.n_wplanes), []).append(i)
    plans = {}
    for key, idx in shapes.items():
        ds0 = jobs[idx[0]]
        plans[key] = rick.Plan.for_dataset(ds0, max_vis=max(jobs[i].nvis for i in idx), fused=fused)
    imgs = [torch.zeros((ds.grid_n, ds.grid_n), dtype=torch.float32, device="cuda:0") for ds in jobs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for i, ds in enumerate(jobs):                      # eager reference (also sets up the kernels)
            _run_eager(plans[(ds.grid_n, ds.n_wplanes)], ds, *dev[i], imgs[i])
        torch.cuda.synchronize()
        eager = [im.double().cpu().numpy() for im in imgs]
        stamps = rick.Stamps(len(jobs) + 1)
        with rick.Graph.record(stream) as graph:
            stamps.stamp(0, stream)
            for i, ds in enumerate(jobs):
                p = plans[(ds.grid_n, ds.n_wplanes)]
                p.retarget(ds.fov, ds.w_min, ds.w_max)
                p.reset(stream)
                p.grid(dev[i][0], dev[i][1], None, ds.freq, stream)
                p.fft(stream)
                p.image(imgs[i], stream)
                stamps.stamp(i + 1, stream)
    for rep in range(3):
        for im in imgs:
            im.fill_(-1.0)
        # other eager work on the same plans between replays
        other = jobs[(rep + 1) % len(jobs)]
        j = (rep + 1) % len(jobs)
        scratch = torch.empty_like(imgs[j])
        _run_eager(plans[(other.grid_n, other.n_wplanes)], other, *dev[j], scratch)
        torch.cuda.synchronize()
        graph.launch(stream)
        stream.synchronize()
        for i in range(len(jobs)):
            got = imgs[i].double().cpu().numpy()
            assert rel_rms(got, eager[i]) <= 1e-6, (rep, i)
        total = stamps.elapsed(0, len(jobs))
        per_job = [stamps.elapsed(i, i + 1) for i in range(len(jobs))]
        assert total > 0 and all(t >= 0 for t in per_job) and sum(per_job) <= total * 1.001 + 1e-3
    graph.close()
    stamps.close()
    for p in plans.values():
        p.close()


def test_autotune_picks_a_valid_shape_that_images_correctly():
    import torch
    ds = synth.tiny(nrow=20000, seed=22)
    uvw, vis, _ = to_device(ds)
    tile, chunk, ms = rick.autotune(ds, uvw, vis, fused=True)
    assert tile in (16, 32, 64) and tile >= ds.support and chunk in (2048, 8192, 32768) and ms > 0
    with rick.Plan.for_dataset(ds, tile=tile, chunk=chunk, fused=True) as p:
        p.reset()
        p.grid(uvw, vis)
        p.fft()
        img = p.image().double().cpu().numpy()
        torch.cuda.synchronize()
        assert p.info()["tile"] == tile
    ref = oracle.wstack.wstack_dataset(ds)
    err = image_errors(img, ref.image, ref.corr)
    assert err["apparent"] <= FP32_IMG and err["central"] <= FP32_IMG, err


def test_sixteen_uneven_jobs_replayed_each_against_the_oracle():
    """The batched form at a size the oracle follows: 16 jobs of uneven grid
    (256 to 1024), plane count and visibility count, one fused plan with
    transposed planes allowed per (grid, planes) shape, recorded into one
    graph and replayed twice.  Every job of every replay is checked against
    the oracle at sampled pixels (apparent image: the taper division is the
    same float64 scale on both sides), and against the eager run."""
    import torch
    jobs = synth.batched_jobs(seed=40, n_jobs=16, grid_sizes=(256, 512, 1024), nvis_range=(2e4, 4e5), n_dumps=300,
                              oversample=32)
    shapes = {}
    for i, ds in enumerate(jobs):
        shapes.setdefault((ds.grid_n, ds.n_wplanes), []).append(i)
    assert len(shapes) >= 3 and max(ds.nvis for ds in jobs) > 5 * min(ds.nvis for ds in jobs)
    dev = [to_device(ds)[:2] for ds in jobs]
    plans = {key: rick.Plan.for_dataset(jobs[idx[0]], max_vis=max(jobs[i].nvis for i in idx), fused=True,
                                        orient=True)
             for key, idx in shapes.items()}
    imgs = [torch.zeros((ds.grid_n, ds.grid_n), dtype=torch.float32, device="cuda:0") for ds in jobs]
    stream = torch.cuda.Stream()
    transposed = []
    with torch.cuda.stream(stream):
        for i, ds in enumerate(jobs):
            p = plans[(ds.grid_n, ds.n_wplanes)]
            _run_eager(p, ds, *dev[i], imgs[i])
            stream.synchronize()
            transposed.append(p.transposed())
        eager = [im.double().cpu().numpy() for im in imgs]
        stamps = rick.Stamps(len(jobs) + 1)
        with rick.Graph.record(stream) as graph:
            stamps.stamp(0, stream)
            for i, ds in enumerate(jobs):
                p = plans[(ds.grid_n, ds.n_wplanes)]
                p.retarget(ds.fov, ds.w_min, ds.w_max)
                p.reset(stream)
                p.grid(dev[i][0], dev[i][1], None, ds.freq, stream)
                p.fft(stream)
                p.image(imgs[i], stream)
                stamps.stamp(i + 1, stream)
    assert any(t.any() for t in transposed) and any((~t).any() for t in transposed)
    # the oracle at sampled pixels of every job: centre, the brightest source, inner-half pixels
    rng = np.random.default_rng(41)
    refs = []
    for ds in jobs:
        N = ds.grid_n
        dl = ds.fov / N
        b = int(np.argmax(ds.sources["flux"]))
        pp = np.r_[N // 2, int(np.rint(ds.sources["l"][b] / dl)) + N // 2, rng.integers(N // 4, 3 * N // 4, 6)]
        qq = np.r_[N // 2, int(np.rint(ds.sources["m"][b] / dl)) + N // 2, rng.integers(N // 4, 3 * N // 4, 6)]
        ref, _, _, _ = oracle.pixels.wstack_pixels(ds.uvw, ds.freq, np.asarray(ds.vis), None, pp, qq,
                                                   **ds.plan_kwargs())
        corr = oracle.wstack.grid_correction(oracle.wstack.tap_table(ds.support, ds.oversample), N)
        refs.append((pp, qq, ref, corr[pp] * corr[qq], np.outer(corr, corr)))
    for rep in range(2):
        for im in imgs:
            im.fill_(-1.0)
        torch.cuda.synchronize()
        graph.launch(stream)
        stream.synchronize()
        for i, (pp, qq, ref, c2, C2) in enumerate(refs):
            got = imgs[i].double().cpu().numpy()
            # (apparent image: split bins add partial tiles with float atomics in
            # no fixed order, which the taper division magnifies at the edges)
            assert rel_rms(got * C2, eager[i] * C2) <= 1e-6, (rep, i)
            e = rel_rms(got[qq, pp] * c2, ref * c2)
            assert e <= FP32_IMG, (rep, i, jobs[i].grid_n, jobs[i].n_wplanes, jobs[i].nvis, e)
        per_job = [stamps.elapsed(i, i + 1) for i in range(len(jobs))]
        assert all(t >= 0 for t in per_job)
    graph.close()
    stamps.close()
    for p in plans.values():
        p.close()
