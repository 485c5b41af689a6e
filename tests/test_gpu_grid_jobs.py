"""Many jobs per launch through the C ABI: the gridding of many jobs in one
persistent launch (rick_grid_jobs) and the fused column passes of many
plans of one grid size in one launch (rick_wstack_image_jobs).

Eight jobs of uneven grid size, plane count and visibility count, each on
its own plan (two tile edges, so two launches; small chunks on some plans,
so bins spanning several work items flush with atomics), are gridded
jointly and checked against the same plans gridded one call at a time:
equal counters and tile bitmaps, planes equal to float rounding, images
equal to float rounding, and every job's image against the oracle's.  The joint call is also recorded into a graph and replayed,
with other work between the replays, and its argument checks are exercised.
The joint column pass must give every plan's image bit for bit, with
planes stored as they are and transposed, in float32 (plain and
compensated sums) and float64.
"""
import numpy as np
import pytest

import oracle
import synth
from paper_2504_00959_amd import rick
from tests.helpers import image_errors, rel_rms, to_device

pytestmark = pytest.mark.gpu

FP32_IMG = 1e-5


def _jobs(n=6, seed=23):
    return synth.batched_jobs(seed=seed, n_jobs=n, grid_sizes=(256, 512), nvis_range=(2e4, 2e5), n_dumps=200,
                              oversample=32)


def _plans(jobs, precision="fp32"):
    # tiles of 32 and 64 cells in turn; small gridding chunks on every third plan
    return [rick.Plan.for_dataset(ds, precision=precision, fused=True, tile=(32, 64)[i % 2],
                                  chunk=(512 if i % 3 == 0 else 0)) for i, ds in enumerate(jobs)]


def _state(p):
    inf = p.info()
    return dict(counts=(inf["n_gridded"], inf["n_dropped"], inf["n_records"]), sum_w=inf["sum_weights"],
                mask=p.tile_mask(), G=p.mesh().cpu().numpy())


def _apparent(ds):
    c = oracle.wstack.grid_correction(oracle.wstack.tap_table(ds.support, ds.oversample), ds.grid_n)
    return np.outer(c, c)


def _image(p):
    import torch
    p.fft()
    img = p.image().double().cpu().numpy()
    torch.cuda.synchronize()
    return img


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_joint_launch_equals_one_call_per_job(precision):
    import torch
    jobs = _jobs(8 if precision == "fp32" else 4)
    dev = [to_device(ds, precision)[:2] for ds in jobs]
    plans = _plans(jobs, precision)
    try:
        single, joint = [], []
        for p, ds, (u, v) in zip(plans, jobs, dev):
            p.reset()
            p.grid(u, v, None, ds.freq)
        torch.cuda.synchronize()
        for p in plans:
            single.append(_state(p))
            single[-1]["img"] = _image(p)
        for p in plans:
            p.reset()
        rick.grid_jobs([(p, u, v, None, ds.freq) for p, ds, (u, v) in zip(plans, jobs, dev)])
        torch.cuda.synchronize()
        for p in plans:
            joint.append(_state(p))
            joint[-1]["img"] = _image(p)
    finally:
        for p in plans:
            p.close()
    g_tol = 1e-12 if precision == "fp64" else 1e-6
    for i, (a, b) in enumerate(zip(single, joint)):
        assert a["counts"] == b["counts"], i
        assert abs(a["sum_w"] - b["sum_w"]) <= 1e-9 * abs(a["sum_w"]), i
        assert np.array_equal(a["mask"], b["mask"]), i
        assert rel_rms(b["G"], a["G"]) <= g_tol, i
        c2 = _apparent(jobs[i])
        assert rel_rms(b["img"] * c2, a["img"] * c2) <= g_tol, i
    # every job against the oracle
    assert len({(ds.grid_n, ds.n_wplanes) for ds in jobs}) >= 2
    for i in range(len(jobs)):
        ref = oracle.wstack.wstack_dataset(jobs[i])
        if precision == "fp64":
            assert rel_rms(joint[i]["img"], ref.image) <= 1e-10
        else:
            err = image_errors(joint[i]["img"], ref.image, ref.corr)
            assert err["apparent"] <= FP32_IMG and err["central"] <= FP32_IMG, (i, err)


def test_joint_launch_recorded_and_replayed():
    import torch
    jobs = _jobs(5, seed=24)
    dev = [to_device(ds)[:2] for ds in jobs]
    plans = _plans(jobs)
    imgs = [torch.zeros((ds.grid_n, ds.grid_n), dtype=torch.float32, device="cuda:0") for ds in jobs]
    stream = torch.cuda.Stream()
    args = [(p, u, v, None, ds.freq) for p, ds, (u, v) in zip(plans, jobs, dev)]

    def run(s):
        for p in plans:
            p.reset(s)
        rick.grid_jobs(args, s)
        for p in plans:
            p.fft(s)
        rick.wstack_image_jobs(list(zip(plans, imgs)), s)

    try:
        with torch.cuda.stream(stream):
            run(stream)                                    # eager reference
            torch.cuda.synchronize()
            eager = [im.double().cpu().numpy() for im in imgs]
            with rick.Graph.record(stream) as graph:
                run(stream)
            for rep in range(3):
                for im in imgs:
                    im.fill_(float("nan"))
                torch.cuda.synchronize()
                graph.launch(stream)
                torch.cuda.synchronize()
                got = [im.double().cpu().numpy() for im in imgs]
                for i, (a, b) in enumerate(zip(eager, got)):
                    # apparent images: bins split over several chunks add their
                    # partial tiles with float atomics in no fixed order, which
                    # the taper division magnifies in the corners
                    c2 = _apparent(jobs[i])
                    assert np.isfinite(b).all(), (rep, i)
                    assert rel_rms(b * c2, a * c2) <= 1e-6, (rep, i)
                _ = torch.ones(1 << 20, device="cuda:0").sum().item()   # other eager work between replays
            graph.close()
    finally:
        for p in plans:
            p.close()
    ref = oracle.wstack.wstack_dataset(jobs[2])
    err = image_errors(got[2], ref.image, ref.corr)
    assert err["apparent"] <= FP32_IMG and err["central"] <= FP32_IMG, err


def test_joint_launch_argument_checks():
    jobs = _jobs(2, seed=25)
    dev = [to_device(ds)[:2] for ds in jobs]
    p = rick.Plan.for_dataset(jobs[0], fused=True)
    q = rick.Plan.for_dataset(jobs[1], precision="fp64", fused=True)
    u = rick.Plan(grid_n=256, n_wplanes=4, support=7, oversample=32, fov=0.2, w_min=-1.0, w_max=1.0,
                  kernel="user_lut", lut_wbins=2)
    try:
        u0, v0 = dev[0]
        with pytest.raises(rick.RickError, match="INVALID_ARG"):      # the same plan twice
            rick.grid_jobs([(p, u0, v0, None, jobs[0].freq), (p, u0, v0, None, jobs[0].freq)])
        u1, v1, _ = to_device(jobs[1], "fp64")
        with pytest.raises(rick.RickError, match="INVALID_ARG"):      # mixed precisions
            rick.grid_jobs([(p, u0, v0, None, jobs[0].freq), (q, u1, v1, None, jobs[1].freq)])
        with pytest.raises(rick.RickError, match="UNSUPPORTED"):      # a user table
            rick.grid_jobs([(u, u0, v0, None, jobs[0].freq)])
    finally:
        for x in (p, q, u):
            x.close()


@pytest.mark.parametrize("precision", ["fp32", "fp32_kahan", "fp64"])
def test_joint_column_pass_equals_one_call_per_plan(precision):
    import torch
    jobs = _jobs(8 if precision != "fp64" else 4, seed=26)
    dev = [to_device(ds, precision)[:2] for ds in jobs]
    # every other plan with transposed planes allowed (a second pass)
    plans = [rick.Plan.for_dataset(ds, precision=precision, fused=True, orient=(i % 2 == 1))
             for i, ds in enumerate(jobs)]
    try:
        for p, ds, (u, v) in zip(plans, jobs, dev):
            p.reset()
            p.grid(u, v, None, ds.freq)
            p.fft()
        single = [p.image() for p in plans]
        joint = [torch.full_like(im, float("nan")) for im in single]
        rick.wstack_image_jobs(list(zip(plans, joint)))
        torch.cuda.synchronize()
        assert any(p.transposed().any() for p in plans)
        for i, (a, b) in enumerate(zip(single, joint)):
            assert torch.equal(a, b), i
        ref = oracle.wstack.wstack_dataset(jobs[3])
        got = joint[3].double().cpu().numpy()
        if precision == "fp64":
            assert rel_rms(got, ref.image) <= 1e-10
        else:
            err = image_errors(got, ref.image, ref.corr)
            assert err["apparent"] <= FP32_IMG and err["central"] <= FP32_IMG, err
        with pytest.raises(rick.RickError, match="STATE"):             # planes not transformed
            plans[0].reset()
            rick.wstack_image_jobs([(plans[0], joint[0])])
    finally:
        for p in plans:
            p.close()


def test_joint_calls_with_an_empty_job():
    """A job without visibilities among others: no work items of its own in
    the joint gridding (the queue's prefix skips it), zero counters and a
    zero image through the joint column pass; the other jobs as one call
    each would give."""
    import torch
    jobs = _jobs(3, seed=27)
    dev = [to_device(ds)[:2] for ds in jobs]
    plans = [rick.Plan.for_dataset(ds, fused=True) for ds in jobs]
    try:
        single = []
        for p, ds, (u, v) in zip(plans, jobs, dev):
            p.reset()
            p.grid(u, v, None, ds.freq)
            p.fft()
            single.append(p.image())
        empty_u = dev[1][0][:0].contiguous()
        empty_v = dev[1][1][:0].contiguous()
        args = [(plans[0], *dev[0], None, jobs[0].freq), (plans[1], empty_u, empty_v, None, jobs[1].freq),
                (plans[2], *dev[2], None, jobs[2].freq)]
        for p in plans:
            p.reset()
        rick.grid_jobs(args)
        for p in plans:
            p.fft()
        imgs = [torch.full_like(im, float("nan")) for im in single]
        rick.wstack_image_jobs(list(zip(plans, imgs)))
        torch.cuda.synchronize()
        inf = plans[1].info()
        assert inf["n_gridded"] == 0 and inf["n_records"] == 0
        assert torch.count_nonzero(imgs[1]) == 0
        for i in (0, 2):
            c2 = _apparent(jobs[i])
            a, b = single[i].double().cpu().numpy(), imgs[i].double().cpu().numpy()
            assert rel_rms(b * c2, a * c2) <= 1e-6, i
    finally:
        for p in plans:
            p.close()
