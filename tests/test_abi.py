"""The C-ABI library loads, exports every declared symbol, and validates
arguments on the host before touching a device (no GPU needed)."""
import ctypes

import pytest

from paper_2504_00959_amd import rick


def test_library_exports_every_header_symbol():
    L = rick.lib()
    names = rick.header_functions()
    assert {"rick_plan", "rick_grid", "rick_fft_planes", "rick_wstack_image", "rick_reset",
            "rick_plan_info", "rick_plan_destroy", "rick_status_str"} <= set(names)
    for n in names:
        assert hasattr(L, n), n


def test_status_strings():
    L = rick.lib()
    for s in range(0, 9):
        assert L.rick_status_str(s)
    assert L.rick_status_str(99) == b"unknown status"


def _plan_status(**over):
    L = rick.lib()
    kw = dict(grid_n=256, n_wplanes=8, support=7, oversample=32, fov=0.2, w_min=-50.0, w_max=50.0)
    kw.update(over)
    d = rick.make_desc(**kw)
    h = ctypes.c_void_p(1234)
    st = L.rick_plan(ctypes.byref(d), ctypes.byref(h))
    return st, h.value


@pytest.mark.parametrize("over", [
    dict(grid_n=100), dict(grid_n=32), dict(grid_n=32768),
    dict(kernel="user_lut", lut_wbins=0), dict(kernel="user_lut", lut_wbins=3), dict(kernel="user_lut", lut_wbins=16), dict(n_wplanes=0), dict(support=4),
    dict(support=17), dict(oversample=3), dict(oversample=512), dict(fov=0.0), dict(fov=1.5),
    dict(w_min=1.0, w_max=1.0), dict(w_min=float("nan")), dict(max_vis=-1), dict(max_vis=1 << 29),
    dict(tile=48), dict(tile=8), dict(tile=128), dict(tile=256),
    dict(device=-1), dict(kernel_param=float("inf")), dict(chunk=-1),
])
def test_invalid_plan_rejected_before_device(over):
    st, h = _plan_status(**over)
    assert st == 1, rick.lib().rick_last_error()      # RICK_E_INVALID_ARG
    assert h is None                                    # *out cleared


def test_null_arguments():
    L = rick.lib()
    assert L.rick_plan(None, None) == 1
    h = ctypes.c_void_p()
    assert L.rick_plan(None, ctypes.byref(h)) == 1
    for call in (lambda: L.rick_grid(None, None, None, None, None, 0, 1, None),
                 lambda: L.rick_fft_planes(None, None), lambda: L.rick_wstack_image(None, None, None),
                 lambda: L.rick_reset(None, None), lambda: L.rick_plan_info(None, None),
                 lambda: L.rick_plan_destroy(None), lambda: L.rick_plan_bin_counts(None, None, 0)):
        assert call() == 6                              # RICK_E_BAD_PLAN


def test_valid_plan_without_device_reports_no_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    st, h = _plan_status()
    assert st == 2 and h is None                        # RICK_E_NO_DEVICE


def test_binding_refuses_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(rick, "_lib", None)
    monkeypatch.setattr(rick, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        rick.lib()


def test_learned_calls_validate_on_the_host():
    """The learned-kernel calls reject bad shapes, NULL pointers and bad
    handles before any device work (no GPU needed)."""
    L = rick.lib()
    fake = ctypes.c_void_p(16)
    assert L.rick_mlp_tabulate(fake, 4, 16, 2, fake, None) == 1          # even support
    assert L.rick_mlp_tabulate(fake, 7, 12, 2, fake, None) == 1          # oversample not a power of two
    assert L.rick_mlp_tabulate(fake, 7, 16, 3, fake, None) == 1          # w-fraction bins
    assert L.rick_mlp_tabulate(None, 7, 16, 2, fake, None) == 1
    assert L.rick_mlp_backward(fake, 7, 16, 2, fake, None, fake, None) == 1
    assert L.rick_adam_step(fake, fake, fake, fake, 0, 1, 1e-3, 0.9, 0.999, 1e-8, None) == 1
    assert L.rick_adam_step(fake, fake, fake, fake, 10, 1, 1e-3, 1.0, 0.999, 1e-8, None) == 1
    assert L.rick_plan_set_lut(None, fake, 1, None) == 6                 # RICK_E_BAD_PLAN
    assert L.rick_image_loss(None, fake, fake, fake, fake, fake, None) == 6
    assert L.rick_table_gradient(None, fake, fake, fake, None, fake, None, 1, 1, fake, None) == 6
    assert L.rick_dft_image(None, fake, None, fake, None, 1, 1, 0, 0, 1, 1, fake, None) == 6


def test_grid_jobs_validates_on_the_host():
    L = rick.lib()
    assert L.rick_grid_jobs(None, 1, None) == 1                     # RICK_E_INVALID_ARG: no jobs
    jobs = (rick.GridJob * 2)()
    assert L.rick_grid_jobs(jobs, 0, None) == 1                     # n out of range
    assert L.rick_grid_jobs(jobs, 65, None) == 1
    assert b"1 ... 64" in L.rick_last_error()
    assert L.rick_grid_jobs(jobs, 2, None) == 6                     # RICK_E_BAD_PLAN: a NULL plan


def test_wstack_image_jobs_validates_on_the_host():
    L = rick.lib()
    assert L.rick_wstack_image_jobs(None, 1, None) == 1              # RICK_E_INVALID_ARG: no jobs
    jobs = (rick.ImageJob * 2)()
    assert L.rick_wstack_image_jobs(jobs, 0, None) == 1              # n out of range
    assert L.rick_wstack_image_jobs(jobs, 65, None) == 1
    assert L.rick_wstack_image_jobs(jobs, 2, None) == 6              # RICK_E_BAD_PLAN: a NULL plan
