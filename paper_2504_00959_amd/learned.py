"""Training of the learned gridding kernel on the GPU.

The paper convolves visibilities with a Gaussian or Kaiser-Bessel kernel
(Sec. 2.1, Eq. 3).  Here the kernel is a 3 -> 32 -> 32 -> 1 MLP over (tap
offset x, tap offset y, w-fraction), tabulated into a non-separable table per
w-fraction bin, and trained so that the dirty image of a scene matches the
direct Fourier sum of Eq. 1 over the inner half of the field.  This module
only orders the library's calls: every step -- tabulation, imaging with the
table, the loss, its gradient through the adjoint of imaging, the MLP's
backward pass, the Adam update, and the direct sum that serves as the target
-- runs in librick's HIP kernels.
"""
from __future__ import annotations

import numpy as np

from . import rick


class LearnedKernel:
    """MLP parameters and Adam state on the device, and the plans that image
    scenes of one shape with the MLP's table (user table) and with the
    Gaussian kernel (the starting point and the reference)."""

    def __init__(self, *, grid_n: int, n_wplanes: int, support: int, oversample: int, fov: float, w_min: float,
                 w_max: float, max_vis: int, n_wbins: int = 4, seed: int = 0, device: int = 0):
        import torch
        self.dev = f"cuda:{device}"
        self.geo = dict(grid_n=grid_n, n_wplanes=n_wplanes, support=support, oversample=oversample, fov=fov,
                        w_min=w_min, w_max=w_max)
        self.n_wbins = n_wbins
        self.shape = (n_wbins, oversample, oversample, support, support)
        # initial parameters: small random values (host generator, an input)
        rng = np.random.default_rng(seed)
        h = 32
        init = np.concatenate([rng.normal(0, 0.5, h * 3), rng.normal(0, 0.5, h),
                               rng.normal(0, 0.5 / np.sqrt(h), h * h), rng.normal(0, 0.5, h),
                               rng.normal(0, 0.5 / np.sqrt(h), h), [0.0]]).astype(np.float32)
        self.theta = torch.as_tensor(init, device=self.dev)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.dtheta = torch.empty_like(self.theta)
        self.t = 0
        self.plan = rick.Plan(**self.geo, max_vis=max_vis, kernel="user_lut", lut_wbins=n_wbins, device=device)
        self.gauss = rick.Plan(**self.geo, max_vis=max_vis, kernel="gaussian", device=device)
        self.table = torch.empty(self.shape, dtype=torch.float32, device=self.dev)
        self.dtable = torch.empty(self.shape, dtype=torch.float64, device=self.dev)
        N = grid_n
        self.dA = torch.empty((N, N), dtype=torch.float64, device=self.dev)
        self.dC = torch.empty((N, N), dtype=torch.float64, device=self.dev)
        self.img = torch.empty((N, N), dtype=torch.float32, device=self.dev)

    def close(self):
        self.plan.close()
        self.gauss.close()

    def _adam(self, lr):
        self.t += 1
        rick.adam_step(self.theta, self.dtheta, self.m, self.v, self.t, lr)

    def fit_table(self, target, steps: int, lr: float):
        """Least-squares fit of the MLP's table to `target` (float32 device table);
        returns the final mean squared difference."""
        import torch
        sums = torch.zeros((steps, 2), dtype=torch.float64, device=self.dev)
        for i in range(steps):
            rick.mlp_tabulate(self.theta, self.geo["support"], self.geo["oversample"], self.n_wbins, out=self.table)
            rick.table_residual(self.table, target, self.dtable, sums[i])
            rick.mlp_backward(self.theta, self.table, self.dtable, self.dtheta)
            self._adam(lr)
        return float(sums[-1, 0])

    def gaussian_table(self):
        return self.gauss.separable_table(self.n_wbins)

    def target(self, uvw, vis):
        """The direct Fourier sum over the whole image (float64, device)."""
        return self.gauss.dft_image(uvw, vis)

    def image(self, plan, uvw, vis):
        plan.reset()
        plan.grid(uvw, vis, None, None)
        plan.fft()
        plan.image(self.img)
        return self.img

    def loss(self, plan, uvw, vis, target, sums):
        """Loss of `plan`'s image against target into sums (device [2]): sums[0] / sums[1]."""
        img = self.image(plan, uvw, vis)
        plan.image_loss(img, target, self.dA, self.dC, sums)

    def snapshot(self):
        return self.theta.clone()

    def restore(self, theta):
        self.theta.copy_(theta)

    def install(self):
        rick.mlp_tabulate(self.theta, self.geo["support"], self.geo["oversample"], self.n_wbins, out=self.table)
        self.plan.set_lut(self.table)

    def step(self, uvw, vis, target, sums, lr: float):
        """One training step on one scene: tabulate, image, loss, gradient through
        the adjoint of imaging and the MLP, Adam.  The loss before the update
        goes to sums."""
        self.install()
        self.loss(self.plan, uvw, vis, target, sums)
        self.plan.table_gradient(self.dA, self.dC, uvw, vis, None, None, self.dtable)
        rick.mlp_backward(self.theta, self.table, self.dtable, self.dtheta)
        self._adam(lr)
