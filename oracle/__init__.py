"""CPU oracle for the w-stacking imager -- TEST INFRASTRUCTURE ONLY.

Plain, slow, float64 implementations of what the imaging path computes,
written from the paper's equations:

* ``oracle.wstack`` -- w-stacking step by step (nearest-w-plane mapping of
  Sec. 2.1, the convolutional gridding of Eq. 3 with a Gaussian or
  Kaiser-Bessel kernel, an inverse 2D FFT per plane, the per-plane w phase
  screen of Eq. 1 and the sum over planes).
* ``oracle.dft`` -- the direct Fourier sum that w-stacking approximates
  (Eq. 1 discretised over the measured samples, with Eq. 2 as the model),
  as brute force in C.
* ``oracle.learned`` -- a learned gridding kernel: an MLP over (tap offset
  x, tap offset y, w-fraction) tabulated into a non-separable table indexed
  by w-fraction bin, imaging with that table and its 2-D taper, the loss
  against the direct Fourier sum and its exact gradient.
* ``oracle.predict`` -- the other direction: visibilities of a model image
  by the same w-stacking discretisation run backwards (plane images with the
  conjugate screen, forward FFT, interpolation with the tap table; Eq. 2),
  and Eq. 2 itself as a sum over pixels.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The GPU path never calls it and shares no code,
tables or helpers with it.
"""
from . import wstack, dft, pixels, predict, learned  # noqa: F401
