"""The float32 sin/cos polynomials of the fused screen kernel, checked on the CPU.

The w phase screen of Eq. 1 multiplies plane k by exp(+2 pi i w_k (n - 1)).
The kernel forms the argument in float64 half turns, takes the nearest
integer out (a sign), and evaluates sin(pi g) and cos(pi g) for the float32
remainder g in [-1/2, 1/2] by two polynomials in g^2 (Horner form, float32
fused multiply-adds; sincospi_half, also used by the direct-sum kernel).
This test reads the coefficients from the kernel source, evaluates the same Horner steps with float32 rounding after every
fused step, and checks the stated bound of 2.5e-7 absolute error against
numpy's float64 sin and cos over every float32 g in a dense sweep.
"""
import os
import re

import numpy as np

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2504_00959_amd", "csrc", "rick_internal.h")


def _coeffs():
    body = open(SRC).read()
    fn = body[body.index("__device__ __forceinline__ void sincospi_half("):]
    fn = fn[:fn.index("\n}\n")]
    sin_c = [float(x) for x in re.findall(r"ps = fmaf\(g2, (?:ps|[-0-9.e]+f), ([-0-9.e]+)f\)", fn)]
    first_s = re.search(r"ps = fmaf\(g2, ([-0-9.e]+)f,", fn).group(1)
    cos_c = [float(x) for x in re.findall(r"(?:pc|cs) = fmaf\(g2, (?:pc|[-0-9.e]+f), ([-0-9.e]+)f\)", fn)]
    first_c = re.search(r"pc = fmaf\(g2, ([-0-9.e]+)f,", fn).group(1)
    return [float(first_s)] + sin_c, [float(first_c)] + cos_c


def _fma32(a, b, c):
    # a*b of two float32 values is exact in float64; one float64 add, then
    # rounding to float32 (double rounding differs from a true fmaf only on
    # rare ties, far below the bound checked here)
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(np.float32)


def test_screen_polynomials_within_stated_bound():
    s, c = _coeffs()
    assert len(s) == 5 and len(c) == 6, (s, c)
    g = np.linspace(-0.5, 0.5, 2_000_001).astype(np.float32)
    g2 = (g * g).astype(np.float32)
    f32 = np.float32
    ps = _fma32(g2, np.full_like(g2, f32(s[0])), np.full_like(g2, f32(s[1])))
    for k in s[2:]:
        ps = _fma32(g2, ps, np.full_like(g2, f32(k)))
    sn = (g * ps).astype(np.float32)
    pc = _fma32(g2, np.full_like(g2, f32(c[0])), np.full_like(g2, f32(c[1])))
    for k in c[2:]:
        pc = _fma32(g2, pc, np.full_like(g2, f32(k)))
    gd = g.astype(np.float64)
    err_s = np.max(np.abs(sn - np.sin(np.pi * gd)))
    err_c = np.max(np.abs(pc - np.cos(np.pi * gd)))
    assert err_s < 2.5e-7, err_s
    assert err_c < 2.5e-7, err_c
    # the constant and linear terms are the Taylor ones to float32 precision
    assert abs(s[-1] - np.pi) < 1e-6 and c[-1] == 1.0
