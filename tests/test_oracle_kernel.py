"""Pins of the oracle's smoothing kernel against facts outside its own formula:
normalisation by quadrature, textbook spline values, continuity, and the
derivatives against finite differences of the kernel itself."""
import math

import numpy as np
import pytest
from scipy import integrate


def test_normalisation_by_quadrature(orc):
    # int W dV = 4 pi int_0^{2h} W r^2 dr = 4 int_0^2 w(q) q^2 dq must be 1
    val, err = integrate.quad(lambda q: orc.w(q) * q * q, 0.0, 2.0, points=[1.0],
                              epsabs=1e-15, epsrel=1e-13)
    assert abs(4.0 * val - 1.0) < 1e-13


def test_normalisation_in_h(orc):
    for h in (0.01, 0.3, 2.5):
        val, _ = integrate.quad(lambda r: orc.W(r, h) * 4.0 * math.pi * r * r, 0.0, 2.0 * h,
                                points=[h], epsabs=1e-15, epsrel=1e-13)
        assert abs(val - 1.0) < 1e-12


def test_textbook_values(orc):
    # M4 spline with support 2h: w(0)=1, w(1)=1/4, w(2)=0, zero beyond
    assert orc.w(0.0) == 1.0
    assert orc.w(1.0) == 0.25
    assert orc.w(2.0) == 0.0
    assert orc.w(2.5) == 0.0 and orc.dw(2.5) == 0.0
    assert orc.dw(0.0) == 0.0
    assert orc.dw(1.0) == -0.75
    assert orc.dw(2.0) == 0.0
    assert orc.W(0.0, 1.0) == 1.0 / math.pi


def test_continuity(orc):
    for q0 in (1.0, 2.0):
        for eps in (1e-7, 1e-9):
            assert abs(orc.w(q0 - eps) - orc.w(q0 + eps)) < 10 * eps
            assert abs(orc.dw(q0 - eps) - orc.dw(q0 + eps)) < 10 * eps


@pytest.mark.parametrize("q", np.linspace(0.05, 1.95, 39))
def test_dw_is_derivative_of_w(orc, q):
    e = 1e-6
    fd = (orc.w(q + e) - orc.w(q - e)) / (2 * e)
    assert abs(fd - orc.dw(q)) < 1e-8


@pytest.mark.parametrize("r,h", [(0.01, 0.1), (0.07, 0.1), (0.15, 0.1), (0.19, 0.1), (1.3, 1.0)])
def test_radial_and_h_derivatives(orc, r, h):
    e = 1e-7 * h
    fd_r = (orc.W(r + e, h) - orc.W(r - e, h)) / (2 * e)
    fd_h = (orc.W(r, h + e) - orc.W(r, h - e)) / (2 * e)
    scale = orc.W(0.0, h) / h
    assert abs(fd_r - orc.dWdr(r, h)) < 1e-7 * scale
    assert abs(fd_h - orc.dWdh(r, h)) < 1e-7 * scale


def test_scaling(orc):
    for r, h in ((0.3, 0.2), (0.05, 0.04)):
        assert math.isclose(orc.W(r, h) * h ** 3, orc.W(r / h, 1.0), rel_tol=1e-14)
