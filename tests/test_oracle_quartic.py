"""Pins of the oracle's quartic M5 spline (the kernel the paper employs,
Sec. 2.1), scaled to support 2h, against facts outside its own formula: the
degree-4 cardinal B-spline of scipy (Cox-de Boor recursion, a different
algorithm), normalisation by quadrature, continuity at the knots, finite
differences, and lattice sums built from the B-spline through the density
entry points (kernel id 1)."""
import itertools
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.interpolate import BSpline

from paper_2502_16517_amd import inputs

Q = 1          # kernel id of the quartic
# M5 is 4! times the degree-4 B-spline on unit-spaced knots centred at 0; with
# support 2h its variable is s = 1.25 q and the 3-D normalisation 1/(10.24 pi h^3)
_B = BSpline.basis_element(np.array([-2.5, -1.5, -0.5, 0.5, 1.5, 2.5]), extrapolate=False)
_dB = _B.derivative()


def w_bspline(q):
    s = 1.25 * np.asarray(q, dtype=float)
    v = np.nan_to_num(_B(s), nan=0.0)
    return 24.0 * v / 10.24


def dw_bspline(q):
    s = 1.25 * np.asarray(q, dtype=float)
    v = np.nan_to_num(_dB(s), nan=0.0)
    return 1.25 * 24.0 * v / 10.24


def test_shape_is_the_degree4_bspline(orc):
    qs = np.concatenate([np.linspace(0.0, 1.999, 401), [0.4, 1.2, 0.3999999, 1.2000001]])
    for q in qs:
        assert abs(orc.w(q, Q) - float(w_bspline(q))) < 1e-14, q
        assert abs(orc.dw(q, Q) - float(dw_bspline(q))) < 1e-13, q


def test_normalisation_by_quadrature(orc):
    # int W dV = 4 int_0^2 w(q) q^2 dq = 1
    val, _ = integrate.quad(lambda q: orc.w(q, Q) * q * q, 0.0, 2.0, points=[0.4, 1.2],
                            epsabs=1e-15, epsrel=1e-13)
    assert abs(4.0 * val - 1.0) < 1e-13


def test_normalisation_in_h(orc):
    for h in (0.01, 0.3, 2.5):
        val, _ = integrate.quad(lambda r: orc.W(r, h, Q) * 4.0 * math.pi * r * r, 0.0, 2.0 * h,
                                points=[0.4 * h, 1.2 * h], epsabs=1e-15, epsrel=1e-13)
        assert abs(val - 1.0) < 1e-12


def test_support_and_centre(orc):
    assert orc.w(2.0, Q) == 0.0 and orc.dw(2.0, Q) == 0.0
    assert orc.w(3.0, Q) == 0.0 and orc.dw(3.0, Q) == 0.0
    assert orc.w(1.999, Q) > 0.0
    assert orc.dw(0.0, Q) == 0.0
    # w(0) = (2.5^4 - 5 1.5^4 + 10 0.5^4) / 10.24 = 14.375 / 10.24
    assert math.isclose(orc.w(0.0, Q), 14.375 / 10.24, rel_tol=1e-15)
    # monotone decreasing inside the support
    qs = np.linspace(0.0, 1.99, 200)
    assert np.all(np.diff([orc.w(q, Q) for q in qs]) < 0.0)


def test_continuity_at_knots(orc):
    for q0 in (0.4, 1.2, 2.0):
        for eps in (1e-7, 1e-9):
            assert abs(orc.w(q0 - eps, Q) - orc.w(q0 + eps, Q)) < 10 * eps
            assert abs(orc.dw(q0 - eps, Q) - orc.dw(q0 + eps, Q)) < 10 * eps


@pytest.mark.parametrize("r,h", [(0.01, 0.1), (0.05, 0.1), (0.13, 0.1), (0.19, 0.1), (1.3, 1.0)])
def test_radial_and_h_derivatives(orc, r, h):
    e = 1e-7 * h
    fd_r = (orc.W(r + e, h, Q) - orc.W(r - e, h, Q)) / (2 * e)
    fd_h = (orc.W(r, h + e, Q) - orc.W(r, h - e, Q)) / (2 * e)
    scale = orc.W(0.0, h, Q) / h
    assert abs(fd_r - orc.dWdr(r, h, Q)) < 1e-7 * scale
    assert abs(fd_h - orc.dWdh(r, h, Q)) < 1e-7 * scale


def test_unknown_kernel_rejected(orc):
    with pytest.raises(ValueError):
        orc.w(0.5, 2)
    x = np.zeros(1)
    box = orc.box_of((0, 0, 0), (1, 1, 1), (1, 1, 1))
    with pytest.raises(ValueError):
        orc.density_at(x, x, x, np.ones(1), np.full(1, 0.1), box, kernel=7)


def _lattice_sum_bspline(h_over_s):
    R = 2.0 * h_over_s
    K = int(math.ceil(R)) + 1
    terms = []
    for k in itertools.product(range(-K, K + 1), repeat=3):
        d = math.sqrt(k[0] ** 2 + k[1] ** 2 + k[2] ** 2)
        if d < R:
            terms.append(float(w_bspline(d / h_over_s)))
    return math.fsum(terms)


def _cols(w):
    S = inputs.SLOT
    return {k: w.rec[:, S[k]].copy() for k in S if k not in inputs.INT_SLOTS}


def test_lattice_density_equals_bspline_sum(orc):
    n = 12
    w = inputs.lattice_box(n, 1, jitter=0.0)
    c = _cols(w)
    s = 1.0 / n
    box = orc.box_of(w.lo, w.length, w.periodic)
    d = orc.density_at(c["x"], c["y"], c["z"], c["m"], c["h"], box, kernel=Q)
    h = 1.2 * s
    expect = c["m"][0] * _lattice_sum_bspline(1.2) / (math.pi * h ** 3)
    assert np.max(np.abs(d["rho"] / expect - 1.0)) < 1e-13
    # the two kernels give different sums on the same lattice
    d0 = orc.density_at(c["x"], c["y"], c["z"], c["m"], c["h"], box)
    assert np.all(np.abs(d0["rho"] / d["rho"] - 1.0) > 1e-4)


def test_converged_h_and_omega_on_the_lattice(orc):
    n = 10
    w = inputs.lattice_box(n, 1, jitter=0.0)
    c = _cols(w)
    s = 1.0 / n
    box = orc.box_of(w.lo, w.length, w.periodic)
    d = orc.density(c["x"], c["y"], c["z"], c["m"], c["h"], box, eta=1.2, tol=1e-13, kernel=Q)
    assert np.all(d["converged"] == 1)
    hs = d["h"][0] / s
    rho = c["m"][0] * _lattice_sum_bspline(hs) / (math.pi * (hs * s) ** 3)
    assert abs(rho * (hs * s) ** 3 / (c["m"][0] * 1.2 ** 3) - 1.0) < 1e-12
    assert np.max(np.abs(d["rho"] / rho - 1.0)) < 1e-13
    e = 1e-6
    rp = c["m"][0] * _lattice_sum_bspline(hs + e) / (math.pi * ((hs + e) * s) ** 3)
    rm = c["m"][0] * _lattice_sum_bspline(hs - e) / (math.pi * ((hs - e) * s) ** 3)
    omega = 1.0 + hs * s / (3.0 * rho) * (rp - rm) / (2 * e * s)
    assert np.max(np.abs(d["omega"] - omega)) < 1e-8
