"""Pins of the oracle's density and smoothing-length iteration: lattice geometry
counts, direct lattice sums, the Newton root condition, finite-difference
Omega, two-particle cases, brute force against the cell list, invariances."""
import itertools
import math

import numpy as np
import pytest

from paper_2502_16517_amd import inputs


def lattice_sum(orc, h_over_s):
    """sum over integer vectors k with |k| < 2 h/s of w(|k| s/h), exact enumeration."""
    R = 2.0 * h_over_s
    K = int(math.ceil(R)) + 1
    terms = []
    for k in itertools.product(range(-K, K + 1), repeat=3):
        d = math.sqrt(k[0] ** 2 + k[1] ** 2 + k[2] ** 2)
        if d < R:
            terms.append(orc.w(d / h_over_s))
    return math.fsum(terms), len(terms)


def unjittered(n_side, seed=1):
    return inputs.lattice_box(n_side, seed, jitter=0.0)


def cols(w):
    r = w.rec
    S = inputs.SLOT
    return {k: r[:, S[k]].copy() for k in S if k not in inputs.INT_SLOTS}


def test_lattice_neighbour_count(orc):
    # integer vectors with |k| < 2.4: 1 + 6 + 12 + 8 + 6 + 24 = 57 including self
    w = unjittered(12)
    c = cols(w)
    box = orc.box_of(w.lo, w.length, w.periodic)
    d = orc.density_at(c["x"], c["y"], c["z"], c["m"], c["h"], box)
    assert np.all(d["count"] == 56)
    assert lattice_sum(orc, 1.2)[1] == 57


def test_lattice_density_equals_direct_sum(orc):
    n = 12
    w = unjittered(n)
    c = cols(w)
    s = 1.0 / n
    box = orc.box_of(w.lo, w.length, w.periodic)
    d = orc.density_at(c["x"], c["y"], c["z"], c["m"], c["h"], box)
    S, _ = lattice_sum(orc, 1.2)
    h = 1.2 * s
    expect = c["m"][0] * S / (math.pi * h ** 3)
    assert np.max(np.abs(d["rho"] / expect - 1.0)) < 2e-15 * 60
    # same value in units of the mean density: rho s^3/m (a property of the spline)
    assert abs(expect * s ** 3 / c["m"][0] - S / (math.pi * 1.2 ** 3)) < 1e-15


def test_converged_h_satisfies_root_condition(orc):
    n = 10
    w = unjittered(n)
    c = cols(w)
    s = 1.0 / n
    box = orc.box_of(w.lo, w.length, w.periodic)
    d = orc.density(c["x"], c["y"], c["z"], c["m"], c["h"], box, eta=1.2, tol=1e-13)
    assert np.all(d["converged"] == 1)
    assert np.all(d["iters"] <= 6)
    hs = d["h"][0] / s
    S, _ = lattice_sum(orc, hs)
    rho = c["m"][0] * S / (math.pi * (hs * s) ** 3)
    # rho(h) h^3 = m eta^3 at the returned h, and rho is the lattice sum there
    assert abs(rho * (hs * s) ** 3 / (c["m"][0] * 1.2 ** 3) - 1.0) < 1e-12
    assert np.max(np.abs(d["rho"] / rho - 1.0)) < 1e-13
    assert abs(hs - 1.19967005248) < 1e-9           # the root on this lattice
    # Omega = 1 + h/(3 rho) drho/dh against a central difference of the lattice sum
    e = 1e-6
    rp = c["m"][0] * lattice_sum(orc, hs + e)[0] / (math.pi * ((hs + e) * s) ** 3)
    rm = c["m"][0] * lattice_sum(orc, hs - e)[0] / (math.pi * ((hs - e) * s) ** 3)
    drho = (rp - rm) / (2 * e * s)
    omega = 1.0 + hs * s / (3.0 * rho) * drho
    assert np.max(np.abs(d["omega"] - omega)) < 1e-8
    # equal masses: n_i = rho_i / m, so wcount = (4 pi/3)(2h)^3 rho/m
    wc = 4.0 * math.pi / 3.0 * (2 * d["h"]) ** 3 * d["rho"] / c["m"]
    assert np.max(np.abs(d["wcount"] / wc - 1.0)) < 1e-13


def _two(orc, r, h=0.1, m=0.5):
    x = np.array([0.0, r]); z = np.zeros(2)
    box = orc.box_of((-5, -5, -5), (10, 10, 10), (0, 0, 0))
    return orc.density_at(x, z, z, np.full(2, m), np.full(2, h), box, brute=True)


def test_two_particles(orc):
    h, m = 0.1, 0.5
    d = _two(orc, h, h, m)                 # q = 1: w = 1/4
    assert math.isclose(d["rho"][0], m * (1.0 + 0.25) / (math.pi * h ** 3), rel_tol=1e-15)
    assert list(d["count"]) == [1, 1]
    d = _two(orc, 2 * h, h, m)             # q = 2 is outside the support
    assert math.isclose(d["rho"][0], m / (math.pi * h ** 3), rel_tol=1e-15)
    assert list(d["count"]) == [0, 0]
    d = _two(orc, 2 * h * (1 - 1e-12), h, m)
    assert list(d["count"]) == [1, 1]


def _random_periodic(n, seed, L=(1.0, 0.7, 1.3)):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, L[0], n); y = rng.uniform(0, L[1], n); z = rng.uniform(0, L[2], n)
    vol = L[0] * L[1] * L[2]
    h = 1.2 * (vol / n) ** (1 / 3) * rng.uniform(0.8, 1.25, n)
    m = rng.uniform(0.5, 1.5, n) / n
    return x, y, z, m, h, L


@pytest.mark.parametrize("periodic", [1, 0])
def test_brute_force_equals_cell_list(orc, periodic):
    x, y, z, m, h, L = _random_periodic(1500, 7)
    box = orc.box_of((0, 0, 0), L, (periodic,) * 3)
    a = orc.density(x, y, z, m, h, box, eta=1.2, brute=True)
    b = orc.density(x, y, z, m, h, box, eta=1.2, brute=False, cell_hint=0.05)
    assert np.array_equal(a["count"], b["count"])
    assert np.array_equal(a["iters"], b["iters"])
    for k in ("h", "rho", "omega", "wcount"):
        assert np.max(np.abs(a[k] / b[k] - 1.0)) < 1e-13, k


def test_permutation_and_translation_invariance(orc):
    x, y, z, m, h, L = _random_periodic(800, 11)
    box = orc.box_of((0, 0, 0), L, (1, 1, 1))
    a = orc.density(x, y, z, m, h, box, eta=1.2)
    p = np.random.default_rng(3).permutation(x.shape[0])
    b = orc.density(x[p], y[p], z[p], m[p], h[p], box, eta=1.2)
    assert np.array_equal(a["count"][p], b["count"])
    assert np.max(np.abs(a["rho"][p] / b["rho"] - 1)) < 1e-13
    sx = np.mod(x + 0.3131, L[0]); sy = np.mod(y + 0.17, L[1])
    c = orc.density(sx, sy, z, m, h, box, eta=1.2)
    assert np.array_equal(a["count"], c["count"])
    assert np.max(np.abs(a["rho"] / c["rho"] - 1)) < 1e-11


def test_iteration_flags(orc):
    x, y, z, m, h, L = _random_periodic(400, 5)
    box = orc.box_of((0, 0, 0), L, (1, 1, 1))
    d = orc.density(x, y, z, m, h * 1.7, box, eta=1.2, max_iter=1)
    assert np.all(d["iters"] == 1)
    assert np.all(d["converged"] == 0)
    # returned h is the last evaluated one (the starting h here)
    assert np.array_equal(d["h"], h * 1.7)
