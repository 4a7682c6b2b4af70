"""Pins of the oracle's force against physics it must satisfy: momentum, angular
momentum and energy conservation, Galilean invariance, the unjittered lattice,
du/dt against a finite difference of the density along the flow, the pressure
force against minus the gradient of the thermal energy, and the viscosity's
switch-off for receding pairs."""
import math

import numpy as np
import pytest

from paper_2502_16517_amd import inputs

G = 5.0 / 3.0


def state(n_side=8, seed=3, jitter=0.15, periodic=True, vscale=0.3, alpha=0.8, converge=True, orc=None,
          kernel=0):
    w = inputs.lattice_box(n_side, seed, jitter=jitter)
    S = inputs.SLOT
    r = w.rec
    rng = np.random.default_rng(seed + 100)
    n = r.shape[0]
    c = {k: r[:, S[k]].copy() for k in ("x", "y", "z", "m", "h")}
    c["m"] = c["m"] * rng.uniform(0.7, 1.3, n)
    c["vx"], c["vy"], c["vz"] = (rng.normal(0, vscale, n) for _ in range(3))
    c["u"] = rng.uniform(0.8, 1.6, n)
    c["alpha"] = np.full(n, alpha)
    per = (1, 1, 1) if periodic else (0, 0, 0)
    box = orc.box_of(w.lo, w.length, per)
    d = orc.density(c["x"], c["y"], c["z"], c["m"], c["h"], box, eta=1.2, tol=1e-14, max_iter=30,
                    kernel=kernel)
    assert np.all(d["converged"] == 1)
    c["h"], c["rho"], c["omega"] = d["h"], d["rho"], d["omega"]
    return c, box


def run_force(orc, c, box, **kw):
    return orc.force(c["x"], c["y"], c["z"], c["vx"], c["vy"], c["vz"], c["m"], c["h"], c["rho"],
                     c["omega"], c["u"], c["alpha"], box, G, **kw)


@pytest.mark.parametrize("kernel", [0, 1])
@pytest.mark.parametrize("periodic", [True, False])
def test_momentum_and_energy_conservation(orc, periodic, kernel):
    c, box = state(periodic=periodic, orc=orc, kernel=kernel)
    f = run_force(orc, c, box, kernel=kernel)
    m = c["m"]
    scale = np.sum(m * f["sa"])
    for k in ("ax", "ay", "az"):
        assert abs(math.fsum(m * f[k])) < 1e-13 * scale
    dE = math.fsum(m * (c["vx"] * f["ax"] + c["vy"] * f["ay"] + c["vz"] * f["az"] + f["udot"]))
    escale = np.sum(m * (f["sa"] * np.sqrt(c["vx"] ** 2 + c["vy"] ** 2 + c["vz"] ** 2) + f["su"]))
    assert abs(dE) < 1e-13 * escale


def test_angular_momentum_open_box(orc):
    c, box = state(periodic=False, orc=orc)
    f = run_force(orc, c, box)
    m = c["m"]
    r = np.stack([c["x"], c["y"], c["z"]], 1)
    a = np.stack([f["ax"], f["ay"], f["az"]], 1)
    L = np.cross(r, a) * m[:, None]
    scale = np.sum(m * f["sa"] * np.linalg.norm(r, axis=1))
    assert np.all(np.abs(L.sum(0)) < 1e-13 * scale)


def test_galilean_invariance(orc):
    c, box = state(orc=orc)
    f0 = run_force(orc, c, box)
    c2 = dict(c)
    c2["vx"] = c["vx"] + 3.7
    c2["vz"] = c["vz"] - 1.1
    f1 = run_force(orc, c2, box)
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(f0[k] - f1[k]) / f0["sa"]) < 1e-13
    assert np.max(np.abs(f0["udot"] - f1["udot"]) / (f0["su"] + 1e-300)) < 1e-12
    assert np.array_equal(f0["count"], f1["count"])


def test_unjittered_lattice_is_in_equilibrium(orc):
    w = inputs.lattice_box(10, 1, jitter=0.0)
    S = inputs.SLOT
    r = w.rec
    c = {k: r[:, S[k]].copy() for k in S if k not in inputs.INT_SLOTS}
    box = orc.box_of(w.lo, w.length, w.periodic)
    d = orc.density(c["x"], c["y"], c["z"], c["m"], c["h"], box, eta=1.2)
    f = orc.force(c["x"], c["y"], c["z"], c["vx"], c["vy"], c["vz"], c["m"], d["h"], d["rho"],
                  d["omega"], c["u"], c["alpha"], box, G)
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(f[k]) / f["sa"]) < 1e-14
    assert np.all(f["udot"] == 0.0)
    cs = math.sqrt(G * (G - 1.0) * 1.0)
    assert np.all(f["vsig"] == 2.0 * cs)
    # dt = C h / (2 c) on the lattice
    assert orc.time_step(d["h"], f["vsig"], 0.3) == 0.3 * (d["h"].min() / (2.0 * cs))


@pytest.mark.parametrize("kernel", [0, 1])
def test_adiabatic_udot_matches_density_rate(orc, kernel):
    """Without viscosity du_i/dt = (P_i / rho_i^2) d rho_i/dt along the flow,
    with h following rho h^3 = m eta^3 (the grad-h construction)."""
    c, box = state(alpha=0.0, jitter=0.2, orc=orc, kernel=kernel)
    f = run_force(orc, c, box, kernel=kernel)
    dt = 1e-6
    dens = []
    for sgn in (+1, -1):
        x = c["x"] + sgn * dt * c["vx"]
        y = c["y"] + sgn * dt * c["vy"]
        z = c["z"] + sgn * dt * c["vz"]
        d = orc.density(x, y, z, c["m"], c["h"], box, eta=1.2, tol=1e-15, max_iter=40, kernel=kernel)
        dens.append(d["rho"])
    drho = (dens[0] - dens[1]) / (2 * dt)
    P = (G - 1.0) * c["rho"] * c["u"]
    expect = P / c["rho"] ** 2 * drho
    assert np.max(np.abs(f["udot"] - expect) / (f["su"] + 1e-30)) < 2e-6


@pytest.mark.parametrize("kernel", [0, 1])
def test_pressure_force_is_minus_energy_gradient(orc, kernel):
    """The grad-h pressure force derives from the thermal energy U = sum m_j u_j
    at fixed entropy u_j / rho_j^(gamma-1): m_i a_i = -dU/dx_i."""
    c, box = state(alpha=0.0, n_side=7, jitter=0.2, orc=orc, kernel=kernel)
    f = run_force(orc, c, box, kernel=kernel)
    K = c["u"] / c["rho"] ** (G - 1.0)
    eps = 2e-7
    for i in (0, 17, 101):
        for axis, key in ((0, "x"), (1, "y"), (2, "z")):
            Us = []
            for sgn in (+1, -1):
                p = {k: c[k].copy() for k in ("x", "y", "z")}
                p[key][i] += sgn * eps
                d = orc.density(p["x"], p["y"], p["z"], c["m"], c["h"], box, eta=1.2, tol=1e-15,
                                max_iter=40, kernel=kernel)
                Us.append(math.fsum(c["m"] * K * d["rho"] ** (G - 1.0)))
            F = -(Us[0] - Us[1]) / (2 * eps)
            a = f[("ax", "ay", "az")[axis]][i]
            assert abs(c["m"][i] * a - F) < 2e-6 * c["m"][i] * f["sa"][i], (i, key)


def test_viscosity_off_for_receding_pairs(orc):
    c, box = state(periodic=False, orc=orc)
    # Hubble flow away from the box centre: every pair recedes
    for k, ax in (("vx", "x"), ("vy", "y"), ("vz", "z")):
        c[k] = 2.0 * (c[ax] - 0.5)
    f0 = run_force(orc, dict(c, alpha=np.zeros_like(c["alpha"])), box)
    f1 = run_force(orc, c, box)
    for k in ("ax", "ay", "az", "udot", "vsig"):
        assert np.array_equal(f0[k], f1[k]), k


def test_viscosity_dissipates_and_is_linear_in_alpha(orc):
    c, box = state(periodic=False, orc=orc)
    for k, ax in (("vx", "x"), ("vy", "y"), ("vz", "z")):
        c[k] = -2.0 * (c[ax] - 0.5)                     # converging flow
    f0 = run_force(orc, dict(c, alpha=np.zeros_like(c["alpha"])), box)
    f1 = run_force(orc, dict(c, alpha=np.full_like(c["alpha"], 0.5)), box)
    f2 = run_force(orc, dict(c, alpha=np.full_like(c["alpha"], 1.0)), box)
    m = c["m"]
    work = sum(math.fsum(m * c[v] * (f1[a] - f0[a])) for v, a in (("vx", "ax"), ("vy", "ay"), ("vz", "az")))
    heat = math.fsum(m * (f1["udot"] - f0["udot"]))
    assert work < 0.0 and heat > 0.0
    assert abs(work + heat) < 1e-12 * heat
    for k in ("ax", "ay", "az", "udot"):
        lin = (f2[k] - f0[k]) - 2.0 * (f1[k] - f0[k])
        assert np.max(np.abs(lin) / (f2["sa"] + f2["su"])) < 1e-13


@pytest.mark.parametrize("periodic", [True, False])
def test_force_brute_equals_cells(orc, periodic):
    c, box = state(periodic=periodic, orc=orc)
    a = run_force(orc, c, box, brute=True)
    b = run_force(orc, c, box, brute=False, cell_hint=0.1)
    assert np.array_equal(a["count"], b["count"])
    assert np.array_equal(a["vsig"], b["vsig"])
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(a[k] - b[k]) / a["sa"]) < 1e-14
    assert np.max(np.abs(a["udot"] - b["udot"]) / a["su"]) < 1e-14
