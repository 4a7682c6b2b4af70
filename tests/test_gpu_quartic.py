"""GPU parity of the pair loops with the quartic M5 spline (the kernel the
paper employs, Sec. 2.1; kernel id 1, support 2h) against the oracle with the
same kernel: density with the smoothing-length iteration and force on small
workloads, layouts and masking bit-identical, the FP32 form within its
budget, one whole step with the kick bit for bit, and a sample of the full
two-state tube in the launch configuration the benchmark times."""
import numpy as np
import pytest

from paper_2502_16517_amd import inputs
from paper_2502_16517_amd import sphview as sv

from gpu_helpers import S, bits, check_density, check_force, cols, oracle_density, oracle_force, \
    run_density, run_density_force

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

Q = sv.KERNEL_QUARTIC

SMALL = {
    "lattice16": (lambda: inputs.config1(), {}),
    "tube16": (lambda: inputs.two_state_tube(16, 7), {}),
    "kh24": (lambda: inputs.kelvin_helmholtz(24, 9), {}),
    "plummer8k": (lambda: inputs.plummer(8192, 5, cell=0.1), {"headroom": 1.6}),
}


@pytest.mark.parametrize("name", list(SMALL))
def test_quartic_density_and_force_match_oracle(orc, name):
    print(f"[quartic fp64] {name}", flush=True)
    mk, pkw = SMALL[name]
    w = mk()
    dens, out, state = run_density_force(w, kernel=Q, **pkw)
    assert state.flags & ~sv.F_OUT_OF_BOX == 0, state.flags
    ref = oracle_density(orc, w, kernel=Q)
    assert np.all(ref["converged"] == 1)
    wd = check_density(dens, ref, tol=1e-12)
    assert state.pairs_density == int(ref["count"].sum())
    rf = oracle_force(orc, w, dens, kernel=Q)
    wf = check_force(out, rf, tol=1e-12, vsig_tol=1e-14)
    assert state.pairs_force == int(rf["count"].sum())
    dt = orc.time_step(dens[:, S["h"]], rf["vsig"], inputs.CFL)
    assert abs(state.dt / dt - 1) < 1e-14
    print(name, "density", wd, "force", wf, flush=True)


def test_quartic_differs_from_cubic(orc):
    w = inputs.two_state_tube(16, 7)
    d3, _ = run_density(w)
    d5, _ = run_density(w, kernel=Q)
    r3, r5 = d3[:, S["rho"]], d5[:, S["rho"]]
    assert np.all(np.abs(r5 / r3 - 1.0) > 0.0)
    check_density(d3, oracle_density(orc, w), tol=1e-12)


LAYOUTS = {
    "soa": sv.layout(sv.LAYOUT_SOA),
    "aosoa8": sv.layout(sv.LAYOUT_AOSOA, 8),
    "direct": sv.layout(sv.LAYOUT_DIRECT),
    "aosoa8_masked": sv.layout(sv.LAYOUT_AOSOA, 8, masked=1),
    "direct_masked": sv.layout(sv.LAYOUT_DIRECT, masked=1),
}


@pytest.mark.parametrize("precision", [sv.PREC_FP64, sv.PREC_FP32])
def test_quartic_layouts_and_masking_bit_identical(precision):
    w = inputs.two_state_tube(16, 11)
    tol = 1e-6 if precision == sv.PREC_FP32 else None
    res = {}
    for name, lay in LAYOUTS.items():
        print(f"[quartic layout] {name} prec={precision}", flush=True)
        _, out, state = run_density_force(w, precision=precision, lay=lay, tol=tol, kernel=Q)
        assert state.flags == 0
        res[name] = (out, state.dt, tuple(state.sums))
    ref = res["soa"]
    for name, (out, dt, sums) in res.items():
        assert np.array_equal(bits(out), bits(ref[0])), name
        assert dt == ref[1] and sums == ref[2], name


def test_quartic_fp32_form_within_budget(orc):
    w = inputs.kelvin_helmholtz(24, 9)
    dens, out, state = run_density_force(w, precision=sv.PREC_FP32, tol=1e-6, kernel=Q)
    assert state.flags == 0
    wd = check_density(dens, oracle_density(orc, w, kernel=Q), tol=1e-5)
    wf = check_force(out, oracle_force(orc, w, dens, kernel=Q), tol=1e-4, vsig_tol=1e-6)
    print("quartic fp32 density", wd, "force", wf, flush=True)


def test_quartic_step_kick_bit_exact(orc):
    w = inputs.config1()
    st = sv.Stepper(w.rec, sv.params_for(w, kernel=Q))
    st.build()
    st.density()
    dens = st.records()
    check_density(dens, oracle_density(orc, w, kernel=Q), tol=1e-12)
    st.force()
    before = st.records()
    check_force(before, oracle_force(orc, w, dens, kernel=Q), tol=1e-12, vsig_tol=1e-14)
    state = st.read_state()
    assert state.flags == 0, state.flags
    st.kick()
    after = st.records()
    st.close()
    ref = before.copy()
    orc.kick_drift(ref, S, state.dt, 0.0, True, w.lo, w.length, w.periodic)
    assert np.array_equal(bits(ref), bits(after))


def test_quartic_full_tube_sampled_parity(orc):
    """The 294,912-particle two-state tube with the benchmark's default launch
    configuration: every output of 400 sampled particles against the oracle."""
    w = inputs.config2()
    st = sv.Stepper(w.rec, sv.params_for(w, kernel=Q))
    st.build()
    st.density()
    dens = st.records()
    st.force()
    out = st.records()
    state = st.read_state()
    st.close()
    assert state.flags & ~sv.F_OUT_OF_BOX == 0, state.flags
    idx = np.sort(np.random.default_rng(3).choice(w.n, size=400, replace=False))
    wd = check_density(dens, oracle_density(orc, w, targets=idx, kernel=Q), idx=idx, tol=1e-12)
    wf = check_force(out, oracle_force(orc, w, dens, targets=idx, kernel=Q), idx=idx, tol=1e-12,
                     vsig_tol=1e-14)
    print("quartic tube64 density", wd, "force", wf, flush=True)


def test_quartic_full_kh128_sampled_parity(orc):
    """The 128^3 Kelvin-Helmholtz shear layer (2,097,152 particles) with the
    quartic kernel: every output of 400 sampled particles against the oracle."""
    w = inputs.config3()
    st = sv.Stepper(w.rec, sv.params_for(w, kernel=Q))
    st.build()
    st.density()
    dens = st.records()
    st.force()
    out = st.records()
    state = st.read_state()
    st.close()
    assert state.flags & ~sv.F_OUT_OF_BOX == 0, state.flags
    idx = np.sort(np.random.default_rng(4).choice(w.n, size=400, replace=False))
    wd = check_density(dens, oracle_density(orc, w, targets=idx, kernel=Q), idx=idx, tol=1e-12)
    wf = check_force(out, oracle_force(orc, w, dens, targets=idx, kernel=Q), idx=idx, tol=1e-12,
                     vsig_tol=1e-14)
    print("quartic kh128 density", wd, "force", wf, flush=True)
