"""Symmetric force evaluation (sphv_params.symmetric = 1 with list walks):
each pair evaluated once, its partner's side stored in the partner's slot and
added in a fixed order.  Against the oracle, bit-identical on reruns and in
graph replay, equal to the twice-evaluated list walk to rounding, the
overflow fallback against the oracle, FP32 refused."""
import numpy as np
import pytest

from paper_2502_16517_amd import inputs
from paper_2502_16517_amd import sphview as sv

from gpu_helpers import S, bits, check_density, check_force, oracle_force, run_density_force

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CAP = 128

SMALL = {
    "lattice16": (lambda: inputs.config1(), {}),
    "tube16": (lambda: inputs.two_state_tube(16, 7), {}),
    "kh24": (lambda: inputs.kelvin_helmholtz(24, 9), {}),
    "plummer8k": (lambda: inputs.plummer(8192, 5, cell=0.1), {"headroom": 1.6}),
}


@pytest.mark.parametrize("name", list(SMALL))
def test_symmetric_force_matches_oracle(orc, name):
    print(f"[symmetric] {name}", flush=True)
    mk, pkw = SMALL[name]
    w = mk()
    dens, out, state = run_density_force(w, list_cap=CAP, symmetric=1, **pkw)
    assert state.flags & ~sv.F_OUT_OF_BOX == 0, state.flags
    ref = oracle_force(orc, w, dens)
    print(check_force(out, ref, tol=1e-12, vsig_tol=1e-14))
    assert state.pairs_force == int(ref["count"].sum())
    dt = orc.time_step(dens[:, S["h"]], ref["vsig"], inputs.CFL)
    assert abs(state.dt / dt - 1) < 1e-14


def test_symmetric_quartic_matches_oracle(orc):
    w = inputs.kelvin_helmholtz(24, 9)
    dens, out, state = run_density_force(w, list_cap=CAP, symmetric=1, kernel=sv.KERNEL_QUARTIC)
    assert state.flags == 0
    check_force(out, oracle_force(orc, w, dens, kernel=sv.KERNEL_QUARTIC), tol=1e-12, vsig_tol=1e-14)


def test_symmetric_rerun_bit_identical_and_close_to_twice(orc):
    w = inputs.two_state_tube(16, 7)
    _, a, sa = run_density_force(w, list_cap=CAP, symmetric=1)
    _, b, sb = run_density_force(w, list_cap=CAP, symmetric=1)
    assert np.array_equal(bits(a), bits(b))
    assert sa.dt == sb.dt and tuple(sa.sums) == tuple(sb.sums)
    _, c, sc = run_density_force(w, list_cap=CAP)
    assert sc.pairs_force == sa.pairs_force
    ref = oracle_force(orc, w, a)
    scale = ref["sa"]
    for k in ("ax", "ay", "az"):
        assert np.max(np.abs(a[:, S[k]] - c[:, S[k]]) / scale) < 1e-12, k
    assert np.array_equal(a[:, S["v_sig"]], c[:, S["v_sig"]])


def test_symmetric_overflow_falls_back_and_matches_oracle(orc):
    """Lists too short for most particles: every particle's pairs are
    evaluated from its window (twice per pair), still against the oracle."""
    w = inputs.config1()
    dens, out, state = run_density_force(w, list_cap=16, symmetric=1)
    assert state.flags == 0
    check_force(out, oracle_force(orc, w, dens), tol=1e-12, vsig_tol=1e-14)


def test_symmetric_step_conserves_momentum_and_replays():
    """Five steps replayed from one captured graph give the eager bits; the
    total force sum m a stays at roundoff of sum m |a|."""
    # a tube whose h stays inside its cells' reach over the steps (with other
    # jitter seeds one interface particle's h meets its cap in the first step)
    w = inputs.two_state_tube(24, 7)
    p = sv.params_for(w, list_cap=CAP, symmetric=1)
    sa = torch.cuda.Stream()
    a = sv.Stepper(w.rec, p, stream=sa)
    for k in range(5):
        a.step()
        s = a.read_state()
        assert s.flags == 0, (k, s.flags)
    ra, sta = a.records(), a.read_state()
    a.close()
    m = ra[:, S["m"]]
    scale = float(np.sum(m * np.sqrt(sum(ra[:, S[k]] ** 2 for k in ("ax", "ay", "az")))))
    assert max(abs(sta.sums[4 + k]) for k in range(3)) <= 1e-13 * scale
    sb = torch.cuda.Stream()
    b = sv.Stepper(w.rec, p, stream=sb)
    sv.graph_begin(sb)
    b.step()
    g = sv.graph_end(sb)
    junk = torch.zeros(1 << 16, device="cuda")
    for _ in range(5):
        sv.graph_launch(g, sb)
        junk.add_(1.0)
        torch.cuda.synchronize()
    rb, stb = b.records(), b.read_state()
    sv.graph_destroy(g)
    b.close()
    assert np.array_equal(bits(ra), bits(rb))
    assert sta.dt == stb.dt and tuple(sta.sums) == tuple(stb.sums)


def test_symmetric_refuses_fp32():
    w = inputs.config1()
    p = sv.params_for(w, list_cap=CAP, symmetric=1, h_tol=1e-6)
    st = sv.Stepper(w.rec, p, sv.PREC_FP32)
    st.build()
    st.density()
    with pytest.raises(sv.SphvError) as e:
        st.force()
    assert e.value.status == sv.E_UNSUPPORTED
    st.close()
